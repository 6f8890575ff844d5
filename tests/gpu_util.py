"""Helpers of the GPU parity tests: device transfer and the flux-scale error norm.

Parity norm per field v (float64):
    err_v = max_n |R_gpu_v - R_orc_v| / ((2/h) max(max_{n,d} |f^d_v(u_n)|, lambda_max max_n |u_v,n|)),
i.e. the difference relative to the scale of the terms that the right-hand side sums: the
physical fluxes, and the dissipation terms lambda (u_R - u_L)/2 of the LLF/HLL interface and
subcell fluxes (lambda_max = max |v_d| + c).  The second term matters where v = 0 makes
the mass and energy fluxes vanish (a blast wave at rest).
Two correct float64 evaluations that only differ in summation order, FMA contraction or an
algebraically equivalent log-mean form differ at the 1e-15 level in this norm; the bar is
1e-12.
"""
import numpy as np
import torch

TOL_FP64 = 1e-12


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def phys_flux_max(u, dim, gamma=1.4):
    """max over nodes and directions of |f^d_v(u)| per variable v (u: [nvar, ...])."""
    uu = u.reshape(dim + 2, -1)
    rho = uu[0]
    v = uu[1:1 + dim] / rho
    p = (gamma - 1) * (uu[dim + 1] - 0.5 * rho * (v * v).sum(0))
    out = np.zeros(dim + 2)
    for d in range(dim):
        f = [uu[1 + d]] + [uu[1 + d] * v[k] + (p if k == d else 0.0) for k in range(dim)] + \
            [v[d] * (uu[dim + 1] + p)]
        out = np.maximum(out, np.array([np.max(np.abs(x)) for x in f]))
    return out


def dissipation_max(u, dim, gamma=1.4):
    """lambda_max * max |u_v| per variable."""
    uu = u.reshape(dim + 2, -1)
    rho = uu[0]
    v = uu[1:1 + dim] / rho
    p = (gamma - 1) * (uu[dim + 1] - 0.5 * rho * (v * v).sum(0))
    lam = np.max(np.abs(v).max(axis=0) + np.sqrt(gamma * np.abs(p) / rho))
    return lam * np.abs(uu).max(axis=1)


def err_v(R_gpu, R_orc, u, dim, h, gamma=1.4):
    scale = (2.0 / h) * np.maximum(phys_flux_max(u, dim, gamma), dissipation_max(u, dim, gamma))
    d = np.abs(np.asarray(R_gpu) - np.asarray(R_orc)).reshape(dim + 2, -1).max(axis=1)
    return d / scale


def rel_to_max(a, b):
    """max |a - b| / max |b| per variable (reported for information)."""
    d = np.abs(a - b).reshape(a.shape[0], -1).max(axis=1)
    return d / np.maximum(np.abs(b).reshape(b.shape[0], -1).max(axis=1), 1e-300)
