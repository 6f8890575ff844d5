"""Helpers of the GPU parity tests: device transfer and the flux-scale error norm.

Parity norm per field v (float64):
    err_v = max_n |R_gpu_v - R_orc_v| / ((2/h) max_{n,d} |f^d_v(u_n)|),
the difference relative to the scale of the flux terms that the right-hand side sums.  Only
for a field whose flux scale is exactly zero (a state at rest: the mass and energy fluxes of
the blast-wave initial state vanish) the scale is lambda_max max_n |u_v,n| instead
(lambda_max = max |v_d| + c): the terms that remain are then the dissipation terms
lambda (u_R - u_L)/2 of the LLF/HLL interface and subcell fluxes.
Two correct float64 evaluations that only differ in summation order, FMA contraction or an
algebraically equivalent log-mean form differ at the 1e-15 level in this norm; the bar is
1e-12.

State norm after time steps: max_n |u_gpu_v - u_orc_v| / max_n |u_orc_v|, where the three
momentum components share one denominator (the largest of the three: a component can start
at zero), also bounded by 1e-12.
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


def err_scale(u, dim, h, gamma=1.4):
    """(2/h) max_{n,d} |f^d_v| per field; (2/h) lambda_max max |u_v| where that is zero."""
    fs = phys_flux_max(u, dim, gamma)
    return (2.0 / h) * np.where(fs > 0.0, fs, dissipation_max(u, dim, gamma))


def err_v(R_gpu, R_orc, u, dim, h, gamma=1.4):
    d = np.abs(np.asarray(R_gpu) - np.asarray(R_orc)).reshape(dim + 2, -1).max(axis=1)
    return d / err_scale(u, dim, h, gamma)


def state_err(u_gpu, u_orc, dim):
    """Per-field state difference after steps: max |du_v| / max |u_v|, the momentum
    components against the largest momentum magnitude."""
    a = np.asarray(u_gpu).reshape(dim + 2, -1)
    b = np.asarray(u_orc).reshape(dim + 2, -1)
    d = np.abs(a - b).max(axis=1)
    m = np.abs(b).max(axis=1)
    m[1:1 + dim] = m[1:1 + dim].max()
    return d / np.maximum(m, 1e-300)


def rel_to_max(a, b):
    """max |a - b| / max |b| per variable (reported for information)."""
    d = np.abs(a - b).reshape(a.shape[0], -1).max(axis=1)
    return d / np.maximum(np.abs(b).reshape(b.shape[0], -1).max(axis=1), 1e-300)
