"""Seeded synthetic inputs: workload definitions and initial states.

This module serves both the HIP path and the oracle-based tests.  It holds no
arithmetic of the method itself (no fluxes, no DG operators): it only evaluates
initial conditions at node coordinates it is given and converts primitive to
conserved variables, so a state can be handed to either side.  Every random
number comes from ``numpy.random.default_rng`` with a stated seed.

State layout: ``u[var][elem][node]`` float64 with var = (rho, rho v_1..rho v_d, rho E).
Coordinates: ``xyz[d][elem][node]`` as produced by either side's node-coordinate call.
"""
import math

import numpy as np

GAMMA = 1.4


def _xp(a):
    """NumPy, or torch for torch tensors (the same formulas evaluated where the data lives)."""
    if type(a).__module__.startswith("torch"):
        import torch
        return torch
    return np


def prim_to_cons(rho, vel, p, gamma=GAMMA):
    """(rho, [v_1..v_d], p) -> u = (rho, rho v, p/(gamma-1) + rho |v|^2 / 2)."""
    xp = _xp(rho)
    if xp is np:
        rho = np.asarray(rho, dtype=np.float64)
        vel = [np.broadcast_to(np.asarray(v, dtype=np.float64), rho.shape) for v in vel]
        p = np.broadcast_to(np.asarray(p, dtype=np.float64), rho.shape)
    else:
        vel = [v if _xp(v) is xp else xp.full_like(rho, float(v)) for v in vel]
        p = p if _xp(p) is xp else xp.full_like(rho, float(p))
    v2 = sum(v * v for v in vel)
    return xp.stack([rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + 0.5 * rho * v2])


# --------------------------------------------------------------------------- workloads
def workload(name):
    """Solver configuration of a named workload (keyword arguments for either side)."""
    pi = math.pi
    if name == "density_wave_2d":   # 2D, N=3, 16^2 on [-2,2]^2, EC volume + LLF
        return dict(dim=2, polydeg=3, cells=(16, 16, 1), xmin=(-2.0, -2.0, 0.0),
                    xmax=(2.0, 2.0, 1.0), gamma=GAMMA, volume="ec", surface="llf")
    if name == "tgv_32":            # 3D, N=3, 32^3 on [-pi,pi]^3, EC + LLF
        return dict(dim=3, polydeg=3, cells=(32, 32, 32), xmin=(-pi,) * 3, xmax=(pi,) * 3,
                    gamma=GAMMA, volume="ec", surface="llf")
    if name == "sedov_32":          # 3D, N=3, 32^3 on [-1,1]^3, HG shock capturing
        return dict(dim=3, polydeg=3, cells=(32, 32, 32), xmin=(-1.0,) * 3, xmax=(1.0,) * 3,
                    gamma=GAMMA, volume="shockcap_hg", surface="llf", fv_flux="llf",
                    alpha_max=0.5, alpha_min=0.001, alpha_smooth=True)
    if name in ("curved_4", "curved_32"):   # the PID study's warped box (Eq. (2)), MMS source
        return dict(polydeg=3, cells=4 if name == "curved_4" else 32, warp=0.15, gamma=GAMMA,
                    volume="ec", surface="llf", source="mms")
    if name in ("alfven_4", "alfven_32"):   # ideal MHD, weak form + HLL, N = 3
        return dict(polydeg=3, cells=4 if name == "alfven_4" else 32, gamma=5.0 / 3.0,
                    surface="hll")
    if name == "tgv_64_mixed":      # mixed precision, N=3 on 64^3
        return dict(dim=3, polydeg=3, cells=(64, 64, 64), xmin=(-pi,) * 3, xmax=(pi,) * 3,
                    gamma=GAMMA, volume="ec", surface="llf", precision="mixed")
    if name == "tgv_n7_32_mixed":   # mixed precision, N=7 on 32^3
        return dict(dim=3, polydeg=7, cells=(32, 32, 32), xmin=(-pi,) * 3, xmax=(pi,) * 3,
                    gamma=GAMMA, volume="ec", surface="llf", precision="mixed")
    raise KeyError(name)


def scaled(cfg, cells=None, polydeg=None, **over):
    """Copy of a workload configuration with a different grid or degree."""
    c = dict(cfg)
    if cells is not None:
        c["cells"] = tuple(cells) + (1,) * (3 - len(cells))
    if polydeg is not None:
        c["polydeg"] = polydeg
    c.update(over)
    return c


# --------------------------------------------------------------------------- initial states
def density_wave(xyz, gamma=GAMMA, t=0.0):
    """rho = 2 + 0.1 sin(pi (x + y - 2t)), v = (1, 1), p = 10 (2D; exact solution at time t)."""
    x, y = xyz[0], xyz[1]
    rho = 2.0 + 0.1 * np.sin(np.pi * (x + y - 2.0 * t))
    return prim_to_cons(rho, [1.0, 1.0], 10.0, gamma)


def tgv_perturbation_modes(seed=2108, nmodes=8):
    """Random smooth density perturbation: wave vectors k_m in {-2..2}^3 minus 0,
    amplitudes a_m ~ U(0,1), phases phi_m ~ U(0, 2 pi), drawn in that order."""
    rng = np.random.default_rng(seed)
    ks = []
    while len(ks) < nmodes:
        k = rng.integers(-2, 3, size=3)
        if np.any(k != 0):
            ks.append(k)
    a = rng.uniform(0.0, 1.0, nmodes)
    phi = rng.uniform(0.0, 2.0 * np.pi, nmodes)
    return np.array(ks, dtype=np.float64), a, phi


def tgv(xyz, gamma=GAMMA, mach=0.1, perturb_seed=2108, perturb_amp=0.01, shift=(0.0, 0.0, 0.0)):
    """Taylor-Green vortex, rho0 = V0 = 1: v = (sin x cos y cos z, -cos x sin y cos z, 0),
    p = 1/(gamma Ma^2) + (cos 2x + cos 2y)(cos 2z + 2)/16, optionally with
    rho <- rho (1 + amp * g / sum a_m), g = sum_m a_m sin(k_m . x + phi_m)."""
    xp = _xp(xyz)
    x, y, z = (xyz[0] + shift[0], xyz[1] + shift[1], xyz[2] + shift[2])
    rho = xp.ones_like(x)
    v1 = xp.sin(x) * xp.cos(y) * xp.cos(z)
    v2 = -xp.cos(x) * xp.sin(y) * xp.cos(z)
    v3 = xp.zeros_like(x)
    p = 1.0 / (gamma * mach * mach) + (xp.cos(2 * x) + xp.cos(2 * y)) * (xp.cos(2 * z) + 2.0) / 16.0
    if perturb_seed is not None and perturb_amp != 0.0:
        ks, a, phi = tgv_perturbation_modes(perturb_seed)
        g = xp.zeros_like(x)
        for m in range(len(a)):
            g += float(a[m]) * xp.sin(float(ks[m, 0]) * x + float(ks[m, 1]) * y +
                                      float(ks[m, 2]) * z + float(phi[m]))
        rho = rho * (1.0 + perturb_amp * g / float(a.sum()))
    return prim_to_cons(rho, [v1, v2, v3], p, gamma)


def sedov(xyz, gamma=GAMMA, sigma=0.25, E0=1.0, p_amb=1.0e-5):
    """rho = 1, v = 0, p = p_amb + (gamma-1) E0 exp(-r^2/(2 sigma^2)) / ((2 pi)^(3/2) sigma^3)."""
    r2 = sum(xyz[d] ** 2 for d in range(len(xyz)))
    dim = len(xyz)
    p = p_amb + (gamma - 1.0) * E0 * np.exp(-r2 / (2 * sigma ** 2)) / ((2 * np.pi) ** 1.5 * sigma ** 3)
    rho = np.ones_like(r2)
    return prim_to_cons(rho, [np.zeros_like(r2)] * dim, p, gamma)


def mms(xyz, t=0.0):
    """Manufactured solution of the curvilinear workload: rho = 2 + 0.1 sin(pi (x+y+z) - 2 pi t),
    v = (1, 1, 1), rho E = rho^2 (3D; numpy or torch coordinates)."""
    xp = _xp(xyz)
    rho = 2.0 + 0.1 * xp.sin(math.pi * (xyz[0] + xyz[1] + xyz[2]) - 2.0 * math.pi * t)
    return xp.stack([rho, rho, rho, rho, rho * rho])


def alfven(xyz, t=0.0, gamma=5.0 / 3.0):
    """Circularly polarised Alfven wave (ideal MHD, 8 variables) along e1 = (1,1,1)/sqrt 3
    with wave vector pi (1,1,1): rho = 1, p = 0.1, B = e1 + 0.1 (cos phi e2 + sin phi e3),
    v = -0.1 (cos phi e2 + sin phi e3), phi = pi (x+y+z) - pi sqrt(3) t, e2 = (1,-1,0)/sqrt 2,
    e3 = e1 x e2 (numpy or torch coordinates)."""
    xp = _xp(xyz)
    r3, r2, r6 = math.sqrt(3.0), math.sqrt(2.0), math.sqrt(6.0)
    e1 = (1 / r3, 1 / r3, 1 / r3)
    e2 = (1 / r2, -1 / r2, 0.0)
    e3 = (1 / r6, 1 / r6, -2 / r6)
    phi = math.pi * (xyz[0] + xyz[1] + xyz[2]) - math.pi * r3 * t
    c, s = xp.cos(phi), xp.sin(phi)
    B = [e1[k] + 0.1 * (c * e2[k] + s * e3[k]) for k in range(3)]
    v = [-0.1 * (c * e2[k] + s * e3[k]) for k in range(3)]
    rho = xp.ones_like(c)
    E = 0.1 / (gamma - 1.0) + 0.5 * sum(vk * vk for vk in v) + 0.5 * sum(Bk * Bk for Bk in B)
    return xp.stack([rho] + v + [E] + B)


def random_smooth(xyz, seed, amp=0.2, vamp=0.5, nmodes=4, periods=None):
    """Random smooth periodic state: rho, p = 1 + amp * g, v_d = vamp * g with independent
    random Fourier sums g (|g| <= 1).  ``periods`` = domain length per direction."""
    rng = np.random.default_rng(seed)
    dim = len(xyz)
    if periods is None:
        periods = [2.0 * np.pi] * dim

    def field():
        g = np.zeros_like(xyz[0])
        amps = rng.uniform(0.2, 1.0, nmodes)
        for m in range(nmodes):
            k = rng.integers(-2, 3, size=dim)
            ph = rng.uniform(0, 2 * np.pi)
            arg = sum(2 * np.pi * k[d] / periods[d] * xyz[d] for d in range(dim))
            g += amps[m] * np.sin(arg + ph)
        return g / amps.sum()

    rho = 1.0 + amp * field()
    vel = [vamp * field() for _ in range(dim)]
    p = 1.0 + amp * field()
    return prim_to_cons(rho, vel, p)


def random_nodal(shape_nodes, dim, seed, rho_range=(0.5, 1.5), p_range=(0.5, 1.5), vamp=1.0,
                 gamma=GAMMA):
    """Non-smooth random state: independent uniform rho, p and v at every node.  Neighbour
    ratios up to 3 put z^2 = ((b - a)/(b + a))^2 across [0, 0.25), so every branch of the
    logarithmic mean (near-equal series, longer series, logarithm) and both signs of every
    wave speed occur."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(*rho_range, size=shape_nodes)
    p = rng.uniform(*p_range, size=shape_nodes)
    vel = [rng.uniform(-vamp, vamp, size=shape_nodes) for _ in range(dim)]
    return prim_to_cons(rho, vel, p, gamma)


def constant_state(shape_nodes, dim, rho=1.3, vel=(0.3, -0.2, 0.1), p=2.1, gamma=GAMMA):
    return prim_to_cons(np.full(shape_nodes, rho), list(vel[:dim]), p, gamma)


# --------------------------------------------------------------------------- ensemble
def ensemble(nruns=256, seed=2109):
    """Ensemble of independent 3D TGV runs: per run K in {8,12,16,24}, N in {3,4,5}
    (uniform), Mach ~ U(0.05, 0.3), phase shift ~ U(0, 2 pi)^3; drawn per run in that
    order from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    runs = []
    for _ in range(nruns):
        K = int(rng.choice([8, 12, 16, 24]))
        N = int(rng.choice([3, 4, 5]))
        mach = float(rng.uniform(0.05, 0.3))
        shift = tuple(float(s) for s in rng.uniform(0.0, 2 * np.pi, 3))
        runs.append(dict(K=K, N=N, mach=mach, shift=shift))
    return runs


def ensemble_config(run):
    pi = math.pi
    return dict(dim=3, polydeg=run["N"], cells=(run["K"],) * 3, xmin=(-pi,) * 3, xmax=(pi,) * 3,
                gamma=GAMMA, volume="ec", surface="llf")


def ensemble_state(run, xyz, gamma=GAMMA):
    return tgv(xyz, gamma, mach=run["mach"], perturb_seed=None, shift=run["shift"])
