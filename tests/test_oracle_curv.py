"""Pins of the curvilinear oracle (the warped periodic box of the PID study, Section 3.1,
Eq. (2); manufactured solution with source terms): geometry identities, free-stream
preservation, reduction to the Cartesian oracle, conservation, entropy conservation, the
source term against symbolic differentiation, and the convergence order."""
import numpy as np
import pytest
import sympy as sp

import oracle
from paper_2108_06476_amd import inputs


def _D(N):
    return oracle.lgl(N)[2]


def _deriv(f, D, j, n):
    """Derivative along element direction j of nodal data f[..., node] (node = i + n j + n^2 k)."""
    g = f.reshape(f.shape[:-1] + (n, n, n))          # [..., k, j, i]
    axis = {0: -1, 1: -2, 2: -3}[j]
    return np.moveaxis(np.tensordot(D, np.moveaxis(g, axis, 0), axes=(1, 0)), 0, axis).reshape(f.shape)


def test_map_fixes_box_faces_and_is_identity_without_warp():
    rng = np.random.default_rng(1)
    for _ in range(50):
        p = rng.uniform(-1, 1, 3)
        np.testing.assert_array_equal(oracle.curv_map(p, warp=0.0), p)
        for d in range(3):
            q = p.copy()
            q[d] = rng.choice([-1.0, 1.0])
            x = oracle.curv_map(q, warp=0.15)
            assert abs(x[d] - q[d]) <= 1e-15         # a box face stays on itself


def test_affine_geometry():
    o = oracle.CurvOracle(3, 4, warp=0.0, source="none")
    _, Ja, J = o.geometry()
    h2 = 0.5 * (2.0 / 4)
    np.testing.assert_allclose(J, h2 ** 3, rtol=5e-14)   # D applied to O(1) coordinates
    for i in range(3):
        for n in range(3):
            np.testing.assert_allclose(Ja[i, n], h2 ** 2 if i == n else 0.0, atol=5e-15)


@pytest.mark.parametrize("N", [2, 3, 5])
def test_discrete_metric_identities(N):
    """sum_i d/ds_i (J a^i)_n = 0 node by node: what makes a constant state stay constant."""
    o = oracle.CurvOracle(N, 2, warp=0.15, source="none")
    _, Ja, J = o.geometry()
    D = _D(N)
    for n in range(3):
        div = sum(_deriv(Ja[i, n], D, i, N + 1) for i in range(3))
        assert np.abs(div).max() <= 1e-13 * np.abs(Ja).max(), (n, np.abs(div).max())


def test_watertight_faces():
    """Coincident face nodes of neighbouring elements share position and contravariant vector."""
    N, K = 3, 3
    n = N + 1
    o = oracle.CurvOracle(N, K, warp=0.15, source="none")
    xyz, Ja, _ = o.geometry()
    X = xyz.reshape(3, K, K, K, n, n, n)            # [c][ez][ey][ex][k][j][i]
    A = Ja.reshape(3, 3, K, K, K, n, n, n)
    # x faces: element ex's i = N face against element ex+1's i = 0 face (interior faces)
    np.testing.assert_allclose(X[:, :, :, :-1, :, :, -1], X[:, :, :, 1:, :, :, 0], atol=1e-15)
    np.testing.assert_allclose(A[0, :, :, :, :-1, :, :, -1], A[0, :, :, :, 1:, :, :, 0], atol=1e-14)
    np.testing.assert_allclose(A[1, :, :, :-1, :, :, -1, :], A[1, :, :, 1:, :, :, 0, :], atol=1e-14)
    np.testing.assert_allclose(A[2, :, :-1, :, :, -1, :, :], A[2, :, 1:, :, :, 0, :, :], atol=1e-14)
    # periodic: the x = -1 and x = +1 faces match too
    np.testing.assert_allclose(A[0, :, :, :, -1, :, :, -1], A[0, :, :, :, 0, :, :, 0], atol=1e-14)


def test_jacobian_positive_and_volume():
    N, K = 5, 4
    o = oracle.CurvOracle(N, K, warp=0.15, source="none")
    _, _, J = o.geometry()
    assert J.min() > 0.0
    w = oracle.lgl(N)[1]
    W = np.einsum("i,j,k->kji", w, w, w).reshape(-1)
    vol = float((J * W[None, :]).sum())
    assert abs(vol - 8.0) <= 1e-4, vol                 # the box [-1,1]^3 keeps its volume


@pytest.mark.parametrize("N", [2, 3, 4])
@pytest.mark.parametrize("vol,surf", [("ec", "llf"), ("ec", "ec"), ("central", "hll"),
                                      ("ec", "hll")])
def test_free_stream_preservation(N, vol, surf):
    o = oracle.CurvOracle(N, 2, warp=0.15, volume=vol, surface=surf, source="none")
    u = inputs.constant_state((o.E, o.NN), 3)
    R = o.rhs(u)
    _, _, J = o.geometry()
    scale = 10.0 / J.min()                               # flux scale (|f| < 10) times 1/J
    assert np.abs(R).max() <= 1e-13 * scale, np.abs(R).max()


@pytest.mark.parametrize("vol,surf", [("ec", "llf"), ("central", "hll"), ("ec", "ec")])
def test_without_warp_equals_cartesian_oracle(vol, surf):
    N, K = 3, 3
    o = oracle.CurvOracle(N, K, warp=0.0, volume=vol, surface=surf, source="none")
    c = oracle.Oracle(dim=3, polydeg=N, cells=(K, K, K), xmin=(-1,) * 3, xmax=(1,) * 3,
                      volume=vol, surface=surf)
    u = inputs.random_smooth(c.node_coords(), 11, periods=[2.0] * 3)
    a, b = o.rhs(u), c.rhs(u)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    np.testing.assert_allclose(o.max_dt(u, 0.5), c.max_dt(u, 0.5), rtol=1e-14)


def _smooth_on(o, seed):
    xyz, _, _ = o.geometry()
    return inputs.random_smooth(xyz, seed, periods=[2.0] * 3)


def test_conservation_on_warped_mesh():
    o = oracle.CurvOracle(3, 3, warp=0.15, volume="ec", surface="llf", source="none")
    u = _smooth_on(o, 5)
    R = o.rhs(u)
    _, _, J = o.geometry()
    w = oracle.lgl(3)[1]
    W = np.einsum("i,j,k->kji", w, w, w).reshape(-1)
    tot = (R * J[None] * W[None, None]).sum(axis=(1, 2))
    scale = (np.abs(R) * J[None] * W[None, None]).sum(axis=(1, 2))
    assert np.all(np.abs(tot) <= 1e-13 * scale), tot / scale


def test_entropy_on_warped_mesh():
    """EC volume + EC surface conserve entropy (rate 0 to roundoff); LLF dissipates it."""
    o = oracle.CurvOracle(3, 3, warp=0.15, volume="ec", surface="ec", source="none")
    ol = oracle.CurvOracle(3, 3, warp=0.15, volume="ec", surface="llf", source="none")
    # independent random states per node: jumps at every interface (smooth data is
    # continuous at the shared face nodes, where LLF then dissipates nothing)
    u = inputs.random_nodal((o.E, o.NN), 3, seed=9)
    _, _, J = o.geometry()
    w = oracle.lgl(3)[1]
    W = np.einsum("i,j,k->kji", w, w, w).reshape(-1)
    wv = np.stack([oracle.entropy_vars(u[:, e, i]) for e in range(o.E) for i in range(o.NN)],
                  axis=1).reshape(5, o.E, o.NN)
    for orc, sign in [(o, 0), (ol, -1)]:
        R = orc.rhs(u)
        rate = float((wv * R * J[None] * W[None, None]).sum())
        scale = float((np.abs(wv * R) * J[None] * W[None, None]).sum())
        if sign == 0:
            assert abs(rate) <= 1e-12 * scale, rate / scale
        else:
            assert rate < 0.0, rate


def test_mms_source_matches_symbolic_differentiation():
    """s = du/dt + div f(u) of the manufactured solution, by sympy from its definition."""
    x, y, z, t = sp.symbols("x y z t", real=True)
    g = sp.Rational(7, 5)
    rho = 2 + sp.Rational(1, 10) * sp.sin(sp.pi * (x + y + z) - 2 * sp.pi * t)
    v = [1, 1, 1]
    rhoE = rho ** 2
    p = (g - 1) * (rhoE - rho * sum(vi * vi for vi in v) / 2)
    u = [rho, rho * v[0], rho * v[1], rho * v[2], rhoE]
    X = [x, y, z]
    F = [[rho * v[d], rho * v[d] * v[0] + (p if d == 0 else 0), rho * v[d] * v[1] + (p if d == 1 else 0),
          rho * v[d] * v[2] + (p if d == 2 else 0), v[d] * (rhoE + p)] for d in range(3)]
    src = [sp.diff(u[k], t) + sum(sp.diff(F[d][k], X[d]) for d in range(3)) for k in range(5)]
    f_u = sp.lambdify((x, y, z, t), u, "numpy")
    f_s = sp.lambdify((x, y, z, t), src, "numpy")
    rng = np.random.default_rng(3)
    for _ in range(40):
        P = rng.uniform(-1, 1, 3)
        tt = rng.uniform(0, 2)
        uo, so = oracle.curv_mms(P, tt)
        np.testing.assert_allclose(uo, np.array(f_u(*P, tt), dtype=float), rtol=1e-15, atol=1e-15)
        np.testing.assert_allclose(so, np.array(f_s(*P, tt), dtype=float), rtol=1e-13, atol=1e-13)


def _mms_error(K, N, warp, T=0.1):
    o = oracle.CurvOracle(N, K, warp=warp, volume="ec", surface="llf", source="mms")
    u = o.initial(0.0)
    nst = int(np.ceil(T / o.max_dt(u, 0.5)))
    u1, t = o.step(u, nst, cfl=0.0, dt_fixed=T / nst)
    _, _, J = o.geometry()
    w = oracle.lgl(N)[1]
    W = np.einsum("i,j,k->kji", w, w, w).reshape(-1)
    return np.sqrt(((u1 - o.initial(t)) ** 2 * J[None] * W[None, None]).sum(axis=(1, 2)) / 8)


@pytest.mark.parametrize("warp", [0.0, 0.05])
def test_mms_convergence(warp):
    """EC volume + LLF surface, N = 3: L2 error of the manufactured solution at t = 0.1 on
    K = 4 and 8; the observed order approaches N + 1 (3.7-4.0 measured; >= 3.5 asserted).
    (The paper's amplitude 0.15 is still pre-asymptotic at these sizes: 3.0-3.3 at K = 16.)"""
    e4, e8 = _mms_error(4, 3, warp), _mms_error(8, 3, warp)
    eoc = np.log2(e4 / e8)
    print("EOC", eoc, flush=True)
    assert np.all(eoc >= 3.5), eoc
