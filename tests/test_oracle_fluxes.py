"""Pins of the oracle's pointwise physics: logarithmic mean, EC flux, LLF and HLL.

Checked against mpmath logarithms at 50 digits, finite differences (entropy variables are
the gradient of the entropy; the entropy flux is compatible with the Euler flux),
Tadmor's entropy-conservation condition, consistency f(u,u) = f(u), mirror symmetry and
the HLL/LLF intermediate-state (integral-form) derivation.
"""
import mpmath
import numpy as np
import pytest

import oracle
from paper_2108_06476_amd.inputs import prim_to_cons

G = 1.4
RNG = np.random.default_rng(7)


def _rand_state(dim, rng, jump=1.0):
    rho = rng.uniform(0.3, 2.0)
    p = rng.uniform(0.3, 2.0)
    v = rng.uniform(-jump, jump, dim)
    return prim_to_cons(np.array(rho), list(v), np.array(p), G).reshape(-1)


def _prim(u, dim):
    rho = u[0]
    v = u[1:1 + dim] / rho
    p = (G - 1) * (u[dim + 1] - 0.5 * rho * np.dot(v, v))
    return rho, v, p


# --------------------------------------------------------------------------- log mean
def _lnmean_mp(x, y):
    mpmath.mp.dps = 50
    X, Y = mpmath.mpf(x), mpmath.mpf(y)
    if X == Y:
        return X
    return (Y - X) / (mpmath.log(Y) - mpmath.log(X))


def test_ln_mean_against_mpmath():
    rng = np.random.default_rng(11)
    worst = 0.0
    # bound: a few ulp, plus, on the log branch, the rounding of the quotient y/x amplified
    # by 1/|ln(y/x)| (at most ~6e-15 just above the series threshold f2 = 1e-4)
    cases = [(rng.uniform(0.01, 100), rng.uniform(0.01, 100)) for _ in range(300)]
    for z in np.logspace(-12, np.log10(0.5), 200):     # zeta = (y-x)/(y+x)
        x = rng.uniform(0.1, 10)
        cases.append((x, x * (1 + z) / (1 - z)))
    for x, y in cases:
        ref = _lnmean_mp(x, y)
        got = oracle.ln_mean(x, y)
        bound = 4.5e-16 + (1.2e-16 / abs(np.log(y / x)) if x != y else 0.0)
        worst = max(worst, float(abs((mpmath.mpf(got) - ref) / ref)) / bound)
    assert worst < 1.0, worst


def test_ln_mean_identities():
    rng = np.random.default_rng(12)
    for _ in range(100):
        x, y = rng.uniform(0.1, 10, 2)
        assert oracle.ln_mean(x, x) == x
        # symmetric up to the rounding of y/x vs x/y on the log branch
        tol = 4.5e-16 + 2.4e-16 / abs(np.log(y / x))
        assert abs(oracle.ln_mean(x, y) - oracle.ln_mean(y, x)) <= tol * oracle.ln_mean(x, y)
        s = 2.0 ** rng.integers(-5, 6)   # exact scaling: homogeneous of degree one
        assert oracle.ln_mean(s * x, s * y) == s * oracle.ln_mean(x, y)
        assert min(x, y) <= oracle.ln_mean(x, y) <= max(x, y)


# --------------------------------------------------------------------------- entropy pair
@pytest.mark.parametrize("dim", [2, 3])
def test_entropy_vars_are_gradient_of_entropy(dim):
    for _ in range(20):
        u = _rand_state(dim, RNG)
        w = oracle.entropy_vars(u, dim, G)
        g = np.zeros_like(u)
        for v in range(dim + 2):
            h = 1e-6 * max(1.0, abs(u[v]))
            up, um = u.copy(), u.copy()
            up[v] += h
            um[v] -= h
            g[v] = (oracle.entropy(up, dim, G) - oracle.entropy(um, dim, G)) / (2 * h)
        np.testing.assert_allclose(w, g, rtol=1e-7, atol=1e-7)


@pytest.mark.parametrize("dim", [2, 3])
def test_entropy_flux_compatibility(dim):
    """w . df^d/du = dF^d/du with entropy flux F^d = S v_d (finite differences)."""
    for _ in range(10):
        u = _rand_state(dim, RNG)
        w = oracle.entropy_vars(u, dim, G)
        for d in range(dim):
            def F(uu):
                return oracle.entropy(uu, dim, G) * uu[1 + d] / uu[0]
            for v in range(dim + 2):
                h = 1e-6 * max(1.0, abs(u[v]))
                up, um = u.copy(), u.copy()
                up[v] += h
                um[v] -= h
                dfl = (oracle.flux_phys(up, d, dim, G) - oracle.flux_phys(um, d, dim, G)) / (2 * h)
                dF = (F(up) - F(um)) / (2 * h)
                assert abs(np.dot(w, dfl) - dF) < 1e-6 * (1 + abs(dF))


# --------------------------------------------------------------------------- EC flux
def _psi(u, d, dim):
    """entropy potential psi_d = w . f^d - F^d, from the oracle's own w, f and S."""
    w = oracle.entropy_vars(u, dim, G)
    f = oracle.flux_phys(u, d, dim, G)
    return np.dot(w, f) - oracle.entropy(u, dim, G) * u[1 + d] / u[0]


@pytest.mark.parametrize("dim", [2, 3])
def test_ec_flux_tadmor_condition(dim):
    """[[w]] . f#(uL, uR) = [[psi_d]] (Tadmor's entropy-conservation condition)."""
    rng = np.random.default_rng(21 + dim)
    worst = 0.0
    for _ in range(200):
        uL, uR = _rand_state(dim, rng), _rand_state(dim, rng)
        for d in range(dim):
            f = oracle.flux_ec(uL, uR, d, dim, G)
            wL, wR = oracle.entropy_vars(uL, dim, G), oracle.entropy_vars(uR, dim, G)
            lhs = np.dot(wR - wL, f)
            rhs = _psi(uR, d, dim) - _psi(uL, d, dim)
            scale = np.abs(wR - wL) @ np.abs(f) + 1.0
            worst = max(worst, abs(lhs - rhs) / scale)
    assert worst < 1e-14, worst


@pytest.mark.parametrize("dim", [2, 3])
def test_ec_flux_consistency_symmetry_kep(dim):
    rng = np.random.default_rng(31 + dim)
    for _ in range(100):
        u, uR = _rand_state(dim, rng), _rand_state(dim, rng)
        for d in range(dim):
            np.testing.assert_allclose(oracle.flux_ec(u, u, d, dim, G),
                                       oracle.flux_phys(u, d, dim, G), rtol=1e-15, atol=1e-15)
            np.testing.assert_allclose(oracle.flux_ec(u, uR, d, dim, G),
                                       oracle.flux_ec(uR, u, d, dim, G), rtol=1e-14, atol=1e-15)
            # kinetic-energy preservation: momentum flux = mass flux * {{v}} + {{p}} e_d
            f = oracle.flux_ec(u, uR, d, dim, G)
            rL, vL, pL = _prim(u, dim)
            rR, vR, pR = _prim(uR, dim)
            mom = f[0] * 0.5 * (vL + vR)
            mom[d] += 0.5 * (pL + pR)
            np.testing.assert_allclose(f[1:1 + dim], mom, rtol=1e-14, atol=1e-14)


def _mirror(u, d):
    m = u.copy()
    m[1 + d] = -m[1 + d]
    return m


@pytest.mark.parametrize("name", ["flux_ec", "flux_llf", "flux_hll", "flux_central"])
@pytest.mark.parametrize("dim", [2, 3])
def test_mirror_symmetry(name, dim):
    """f*(M uR, M uL) = -M f*(uL, uR) for the reflection M of the normal velocity."""
    fn = getattr(oracle, name)
    rng = np.random.default_rng(41 + dim)
    for _ in range(100):
        uL, uR = _rand_state(dim, rng, jump=3.0), _rand_state(dim, rng, jump=3.0)
        for d in range(dim):
            a = fn(_mirror(uR, d), _mirror(uL, d), d, dim, G)
            b = -_mirror(fn(uL, uR, d, dim, G), d)
            np.testing.assert_allclose(a, b, rtol=1e-14, atol=1e-14)


# --------------------------------------------------------------------------- LLF / HLL
@pytest.mark.parametrize("name", ["flux_llf", "flux_hll", "flux_central"])
@pytest.mark.parametrize("dim", [2, 3])
def test_surface_flux_consistency(name, dim):
    fn = getattr(oracle, name)
    for _ in range(50):
        u = _rand_state(dim, RNG, jump=3.0)
        for d in range(dim):
            np.testing.assert_allclose(fn(u, u, d, dim, G), oracle.flux_phys(u, d, dim, G),
                                       rtol=1e-15, atol=1e-15)


def _speeds(u, d, dim):
    rho, v, p = _prim(u, dim)
    c = np.sqrt(G * p / rho)
    return v[d], c


def _flux_jacobian(u, d, dim):
    """df_d/du by central differences of the oracle's physical flux (step 1e-6 per column)."""
    n = dim + 2
    A = np.zeros((n, n))
    for j in range(n):
        h = 1e-6 * max(1.0, abs(u[j]))
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        A[:, j] = (oracle.flux_phys(up, d, dim, G) - oracle.flux_phys(um, d, dim, G)) / (2 * h)
    return A


@pytest.mark.parametrize("dim", [2, 3])
def test_wave_speeds_are_flux_jacobian_eigenvalues(dim):
    """The speeds in the HLL and LLF pins below, v_d -+ c with c = sqrt(gamma p / rho), are
    the extreme eigenvalues of the flux Jacobian df_d/du (eigenvalues of a difference
    Jacobian of the physical flux), and the others equal v_d; so those pins do not rest on
    a restated sound speed."""
    rng = np.random.default_rng(91 + dim)
    for _ in range(50):
        u = _rand_state(dim, rng, jump=3.0)
        for d in range(dim):
            lam = np.linalg.eigvals(_flux_jacobian(u, d, dim))
            v, c = _speeds(u, d, dim)
            tol = 1e-6 * (abs(v) + c)
            assert np.abs(lam.imag).max() < tol
            ev = np.sort(lam.real)
            np.testing.assert_allclose([ev[0], ev[-1]], [v - c, v + c], rtol=0, atol=tol)
            np.testing.assert_allclose(ev[1:-1], v, rtol=0, atol=tol)


@pytest.mark.parametrize("dim", [2, 3])
def test_hll_intermediate_state(dim):
    """HLL = f_L + s_L (u* - u_L) = f_R + s_R (u* - u_R) with the integral-average state
    u* = (s_R u_R - s_L u_L - (f_R - f_L))/(s_R - s_L); upwind f_L / f_R when supersonic."""
    rng = np.random.default_rng(51 + dim)
    n_sub = 0
    for _ in range(300):
        uL, uR = _rand_state(dim, rng, jump=3.0), _rand_state(dim, rng, jump=3.0)
        for d in range(dim):
            vl, cl = _speeds(uL, d, dim)
            vr, cr = _speeds(uR, d, dim)
            sL, sR = min(vl - cl, vr - cr), max(vl + cl, vr + cr)
            fL, fR = oracle.flux_phys(uL, d, dim, G), oracle.flux_phys(uR, d, dim, G)
            f = oracle.flux_hll(uL, uR, d, dim, G)
            if sL >= 0:
                np.testing.assert_array_equal(f, fL)
            elif sR <= 0:
                np.testing.assert_array_equal(f, fR)
            else:
                n_sub += 1
                us = (sR * uR - sL * uL - (fR - fL)) / (sR - sL)
                np.testing.assert_allclose(f, fL + sL * (us - uL), rtol=1e-12, atol=1e-12)
                np.testing.assert_allclose(f, fR + sR * (us - uR), rtol=1e-12, atol=1e-12)
    assert n_sub > 100


@pytest.mark.parametrize("dim", [2, 3])
def test_llf_is_hll_with_symmetric_speeds(dim):
    """LLF = HLL-type integral form with s_L = -lambda, s_R = lambda,
    lambda = max(|v_dL| + c_L, |v_dR| + c_R)."""
    rng = np.random.default_rng(61 + dim)
    for _ in range(200):
        uL, uR = _rand_state(dim, rng, jump=3.0), _rand_state(dim, rng, jump=3.0)
        for d in range(dim):
            vl, cl = _speeds(uL, d, dim)
            vr, cr = _speeds(uR, d, dim)
            lam = max(abs(vl) + cl, abs(vr) + cr)
            fL, fR = oracle.flux_phys(uL, d, dim, G), oracle.flux_phys(uR, d, dim, G)
            us = (lam * uR + lam * uL - (fR - fL)) / (2 * lam)
            np.testing.assert_allclose(oracle.flux_llf(uL, uR, d, dim, G), fL - lam * (us - uL),
                                       rtol=1e-12, atol=1e-12)


def test_supersonic_hll_upwinds():
    rho, p = 1.0, 1.0
    c = np.sqrt(G * p / rho)
    uL = prim_to_cons(np.array(rho), [3 * c, 0.1, 0.0], np.array(p), G).reshape(-1)
    uR = prim_to_cons(np.array(1.2 * rho), [2.5 * c, -0.1, 0.2], np.array(1.1 * p), G).reshape(-1)
    np.testing.assert_array_equal(oracle.flux_hll(uL, uR, 0, 3, G), oracle.flux_phys(uL, 0, 3, G))
    np.testing.assert_array_equal(oracle.flux_hll(_mirror(uR, 0), _mirror(uL, 0), 0, 3, G),
                                  oracle.flux_phys(_mirror(uL, 0), 0, 3, G))
