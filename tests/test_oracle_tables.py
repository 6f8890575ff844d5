"""Pins of the oracle's tables: LGL operator, Legendre Vandermonde, CK(5,4) coefficients.

Each check is against something other than the oracle: closed forms, NumPy's Legendre
routines, exact rational arithmetic of the Runge-Kutta order conditions.
"""
from fractions import Fraction

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle

CLOSED_FORMS = {
    1: ([-1.0, 1.0], [1.0, 1.0]),
    2: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1.0, -1 / np.sqrt(5), 1 / np.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1.0, -np.sqrt(3 / 7), 0.0, np.sqrt(3 / 7), 1.0],
        [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("N", sorted(CLOSED_FORMS))
def test_lgl_closed_forms(N):
    x, w, _ = oracle.lgl(N)
    xe, we = CLOSED_FORMS[N]
    np.testing.assert_allclose(x, xe, rtol=0, atol=2e-16)
    np.testing.assert_allclose(w, we, rtol=3e-16, atol=0)


@pytest.mark.parametrize("N", range(1, 16))
def test_lgl_against_numpy_roots(N):
    """Interior nodes are the roots of P_N' (NumPy's Legendre class); weights sum to 2."""
    x, w, _ = oracle.lgl(N)
    if N > 1:
        r = np.sort(npleg.Legendre.basis(N).deriv().roots().real)
        np.testing.assert_allclose(x[1:-1], r, rtol=0, atol=1e-14)
    assert abs(w.sum() - 2.0) < 1e-14
    # quadrature is exact up to degree 2N-1
    for k in range(2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-13


@pytest.mark.parametrize("N", range(1, 16))
def test_sbp_property_and_exactness(N):
    """M D + D^T M = B = diag(-1, 0..0, 1), and D differentiates degree <= N exactly."""
    x, w, D = oracle.lgl(N)
    M = np.diag(w)
    B = np.zeros((N + 1, N + 1))
    B[0, 0], B[-1, -1] = -1.0, 1.0
    np.testing.assert_allclose(M @ D + D.T @ M, B, rtol=0, atol=5e-13 * max(1, N))
    for k in range(N + 1):
        dk = k * x ** (k - 1) if k > 0 else np.zeros_like(x)
        np.testing.assert_allclose(D @ x ** k, dk, rtol=0, atol=1e-11 * (N + 1) ** 2)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7, 9])
def test_vandermonde_inverse(N):
    """Vinv inverts V_ia = sqrt((2a+1)/2) P_a(x_i), built from NumPy's legval."""
    x, _, _ = oracle.lgl(N)
    V = np.zeros((N + 1, N + 1))
    for a in range(N + 1):
        c = np.zeros(a + 1)
        c[a] = 1.0
        V[:, a] = np.sqrt((2 * a + 1) / 2) * npleg.legval(x, c)
    Vinv = oracle.legendre_vinv(N)
    np.testing.assert_allclose(Vinv @ V, np.eye(N + 1), rtol=0, atol=1e-13)


def _butcher_from_2n(A, B):
    """Williamson 2N-storage -> Butcher (a, b, c):  k_s = A_s k_{s-1} + dt F_s,
    Y_{s+1} = Y_s + B_s k_s."""
    s = len(A)
    kappa = [[Fraction(0)] * s for _ in range(s)]
    for r in range(s):
        for j in range(r):
            kappa[r][j] = A[r] * kappa[r - 1][j]
        kappa[r][r] = Fraction(1)
    a = [[Fraction(0)] * s for _ in range(s + 1)]
    for i in range(1, s + 1):
        for j in range(i):
            a[i][j] = sum(B[r] * kappa[r][j] for r in range(j, i))
    b = a[s]
    c = [sum(a[i]) for i in range(s)]
    return [row for row in a[:s]], b, c


def test_ck45_order_conditions():
    """The eight order-4 conditions of the equivalent Butcher tableau, exactly in rational
    arithmetic on the oracle's coefficients (as stored doubles)."""
    A, B, c_given = oracle.lsrk_coeffs()
    assert A[0] == 0.0
    Af = [Fraction(v) for v in A]
    Bf = [Fraction(v) for v in B]
    a, b, c = _butcher_from_2n(Af, Bf)
    s = 5
    ac = [sum(a[i][j] * c[j] for j in range(s)) for i in range(s)]
    ac2 = [sum(a[i][j] * c[j] ** 2 for j in range(s)) for i in range(s)]
    aac = [sum(a[i][j] * ac[j] for j in range(s)) for i in range(s)]
    conds = {
        "b": (sum(b), Fraction(1)),
        "bc": (sum(b[i] * c[i] for i in range(s)), Fraction(1, 2)),
        "bc2": (sum(b[i] * c[i] ** 2 for i in range(s)), Fraction(1, 3)),
        "bac": (sum(b[i] * ac[i] for i in range(s)), Fraction(1, 6)),
        "bc3": (sum(b[i] * c[i] ** 3 for i in range(s)), Fraction(1, 4)),
        "bcac": (sum(b[i] * c[i] * ac[i] for i in range(s)), Fraction(1, 8)),
        "bac2": (sum(b[i] * ac2[i] for i in range(s)), Fraction(1, 12)),
        "baac": (sum(b[i] * aac[i] for i in range(s)), Fraction(1, 24)),
    }
    for name, (val, exact) in conds.items():
        assert abs(float(val - exact)) < 1e-15, (name, float(val - exact))
    # c from the tableau equals the published stage times; the published c_3 is a separate
    # rational approximation that differs from the tableau's row sum by 4.2e-8 (stage times
    # only matter for a time-dependent right-hand side, which no workload here has)
    np.testing.assert_allclose([float(v) for v in c], c_given, rtol=0, atol=5e-8)
    # fifth-order term of the stability polynomial differs from 1/120 (not order 5)
    aaac = [sum(a[i][j] * aac[j] for j in range(s)) for i in range(s)]
    z5 = float(sum(b[i] * aaac[i] for i in range(s)))
    assert abs(z5 - 1 / 200) < 1e-12 and abs(z5 - 1 / 120) > 1e-3
