"""Coefficients of the log means' middle branch in physics.h (not run by the build).

With z = (b - a)/(b + a) and x = z^2, the logarithmic mean of a and b is (a + b) * P(x) with
P(x) = z / (2 artanh z), and its reciprocal (2/(a + b)) * Q(x) with Q(x) = artanh(z) / z.
On 1e-4 <= x < 0.1 (states within a factor 1.9) the kernels evaluate P and Q as polynomials
in x of degree DEG: interpolants at Chebyshev nodes of [0, 0.1], formed at 60 digits and
rounded to float64.  Both functions are analytic in x for |x| < 1 (the branch point of
artanh is at z = 1), so the interpolation error falls by about 38 per degree on this
interval; degree 10 leaves about 1e-18 relative with the rounded coefficients.

    python paper_2108_06476_amd/csrc/logmean_fit.py      # prints the two arrays
"""
import mpmath as mp

DEG = 10
LO, HI = 0, "0.1"


def q_exact(x):
    """artanh(z)/z at x = z^2."""
    x = mp.mpf(x)
    if x == 0:
        return mp.mpf(1)
    z = mp.sqrt(x)
    return mp.atanh(z) / z


def p_exact(x):
    """z/(2 artanh z) at x = z^2."""
    return 1 / (2 * q_exact(x))


def fit(f, deg=DEG, lo=LO, hi=HI):
    """Monomial coefficients (constant first) of f's interpolant at Chebyshev nodes."""
    with mp.workdps(60):
        a, b = mp.mpf(lo), mp.mpf(hi)
        xs = [(a + b) / 2 + (b - a) / 2 * mp.cos(mp.pi * (2 * k + 1) / (2 * (deg + 1)))
              for k in range(deg + 1)]
        A = mp.matrix(deg + 1, deg + 1)
        y = mp.matrix(deg + 1, 1)
        for i, x in enumerate(xs):
            for j in range(deg + 1):
                A[i, j] = x ** j
            y[i] = f(x)
        c = mp.lu_solve(A, y)
        return [float(c[j]) for j in range(deg + 1)]


if __name__ == "__main__":
    for name, f in (("P (ln_mean)", p_exact), ("Q (inv_ln_mean)", q_exact)):
        print(name)
        print(",\n".join(repr(c) for c in fit(f)))
