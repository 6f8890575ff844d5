"""The stage kernels' log-mean middle branch (1e-4 <= z^2 < 0.1), checked on the host.

The coefficients are read from the HIP source and compared with artanh at 50 digits: the
logarithmic mean {{a}}_ln = (b - a)/(ln b - ln a) with z = (b - a)/(b + a) is
(a + b) z/(2 artanh z), and its reciprocal (2/(a + b)) artanh(z)/z (ln(b/a) = 2 artanh z).
"""
import os
import re

import mpmath
import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
PHYSICS = os.path.join(HERE, "..", "paper_2108_06476_amd", "csrc", "physics.h")


def _coeffs(name):
    src = open(PHYSICS).read()
    m = re.search(r"constexpr double " + name + r"\[11\] = \{([^}]*)\}", src)
    assert m, name
    body = re.sub(r"//[^\n]*", "", m.group(1))
    return [float(t) for t in body.replace("\n", " ").split(",") if t.strip()]


def _exact_q(x):
    z = mpmath.sqrt(x)
    return mpmath.atanh(z) / z


def _grid():
    # both ends of the branch, a log-spaced sweep and the values where it meets its neighbours
    xs = list(np.geomspace(1e-4, 0.1, 400)) + list(np.linspace(1e-4, 0.1, 400))
    return [x for x in xs if 1e-4 <= x < 0.1] + [np.nextafter(0.1, 0.0)]


@pytest.mark.parametrize("name", ["kP", "kQ"])
def test_middle_branch_polynomial_error(name):
    """Relative error of the float64-coefficient polynomial, in exact arithmetic, <= 2e-17."""
    c = [mpmath.mpf(v) for v in _coeffs(name)]
    mpmath.mp.dps = 50
    worst = mpmath.mpf(0)
    for x in _grid():
        X = mpmath.mpf(float(x))
        q = _exact_q(X)
        want = 1 / (2 * q) if name == "kP" else q
        got = mpmath.polyval(c[::-1], X)
        worst = max(worst, abs(got / want - 1))
    assert worst <= 2e-17, float(worst)


def test_middle_branch_log_means_in_float64():
    """The two log means as the kernels form them (float64 Horner with fused steps emulated
    by mpmath rounding to float64), against the 50-digit definitions, for pairs of states
    spread over the branch: relative error below 4e-16."""
    kP, kQ = _coeffs("kP"), _coeffs("kQ")
    mpmath.mp.dps = 50
    rng = np.random.default_rng(7)
    worst = 0.0
    for _ in range(300):
        a = float(rng.uniform(0.1, 10.0))
        ratio = float(np.exp(rng.uniform(np.log(1.0202), np.log(1.89))))
        b = a * ratio if rng.random() < 0.5 else a / ratio
        s, d = a + b, b - a
        r = 1.0 / s
        z = d * r
        x = z * z
        if not (1e-4 <= x < 0.1):
            continue

        def fma(p, q, t):
            return float(mpmath.mpf(p) * mpmath.mpf(q) + mpmath.mpf(t))

        p = kP[10]
        for k in range(9, -1, -1):
            p = fma(p, x, kP[k])
        ln = s * p
        q = 2.0 * kQ[10]
        for k in range(9, -1, -1):
            q = fma(q, x, 2.0 * kQ[k])
        iln = r * q
        A, B = mpmath.mpf(a), mpmath.mpf(b)
        exact = (B - A) / (mpmath.log(B) - mpmath.log(A))
        worst = max(worst, float(abs(ln / exact - 1)), float(abs(iln * exact - 1)))
    assert worst < 4e-16, worst


def test_coefficients_match_their_generator():
    """The arrays in the source are what the committed fit script produces."""
    import importlib.util

    path = os.path.join(HERE, "..", "paper_2108_06476_amd", "csrc", "logmean_fit.py")
    spec = importlib.util.spec_from_file_location("logmean_fit", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    assert _coeffs("kP") == mod.fit(mod.p_exact)
    assert _coeffs("kQ") == mod.fit(mod.q_exact)
