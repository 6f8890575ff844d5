"""The wave-speed slots of mid-size Cartesian meshes, checked on the host.

The last RK stage folds each element's wave speed into slot e mod 64 with an unsigned 64-bit
atomic max on the bits of the double, and the next step's first stage takes dt from the max
over the slots.  That gives the same dt as the reduction of the per-element partials only
if non-negative doubles order as their bit patterns do and the slot maxima keep the overall
maximum whatever the order of the atomics; both are checked here (IEEE 754 binary64).
"""
import numpy as np


def _bits(x):
    return np.asarray(x, dtype=np.float64).view(np.uint64)


def test_nonnegative_doubles_order_as_their_bits():
    rng = np.random.default_rng(11)
    x = np.concatenate([
        rng.uniform(0.0, 10.0, 4000),
        np.exp(rng.uniform(-700.0, 700.0, 4000)),          # the whole normal range
        np.array([0.0, 5e-324, 2.2e-308, 1.0, np.nextafter(1.0, 2.0), 1.7e308, np.inf]),
    ])
    a, b = rng.permutation(x), rng.permutation(x)
    assert np.array_equal(a < b, _bits(a) < _bits(b))
    assert np.array_equal(a == b, _bits(a) == _bits(b))


def test_slot_maxima_keep_the_maximum_in_any_order():
    rng = np.random.default_rng(12)
    for E in (513, 1000, 4096, 16383):
        lam = rng.uniform(0.5, 3.0, E) * np.exp(rng.uniform(-3, 3, E))
        want = lam.max()
        for _ in range(3):
            slots = np.zeros(64, dtype=np.uint64)
            for e in rng.permutation(E):                     # any order of the atomics
                slots[e % 64] = max(slots[e % 64], _bits(lam[e]))
            got = slots.view(np.float64).max()
            assert got == want                               # bit for bit
            assert 2.0 * 0.5 / (4.0 * got) == 2.0 * 0.5 / (4.0 * want)
