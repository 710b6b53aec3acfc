"""The collide-stream kernels turn a site index into (x, y, z) by multiplying
with m = ceil(2^L / d), L = 27 + ceil(log2 d), and shifting by L instead of
dividing by the box edges (the site index is below 2^27).  The claim that
this is exact for every n < 2^27 is checked here against integer division:
every edge length a box can have up to 2^14, each with the sites around every
multiple of d near the top of the range, the largest indices, and random ones."""
import numpy as np

SITE_BITS = 27


def magic(d):
    c = 0
    while (1 << c) < d:
        c += 1
    L = SITE_BITS + c
    return ((1 << L) + d - 1) // d, L


def test_magic_division_is_exact():
    rng = np.random.default_rng(5)
    top = (1 << SITE_BITS) - 1
    for d in list(range(1, 1025)) + sorted(set(rng.integers(1025, 1 << 14, 300).tolist())):
        m, L = magic(d)
        assert m < (1 << 29)
        k = top // d
        ns = [0, 1, d - 1, d, d + 1, top, top - 1]
        for q in (k, k - 1, k // 2, 1):
            ns += [q * d - 1, q * d, q * d + d - 1]
        ns += rng.integers(0, top + 1, 200).tolist()
        for n in ns:
            if 0 <= n <= top:
                assert (n * m) >> L == n // d, (n, d)
