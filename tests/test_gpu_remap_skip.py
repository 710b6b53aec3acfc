"""The remap skips testing a particle's window while no node can have
changed side since its last test, and between full tests it tests only the
narrow band of nodes near the surface that the last full test recorded.  A
slowly moving and turning particle crosses nodes now and then: its node map
must equal the oracle's (which tests every node every step) after every
single step, and the trajectory must stay within the FP64 parity bar; with
the band switched off (LBELL_BAND=0, every rescan full) the library must
give the same node maps and links."""
import os

import numpy as np
import pytest

from test_gpu_parity import compare_particles, pair, rand_q, snapshot

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    from paper_2403_05443_amd import lbell
    lbell.load()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lbell


class _band:
    """LBELL_BAND for the contexts created inside the block."""

    def __init__(self, on):
        self.on = on

    def __enter__(self):
        self.old = os.environ.get("LBELL_BAND")
        os.environ["LBELL_BAND"] = "1" if self.on else "0"

    def __exit__(self, *exc):
        if self.old is None:
            os.environ.pop("LBELL_BAND", None)
        else:
            os.environ["LBELL_BAND"] = self.old


@pytest.mark.parametrize("band", [True, False], ids=["band", "full-scans"])
@pytest.mark.parametrize("fused", [True, False], ids=["one-particle", "two-particles"])
def test_node_map_every_step(lb, fused, band):
    shape = (30, 24, 26) if fused else (44, 24, 26)
    with _band(band):
        g, o = pair(lb, shape, "trt", 0.8, "fp64")
    rng = np.random.default_rng(77)
    centres = [(14.3, 11.6, 12.8)] if fused else [(10.3, 11.6, 12.8), (32.6, 12.1, 13.4)]
    ids = []
    for k, c in enumerate(centres):
        q = rand_q(rng)
        pg, po = g.add_ellipsoid(c, (5.0, 3.0, 2.0), q), o.add_ellipsoid(c, (5.0, 3.0, 2.0), q)
        for s, p in ((g, pg), (o, po)):
            s.set_density(p, 5.0)
            s.set_velocity(p, (2e-3, -1e-3 * (k + 1), 1.5e-3), (1e-3, -5e-4, 8e-4))
        ids.append((pg, po))
    x0 = [snapshot(o, po) for _, po in ids]
    m_prev, changes = g.mask(), 0
    for step in range(240):
        g.step(1)
        o.step(1)
        m = g.mask()
        assert np.array_equal(m, o.mask()), step
        changes += int((m != m_prev).any())
        m_prev = m
    print("steps with a node change:", changes)
    assert 5 < changes < 200      # nodes change side on some steps, not on most
    for (pg, po), s in zip(ids, x0):
        compare_particles(g, o, pg, po, 1e-9, s, a=5.0)


@pytest.mark.parametrize("fused", [True, False], ids=["one-particle", "two-particles"])
def test_band_rescans_equal_full_rescans(lb, fused):
    """Fast-turning particles (a full rescan every few steps, band rescans in
    between) with FP32 storage: the node maps and every particle's link set
    equal those of full rescans after each of 200 steps, and the velocities
    agree to rounding (the uncovered nodes' momenta are summed in another
    order)."""
    shape = (36, 30, 32) if fused else (60, 30, 32)
    centres = [(17.3, 14.6, 15.8)] if fused else [(14.3, 14.6, 15.8), (44.6, 15.1, 16.4)]
    rng = np.random.default_rng(91)
    qs = [rand_q(rng) for _ in centres]
    runs = []
    for band in (True, False):
        with _band(band):
            g = lb.Lattice([shape], collision="trt", tau=0.8, storage="fp32", max_particles=4)
        ids = []
        for k, (c, q) in enumerate(zip(centres, qs)):
            p = g.add_ellipsoid(c, (7.0, 3.0, 2.5), q)
            g.set_density(p, 3.0)
            g.set_velocity(p, (3e-3, -2e-3 * (k + 1), 2.5e-3), (6e-3, -4e-3, 5e-3))
            ids.append(p)
        runs.append((g, ids))
    (ga, ia), (gb, ib) = runs
    for step in range(200):
        ga.step(1)
        gb.step(1)
        assert np.array_equal(ga.mask(), gb.mask()), step
        if step % 20 == 19:
            for pa, pb in zip(ia, ib):
                (sa, da), (sb, db) = ga.links(pa), gb.links(pb)
                assert np.array_equal(sa, sb) and np.array_equal(da, db), step
    for pa, pb in zip(ia, ib):
        A, B = ga.particle(pa), gb.particle(pb)
        for k in ("U", "W"):
            assert np.abs(A[k] - B[k]).max() <= 1e-12 * np.abs(B[k]).max() + 1e-300, (k, A[k], B[k])
