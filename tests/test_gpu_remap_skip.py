"""The remap skips testing a particle's window while no node can have
changed side since its last test.  A slowly moving and turning particle
crosses nodes now and then: its node map must equal the oracle's (which
tests every node every step) after every single step, and the trajectory
must stay within the FP64 parity bar."""
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


@pytest.mark.parametrize("fused", [True, False], ids=["one-particle", "two-particles"])
def test_node_map_every_step(lb, fused):
    shape = (30, 24, 26) if fused else (44, 24, 26)
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
