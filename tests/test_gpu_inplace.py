"""The in-place collide-stream variants (11-14): one population buffer,
alternating an even step on each node's own slots with an odd step that
gathers from and scatters to the neighbours.  They run the same arithmetic
on the same populations as the two-buffer pull variants, so every observable
(particle states, forces, node maps, fields, mass) must come out bit for bit
equal; the layout switches (tuner, checkpoints across layouts) permute slots
and must not change a bit either."""
import os
import tempfile

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

INPLACE = (11, 12, 13, 14)


@pytest.fixture(scope="module")
def lb():
    import torch
    from paper_2403_05443_amd import lbell
    lbell.load()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lbell


def _lattice(lb, variant, shape, storage, walls=False, nparts=1, coll="trt"):
    os.environ["LBELL_K1_VARIANT"] = str(variant)
    try:
        U = 0.01
        box = lb.make_box(*shape, walls=walls, wall_lo=(-U, 0, 0) if walls else (0, 0, 0),
                          wall_hi=(U, 0, 0) if walls else (0, 0, 0), init="couette" if walls else "rest")
        g = lb.Lattice([box], collision=coll, tau=0.8, storage=storage, counterforce=not walls,
                       max_particles=nparts)
    finally:
        del os.environ["LBELL_K1_VARIANT"]
    ids = []
    q = np.array([0.8, 0.3, -0.4, 0.33])
    centres = [(shape[0] / 2 + 0.3, shape[1] / 2 - 0.4, shape[2] / 2 + 0.2),
               (shape[0] / 2 - 13.7, shape[1] / 2 + 0.6, shape[2] / 2 - 0.3)]
    for k in range(nparts):
        p = g.add_ellipsoid(centres[k], (5, 2.5, 2), q / np.linalg.norm(q))
        g.set_density(p, 4.0)
        g.set_velocity(p, (0.03, -0.02, 0.01 * (k + 1)), (0.001, -0.002, 0.0015))
        if not walls:
            g.set_external(p, (1e-4, -5e-5, 2e-4), (1e-3, 0, 0))
        ids.append(p)
    return g, ids


def _same(a, ia, b, ib):
    for pa, pb in zip(ia, ib):
        for k, v in a.particle(pa).items():
            assert np.array_equal(v, b.particle(pb)[k]), k
        Fa, Ta = a.force_torque(pa)
        Fb, Tb = b.force_torque(pb)
        assert np.array_equal(Fa, Fb) and np.array_equal(Ta, Tb)
    ra, ua = a.fields()
    rb, ub = b.fields()
    assert np.array_equal(ra, rb) and np.array_equal(ua, ub)
    assert np.array_equal(a.mask(), b.mask())
    assert a.mass() == b.mass()


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("walls", [False, True])
def test_inplace_matches_pull(lb, storage, walls):
    """Every in-place shape against the pull kernel, with a moving particle
    that crosses nodes, periodic or between moving walls (Couette start),
    over an odd and then an even number of steps."""
    shape = (48, 22, 26)
    ref, ir = _lattice(lb, 0, shape, storage, walls)
    ref.step(25)
    for v in INPLACE:
        g, ig = _lattice(lb, v, shape, storage, walls)
        g.step(25)
        _same(g, ig, ref, ir)
    ref.step(24)
    g.step(24)
    _same(g, ig, ref, ir)


def test_inplace_two_particles_in_one_box(lb):
    """Two particles in one box take the two-kernel particle path."""
    ref, ir = _lattice(lb, 0, (56, 24, 24), "fp32", nparts=2)
    g, ig = _lattice(lb, 12, (56, 24, 24), "fp32", nparts=2)
    ref.step(41)
    g.step(41)
    _same(g, ig, ref, ir)


@pytest.mark.parametrize("src,dst", [(12, 0), (0, 12), (13, 11)])
def test_checkpoint_across_layouts(lb, src, dst):
    """A checkpoint written in one layout and loaded into a context of the
    other continues the uninterrupted run bit for bit."""
    a, ia = _lattice(lb, src, (40, 22, 24), "fp32")
    b, ib = _lattice(lb, dst, (40, 22, 24), "fp32")
    a.step(17)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.bin")
        a.save(path)
        a.step(20)
        b.load(path)
        b.step(20)
    _same(a, ia, b, ib)


@pytest.mark.parametrize("gsteps", [1, 2, 3])
def test_inplace_graph_replay(lb, gsteps):
    """Graph replay of in-place steps in groups of 1, 2 and 3 (odd groups
    alternate the parity a replay starts from)."""
    ref, ir = _lattice(lb, 0, (40, 22, 24), "fp16")
    g, ig = _lattice(lb, 12, (40, 22, 24), "fp16")
    g.set_graph(gsteps)
    for _ in range(4):
        ref.step(6 * gsteps)
        g.step(6 * gsteps)
        _same(g, ig, ref, ir)


def test_inplace_stokes_start(lb):
    """The Stokes start field written into the in-place layout."""
    runs = []
    for v in (0, 12):
        g, ids = _lattice(lb, v, (40, 22, 24), "fp32")
        g.step(3)  # start from the odd parity of the in-place layout
        g.stokes_start()
        g.step(12)
        runs.append((g, ids))
    _same(runs[0][0], runs[0][1], runs[1][0], runs[1][1])


def test_inplace_nonfinite_watchdog(lb):
    g, _ = _lattice(lb, 12, (24, 20, 22), "fp32")
    g.step(2)
    assert g.nonfinite() == 0
    g.poke(0, 3 + 24 * (4 + 20 * 5), 3, float("nan"))
    assert g.nonfinite() >= 1


def test_inplace_ensemble_matches_oracle(lb):
    """Uneven boxes in one in-place launch, FP64, against the oracle."""
    import oracle
    specs = [((24, 20, 28), (11.2, 9.7, 13.1), (5, 2.5, 2.5), (0.9, 0.1, -0.2, 0.3)),
             ((17, 19, 21), (8.4, 9.1, 10.3), (4, 2, 2), (0.6, -0.5, 0.4, 0.2))]
    os.environ["LBELL_K1_VARIANT"] = "13"
    try:
        g = lb.Lattice([lb.make_box(*s[0]) for s in specs], collision="trt", tau=0.8, storage="fp64",
                       counterforce=True, max_particles=2)
    finally:
        del os.environ["LBELL_K1_VARIANT"]
    sims = []
    for b, (shape, c, a, q) in enumerate(specs):
        q = np.array(q) / np.linalg.norm(q)
        pid = g.add_ellipsoid(c, a, q, box=b)
        g.set_external(pid, (1e-4, 2e-5 * (b + 1), -3e-5), (0, 2e-4, 1e-4))
        o = oracle.OracleSim(shape, "trt", 0.8, counterforce=True)
        po = o.add_ellipsoid(c, a, q)
        o.set_external(po, (1e-4, 2e-5 * (b + 1), -3e-5), (0, 2e-4, 1e-4))
        sims.append((pid, o, po))
    g.step(61)
    for pid, o, po in sims:
        o.step(61)
        U, Uo = g.particle(pid)["U"], o.particle(po)["U"]
        assert np.abs(U - Uo).max() / np.linalg.norm(Uo) < 1e-9
