"""Batched ensembles: many independent boxes in one collide-stream launch and
one particle launch, the tuner's tile shapes, and graph replay.

Every collide-stream variant computes each site with the same arithmetic, so
the variants, graph replay and the batch itself must reproduce the bits of a
plain run of each box alone; FP64 batches must match the oracle to 1e-9
(the FP64 bar of the parity tests).
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# generic tile shapes: pull (0, 3-10, 15) and in place (11-14)
GENERIC = (0, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15)


@pytest.fixture(scope="module")
def lb():
    import torch
    from paper_2403_05443_amd import lbell
    lbell.load()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lbell


SPECS = [((24, 20, 28), (11.2, 9.7, 13.1), (5, 2.5, 2.5), (0.9, 0.1, -0.2, 0.3)),
         ((17, 19, 21), (8.4, 9.1, 10.3), (4, 2, 2), (0.6, -0.5, 0.4, 0.2)),
         ((33, 16, 18), (15.1, 7.6, 8.8), (6, 2, 3), (0.2, 0.7, 0.1, -0.6))]


def _batch(lb, storage="fp32", variant=None, specs=SPECS, spare=0):
    if variant is not None:
        os.environ["LBELL_K1_VARIANT"] = str(variant)
    try:
        g = lb.Lattice([lb.make_box(*s[0]) for s in specs], collision="trt", tau=0.8, storage=storage,
                       counterforce=True, max_particles=len(specs) + spare)
    finally:
        os.environ.pop("LBELL_K1_VARIANT", None)
    for b, (shape, c, a, q) in enumerate(specs):
        q = np.array(q) / np.linalg.norm(q)
        pid = g.add_ellipsoid(c, a, q, box=b)
        g.set_external(pid, (1e-4, 2e-5 * (b + 1), -3e-5), (0, 2e-4, 1e-4))
        g.set_density(pid, 3.0)
        g.set_velocity(pid, (0.02, -0.01, 0.015 * (b - 1)), (0.001, -0.002, 0.0015))
    return g


def _same(a, b, nboxes, nparts=None):
    for p in range(nboxes if nparts is None else nparts):
        pa, pb = a.particle(p), b.particle(p)
        for k in pa:
            assert np.array_equal(pa[k], pb[k]), (p, k)
        Fa, Ta = a.force_torque(p)
        Fb, Tb = b.force_torque(p)
        assert np.array_equal(Fa, Fb) and np.array_equal(Ta, Tb), p
    for bx in range(nboxes):
        assert np.array_equal(a.fields(bx)[1], b.fields(bx)[1]), bx
        assert np.array_equal(a.mask(bx), b.mask(bx)), bx


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_generic_tile_shapes_bitwise(lb, storage):
    """Two tiles per block, XCD-chunked order and the persistent grid give the
    bits of one tile per block, on uneven boxes with moving particles that
    cross nodes."""
    ref = _batch(lb, storage, 0)
    ref.step(40)
    for v in GENERIC[1:]:
        g = _batch(lb, storage, v)
        g.step(40)
        _same(g, ref, len(SPECS))


def test_all_variants_single_box_bitwise(lb):
    """On a box the row-wave kernel also fits (nx = 128) all sixteen variants
    agree."""
    spec = [((128, 20, 18), (60.3, 9.6, 8.7), (6, 2.5, 2), (0.8, 0.3, -0.4, 0.33))]
    ref = _batch(lb, "fp32", 0, spec)
    ref.step(30)
    for v in range(1, 16):
        g = _batch(lb, "fp32", v, spec)
        g.step(30)
        _same(g, ref, 1)


def test_tuner_covers_generic_shapes(lb):
    """On a batch the tuner picks one of the generic shapes; the steps it
    times are ordinary steps (same bits as plain stepping)."""
    g, h = _batch(lb), _batch(lb)
    g.step(10)
    h.step(10)
    t0 = g.step_count()
    v, ms = g.autotune(3)
    assert v in GENERIC and ms > 0
    taken = g.step_count() - t0
    assert taken == 2 * len(GENERIC) * 5  # two sweeps of two warm-up + 3 timed steps per variant
    h.step(taken)
    g.step(10)
    h.step(10)
    _same(g, h, len(SPECS))


@pytest.mark.parametrize("gsteps", [1, 2, 3])
def test_graph_replay_bitwise(lb, gsteps):
    """Steps replayed from a HIP graph (groups of 1, 2, 3 steps, so both
    buffer parities are captured) give the bits of plain launches; replays are
    interleaved with the program's own reads and synchronisations, and every
    chunk is checked."""
    a, b = _batch(lb), _batch(lb)
    b.set_graph(gsteps)
    for chunk in (7, 5, 6):
        a.step(chunk)
        b.step(chunk)
        b.sync()
        _same(a, b, len(SPECS))
        b.mass(0)  # eager work on the stream between replays
    b.set_graph(0)
    a.step(4)
    b.step(4)
    _same(a, b, len(SPECS))


def test_graph_recaptured_after_add(lb):
    """Adding a particle changes the launch arguments: the graph is captured
    again and the run matches plain launches."""
    specs = SPECS[:2]
    a, b = _batch(lb, specs=specs, spare=1), _batch(lb, specs=specs, spare=1)
    b.set_graph(2)
    a.step(6)
    b.step(6)
    # a third particle, a sphere clear of the first one in box 0: box 0 now
    # holds two particles, so the particle phase also changes kernels
    for g in (a, b):
        pid = g.add_ellipsoid((2.5, 2.5, 2.5), (2.0, 2.0, 2.0), (1.0, 0.0, 0.0, 0.0), box=0)
        g.set_external(pid, (0, 0, 5e-5))
    a.step(7)
    b.step(7)
    _same(a, b, 2, nparts=3)


def _sample_boxes(W, k=3):
    """Indices of the smallest box, the largest box and the longest particle."""
    sizes = [b.shape[0] for b in W.boxes]
    longest = int(np.argmax([p.axes[0] for p in W.particles]))
    return sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), longest})[:k]


def _single(lb, W, i):
    from paper_2403_05443_amd.runner import build_lattice
    from paper_2403_05443_amd import workloads
    Wi = workloads.Workload(W.name, [W.boxes[i]], [W.particles[i]], W.collision, W.tau, W.storage, 0,
                            magic=W.magic, counterforce=W.counterforce, velocity_scale=W.velocity_scale,
                            max_semi_axis=W.max_semi_axis)
    Wi.particles[0] = workloads.Particle(**{**W.particles[i].__dict__, "box": 0})
    return build_lattice(Wi)


def test_full_ensemble_fp16_matches_single_boxes(lb):
    """The 256-box FP16 ensemble (edges 32-64, one spheroid each) in one
    launch per phase, graph-replayed, tuner-chosen tile shape: sampled boxes
    match the same box run alone bit for bit, and every box stays finite."""
    from paper_2403_05443_amd.runner import build_lattice
    from paper_2403_05443_amd import workloads
    W = workloads.c4("fp16")
    g = build_lattice(W)
    v, _ = g.autotune(3)
    g.set_graph(10)
    g.step(60)
    g.sync()
    bad = sum(g.nonfinite(b) for b in range(len(W.boxes)))
    assert bad == 0
    total = g.step_count()  # the tuner's steps included
    for i in _sample_boxes(W):
        s = _single(lb, W, i)
        s.step(total)
        ps, pg = s.particle(0), g.particle(i)
        for k in ps:
            assert np.array_equal(ps[k], pg[k]), (i, k)
        assert np.array_equal(s.fields(0)[1], g.fields(i)[1]), i
        del s
    print("variant", v)


def test_full_ensemble_fp64_matches_oracle(lb):
    """The same 256-box ensemble with FP64 storage, 60 steps: the smallest
    box, the largest box and the box of the longest particle (a = 18 in a
    45^3 box, the largest remap window) against the oracle at the FP64 bar."""
    import oracle
    from paper_2403_05443_amd.runner import build_lattice
    from paper_2403_05443_amd import workloads
    W = workloads.c4("fp64")
    g = build_lattice(W)
    g.step(60)
    boxes = _sample_boxes(W)
    assert len(boxes) == 3 and max(W.particles[i].axes[0] for i in boxes) > 17.9
    for i in boxes:
        p, b = W.particles[i], W.boxes[i]
        o = oracle.OracleSim(b.shape, W.collision, W.tau, magic=W.magic, counterforce=True)
        po = o.add_ellipsoid(p.centre, p.axes, p.quat)
        o.set_external(po, p.force, p.torque)
        o.step(60)
        A, B = g.particle(i), o.particle(po)
        Fg, Tg = g.force_torque(i)
        Fo, To = o.force_torque(po)
        a = p.axes[0]
        # natural velocity scale: the larger of |U| and the Stokes speed of the
        # load, |F_ext| / (6 pi mu a).  A heavy particle started from rest
        # (a = 18: M ~ 1000) moves at |U| ~ 3e-7 after 60 steps, a few percent
        # of that scale, and the oracle's full populations (rounding ~6e-17
        # near 1/3) resolve flow deviations of ~|U| / 6 only to ~1e-9
        # relative there: the bar stays 1e-9 of the velocity scale
        mu = (W.tau - 0.5) / 3.0
        Us = np.linalg.norm(p.force) / (6 * np.pi * mu * a)
        nU, nF = max(np.linalg.norm(B["U"]), Us), np.linalg.norm(Fo)
        errs = {"U": np.abs(A["U"] - B["U"]).max() / nU,
                "W": np.abs(A["W"] - B["W"]).max() / max(np.linalg.norm(B["W"]), nU / a),
                "F": np.abs(Fg - Fo).max() / nF,
                "T": np.abs(Tg - To).max() / max(np.linalg.norm(To), nF * a)}
        print(i, b.shape, {k: float(f"{e:.3g}") for k, e in errs.items()})
        assert all(e < 1e-9 for e in errs.values()), errs
        assert np.array_equal(g.mask(i) != 0, o.mask() != 0)
