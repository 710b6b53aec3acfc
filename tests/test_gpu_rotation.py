"""The three inertia treatments of the rotational update (Sec. II.D) on the
GPU against the FP64 oracle run in the same mode: the analytic dI/dt, the
backward difference I(t) - I(t - dt) over the last two orientations, and the
predictor-corrector that solves the rotational rows again with the inertia
at the predicted orientation.  FP64 storage, 1e-9 relative (the parity bar
of the other FP64 trajectories).  Each case also checks that the modes give
measurably different trajectories, so a mode mixed up with another fails."""
import os
import tempfile

import numpy as np
import pytest

from test_gpu_parity import compare_particles, rand_q, snapshot

pytestmark = pytest.mark.gpu

MODES = {"analytic": 0, "fd": 1, "pc": 2}


@pytest.fixture(scope="module")
def lb():
    import torch
    from paper_2403_05443_amd import lbell
    lbell.load()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lbell


def pair(lb, mode, shape, coll="trt", tau=0.8, counterforce=False, max_particles=2):
    import oracle
    g = lb.Lattice([lb.make_box(*shape)], collision=coll, tau=tau, storage="fp64", counterforce=counterforce,
                   max_particles=max_particles, rotation=mode)
    o = oracle.OracleSim(shape, coll, tau, counterforce=counterforce, rotation=MODES[mode])
    return g, o


def other_mode_gap(shape, coll, tau, counterforce, setup, steps, mode):
    """Largest relative difference of Omega between the oracle in `mode` and
    in each of the other modes after `steps` steps."""
    import oracle
    W = {}
    for m, k in MODES.items():
        o = oracle.OracleSim(shape, coll, tau, counterforce=counterforce, rotation=k)
        po = setup(o)
        o.step(steps)
        W[m] = o.particle(po)["W"]
    return min(np.abs(W[m] - W[mode]).max() / np.linalg.norm(W[mode]) for m in MODES if m != mode)


@pytest.mark.parametrize("mode", list(MODES))
def test_rotation_mode_random_pose(lb, mode):
    """Triaxial ellipsoid at a random orientation, started spinning, under a
    force and a torque, counter-force on (without the initial spin the modes
    differ by only ~4e-9 over 300 steps, too little to tell them apart)."""
    shape, axes = (32, 28, 30), (6.0, 4.0, 2.0)
    q = rand_q(np.random.default_rng(2403054421))
    c = (15.2, 13.7, 14.9)
    F, T = (1e-4, -2e-4, 5e-5), (2e-3, 1e-3, -1e-3)

    def setup(s):
        p = s.add_ellipsoid(c, axes, q)
        s.set_external(p, F, T)
        s.set_velocity(p, (0, 0, 0), (0.004, -0.006, 0.008))
        return p

    g, o = pair(lb, mode, shape, counterforce=True)
    pg, po = setup(g), setup(o)
    x0 = snapshot(o, po)
    for _ in range(3):
        g.step(100)
        o.step(100)
        compare_particles(g, o, pg, po, 1e-9, x0, a=max(axes))
    gap = other_mode_gap(shape, "trt", 0.8, True, setup, 300, mode)
    print("nearest other mode", gap)
    assert gap > 1e-6


@pytest.mark.parametrize("mode", ["fd", "pc"])
def test_rotation_mode_with_transitions(lb, mode):
    """A heavy, fast-spinning ellipsoid that covers and uncovers many nodes."""
    shape, axes = (20, 18, 22), (5.0, 2.5, 2.0)
    q = np.array([0.7, 0.3, -0.5, 0.4])
    q /= np.linalg.norm(q)
    c = (9.3, 8.7, 10.1)

    def setup(s):
        p = s.add_ellipsoid(c, axes, q)
        s.set_density(p, 20.0)
        s.set_velocity(p, (0.04, -0.03, 0.02), (0.004, -0.006, 0.008))
        return p

    g, o = pair(lb, mode, shape, coll="bgk", tau=1.0)
    pg, po = setup(g), setup(o)
    m0, mass0 = g.mask(), g.mass()
    x0 = snapshot(o, po)
    for _ in range(3):
        g.step(20)
        o.step(20)
        compare_particles(g, o, pg, po, 1e-9, x0, a=5.0)
        assert np.array_equal(g.mask(), o.mask())
    assert int((g.mask() != m0).sum()) > 20
    assert abs(g.mass() / mass0 - 1) < 1e-13
    gap = other_mode_gap(shape, "bgk", 1.0, False, setup, 60, mode)
    print("nearest other mode", gap)
    assert gap > 1e-6


def test_rotation_pc_two_particles(lb):
    """Two particles in one box (the two-kernel particle path)."""
    shape = (40, 26, 28)
    rng = np.random.default_rng(21)
    specs = [((10.3, 12.6, 13.1), rand_q(rng)), ((28.7, 13.2, 14.4), rand_q(rng))]
    g, o = pair(lb, "pc", shape, coll="trt", tau=1.0)
    ids = []
    for k, (c, q) in enumerate(specs):
        pg, po = g.add_ellipsoid(c, (5, 3, 2), q), o.add_ellipsoid(c, (5, 3, 2), q)
        for s, p in ((g, pg), (o, po)):
            s.set_external(p, (0, 0, 1e-4 * (k + 1)), (1e-3, -2e-3 * k, 5e-4))
        ids.append((pg, po))
    x0 = [snapshot(o, po) for _, po in ids]
    g.step(150)
    o.step(150)
    for (pg, po), s in zip(ids, x0):
        compare_particles(g, o, pg, po, 1e-9, s, a=5.0)


def test_rotation_fd_checkpoint_bitwise(lb):
    """The previous orientation travels with the checkpoint: a run resumed
    from one continues the uninterrupted backward-difference run bit for bit."""
    def make():
        g = lb.Lattice([lb.make_box(20, 18, 22)], collision="trt", tau=0.8, storage="fp32", counterforce=True,
                       max_particles=1, rotation="fd")
        p = g.add_ellipsoid((9.3, 8.7, 10.1), (5.0, 3.0, 2.0), (0.9, 0.1, -0.3, 0.3) / np.linalg.norm((0.9, 0.1, -0.3, 0.3)))
        g.set_external(p, (1e-4, 0, 5e-5), (1e-3, 2e-3, 0))
        return g, p
    a, pa = make()
    a.step(31)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.bin")
        a.save(path)
        a.step(30)
        b, pb = make()
        b.load(path)
        b.step(30)
    for k, v in a.particle(pa).items():
        assert np.array_equal(v, b.particle(pb)[k]), k
