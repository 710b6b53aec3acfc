"""D3Q27 on the GPU (the paper's lattice-independence check, Sec. III.A,
Fig. 3d): the same parity bars as D3Q19 against the FP64 oracle on its D3Q27
lattice (masks and link lists bit-exact, FP64 storage within 1e-9, FP32 within
1e-5), the collide-stream shapes it takes (pull and in place, plain and
XCD-chunked) bit for bit against each other, and the tuner's choices."""
import os
import tempfile

import numpy as np
import pytest

from test_gpu_parity import compare_particles, rand_q, snapshot, sorted_links

pytestmark = pytest.mark.gpu

SHAPES27 = (0, 3, 11, 12)


@pytest.fixture(scope="module")
def lb():
    import torch
    from paper_2403_05443_amd import lbell
    lbell.load()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lbell


def pair27(lb, shape, coll="bgk", tau=1.0, storage="fp64", counterforce=False, walls=False,
           wall_lo=(0, 0, 0), wall_hi=(0, 0, 0), init="rest", max_particles=4, magic=3 / 16, variant=None):
    import oracle
    if variant is not None:
        os.environ["LBELL_K1_VARIANT"] = str(variant)
    try:
        box = lb.make_box(*shape, walls=walls, wall_lo=wall_lo, wall_hi=wall_hi, init=init)
        g = lb.Lattice([box], collision=coll, tau=tau, storage=storage, counterforce=counterforce,
                       max_particles=max_particles, magic=magic, lattice=27)
    finally:
        os.environ.pop("LBELL_K1_VARIANT", None)
    o = oracle.OracleSim(shape, coll, tau, magic=magic, walls=walls, wall_lo=wall_lo, wall_hi=wall_hi,
                         init=init, counterforce=counterforce, lattice=27)
    return g, o


@pytest.mark.parametrize("seed", range(4))
def test_d3q27_geometry_bit_exact(lb, seed):
    rng = np.random.default_rng(2700 + seed)
    shape = (20, 17, 23) if seed % 2 else (32, 32, 32)
    g, o = pair27(lb, shape)
    centre = rng.random(3) * np.array(shape)
    axes = np.array([5.0, 2.5, 2.0]) * (0.8 + 0.4 * rng.random())
    q = rand_q(rng)
    pg, po = g.add_ellipsoid(centre, axes, q), o.add_ellipsoid(centre, axes, q)
    assert np.array_equal(g.mask(), o.mask())
    sg, so = g.links(pg), o.links(po)
    assert len(sg[0]) == len(so[0]) == g.aux(pg)["nlinks"]
    assert np.array_equal(sorted_links(*sg), sorted_links(*so))
    assert (sg[1] >= 19).any()           # corner links present


@pytest.mark.parametrize("storage,tol", [("fp64", 1e-9), ("fp32", 1e-5)])
def test_d3q27_settling_spheroid(lb, storage, tol):
    """Inclined spheroid under a force and a torque, counter-force, TRT."""
    g, o = pair27(lb, (28, 26, 30), "trt", 0.8, storage, counterforce=True)
    q = rand_q(np.random.default_rng(27))
    c = (13.6, 12.3, 14.8)
    pg, po = g.add_ellipsoid(c, (5.0, 2.5, 2.5), q), o.add_ellipsoid(c, (5.0, 2.5, 2.5), q)
    for s, p in ((g, pg), (o, po)):
        s.set_external(p, (2e-5, -1e-5, 1e-4), (0, 2e-4, -1e-4))
    x0 = snapshot(o, po)
    for _ in range(3):
        g.step(100)
        o.step(100)
        compare_particles(g, o, pg, po, tol, x0, a=5.0)
    assert abs(g.mass() / o.mass() - 1) < (1e-13 if storage == "fp64" else 1e-11)


@pytest.mark.parametrize("coll,tau", [("bgk", 1.0), ("trt", 0.8), ("reg", 0.7)])
def test_d3q27_moving_particle_with_transitions(lb, coll, tau):
    g, o = pair27(lb, (20, 18, 22), coll, tau, "fp64")
    q = np.array([0.7, 0.3, -0.5, 0.4])
    q /= np.linalg.norm(q)
    c = (9.3, 8.7, 10.1)
    pg, po = g.add_ellipsoid(c, (5.0, 2.5, 2.0), q), o.add_ellipsoid(c, (5.0, 2.5, 2.0), q)
    for s, p in ((g, pg), (o, po)):
        s.set_density(p, 20.0)
        s.set_velocity(p, (0.04, -0.03, 0.02), (0.002, -0.003, 0.004))
    m0, mass0 = g.mask(), g.mass()
    x0 = snapshot(o, po)
    for _ in range(3):
        g.step(20)
        o.step(20)
        compare_particles(g, o, pg, po, 1e-9, x0, a=5.0)
        assert np.array_equal(g.mask(), o.mask())
    assert int((g.mask() != m0).sum()) > 20
    assert abs(g.mass() / mass0 - 1) < 1e-13
    ag, ao = g.aux(pg), o.aux(po)
    assert ag["nlinks"] == ao["nlinks"]
    assert abs(ag["dm"] - ao["dm"]) < 1e-12


def test_d3q27_particle_between_moving_walls(lb):
    U = 0.01
    g, o = pair27(lb, (30, 28, 26), "bgk", 0.9, "fp64", walls=True, wall_lo=(-U, 0, 0), wall_hi=(U, 0, 0),
                  init="couette")
    q = rand_q(np.random.default_rng(3))
    c = (14.2, 13.6, 12.7)
    pg, po = g.add_ellipsoid(c, (6.0, 3.0, 3.0), q), o.add_ellipsoid(c, (6.0, 3.0, 3.0), q)
    x0 = snapshot(o, po)
    for _ in range(2):
        g.step(100)
        o.step(100)
        compare_particles(g, o, pg, po, 1e-9, x0, a=6.0)


def test_d3q27_squirmer_and_two_particles(lb):
    """Two particles in one box (two-kernel particle path), one a squirmer."""
    g, o = pair27(lb, (40, 26, 28), "trt", 1.0, "fp64")
    rng = np.random.default_rng(9)
    specs = [((10.3, 12.6, 13.1), rand_q(rng)), ((28.7, 13.2, 14.4), rand_q(rng))]
    ids = []
    for c, q in specs:
        ids.append((g.add_ellipsoid(c, (5, 2.5, 2.5), q), o.add_ellipsoid(c, (5, 2.5, 2.5), q)))
    g.set_squirmer(ids[0][0], 1e-3, 2e-3)
    o.set_squirmer(ids[0][1], 1e-3, 2e-3)
    g.set_external(ids[1][0], (0, 0, 1e-4))
    o.set_external(ids[1][1], (0, 0, 1e-4))
    x0 = [snapshot(o, po) for _, po in ids]
    g.step(150)
    o.step(150)
    for (pg, po), s in zip(ids, x0):
        compare_particles(g, o, pg, po, 1e-9, s, a=5.0)


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
@pytest.mark.parametrize("walls", [False, True])
def test_d3q27_shapes_bitwise(lb, storage, walls):
    """Pull and in-place, plain and XCD-chunked D3Q27 launches give the same
    bits (moving particle, periodic or between moving walls)."""
    runs = []
    U = 0.01
    for v in SHAPES27:
        g, _ = pair27(lb, (40, 22, 26), "trt", 0.8, storage, walls=walls, wall_lo=(-U, 0, 0) if walls else (0, 0, 0),
                      wall_hi=(U, 0, 0) if walls else (0, 0, 0), init="couette" if walls else "rest", variant=v)
        q = np.array([0.8, 0.3, -0.4, 0.33])
        p = g.add_ellipsoid((19.3, 10.6, 13.2), (5, 2.5, 2), q / np.linalg.norm(q))
        g.set_density(p, 4.0)
        g.set_velocity(p, (0.03, -0.02, 0.01), (0.001, -0.002, 0.0015))
        g.step(31)
        runs.append((g.particle(p), g.force_torque(p), g.fields(), g.mask(), g.mass()))
    for r in runs[1:]:
        for k in r[0]:
            assert np.array_equal(r[0][k], runs[0][0][k]), k
        assert all(np.array_equal(a, b) for a, b in zip(r[1], runs[0][1]))
        assert all(np.array_equal(a, b) for a, b in zip(r[2], runs[0][2]))
        assert np.array_equal(r[3], runs[0][3])
        assert r[4] == runs[0][4]


def test_d3q27_tuner_and_checkpoint(lb):
    """The tuner picks among the D3Q27 shapes; a checkpoint taken in one
    layout and loaded into a pull context continues bit for bit."""
    def make(v):
        g, _ = pair27(lb, (48, 24, 24), "trt", 0.8, "fp32", counterforce=True, variant=v)
        q = np.array([0.9, 0.1, -0.2, 0.3])
        p = g.add_ellipsoid((23.1, 11.7, 12.2), (5, 2.5, 2.5), q / np.linalg.norm(q))
        g.set_external(p, (0, 1e-4, 0), (1e-4, 0, 0))
        return g, p
    a, pa = make(None)
    v, ms = a.autotune(2)
    assert v in SHAPES27 and ms > 0
    b, pb = make(0)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.bin")
        a.save(path)
        a.step(21)
        b.load(path)
        b.step(21)
    for k, val in a.particle(pa).items():
        assert np.array_equal(val, b.particle(pb)[k]), k
    assert np.array_equal(a.fields()[1], b.fields()[1])
