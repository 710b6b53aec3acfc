"""Seeded synthetic workloads shaped like the paper's set-ups.

This module only draws numbers and states parameters (box sizes, particle
poses, loads); it holds none of the method's arithmetic, so both the oracle
tests and the GPU library can take their inputs from it.  All randomness
comes from one SplitMix64 stream (Steele, Lea & Flood 2014) per workload,
seed = 2403054430 + workload index.
"""
import math
from dataclasses import dataclass, field
from typing import List, Tuple

SEED0 = 2403054430
MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator with its published constants."""

    def __init__(self, seed):
        self.s = seed & MASK64

    def next_u64(self):
        self.s = (self.s + 0x9E3779B97F4A7C15) & MASK64
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self, lo=0.0, hi=1.0):
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / (1 << 53)))

    def normal(self):
        u1 = max(self.uniform(), 1e-300)
        u2 = self.uniform()
        return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)

    def unit_quaternion(self):
        """Uniform on S^3: normalised 4-D Gaussian."""
        while True:
            q = [self.normal() for _ in range(4)]
            n = math.sqrt(sum(v * v for v in q))
            if n > 1e-12:
                return tuple(v / n for v in q)

    def unit_vector(self):
        while True:
            v = [self.normal() for _ in range(3)]
            n = math.sqrt(sum(x * x for x in v))
            if n > 1e-12:
                return tuple(x / n for x in v)


@dataclass
class Particle:
    centre: Tuple[float, float, float]
    axes: Tuple[float, float, float]
    quat: Tuple[float, float, float, float]
    force: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    torque: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    squirmer: Tuple[float, float] = (0.0, 0.0)
    box: int = 0


@dataclass
class Box:
    shape: Tuple[int, int, int]
    walls: bool = False
    wall_lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    wall_hi: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    init: str = "rest"


@dataclass
class Workload:
    name: str
    boxes: List[Box]
    particles: List[Particle]
    collision: str
    tau: float
    storage: str
    steps: int
    magic: float = 3.0 / 16.0
    counterforce: bool = False
    velocity_scale: float = 1e-3
    max_semi_axis: float = 8.0
    notes: dict = field(default_factory=dict)
    lattice: int = 19

    @property
    def sites(self):
        return sum(b.shape[0] * b.shape[1] * b.shape[2] for b in self.boxes)


def quat_axis_angle(axis, angle):
    n = math.sqrt(sum(a * a for a in axis))
    s = math.sin(0.5 * angle) / n
    return (math.cos(0.5 * angle), axis[0] * s, axis[1] * s, axis[2] * s)


def c1(storage="fp64"):
    """32^3 periodic, BGK tau=1, a=4 b=c=2 along x, centred, F = 1e-4 x, 500 steps."""
    return Workload("c1_settling_32", [Box((32, 32, 32))],
                    [Particle((15.5, 15.5, 15.5), (4.0, 2.0, 2.0), (1.0, 0.0, 0.0, 0.0), force=(1e-4, 0, 0))],
                    "bgk", 1.0, storage, 500, counterforce=True, velocity_scale=2e-5)


def c1r(storage="fp64"):
    """c1 with a seeded random orientation and a torque (non-zero rotation)."""
    g = SplitMix64(SEED0 + 0)
    q = g.unit_quaternion()
    return Workload("c1r_settling_32_random", [Box((32, 32, 32))],
                    [Particle((15.5, 15.5, 15.5), (4.0, 2.0, 2.0), q, force=(1e-4, 0, 0),
                              torque=(0.0, 0.0, 1e-3))],
                    "bgk", 1.0, storage, 500, counterforce=True, velocity_scale=2e-5)


def c2(storage="fp32", L=128, lattice=19):
    """L^3 periodic (128 by default), TRT Lambda=3/16 with tau+ = 0.8
    (nu = 0.1), spheroid a=6, b=c=2, long axis at 45 deg to a force 5e-4
    along z, 20 000 steps; D3Q19, or D3Q27 with lattice=27."""
    # body x -> (sin 45, 0, cos 45): rotation about y by +45 deg maps x -> (cos, 0, -sin)
    q = quat_axis_angle((0.0, 1.0, 0.0), -math.pi / 4)
    c = (L - 1) / 2.0
    return Workload(f"c2_inclined_{L}" + ("_d3q27" if lattice == 27 else ""), [Box((L, L, L))],
                    [Particle((c, c, c), (6.0, 2.0, 2.0), q, force=(0.0, 0.0, 5e-4))],
                    "trt", 0.8, storage, 20000, counterforce=True, velocity_scale=1e-4, lattice=lattice)


def settling(L, a=7.5, b=2.5, orientation="end-on", nu=0.1, force=1e-3, storage="fp32", lattice=19, c=None):
    """An ellipsoid (a, b, c) (c = b by default: a spheroid) settling under a
    force at the centre of a periodic L^3 box (Sec. III.A, Figs. 3-4 and 9):
    body x axis along the lab x axis, the force along x ("end-on": along the
    a axis) or along y ("broadside"); TRT with tau = 3 nu + 1/2,
    counter-force on."""
    c_ax = b if c is None else c
    c0 = (L - 1) / 2.0
    F = (force, 0.0, 0.0) if orientation == "end-on" else (0.0, force, 0.0)
    u_est = force / (6 * math.pi * nu * min(a, b, c_ax))
    return Workload(f"settling_{orientation}_L{L}_a{a:g}_b{b:g}_c{c_ax:g}", [Box((L, L, L))],
                    [Particle((c0, c0, c0), (a, b, c_ax), (1.0, 0.0, 0.0, 0.0), force=F)],
                    "trt", 3 * nu + 0.5, storage, 0, counterforce=True, velocity_scale=2 * u_est,
                    max_semi_axis=max(8.0, a, b, c_ax), lattice=lattice, notes={"nu": nu, "orientation": orientation})


def jeffery_box(L, a=6.0, b=2.0, rate=2e-4, nu=0.1, storage="fp32"):
    """A prolate spheroid (a, b, b) at the centre of an L^3 box between walls
    y = 0 and y = L-1 moving at -/+U along x, U chosen for the shear rate
    `rate` between the half-way planes (Sec. III.C, Fig. 6c), started in the
    flow-gradient plane along the flow (body x = lab x); Couette start."""
    U = rate * (L - 2) / 2.0
    c = (L - 1) / 2.0
    return Workload(f"jeffery_L{L}_a{a:g}_b{b:g}",
                    [Box((L, L, L), walls=True, wall_lo=(-U, 0, 0), wall_hi=(U, 0, 0), init="couette")],
                    [Particle((c, c, c), (a, b, b), (1.0, 0.0, 0.0, 0.0))], "trt", 3 * nu + 0.5, storage, 0,
                    velocity_scale=2 * U, max_semi_axis=max(8.0, a), notes={"shear_rate": rate, "nu": nu})


def c3(r=3, seed_index=1, storage="fp32"):
    """64 x 128 x 64 between walls y=0 and y=127 moving at -/+0.01 along x,
    BGK tau=0.8, neutrally buoyant spheroid b=c=3, a=3r, seeded orientation."""
    g = SplitMix64(SEED0 + 2 + 1000 * seed_index + r)
    q = g.unit_quaternion()
    return Workload(f"c3_jeffery_r{r}_s{seed_index}",
                    [Box((64, 128, 64), walls=True, wall_lo=(-0.01, 0, 0), wall_hi=(0.01, 0, 0), init="couette")],
                    [Particle((31.5, 63.5, 31.5), (3.0 * r, 3.0, 3.0), q)],
                    "bgk", 0.8, storage, 0, velocity_scale=0.01, max_semi_axis=12.0,
                    notes={"shear_rate": 0.02 / 126.0})


def c4(storage="fp16", nboxes=256, seed_index=0, torque=True):
    """Ensemble of independent periodic cubic boxes, one spheroid each.

    Edge L uniform on the integers 32..64; aspect ratio r uniform in [1, 5]
    and semi-minor axis b uniform in [2, 4], redrawn until L - 2a >= 8
    (a = r b); body axes (a, b, b); orientation uniform on S^3; centre at the
    box centre plus a uniform sub-lattice offset in [-0.5, 0.5)^3; force of
    magnitude uniform in [1e-5, 1e-4] and torque of magnitude uniform in
    [1e-4, 1e-3], both in uniformly random directions (torque=False keeps
    the same draws and zeroes the torques: force-driven boxes reach a true
    steady state).  TRT, Lambda = 3/16, tau+ = 1 (nu = 1/6), counter-force on."""
    g = SplitMix64(SEED0 + 3 + 1000 * seed_index)
    boxes, parts = [], []
    for i in range(nboxes):
        L = 32 + int(g.uniform() * 33)
        while True:
            r = g.uniform(1.0, 5.0)
            b = g.uniform(2.0, 4.0)
            if L - 2.0 * r * b >= 8.0:
                break
        q = g.unit_quaternion()
        c = tuple((L - 1) / 2.0 + g.uniform(-0.5, 0.5) for _ in range(3))
        fm, tm = g.uniform(1e-5, 1e-4), g.uniform(1e-4, 1e-3)
        fd, td = g.unit_vector(), g.unit_vector()
        boxes.append(Box((L, L, L)))
        parts.append(Particle(c, (r * b, b, b), q, force=tuple(fm * v for v in fd),
                              torque=tuple(tm * v for v in td) if torque else (0.0, 0.0, 0.0), box=i))
    name = f"c4_ensemble_{nboxes}" + (f"_s{seed_index}" if seed_index else "") + ("" if torque else "_force")
    return Workload(name, boxes, parts, "trt", 1.0, storage, 0, counterforce=True,
                    velocity_scale=1e-3, max_semi_axis=20.0)


def empty(storage="fp16", L=256):
    """A periodic L^3 box with no particle (TRT, Lambda = 3/16, tau+ = 1,
    fluid at rest): the collide-stream kernel alone, for its roofline."""
    return Workload(f"empty_{L}", [Box((L, L, L))], [], "trt", 1.0, storage, 0)


MLP_LAYERS = ((64, 8), (64, 64), (6, 64))   # (fan_out, fan_in) of the surrogate's three layers


def xavier_params(gen):
    """Initial surrogate parameters, flat in the order W1, b1, W2, b2, W3, b3:
    weights uniform in +-sqrt(6 / (fan_in + fan_out)) (Glorot & Bengio 2010),
    drawn row by row from `gen` (a SplitMix64), biases zero."""
    out = []
    for fo, fi in MLP_LAYERS:
        lim = math.sqrt(6.0 / (fi + fo))
        out += [gen.uniform(-lim, lim) for _ in range(fo * fi)]
        out += [0.0] * fo
    import numpy as np
    return np.array(out)


def _aabb_half(axes, q):
    """Half-extents of the axis-aligned box around an ellipsoid: sqrt(sum_j (R_kj a_j)^2)."""
    q0, q1, q2, q3 = q
    R = ((1 - 2 * (q2 * q2 + q3 * q3), 2 * (q1 * q2 - q0 * q3), 2 * (q1 * q3 + q0 * q2)),
         (2 * (q1 * q2 + q0 * q3), 1 - 2 * (q1 * q1 + q3 * q3), 2 * (q2 * q3 - q0 * q1)),
         (2 * (q1 * q3 - q0 * q2), 2 * (q2 * q3 + q0 * q1), 1 - 2 * (q1 * q1 + q2 * q2)))
    return tuple(math.sqrt(sum((R[k][j] * axes[j]) ** 2 for j in range(3))) for k in range(3))


def c5(storage="fp16", L=256, n=512, seed_index=0):
    """Suspension of n spheroidal squirmers a=5, b=c=2.5 in a periodic L^3
    box (defaults 256^3, 512): centres uniform, orientations uniform on S^3,
    placed one by one and redrawn while the bounding boxes (with a gap of 2
    nodes) of two particles overlap under the minimum image; B1 = 1e-3,
    B2 = beta B1 with beta uniform in [-3, 3].  TRT, Lambda = 3/16, tau+ = 1."""
    import numpy as np
    g = SplitMix64(SEED0 + 5 + 1000 * seed_index)
    axes = (5.0, 2.5, 2.5)
    parts = []
    cs = np.zeros((n, 3))
    hs = np.zeros((n, 3))
    while len(parts) < n:
        c = tuple(g.uniform(0.0, float(L)) for _ in range(3))
        q = g.unit_quaternion()
        h = _aabb_half(axes, q)
        m = len(parts)
        if m:
            d = np.abs(np.asarray(c) - cs[:m])
            d = np.minimum(d, L - d)
            if np.any(np.all(d < np.asarray(h) + hs[:m] + 2.0, axis=1)):
                continue
        beta = g.uniform(-3.0, 3.0)
        cs[m], hs[m] = c, h
        parts.append(Particle(c, axes, q, squirmer=(1e-3, beta * 1e-3)))
    return Workload(f"c5_squirmers_{L}_{n}" + (f"_s{seed_index}" if seed_index else ""), [Box((L, L, L))], parts,
                    "trt", 1.0, storage, 10000,
                    velocity_scale=2e-3, max_semi_axis=5.0)
