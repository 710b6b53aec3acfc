"""FP64 CPU oracle for the lattice Boltzmann method with rigid ellipsoids.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by the package smoke check
and by the CPU-baseline leg of ``bench.py``; never by the product path.  The
arithmetic lives in ``lbe_oracle.c`` (plain C, full populations, the paper's
Appendix A order); this module only marshals arguments through ctypes.
It shares no code with the HIP library.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbe_oracle.c")
_LIB = os.path.join(_HERE, "liblbe_oracle.so")

COLLISIONS = {"bgk": 0, "trt": 1, "reg": 2}


def build(force=True):
    """Compile the oracle with gcc (FP contraction off, OpenMP over sites)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-shared", "-fPIC", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None
_D = C.POINTER(C.c_double)


def _arr(a, dtype=np.float64):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def _ptr(a):
    return a.ctypes.data_as(_D)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        vp = C.c_void_p
        L.or_create.restype = vp
        L.or_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                C.c_int, _D, _D, C.c_int, C.c_int]
        L.or_create_q.restype = vp
        L.or_create_q.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                  C.c_int, _D, _D, C.c_int, C.c_int, C.c_int]
        L.or_equilibrium_q.argtypes = [C.c_int, C.c_double, _D, _D]
        L.or_lattice_q.argtypes = [C.c_int, C.POINTER(C.c_int), _D]
        L.or_set_rotation.argtypes = [vp, C.c_int]
        L.or_destroy.argtypes = [vp]
        L.or_add_ellipsoid.argtypes = [vp, _D, _D, _D]
        for name in ("or_set_external", "or_set_velocity"):
            getattr(L, name).argtypes = [vp, C.c_int, _D, _D]
        L.or_set_squirmer.argtypes = [vp, C.c_int, C.c_double, C.c_double]
        L.or_set_density.argtypes = [vp, C.c_int, C.c_double]
        L.or_step.argtypes = [vp, C.c_int]
        L.or_get_particle.argtypes = [vp, C.c_int, _D, _D, _D, _D]
        L.or_get_force_torque.argtypes = [vp, C.c_int, _D, _D]
        L.or_get_aux.argtypes = [vp, C.c_int, _D, _D, _D, _D, C.POINTER(C.c_int)]
        L.or_get_zeta.argtypes = [vp, C.c_int, _D]
        L.or_get_links.argtypes = [vp, C.c_int, C.POINTER(C.c_uint32), C.POINTER(C.c_uint8),
                                   C.c_int]
        L.or_get_mask.argtypes = [vp, C.POINTER(C.c_uint16)]
        L.or_get_fields.argtypes = [vp, _D, _D]
        L.or_get_mass.argtypes = [vp]
        L.or_get_mass.restype = C.c_double
        L.or_get_momentum.argtypes = [vp, _D]
        L.or_get_step.argtypes = [vp]
        L.or_get_step.restype = C.c_longlong
        L.or_overlap_count.argtypes = [vp]
        L.or_get_f.argtypes = [vp, _D]
        L.or_set_f.argtypes = [vp, _D]
        L.or_stream_only.argtypes = [vp]
        L.or_equilibrium.argtypes = [C.c_double, _D, _D]
        L.or_collide_node.argtypes = [vp, _D, _D]
        L.or_inside.argtypes = [C.c_int, C.c_int, C.c_int, _D, _D, _D, C.c_int, C.c_int,
                                C.c_int]
        L.or_inertia_lab.argtypes = [_D, _D, _D]
        L.or_inertia_dot.argtypes = [_D, _D, _D, _D]
        L.or_solve6.argtypes = [_D, _D, _D]
        L.or_quat_update.argtypes = [_D, _D, _D]
        L.or_squirmer_slip.argtypes = [_D, _D, C.c_double, C.c_double, _D, _D]
        L.or_lattice.argtypes = [C.POINTER(C.c_int), _D]
        _lib = L
    return _lib


# ----------------------------- single pieces --------------------------------

def lattice(q=19):
    """Velocities (q, 3) and weights of the D3Q19 (q = 19) or D3Q27 set."""
    c = np.zeros(3 * q, dtype=np.int32)
    w = np.zeros(q)
    lib().or_lattice_q(int(q), c.ctypes.data_as(C.POINTER(C.c_int)), _ptr(w))
    return c.reshape(q, 3), w


def equilibrium(rho, u, q=19):
    u = _arr(u)
    out = np.zeros(q)
    lib().or_equilibrium_q(int(q), float(rho), _ptr(u), _ptr(out))
    return out


def inside(shape, centre, axes, quat, x, y, z):
    c, a, q = _arr(centre), _arr(axes), _arr(quat)
    return bool(lib().or_inside(shape[0], shape[1], shape[2], _ptr(c), _ptr(a), _ptr(q),
                                int(x), int(y), int(z)))


def inertia_lab(q, Ib):
    q, Ib = _arr(q), _arr(Ib)
    out = np.zeros(9)
    lib().or_inertia_lab(_ptr(q), _ptr(Ib), _ptr(out))
    return out.reshape(3, 3)


def inertia_dot(q, Ib, W):
    q, Ib, W = _arr(q), _arr(Ib), _arr(W)
    out = np.zeros(9)
    lib().or_inertia_dot(_ptr(q), _ptr(Ib), _ptr(W), _ptr(out))
    return out.reshape(3, 3)


def solve6(A, b):
    A, b = _arr(A).reshape(36), _arr(b)
    x = np.zeros(6)
    rc = lib().or_solve6(_ptr(A), _ptr(b), _ptr(x))
    if rc != 0:
        raise ZeroDivisionError("singular 6x6 system")
    return x


def quat_update(q, Wmean):
    q, W = _arr(q), _arr(Wmean)
    out = np.zeros(4)
    lib().or_quat_update(_ptr(q), _ptr(W), _ptr(out))
    return out


def squirmer_slip(axes, q, B1, B2, d):
    a, q, d = _arr(axes), _arr(q), _arr(d)
    out = np.zeros(3)
    lib().or_squirmer_slip(_ptr(a), _ptr(q), float(B1), float(B2), _ptr(d), _ptr(out))
    return out


# ------------------------------- simulation ---------------------------------

class OracleSim:
    """One periodic (or wall-bounded) box stepped by the FP64 oracle."""

    def __init__(self, shape, collision="bgk", tau=1.0, magic=3.0 / 16.0, walls=False,
                 wall_lo=(0, 0, 0), wall_hi=(0, 0, 0), init="rest", counterforce=False, lattice=19,
                 rotation=0):
        self.shape = tuple(int(v) for v in shape)
        self.n = self.shape[0] * self.shape[1] * self.shape[2]
        self.q = int(lattice)
        ulo, uhi = _arr(wall_lo), _arr(wall_hi)
        self._h = lib().or_create_q(self.shape[0], self.shape[1], self.shape[2],
                                    COLLISIONS[collision], float(tau), float(magic),
                                    int(bool(walls)), _ptr(ulo), _ptr(uhi),
                                    {"rest": 0, "couette": 1}[init], int(bool(counterforce)), self.q)
        if not self._h:
            raise ValueError(f"lattice must be 19 or 27, got {lattice}")
        if lib().or_set_rotation(self._h, int(rotation)) != 0:
            raise ValueError(f"rotation must be 0, 1 or 2, got {rotation}")
        self.np = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_destroy(h)
            self._h = None

    def add_ellipsoid(self, centre, axes, quat):
        c, a, q = _arr(centre), _arr(axes), _arr(quat)
        rc = lib().or_add_ellipsoid(self._h, _ptr(c), _ptr(a), _ptr(q))
        if rc < 0:
            raise ValueError("overlap while adding the ellipsoid")
        self.np += 1
        return rc

    def set_external(self, pid, F, T=(0, 0, 0)):
        F, T = _arr(F), _arr(T)
        lib().or_set_external(self._h, pid, _ptr(F), _ptr(T))

    def set_squirmer(self, pid, B1, B2):
        lib().or_set_squirmer(self._h, pid, float(B1), float(B2))

    def set_velocity(self, pid, U, W=(0, 0, 0)):
        U, W = _arr(U), _arr(W)
        lib().or_set_velocity(self._h, pid, _ptr(U), _ptr(W))

    def set_density(self, pid, rho_p):
        lib().or_set_density(self._h, pid, float(rho_p))

    def step(self, n=1):
        rc = lib().or_step(self._h, int(n))
        if rc == -6:
            raise FloatingPointError("singular system or non-finite particle velocity")
        return rc

    def particle(self, pid):
        x, q, U, W = np.zeros(3), np.zeros(4), np.zeros(3), np.zeros(3)
        lib().or_get_particle(self._h, pid, _ptr(x), _ptr(q), _ptr(U), _ptr(W))
        return {"x": x, "q": q, "U": U, "W": W}

    def force_torque(self, pid):
        F, T = np.zeros(3), np.zeros(3)
        lib().or_get_force_torque(self._h, pid, _ptr(F), _ptr(T))
        return F, T

    def aux(self, pid):
        M, dm, P, L = np.zeros(1), np.zeros(1), np.zeros(3), np.zeros(3)
        nl = C.c_int(0)
        lib().or_get_aux(self._h, pid, _ptr(M), _ptr(dm), _ptr(P), _ptr(L), C.byref(nl))
        return {"M": M[0], "dm": dm[0], "P": P, "L": L, "nlinks": nl.value}

    def zeta(self, pid):
        z = np.zeros(36)
        lib().or_get_zeta(self._h, pid, _ptr(z))
        return z.reshape(6, 6)

    def links(self, pid):
        n = lib().or_get_links(self._h, pid, None, None, 0)
        site = np.zeros(max(n, 1), dtype=np.uint32)
        d = np.zeros(max(n, 1), dtype=np.uint8)
        lib().or_get_links(self._h, pid, site.ctypes.data_as(C.POINTER(C.c_uint32)),
                           d.ctypes.data_as(C.POINTER(C.c_uint8)), n)
        return site[:n], d[:n]

    def mask(self):
        m = np.zeros(self.n, dtype=np.uint16)
        lib().or_get_mask(self._h, m.ctypes.data_as(C.POINTER(C.c_uint16)))
        return m

    def fields(self):
        rho, u = np.zeros(self.n), np.zeros(3 * self.n)
        lib().or_get_fields(self._h, _ptr(rho), _ptr(u))
        return rho, u.reshape(self.n, 3)

    def mass(self):
        return lib().or_get_mass(self._h)

    def momentum(self):
        P = np.zeros(3)
        lib().or_get_momentum(self._h, _ptr(P))
        return P

    def step_count(self):
        return lib().or_get_step(self._h)

    def overlaps(self):
        return lib().or_overlap_count(self._h)

    def get_f(self):
        f = np.zeros(self.n * self.q)
        lib().or_get_f(self._h, _ptr(f))
        return f.reshape(self.n, self.q)

    def set_f(self, f):
        f = _arr(f).reshape(self.n * self.q)
        lib().or_set_f(self._h, _ptr(f))

    def stream_only(self):
        lib().or_stream_only(self._h)

    def collide_node(self, f):
        f = _arr(f)
        out = np.zeros(self.q)
        lib().or_collide_node(self._h, _ptr(f), _ptr(out))
        return out
