"""Python binding of the C ABI in include/lbell.h (argument marshalling only).

Every step of the method runs in the HIP kernels of liblbell.so; PyTorch only
supplies the device arena (one uint8 tensor) and the HIP stream.  Loading
fails loudly when the library has not been built: there is no fallback.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbell.so")

BGK, TRT, REG = 0, 1, 2
FP64, FP32, FP16, BF16 = 0, 1, 2, 3
COLLISION = {"bgk": BGK, "trt": TRT, "reg": REG}
STORAGE = {"fp64": FP64, "fp32": FP32, "fp16": FP16, "bf16": BF16}
# inertia term of the rotational update (Sec. II.D): analytic rate, backward
# difference, predictor-corrector
ROTATION = {"analytic": 0, "fd": 1, "pc": 2}

STATUS = {0: "LB_OK", -1: "LB_EINVAL", -2: "LB_ENOMEM", -3: "LB_EDEVICE", -4: "LB_ESTATE",
          -5: "LB_EOVERLAP", -6: "LB_ENONFINITE", -7: "LB_ERANGE", -8: "LB_EIO"}
LB_EOVERLAP = -5


class LBError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {msg}")


class Config(C.Structure):
    _fields_ = [("lattice", C.c_int), ("collision", C.c_int), ("tau", C.c_double),
                ("magic", C.c_double), ("storage", C.c_int), ("scale_log2", C.c_int),
                ("velocity_scale", C.c_double), ("rho0", C.c_double), ("counterforce", C.c_int),
                ("max_particles", C.c_int), ("max_semi_axis", C.c_double), ("rotation", C.c_int),
                ("monitor_period", C.c_int)]


class Box(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("walls", C.c_int),
                ("wall_lo", C.c_double * 3), ("wall_hi", C.c_double * 3), ("init", C.c_int)]


# every entry point of include/lbell.h with its argument types
_D = C.POINTER(C.c_double)
_F = C.POINTER(C.c_float)
_VP = C.c_void_p
SIGNATURES = {
    "lb_config_default": (C.c_int, [C.POINTER(Config)]),
    "lb_arena_bytes": (C.c_size_t, [C.POINTER(Config), C.c_int, C.POINTER(Box)]),
    "lb_init": (C.c_int, [C.POINTER(Config), C.c_int, C.POINTER(Box), _VP, C.c_size_t, _VP,
                          C.POINTER(_VP)]),
    "lb_add_ellipsoid": (C.c_int, [_VP, C.c_int, _D, _D, _D, C.POINTER(C.c_int)]),
    "lb_set_external": (C.c_int, [_VP, C.c_int, _D, _D]),
    "lb_set_squirmer": (C.c_int, [_VP, C.c_int, C.c_double, C.c_double]),
    "lb_set_velocity": (C.c_int, [_VP, C.c_int, _D, _D]),
    "lb_set_particle_density": (C.c_int, [_VP, C.c_int, C.c_double]),
    "lb_step": (C.c_int, [_VP, C.c_int]),
    "lb_profile_step": (C.c_int, [_VP, C.c_int, _D, _D]),
    "lb_autotune": (C.c_int, [_VP, C.c_int, C.POINTER(C.c_int), _D]),
    "lb_bandwidth_probe": (C.c_int, [_VP, _VP, C.c_size_t, _VP, C.c_int, _D]),
    "lb_set_graph": (C.c_int, [_VP, C.c_int]),
    "lb_sync": (C.c_int, [_VP]),
    "lb_get_force_torque": (C.c_int, [_VP, C.c_int, _D, _D]),
    "lb_get_particle": (C.c_int, [_VP, C.c_int, _D, _D, _D, _D]),
    "lb_get_particle_aux": (C.c_int, [_VP, C.c_int, _D, _D, _D, _D, C.POINTER(C.c_int)]),
    "lb_get_links": (C.c_int, [_VP, C.c_int, C.POINTER(C.c_uint32), C.POINTER(C.c_uint8), C.c_int,
                               C.POINTER(C.c_int)]),
    "lb_get_mask": (C.c_int, [_VP, C.c_int, C.POINTER(C.c_uint16)]),
    "lb_get_fields": (C.c_int, [_VP, C.c_int, _D, _D]),
    "lb_get_mass": (C.c_int, [_VP, C.c_int, _D]),
    "lb_get_momentum": (C.c_int, [_VP, C.c_int, _D]),
    "lb_check_finite": (C.c_int, [_VP, C.c_int, C.POINTER(C.c_longlong)]),
    "lb_get_step": (C.c_int, [_VP, C.POINTER(C.c_longlong)]),
    "lb_save": (C.c_int, [_VP, C.c_char_p]),
    "lb_load": (C.c_int, [_VP, C.c_char_p]),
    "lb_debug_poke": (C.c_int, [_VP, C.c_int, C.c_int, C.c_int, C.c_double]),
    "lb_get_particles": (C.c_int, [_VP, C.c_int, C.c_int, _D, _D, _D, _D]),
    "lb_stokes_start": (C.c_int, [_VP]),
    "lb_warm_start": (C.c_int, [_VP, C.c_int, _VP, C.c_double, _D]),
    "lb_warm_status": (C.c_int, [_VP, C.POINTER(C.c_int), C.POINTER(C.c_longlong)]),
    "lb_surrogate_sample": (C.c_int, [_VP, _F, _F]),
    "lbs_arena_bytes": (C.c_size_t, [C.c_int]),
    "lbs_create": (C.c_int, [C.c_int, _VP, C.c_size_t, _VP, C.POINTER(_VP)]),
    "lbs_set_params": (C.c_int, [_VP, _F]),
    "lbs_get_params": (C.c_int, [_VP, _F]),
    "lbs_train": (C.c_int, [_VP, _F, _F, C.c_int, C.c_int, C.c_int, C.c_float, _F]),
    "lbs_predict": (C.c_int, [_VP, _F, C.c_int, _F]),
    "lbs_grad": (C.c_int, [_VP, _F, _F, C.c_int, _F, _F]),
    "lbs_grad_noalloc": (C.c_int, [_VP, _VP, _VP, C.c_int, _VP, _VP, _VP]),
    "lbs_destroy": (C.c_int, [_VP]),
    "lb_destroy": (C.c_int, [_VP]),
    "lb_status_str": (C.c_char_p, [C.c_int]),
    "lb_last_error": (C.c_char_p, [_VP]),
}

_lib = None


def load():
    """Load liblbell.so (built in-tree by __graft_entry__.build()).

    torch is imported first: its wheel carries its own HIP runtime, and the
    library must bind to that same runtime (same soname) rather than bring a
    second one into the process."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (load order: one HIP runtime per process)
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _vec(x, n):
    a = np.ascontiguousarray(x, dtype=np.float64).reshape(n)
    return a


def _p(a):
    return a.ctypes.data_as(_D)


def make_box(nx, ny, nz, walls=False, wall_lo=(0, 0, 0), wall_hi=(0, 0, 0), init="rest"):
    b = Box()
    b.nx, b.ny, b.nz = int(nx), int(ny), int(nz)
    b.walls = int(bool(walls))
    for k in range(3):
        b.wall_lo[k] = float(wall_lo[k])
        b.wall_hi[k] = float(wall_hi[k])
    b.init = {"rest": 0, "couette": 1}[init]
    return b


def bandwidth_probe(nbytes=1 << 30, reps=10, device="cuda:0"):
    """Achieved device copy bandwidth (read + write) in GB/s of the library's
    16-byte-access copy kernel; buffers come from torch."""
    import torch
    lib = load()
    nbytes = (int(nbytes) // 16) * 16
    src = torch.empty(nbytes, dtype=torch.uint8, device=device)
    dst = torch.empty_like(src)
    gbs = np.zeros(1)
    st = lib.lb_bandwidth_probe(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), C.c_size_t(nbytes),
                                C.c_void_p(torch.cuda.current_stream(device).cuda_stream), int(reps), _p(gbs))
    if st != 0:
        raise LBError(st, "bandwidth probe failed")
    return gbs[0]


class Lattice:
    """A context of one or more boxes on one GPU.

    boxes: list of Box (make_box) or (nx, ny, nz) tuples."""

    def __init__(self, boxes, collision="bgk", tau=1.0, magic=3.0 / 16.0, storage="fp32",
                 scale_log2=0, velocity_scale=1e-3, counterforce=False, max_particles=0,
                 max_semi_axis=8.0, lattice=19, rotation="analytic", monitor_period=25, device="cuda:0"):
        import torch
        self.lib = load()
        self.torch = torch
        cfg = Config()
        self.lib.lb_config_default(C.byref(cfg))
        cfg.collision = COLLISION[collision] if isinstance(collision, str) else int(collision)
        cfg.tau = float(tau)
        cfg.magic = float(magic)
        cfg.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        cfg.scale_log2 = int(scale_log2)
        cfg.velocity_scale = float(velocity_scale)
        cfg.counterforce = int(bool(counterforce))
        cfg.max_particles = int(max_particles)
        cfg.max_semi_axis = float(max_semi_axis)
        cfg.lattice = int(lattice)
        cfg.rotation = ROTATION[rotation] if isinstance(rotation, str) else int(rotation)
        cfg.monitor_period = int(monitor_period)
        self.cfg = cfg
        bl = [b if isinstance(b, Box) else make_box(*b) for b in boxes]
        self.nboxes = len(bl)
        self.boxes = (Box * len(bl))(*bl)
        self.shapes = [(b.nx, b.ny, b.nz) for b in bl]
        nbytes = self.lib.lb_arena_bytes(C.byref(cfg), self.nboxes, self.boxes)
        if nbytes == 0:
            raise LBError(-1, "invalid configuration")
        self.device = torch.device(device)
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.arena.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        st = self.lib.lb_init(C.byref(cfg), self.nboxes, self.boxes, C.c_void_p(aligned),
                              C.c_size_t(nbytes), C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        if st != 0:
            raise LBError(st, "lb_init failed")
        self.ctx = ctx
        self.np = 0

    # -- helpers --------------------------------------------------------------
    def _chk(self, st):
        if st != 0:
            msg = self.lib.lb_last_error(self.ctx)
            raise LBError(st, msg.decode() if msg else "")
        return st

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.lb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- set-up ---------------------------------------------------------------
    def add_ellipsoid(self, centre, axes, quat, box=0):
        c, a, q = _vec(centre, 3), _vec(axes, 3), _vec(quat, 4)
        pid = C.c_int(-1)
        self._chk(self.lib.lb_add_ellipsoid(self.ctx, int(box), _p(c), _p(a), _p(q), C.byref(pid)))
        self.np += 1
        return pid.value

    def set_external(self, pid, F, T=(0, 0, 0)):
        F, T = _vec(F, 3), _vec(T, 3)
        self._chk(self.lib.lb_set_external(self.ctx, int(pid), _p(F), _p(T)))

    def set_squirmer(self, pid, B1, B2):
        self._chk(self.lib.lb_set_squirmer(self.ctx, int(pid), float(B1), float(B2)))

    def set_velocity(self, pid, U, W=(0, 0, 0)):
        U, W = _vec(U, 3), _vec(W, 3)
        self._chk(self.lib.lb_set_velocity(self.ctx, int(pid), _p(U), _p(W)))

    def set_density(self, pid, rho_p):
        self._chk(self.lib.lb_set_particle_density(self.ctx, int(pid), float(rho_p)))

    # -- stepping -------------------------------------------------------------
    def step(self, n=1):
        self._chk(self.lib.lb_step(self.ctx, int(n)))

    def profile_step(self, n):
        """(ms in collide-stream, ms in the particle phase) summed over n steps."""
        a, b = np.zeros(1), np.zeros(1)
        self._chk(self.lib.lb_profile_step(self.ctx, int(n), _p(a), _p(b)))
        return a[0], b[0]

    def autotune(self, reps=20):
        """Pick the fastest collide-stream variant, timed inside real steps (the
        simulation advances by those steps); returns (variant, ms per launch)."""
        v, ms = C.c_int(0), np.zeros(1)
        self._chk(self.lib.lb_autotune(self.ctx, int(reps), C.byref(v), _p(ms)))
        return v.value, ms[0]

    def set_graph(self, steps):
        """Run lb_step in HIP graphs of `steps` steps (0: plain launches)."""
        self._chk(self.lib.lb_set_graph(self.ctx, int(steps)))

    def sync(self):
        self._chk(self.lib.lb_sync(self.ctx))

    # -- read-back ------------------------------------------------------------
    def particle(self, pid):
        x, q, U, W = np.zeros(3), np.zeros(4), np.zeros(3), np.zeros(3)
        self._chk(self.lib.lb_get_particle(self.ctx, int(pid), _p(x), _p(q), _p(U), _p(W)))
        return {"x": x, "q": q, "U": U, "W": W}

    def force_torque(self, pid):
        F, T = np.zeros(3), np.zeros(3)
        self._chk(self.lib.lb_get_force_torque(self.ctx, int(pid), _p(F), _p(T)))
        return F, T

    def aux(self, pid):
        M, dm, P, L = np.zeros(1), np.zeros(1), np.zeros(3), np.zeros(3)
        nl = C.c_int(0)
        self._chk(self.lib.lb_get_particle_aux(self.ctx, int(pid), _p(M), _p(dm), _p(P), _p(L),
                                               C.byref(nl)))
        return {"M": M[0], "dm": dm[0], "P": P, "L": L, "nlinks": nl.value}

    def links(self, pid):
        n = C.c_int(0)
        st = self.lib.lb_get_links(self.ctx, int(pid), None, None, 0, C.byref(n))
        if st not in (0, -7):
            self._chk(st)
        cnt = n.value
        site = np.zeros(max(cnt, 1), dtype=np.uint32)
        d = np.zeros(max(cnt, 1), dtype=np.uint8)
        self._chk(self.lib.lb_get_links(self.ctx, int(pid), site.ctypes.data_as(C.POINTER(C.c_uint32)),
                                        d.ctypes.data_as(C.POINTER(C.c_uint8)), cnt, C.byref(n)))
        return site[:cnt], d[:cnt]

    def mask(self, box=0):
        nx, ny, nz = self.shapes[box]
        m = np.zeros(nx * ny * nz, dtype=np.uint16)
        self._chk(self.lib.lb_get_mask(self.ctx, int(box), m.ctypes.data_as(C.POINTER(C.c_uint16))))
        return m

    def fields(self, box=0):
        nx, ny, nz = self.shapes[box]
        n = nx * ny * nz
        rho, u = np.zeros(n), np.zeros(3 * n)
        self._chk(self.lib.lb_get_fields(self.ctx, int(box), _p(rho), _p(u)))
        return rho, u.reshape(n, 3)

    def mass(self, box=0):
        m = np.zeros(1)
        self._chk(self.lib.lb_get_mass(self.ctx, int(box), _p(m)))
        return m[0]

    def momentum(self, box=0):
        P = np.zeros(3)
        self._chk(self.lib.lb_get_momentum(self.ctx, int(box), _p(P)))
        return P

    def nonfinite(self, box=0):
        c = C.c_longlong(0)
        self._chk(self.lib.lb_check_finite(self.ctx, int(box), C.byref(c)))
        return c.value

    def step_count(self):
        c = C.c_longlong(0)
        self._chk(self.lib.lb_get_step(self.ctx, C.byref(c)))
        return c.value

    def save(self, path):
        self._chk(self.lib.lb_save(self.ctx, str(path).encode()))

    def load(self, path):
        self._chk(self.lib.lb_load(self.ctx, str(path).encode()))

    def poke(self, box, site, direction, value):
        self._chk(self.lib.lb_debug_poke(self.ctx, int(box), int(site), int(direction), float(value)))

    def particles(self, first=0, count=None):
        """Bulk read-back: dict of arrays x (n,3), q (n,4), U (n,3), W (n,3)."""
        n = self.np - first if count is None else int(count)
        x, q, U, W = np.zeros((n, 3)), np.zeros((n, 4)), np.zeros((n, 3)), np.zeros((n, 3))
        self._chk(self.lib.lb_get_particles(self.ctx, int(first), n, _p(x), _p(q), _p(U), _p(W)))
        return {"x": x, "q": q, "U": U, "W": W}

    def stokes_start(self):
        """Start the fluid from the creeping flow of the particles' current velocities."""
        self._chk(self.lib.lb_stokes_start(self.ctx))

    def warm_start(self, surrogate, box=-1, tol=0.0):
        """Surrogate warm start of the particles of `box` (-1: every box);
        with tol > 0 the boxes are watched on the device and fall back to
        the plain start when the prediction fails (lb_warm_start).  Returns
        the predicted lab-frame (U, Omega) per particle, shape (np, 6)."""
        pred = np.zeros((max(self.np, 1), 6))
        self._chk(self.lib.lb_warm_start(self.ctx, int(box), surrogate.handle, float(tol), _p(pred)))
        return pred[:self.np]

    WARM_STATUS = {0: "off", 1: "pending", 2: "accepted", 3: "fallback", 4: "steady_miss"}

    def warm_status(self):
        """(status per box as LB_WARM_* codes, decision step per box)."""
        st = np.zeros(self.nboxes, dtype=np.int32)
        at = np.zeros(self.nboxes, dtype=np.int64)
        self._chk(self.lib.lb_warm_status(self.ctx, st.ctypes.data_as(C.POINTER(C.c_int)),
                                          at.ctypes.data_as(C.POINTER(C.c_longlong))))
        return st, at


def _fp(a):
    return a.ctypes.data_as(_F)


def _lattice_sample(self):
    """(X, Y): surrogate inputs and normalised responses of every particle now."""
    X = np.zeros((max(self.np, 1), 8), dtype=np.float32)
    Y = np.zeros((max(self.np, 1), 6), dtype=np.float32)
    self._chk(self.lib.lb_surrogate_sample(self.ctx, _fp(X), _fp(Y)))
    return X[:self.np], Y[:self.np]


Lattice.surrogate_sample = _lattice_sample


class Surrogate:
    """The warm-start network on the GPU (8 -> 64 -> 64 -> 6, bfloat16 matrix
    products); parameters, Adam state and data live in a torch-allocated arena."""

    N_PARAMS = 5126

    def __init__(self, max_samples=65536, params=None, device="cuda:0"):
        import torch
        self.lib = load()
        self.max_samples = int(max_samples)
        nbytes = self.lib.lbs_arena_bytes(self.max_samples)
        if nbytes == 0:
            raise LBError(-1, "invalid surrogate capacity")
        self.device = torch.device(device)
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.arena.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = self.lib.lbs_create(self.max_samples, C.c_void_p(aligned), C.c_size_t(nbytes),
                                 C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != 0:
            raise LBError(st, "lbs_create failed")
        self.handle = h
        if params is not None:
            self.set_params(params)

    def _chk(self, st, what):
        if st != 0:
            raise LBError(st, what)

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32).reshape(self.N_PARAMS)
        self._chk(self.lib.lbs_set_params(self.handle, _fp(p)), "lbs_set_params")

    def params(self):
        p = np.zeros(self.N_PARAMS, dtype=np.float32)
        self._chk(self.lib.lbs_get_params(self.handle, _fp(p)), "lbs_get_params")
        return p

    @staticmethod
    def _xy(X, Y=None):
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, 8)
        if Y is not None:
            Y = np.ascontiguousarray(Y, dtype=np.float32).reshape(-1, 6)
        return X, Y

    def train(self, X, Y, epochs, batch=256, lr=1e-3):
        """Adam over the samples in their given order; returns the last epoch's mean loss."""
        X, Y = self._xy(X, Y)
        loss = np.zeros(1, dtype=np.float32)
        self._chk(self.lib.lbs_train(self.handle, _fp(X), _fp(Y), X.shape[0], int(epochs), int(batch),
                                     float(lr), _fp(loss)), "lbs_train")
        return float(loss[0])

    def predict(self, X):
        X, _ = self._xy(X)
        Y = np.zeros((X.shape[0], 6), dtype=np.float32)
        self._chk(self.lib.lbs_predict(self.handle, _fp(X), X.shape[0], _fp(Y)), "lbs_predict")
        return Y

    def grad(self, X, Y):
        """(loss, gradient) of the mean squared error."""
        X, Y = self._xy(X, Y)
        g = np.zeros(self.N_PARAMS, dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        self._chk(self.lib.lbs_grad(self.handle, _fp(X), _fp(Y), X.shape[0], _fp(g), _fp(loss)), "lbs_grad")
        return float(loss[0]), g

    def close(self):
        if getattr(self, "handle", None):
            self.lib.lbs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
