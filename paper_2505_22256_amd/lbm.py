"""Python binding of the C ABI in include/lbm.h (argument marshalling only).

Every compute step runs in the HIP library ``liblbm.so`` built for gfx950;
this module converts NumPy arrays to pointers and return codes to
exceptions.  The module-level functions carry the C names; ``Lattice`` and
``Batch`` wrap a context for convenience.  Importing works without a GPU;
creating a context needs an MI355X and raises ``LbmError`` otherwise.  There
is no CPU fallback: a missing library raises at load time.

Device pointers handed to the library (``Lattice(buffers=...)``, stream
handles) must come from the HIP runtime it is bound to.  PyTorch for ROCm
ships its own copy of that runtime under the same soname, so
``load_library`` imports torch (when it is installed) before it loads the
library: the library then binds to torch's copy, and torch tensors and
streams are valid here.  A process that loaded liblbm.so by other means
before importing torch would hold two runtimes, whose pointers the other
does not know (``lbm_create_ex`` refuses them).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

OK, EINVAL, ESTATE, ENOMEM, EDEVICE, EUNSTABLE, EIO = 0, -1, -2, -3, -4, -5, -6
F64, F32, F16, BF16 = 0, 1, 2, 3
PERIODIC_X, PERIODIC_Y = 1, 2
SCHEME_ORIGINAL, E8_COPY_OFF, WALLPSI_SELF, VEL_LITERAL, FORCE_DENSITY = 4, 8, 16, 32, 64
ROUND_STOCHASTIC = 128
INLET, OUTFLOW = 256, 512
ROUND_NEAREST = 1024
WALL_FLAT, WALL_CYLINDER = 0, 1
L3_PERIODIC_Z = 2048
L3_WALL_FLAT, L3_WALL_SPHERE = 0, 1
SCHED_ALIGN, SCHED_BANDS, SCHED_XCD_SLABS, SCHED_TWO_STEP, SCHED_REPULL = 1, 2, 4, 8, 16
STORAGE_NAMES = {F64: "f64", F32: "f32", F16: "f16", BF16: "bf16"}

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_U = ctypes.c_uint
_L = ctypes.c_long


class LbmRunDesc(ctypes.Structure):
    _fields_ = [("nx", _I), ("ny", _I), ("flags", _U), ("G_c", _D), ("G_ads", _D), ("tau", _D),
                ("wall_kind", _I), ("wall", _D * 3), ("solid", _P), ("rho1", _P), ("rho2", _P),
                ("accel", _P)]


# name -> (restype, argtypes); the exported symbol set of include/lbm.h
SIGNATURES = {
    "lbm_create": (_I, [ctypes.POINTER(_P), _I, _I, _I, _U]),
    "lbm_create_ex": (_I, [ctypes.POINTER(_P), _I, _I, _I, _U, _P, _P, ctypes.c_size_t]),
    "lbm_population_bytes": (ctypes.c_size_t, [_I, _I, _I]),
    "lbm_current_buffer": (_I, [_P]),
    "lbm_get_flags": (_U, [_P]),
    "lbm_set_geometry": (_I, [_P, _P]),
    "lbm_set_params": (_I, [_P, _D, _D, _D]),
    "lbm_set_adhesion": (_I, [_P, _D, _D, _D]),
    "lbm_set_body_accel": (_I, [_P, _D, _D, _D, _D]),
    "lbm_set_wall_velocity": (_I, [_P, _D, _D, _D, _D]),
    "lbm_set_inlet_velocity": (_I, [_P, _P, _P]),
    "lbm_init_fields": (_I, [_P, _P, _P]),
    "lbm_set_populations": (_I, [_P, _P]),
    "lbm_get_populations": (_I, [_P, _P]),
    "lbm_get_populations_window": (_I, [_P, _I, _I, _I, _I, _P]),
    "lbm_step": (_I, [_P, _I]),
    "lbm_set_diag_interval": (_I, [_P, _I]),
    "lbm_get_diag": (_I, [_P, _P, ctypes.POINTER(_L)]),
    "lbm_synchronize": (_I, [_P]),
    "lbm_time": (_L, [_P]),
    "lbm_get_fields": (_I, [_P, _P, _P, _P, _P]),
    "lbm_reduce": (_I, [_P, _P]),
    "lbm_reduce_noalloc": (_I, [_P, _P]),
    "lbm_contact_angle": (_I, [_P, _I, _P, ctypes.POINTER(_D)]),
    "lbm_get_tables": (_I, [_P, _P, _P, _P, ctypes.POINTER(_I)]),
    "lbm_set_stream": (_I, [_P, _P]),
    "lbm_set_tile": (_I, [_P, _I, _I, _U]),
    "lbm_get_tile": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_U)]),
    "lbm_autotune": (_I, [_P, _I]),
    "lbm_save": (_I, [_P, ctypes.c_char_p]),
    "lbm_load": (_I, [_P, ctypes.c_char_p]),
    "lbm_fluid_nodes": (_L, [_P]),
    "lbm_bytes_per_update": (_I, [_P]),
    "lbm_last_error": (ctypes.c_char_p, [_P]),
    "lbm_destroy": (None, [_P]),
    "lbm_batch_create": (_I, [ctypes.POINTER(_P), _I, ctypes.POINTER(LbmRunDesc), _I]),
    "lbm_batch_set_tile": (_I, [_P, _I, _I]),
    "lbm_batch_autotune": (_I, [_P, _I]),
    "lbm_batch_get_tile": (_I, [_P, _P, _P]),
    "lbm_batch_set_sched": (_I, [_P, _U]),
    "lbm_batch_get_sched": (_U, [_P]),
    "lbm_batch_step": (_I, [_P, _I]),
    "lbm_batch_use_graph": (_I, [_P, _I, _I]),
    "lbm_batch_get_fields": (_I, [_P, _I, _P, _P, _P, _P]),
    "lbm_batch_contact_angles": (_I, [_P, _P]),
    "lbm_batch_set_stream": (_I, [_P, _P]),
    "lbm_batch_fluid_nodes": (_L, [_P]),
    "lbm_batch_last_error": (ctypes.c_char_p, [_P]),
    "lbm_batch_destroy": (None, [_P]),
    # three dimensions (include/lbm3d.h)
    "lbm3d_create": (_I, [ctypes.POINTER(_P), _I, _I, _I, _I, _U]),
    "lbm3d_get_flags": (_U, [_P]),
    "lbm3d_set_geometry": (_I, [_P, _P]),
    "lbm3d_set_params": (_I, [_P, _D, _D, _D]),
    "lbm3d_set_adhesion": (_I, [_P, _D, _D, _D]),
    "lbm3d_set_body_accel": (_I, [_P, _P]),
    "lbm3d_init_fields": (_I, [_P, _P, _P]),
    "lbm3d_set_populations": (_I, [_P, _P]),
    "lbm3d_get_populations": (_I, [_P, _P]),
    "lbm3d_step": (_I, [_P, _I]),
    "lbm3d_synchronize": (_I, [_P]),
    "lbm3d_time": (_L, [_P]),
    "lbm3d_get_fields": (_I, [_P, _P, _P, _P, _P, _P]),
    "lbm3d_reduce": (_I, [_P, _P]),
    "lbm3d_contact_angle": (_I, [_P, _I, _P, ctypes.POINTER(_D)]),
    "lbm3d_set_tile": (_I, [_P, _I, _I, _I, _I]),
    "lbm3d_get_tile": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "lbm3d_set_stream": (_I, [_P, _P]),
    "lbm3d_fluid_nodes": (_L, [_P]),
    "lbm3d_bytes_per_update": (_I, [_P]),
    "lbm3d_last_error": (ctypes.c_char_p, [_P]),
    "lbm3d_destroy": (None, [_P]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblbm.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"HIP library {path} is not built; run __graft_entry__.build() "
                               "or python -m paper_2505_22256_amd.build")
        try:
            # torch first: the library then binds to torch's HIP runtime,
            # the one process-wide runtime (see the module docstring)
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_P)


# ---- module-level functions with the C names --------------------------------

def lbm_create(nx: int, ny: int, storage: int = F32, flags: int = 0):
    h = _P()
    rc = load_library().lbm_create(ctypes.byref(h), nx, ny, storage, flags)
    if rc:
        raise LbmError(rc, "lbm_create failed")
    return h


def lbm_create_ex(nx: int, ny: int, storage: int, flags: int, buf_a: int, buf_b: int, bytes_each: int):
    h = _P()
    rc = load_library().lbm_create_ex(ctypes.byref(h), nx, ny, storage, flags, buf_a, buf_b, bytes_each)
    if rc:
        raise LbmError(rc, "lbm_create_ex failed")
    return h


def lbm_population_bytes(nx: int, ny: int, storage: int) -> int:
    return load_library().lbm_population_bytes(nx, ny, storage)


def _device_span(t):
    """(address, bytes) of a device array given as an object with
    data_ptr() (a torch tensor; its bytes are numel * element_size) or as an
    (address, bytes) pair.  A tensor must be contiguous and lie on the
    current HIP device: the library treats the span as one contiguous
    buffer of that device."""
    if hasattr(t, "data_ptr"):
        if hasattr(t, "is_contiguous") and not t.is_contiguous():
            raise ValueError("population buffer must be a contiguous tensor")
        dev = getattr(t, "device", None)
        if dev is not None:
            import torch
            if dev.type != "cuda" or dev.index != torch.cuda.current_device():
                raise ValueError(f"population buffer lies on {dev}, not on the current HIP device "
                                 f"cuda:{torch.cuda.current_device()}")
        return int(t.data_ptr()), int(t.numel() * t.element_size())
    a, n = t
    return int(a), int(n)


def lbm_destroy(h):
    load_library().lbm_destroy(h)


def lbm_last_error(h) -> str:
    return load_library().lbm_last_error(h).decode()


def _check(h, rc):
    if rc:
        raise LbmError(rc, lbm_last_error(h))
    return rc


class Lattice:
    """One context: a lattice with its geometry, parameters and state."""

    def __init__(self, nx: int, ny: int, storage: int = F32, flags: int = 0, buffers=None):
        """buffers: None (the library allocates), or two device arrays (torch
        tensors or (address, bytes) pairs) that become the population
        buffers (lbm_create_ex); they are kept referenced while the
        lattice lives and never freed by the library."""
        self._L = load_library()
        self._ext = None
        if buffers is None:
            self.h = lbm_create(nx, ny, storage, flags)
        else:
            (pa, na), (pb, nb) = (_device_span(b) for b in buffers)
            self.h = lbm_create_ex(nx, ny, storage, flags, pa, pb, min(na, nb))
            self._ext = tuple(buffers)
        self.nx, self.ny, self.storage, self.flags = nx, ny, storage, flags

    def flags_in_effect(self) -> int:
        """Creation flags with the storage's rounding resolved (lbm_get_flags)."""
        return int(self._L.lbm_get_flags(self.h))

    def close(self):
        if getattr(self, "h", None):
            self._L.lbm_destroy(self.h)
            self.h = None
        self._ext = None

    def __del__(self):
        self.close()

    @property
    def shape(self):
        return (self.ny, self.nx)

    def current_buffer(self) -> int:
        """Index (0 or 1) of the population buffer holding the current state."""
        rc = self._L.lbm_current_buffer(self.h)
        if rc < 0:
            raise LbmError(rc, "lbm_current_buffer failed")
        return rc

    def _c(self, rc):
        return _check(self.h, rc)

    def set_geometry(self, solid):
        s = np.ascontiguousarray(solid, dtype=np.uint8).reshape(self.shape)
        self._c(self._L.lbm_set_geometry(self.h, _ptr(s)))

    def set_params(self, G_c, G_ads, tau):
        self._c(self._L.lbm_set_params(self.h, G_c, G_ads, tau))

    def set_adhesion(self, G_w1, G_w2, delta=0.8):
        self._c(self._L.lbm_set_adhesion(self.h, G_w1, G_w2, delta))

    def set_body_accel(self, g1x, g1y, g2x, g2y):
        self._c(self._L.lbm_set_body_accel(self.h, g1x, g1y, g2x, g2y))

    def set_wall_velocity(self, ubx, uby, utx, uty):
        self._c(self._L.lbm_set_wall_velocity(self.h, ubx, uby, utx, uty))

    def set_inlet_velocity(self, ux, uy):
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(ux, dtype=np.float64), (self.ny,)))
        b = np.ascontiguousarray(np.broadcast_to(np.asarray(uy, dtype=np.float64), (self.ny,)))
        self._c(self._L.lbm_set_inlet_velocity(self.h, _ptr(a), _ptr(b)))

    def init_fields(self, rho1, rho2):
        r1 = np.ascontiguousarray(rho1, dtype=np.float64).reshape(self.shape)
        r2 = np.ascontiguousarray(rho2, dtype=np.float64).reshape(self.shape)
        self._c(self._L.lbm_init_fields(self.h, _ptr(r1), _ptr(r2)))

    def set_populations(self, f):
        a = np.ascontiguousarray(f, dtype=np.float64).reshape(2, 9, self.ny, self.nx)
        self._c(self._L.lbm_set_populations(self.h, _ptr(a)))

    def get_populations(self):
        a = np.empty((2, 9, self.ny, self.nx))
        self._c(self._L.lbm_get_populations(self.h, _ptr(a)))
        return a

    def get_populations_window(self, x0, y0, w, h):
        a = np.empty((2, 9, h, w))
        self._c(self._L.lbm_get_populations_window(self.h, x0, y0, w, h, _ptr(a)))
        return a

    def step(self, n=1):
        self._c(self._L.lbm_step(self.h, int(n)))

    def set_diag_interval(self, every):
        self._c(self._L.lbm_set_diag_interval(self.h, int(every)))

    def get_diag(self):
        out = np.empty(8)
        t = _L()
        self._c(self._L.lbm_get_diag(self.h, _ptr(out), ctypes.byref(t)))
        return out, t.value

    def synchronize(self):
        self._c(self._L.lbm_synchronize(self.h))

    @property
    def time(self):
        return self._L.lbm_time(self.h)

    def get_fields(self):
        out = [np.empty(self.shape) for _ in range(4)]
        self._c(self._L.lbm_get_fields(self.h, *[_ptr(a) for a in out]))
        return out

    def reduce(self):
        out = np.empty(8)
        self._c(self._L.lbm_reduce(self.h, _ptr(out)))
        return out

    def reduce_noalloc(self, d_out: int):
        """lbm_reduce into the caller's device memory d_out (address of 8
        doubles), asynchronous on the context's stream, allocating nothing."""
        self._c(self._L.lbm_reduce_noalloc(self.h, _P(int(d_out))))

    def contact_angle(self, wall_kind, wall):
        w = np.ascontiguousarray(wall, dtype=np.float64)
        th = _D()
        self._c(self._L.lbm_contact_angle(self.h, wall_kind, _ptr(w), ctypes.byref(th)))
        return th.value

    def get_tables(self):
        link = np.empty(self.shape, dtype=np.uint8)
        n = _I()
        self._c(self._L.lbm_get_tables(self.h, _ptr(link), None, None, ctypes.byref(n)))
        lst = np.empty(n.value, dtype=np.int32)
        src = np.empty((n.value, 24), dtype=np.int32)
        self._c(self._L.lbm_get_tables(self.h, _ptr(link), _ptr(lst), _ptr(src), ctypes.byref(n)))
        return link, lst, src

    def set_stream(self, stream_handle: Optional[int]):
        self._c(self._L.lbm_set_stream(self.h, stream_handle))

    def set_tile(self, block, seg_rows, sched=0):
        self._c(self._L.lbm_set_tile(self.h, block, seg_rows, sched))

    def get_tile(self):
        b, r, s = _I(), _I(), _U()
        self._c(self._L.lbm_get_tile(self.h, ctypes.byref(b), ctypes.byref(r), ctypes.byref(s)))
        return b.value, r.value, s.value

    def autotune(self, steps=5):
        self._c(self._L.lbm_autotune(self.h, steps))
        return self.get_tile()

    def save(self, path):
        self._c(self._L.lbm_save(self.h, os.fsencode(path)))

    def load(self, path):
        self._c(self._L.lbm_load(self.h, os.fsencode(path)))

    @property
    def fluid_nodes(self):
        return self._L.lbm_fluid_nodes(self.h)

    @property
    def bytes_per_update(self):
        return self._L.lbm_bytes_per_update(self.h)


def lattice_from_workload(wl, storage: int = F32, flags_extra: int = 0) -> Lattice:
    """Context initialised from a ``workloads.Workload``."""
    lat = Lattice(wl.nx, wl.ny, storage, wl.flags | flags_extra)
    lat.set_geometry(wl.solid)
    lat.set_params(wl.G_c, wl.G_ads, wl.tau)
    lat.set_body_accel(*wl.accel)
    if any(v != 0.0 for v in wl.wall_velocity):
        lat.set_wall_velocity(*wl.wall_velocity)
    if wl.inlet_u is not None:
        lat.set_inlet_velocity(wl.inlet_u[0], wl.inlet_u[1])
    lat.init_fields(wl.rho1, wl.rho2)
    return lat


class Batch:
    """Many independent runs advanced together (lbm_batch_*)."""

    def __init__(self, workloads: Sequence, storage: int = F32):
        self._L = load_library()
        self._keep = []
        descs = (LbmRunDesc * len(workloads))()
        for d, wl in zip(descs, workloads):
            solid = np.ascontiguousarray(wl.solid, dtype=np.uint8)
            r1 = np.ascontiguousarray(wl.rho1, dtype=np.float64)
            r2 = np.ascontiguousarray(wl.rho2, dtype=np.float64)
            acc = np.ascontiguousarray(wl.accel, dtype=np.float64)
            self._keep += [solid, r1, r2, acc]
            d.nx, d.ny, d.flags = wl.nx, wl.ny, wl.flags
            d.G_c, d.G_ads, d.tau = wl.G_c, wl.G_ads, wl.tau
            d.wall_kind = wl.wall_kind if wl.wall_kind is not None else WALL_FLAT
            for q, v in enumerate(wl.wall if wl.wall is not None else (0.0, 0.0, 0.0)):
                d.wall[q] = v
            d.solid, d.rho1, d.rho2, d.accel = _ptr(solid), _ptr(r1), _ptr(r2), _ptr(acc)
        h = _P()
        rc = self._L.lbm_batch_create(ctypes.byref(h), len(workloads), descs, storage)
        self._keep = []
        if rc:
            raise LbmError(rc, "lbm_batch_create failed")
        self.h = h
        self.n = len(workloads)
        self.shapes = [(wl.ny, wl.nx) for wl in workloads]

    def close(self):
        if getattr(self, "h", None):
            self._L.lbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _c(self, rc):
        if rc:
            raise LbmError(rc, self._L.lbm_batch_last_error(self.h).decode())

    def set_tile(self, block, seg_rows):
        self._c(self._L.lbm_batch_set_tile(self.h, block, seg_rows))

    def get_tile(self):
        b, r = _I(), _I()
        self._c(self._L.lbm_batch_get_tile(self.h, ctypes.byref(b), ctypes.byref(r)))
        return b.value, r.value

    def set_sched(self, sched):
        self._c(self._L.lbm_batch_set_sched(self.h, int(sched)))

    @property
    def sched(self):
        return self._L.lbm_batch_get_sched(self.h)

    def autotune(self, steps=3):
        """Time the tile candidates on the current state (restored after)
        and keep the fastest; returns (block, seg_rows, sched)."""
        self._c(self._L.lbm_batch_autotune(self.h, int(steps)))
        return self.get_tile() + (self.sched,)

    def use_graph(self, on=True, steps_per_graph=100):
        self._c(self._L.lbm_batch_use_graph(self.h, 1 if on else 0, steps_per_graph))

    def step(self, n=1):
        self._c(self._L.lbm_batch_step(self.h, int(n)))

    def get_fields(self, run):
        out = [np.empty(self.shapes[run]) for _ in range(4)]
        self._c(self._L.lbm_batch_get_fields(self.h, run, *[_ptr(a) for a in out]))
        return out

    def contact_angles(self, allow_failures=True):
        th = np.empty(self.n)
        rc = self._L.lbm_batch_contact_angles(self.h, _ptr(th))
        if rc and not (allow_failures and rc == EUNSTABLE):
            self._c(rc)
        return th

    def set_stream(self, stream_handle):
        self._c(self._L.lbm_batch_set_stream(self.h, stream_handle))

    @property
    def fluid_nodes(self):
        return self._L.lbm_batch_fluid_nodes(self.h)


class Lattice3D:
    """One 3-D context (include/lbm3d.h): arrays are [nz, ny, nx],
    populations [2, 19, nz, ny, nx]."""

    def __init__(self, nx: int, ny: int, nz: int, storage: int = F32, flags: int = 0):
        self._L = load_library()
        h = _P()
        rc = self._L.lbm3d_create(ctypes.byref(h), nx, ny, nz, storage, flags)
        if rc:
            raise LbmError(rc, "lbm3d_create failed")
        self.h = h
        self.nx, self.ny, self.nz, self.storage, self.flags = nx, ny, nz, storage, flags

    def close(self):
        if getattr(self, "h", None):
            self._L.lbm3d_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def _c(self, rc):
        if rc:
            raise LbmError(rc, self._L.lbm3d_last_error(self.h).decode())
        return rc

    def flags_in_effect(self) -> int:
        return int(self._L.lbm3d_get_flags(self.h))

    def set_geometry(self, solid):
        a = np.ascontiguousarray(solid, dtype=np.uint8).reshape(self.shape)
        self._c(self._L.lbm3d_set_geometry(self.h, _ptr(a)))

    def set_params(self, G_c, G_ads, tau):
        self._c(self._L.lbm3d_set_params(self.h, G_c, G_ads, tau))

    def set_adhesion(self, G_w1, G_w2, delta=0.8):
        self._c(self._L.lbm3d_set_adhesion(self.h, G_w1, G_w2, delta))

    def set_body_accel(self, g):
        a = np.ascontiguousarray(g, dtype=np.float64).reshape(6)
        self._c(self._L.lbm3d_set_body_accel(self.h, _ptr(a)))

    def init_fields(self, rho1, rho2):
        a = np.ascontiguousarray(rho1, dtype=np.float64).reshape(self.shape)
        b = np.ascontiguousarray(rho2, dtype=np.float64).reshape(self.shape)
        self._c(self._L.lbm3d_init_fields(self.h, _ptr(a), _ptr(b)))

    def set_populations(self, f):
        a = np.ascontiguousarray(f, dtype=np.float64).reshape((2, 19) + self.shape)
        self._c(self._L.lbm3d_set_populations(self.h, _ptr(a)))

    def get_populations(self):
        a = np.empty((2, 19) + self.shape)
        self._c(self._L.lbm3d_get_populations(self.h, _ptr(a)))
        return a

    def step(self, n=1):
        self._c(self._L.lbm3d_step(self.h, int(n)))

    def synchronize(self):
        self._c(self._L.lbm3d_synchronize(self.h))

    @property
    def time(self):
        return self._L.lbm3d_time(self.h)

    def get_fields(self):
        out = [np.empty(self.shape) for _ in range(5)]
        self._c(self._L.lbm3d_get_fields(self.h, *[_ptr(a) for a in out]))
        return out

    def reduce(self):
        out = np.empty(9)
        self._c(self._L.lbm3d_reduce(self.h, _ptr(out)))
        return out

    def contact_angle(self, wall_kind, wall):
        w = np.ascontiguousarray(wall, dtype=np.float64).reshape(4)
        th = _D()
        self._c(self._L.lbm3d_contact_angle(self.h, wall_kind, _ptr(w), ctypes.byref(th)))
        return th.value

    def set_tile(self, bx, by, bz, tz=1):
        """Brick of the collide pass and its threads in z (lbm3d_set_tile)."""
        self._c(self._L.lbm3d_set_tile(self.h, bx, by, bz, tz))

    def get_tile(self):
        a, b, c, d = _I(), _I(), _I(), _I()
        self._c(self._L.lbm3d_get_tile(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
        return a.value, b.value, c.value, d.value

    def set_stream(self, stream_handle: Optional[int]):
        self._c(self._L.lbm3d_set_stream(self.h, None if stream_handle is None else _P(stream_handle)))

    @property
    def fluid_nodes(self):
        return self._L.lbm3d_fluid_nodes(self.h)

    @property
    def bytes_per_update(self):
        return self._L.lbm3d_bytes_per_update(self.h)


def lattice3d_from_workload(wl, storage: int = F32, flags_extra: int = 0) -> Lattice3D:
    """3-D context initialised from a ``workloads.Workload3D``."""
    lat = Lattice3D(wl.nx, wl.ny, wl.nz, storage, wl.flags | flags_extra)
    lat.set_geometry(wl.solid)
    lat.set_params(wl.G_c, wl.G_ads, wl.tau)
    lat.set_body_accel(wl.accel)
    lat.init_fields(wl.rho1, wl.rho2)
    return lat
