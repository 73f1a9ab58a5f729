"""FP64 CPU oracle of the two-component pseudopotential LBM (arXiv 2505.22256).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow, serial-order C code
in ``lbm_oracle.c``; this module builds it with gcc and wraps it with ctypes.
Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import it.  It shares no code with the GPU library in
``paper_2505_22256_amd``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
SRC3 = os.path.join(HERE, "lbm_oracle3d.c")
LIB = os.path.join(HERE, "liboracle.so")

OK, EINVAL, ESTATE, ENOMEM, EUNSTABLE = 0, -1, -2, -3, -5
PERIODIC_X, PERIODIC_Y = 1, 2
SCHEME_ORIGINAL, E8_COPY_OFF, WALLPSI_SELF, VEL_LITERAL, FORCE_DENSITY = 4, 8, 16, 32, 64
INLET, OUTFLOW = 256, 512
ADH_D2Q9 = 4096  # reading exploration: S(x) with the D2Q9 weights (CPU only)


def build(force: bool = True) -> str:
    """Compile liboracle.so (2-D and 3-D oracles) with gcc (plain -O2: no
    FMA contraction on x86-64)."""
    srcs = [SRC, SRC3]
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(
            os.path.getmtime(f) for f in srcs + [SRC[:-1] + "h", SRC3[:-1] + "h"]):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(LIB)
        P, I, D, U = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint
        dp = ctypes.POINTER(ctypes.c_double)
        sig = {
            "oracle_create": (I, [ctypes.POINTER(P), I, I, U]),
            "oracle_destroy": (None, [P]),
            "oracle_last_error": (ctypes.c_char_p, [P]),
            "oracle_set_geometry": (I, [P, P]),
            "oracle_set_params": (I, [P, D, D, D]),
            "oracle_set_adhesion": (I, [P, D, D, D]),
            "oracle_set_body_accel": (I, [P, D, D, D, D]),
            "oracle_set_wall_velocity": (I, [P, D, D, D, D]),
            "oracle_set_inlet_velocity": (I, [P, P, P]),
            "oracle_init_fields": (I, [P, P, P]),
            "oracle_set_populations": (I, [P, P]),
            "oracle_get_populations": (I, [P, P]),
            "oracle_step": (I, [P, I]),
            "oracle_time": (ctypes.c_long, [P]),
            "oracle_get_fields": (I, [P, P, P, P, P]),
            "oracle_reduce": (I, [P, P]),
            "oracle_contact_angle": (I, [P, I, P, dp]),
            "oracle_interface_points": (I, [P, I, P, P, P, I, ctypes.POINTER(I)]),
            "oracle_get_tables": (I, [P, P, P, P, ctypes.POINTER(I)]),
            "oracle_d2q9": (None, [P, P, P, P]),
            "oracle_e8": (None, [P, P, P, P]),
            "oracle_local_G": (D, [D, D, D, D]),
            "oracle_equilibrium": (None, [D, P, P]),
            "oracle_forcing": (None, [P, P, P]),
            "oracle_node_forces": (I, [P, I, I, P]),
            "oracle_adhesion_vector": (I, [P, I, I, P]),
            "oracle_circle_fit": (I, [P, P, I, P]),
            "oracle_threads": (I, []),
            "oracle_set_threads": (I, [I]),
            "oracle3d_create": (I, [ctypes.POINTER(P), I, I, I, U]),
            "oracle3d_destroy": (None, [P]),
            "oracle3d_last_error": (ctypes.c_char_p, [P]),
            "oracle3d_set_geometry": (I, [P, P]),
            "oracle3d_set_params": (I, [P, D, D, D]),
            "oracle3d_set_adhesion": (I, [P, D, D, D]),
            "oracle3d_set_body_accel": (I, [P, P]),
            "oracle3d_init_fields": (I, [P, P, P]),
            "oracle3d_set_populations": (I, [P, P]),
            "oracle3d_get_populations": (I, [P, P]),
            "oracle3d_step": (I, [P, I]),
            "oracle3d_time": (ctypes.c_long, [P]),
            "oracle3d_get_fields": (I, [P, P, P, P, P, P]),
            "oracle3d_reduce": (I, [P, P]),
            "oracle3d_node_forces": (I, [P, I, I, I, P]),
            "oracle3d_adhesion_vector": (I, [P, I, I, I, P]),
            "oracle3d_d3q19": (None, [P, P, P, P, P]),
            "oracle3d_stencil": (I, [P, P, P, P, P]),
            "oracle3d_equilibrium": (None, [D, P, P]),
            "oracle3d_forcing": (None, [P, P, P]),
            "oracle3d_interface_points": (I, [P, I, P, P, P, P, I, ctypes.POINTER(I)]),
            "oracle3d_sphere_fit": (I, [P, P, P, I, P]),
            "oracle3d_contact_angle": (I, [P, I, P, dp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


class Oracle:
    """ctypes wrapper around one oracle context."""

    def __init__(self, nx: int, ny: int, flags: int = 0):
        self._L = lib()
        h = ctypes.c_void_p()
        rc = self._L.oracle_create(ctypes.byref(h), nx, ny, flags)
        if rc:
            raise OracleError(rc, "create failed")
        self.h, self.nx, self.ny, self.flags = h, nx, ny, flags

    def __del__(self):
        if getattr(self, "h", None):
            self._L.oracle_destroy(self.h)
            self.h = None

    def _chk(self, rc):
        if rc:
            raise OracleError(rc, self._L.oracle_last_error(self.h).decode())
        return rc

    @property
    def shape(self):
        return (self.ny, self.nx)

    def set_geometry(self, solid):
        s = np.ascontiguousarray(solid, dtype=np.uint8).reshape(self.shape)
        self._solid = s
        self._chk(self._L.oracle_set_geometry(self.h, _ptr(s)))

    def set_params(self, G_c, G_ads, tau):
        self._chk(self._L.oracle_set_params(self.h, G_c, G_ads, tau))

    def set_adhesion(self, G_w1, G_w2, delta=0.8):
        self._chk(self._L.oracle_set_adhesion(self.h, G_w1, G_w2, delta))

    def set_body_accel(self, g1x, g1y, g2x, g2y):
        self._chk(self._L.oracle_set_body_accel(self.h, g1x, g1y, g2x, g2y))

    def set_wall_velocity(self, ubx, uby, utx, uty):
        self._chk(self._L.oracle_set_wall_velocity(self.h, ubx, uby, utx, uty))

    def set_inlet_velocity(self, ux, uy):
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(ux, dtype=np.float64), (self.ny,)))
        b = np.ascontiguousarray(np.broadcast_to(np.asarray(uy, dtype=np.float64), (self.ny,)))
        self._chk(self._L.oracle_set_inlet_velocity(self.h, _ptr(a), _ptr(b)))

    def init_fields(self, rho1, rho2):
        r1 = np.ascontiguousarray(rho1, dtype=np.float64).reshape(self.shape)
        r2 = np.ascontiguousarray(rho2, dtype=np.float64).reshape(self.shape)
        self._chk(self._L.oracle_init_fields(self.h, _ptr(r1), _ptr(r2)))

    def set_populations(self, f):
        a = np.ascontiguousarray(f, dtype=np.float64).reshape(2, 9, self.ny, self.nx)
        self._chk(self._L.oracle_set_populations(self.h, _ptr(a)))

    def get_populations(self):
        a = np.empty((2, 9, self.ny, self.nx))
        self._chk(self._L.oracle_get_populations(self.h, _ptr(a)))
        return a

    def step(self, n=1):
        self._chk(self._L.oracle_step(self.h, int(n)))

    @property
    def time(self):
        return self._L.oracle_time(self.h)

    def get_fields(self):
        out = [np.empty(self.shape) for _ in range(4)]
        self._chk(self._L.oracle_get_fields(self.h, *[_ptr(a) for a in out]))
        return out

    def reduce(self):
        out = np.empty(8)
        self._chk(self._L.oracle_reduce(self.h, _ptr(out)))
        return out

    def contact_angle(self, wall_kind, wall):
        w = np.ascontiguousarray(wall, dtype=np.float64)
        th = ctypes.c_double()
        self._chk(self._L.oracle_contact_angle(self.h, wall_kind, _ptr(w), ctypes.byref(th)))
        return th.value

    def interface_points(self, wall_kind, wall):
        w = np.ascontiguousarray(wall, dtype=np.float64)
        n = ctypes.c_int()
        self._chk(self._L.oracle_interface_points(self.h, wall_kind, _ptr(w), None, None, 0,
                                                  ctypes.byref(n)))
        px, py = np.empty(n.value), np.empty(n.value)
        self._chk(self._L.oracle_interface_points(self.h, wall_kind, _ptr(w), _ptr(px), _ptr(py),
                                                  n.value, ctypes.byref(n)))
        return px, py

    def get_tables(self):
        link = np.empty(self.shape, dtype=np.uint8)
        n = ctypes.c_int()
        self._chk(self._L.oracle_get_tables(self.h, _ptr(link), None, None, ctypes.byref(n)))
        lst = np.empty(n.value, dtype=np.int32)
        src = np.empty((n.value, 24), dtype=np.int32)
        self._chk(self._L.oracle_get_tables(self.h, _ptr(link), _ptr(lst), _ptr(src),
                                            ctypes.byref(n)))
        return link, lst, src

    def node_forces(self, x, y):
        out = np.empty(12)
        self._chk(self._L.oracle_node_forces(self.h, x, y, _ptr(out)))
        return out.reshape(6, 2)

    def adhesion_vector(self, x, y):
        out = np.empty(2)
        self._chk(self._L.oracle_adhesion_vector(self.h, x, y, _ptr(out)))
        return out


def d2q9():
    L = lib()
    ex, ey, opp = (np.empty(9, dtype=np.int32) for _ in range(3))
    w = np.empty(9)
    L.oracle_d2q9(_ptr(ex), _ptr(ey), _ptr(w), _ptr(opp))
    return ex, ey, w, opp


def e8():
    L = lib()
    ex, ey, cp = (np.empty(24, dtype=np.int32) for _ in range(3))
    W = np.empty(24)
    L.oracle_e8(_ptr(ex), _ptr(ey), _ptr(W), _ptr(cp))
    return ex, ey, W, cp


def local_G(rho_e, G_w1, G_w2, delta=0.8):
    return lib().oracle_local_G(float(rho_e), G_w1, G_w2, delta)


def equilibrium(rho, u):
    uu = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty(9)
    lib().oracle_equilibrium(float(rho), _ptr(uu), _ptr(out))
    return out


def forcing(F, u):
    FF = np.ascontiguousarray(F, dtype=np.float64)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty(9)
    lib().oracle_forcing(_ptr(FF), _ptr(uu), _ptr(out))
    return out


def circle_fit(px, py):
    x = np.ascontiguousarray(px, dtype=np.float64)
    y = np.ascontiguousarray(py, dtype=np.float64)
    out = np.empty(3)
    rc = lib().oracle_circle_fit(_ptr(x), _ptr(y), len(x), _ptr(out))
    if rc:
        raise OracleError(rc, "circle fit failed")
    return out


def threads():
    return lib().oracle_threads()


def set_threads(n):
    """Threads of the oracle's row loops (results are independent of it);
    returns the previous count."""
    return lib().oracle_set_threads(int(n))


# ---------------------------------------------------------------------------
# Three dimensions (Sec. 3.5): D3Q19 and the 92-position 3-D stencil
# ---------------------------------------------------------------------------
PERIODIC_Z = 2048


class Oracle3D:
    """ctypes wrapper around one 3-D oracle context.  Arrays are [nz, ny, nx];
    populations [2, 19, nz, ny, nx]."""

    def __init__(self, nx: int, ny: int, nz: int, flags: int = 0):
        self._L = lib()
        h = ctypes.c_void_p()
        rc = self._L.oracle3d_create(ctypes.byref(h), nx, ny, nz, flags)
        if rc:
            raise OracleError(rc, "create failed")
        self.h, self.nx, self.ny, self.nz, self.flags = h, nx, ny, nz, flags

    def __del__(self):
        if getattr(self, "h", None):
            self._L.oracle3d_destroy(self.h)
            self.h = None

    def _chk(self, rc):
        if rc:
            raise OracleError(rc, self._L.oracle3d_last_error(self.h).decode())
        return rc

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def set_geometry(self, solid):
        s = np.ascontiguousarray(solid, dtype=np.uint8).reshape(self.shape)
        self._solid = s
        self._chk(self._L.oracle3d_set_geometry(self.h, _ptr(s)))

    def set_params(self, G_c, G_ads, tau):
        self._chk(self._L.oracle3d_set_params(self.h, G_c, G_ads, tau))

    def set_adhesion(self, G_w1, G_w2, delta=0.8):
        self._chk(self._L.oracle3d_set_adhesion(self.h, G_w1, G_w2, delta))

    def set_body_accel(self, g):
        a = np.ascontiguousarray(g, dtype=np.float64).reshape(6)
        self._chk(self._L.oracle3d_set_body_accel(self.h, _ptr(a)))

    def init_fields(self, rho1, rho2):
        r1 = np.ascontiguousarray(rho1, dtype=np.float64).reshape(self.shape)
        r2 = np.ascontiguousarray(rho2, dtype=np.float64).reshape(self.shape)
        self._chk(self._L.oracle3d_init_fields(self.h, _ptr(r1), _ptr(r2)))

    def set_populations(self, f):
        a = np.ascontiguousarray(f, dtype=np.float64).reshape((2, 19) + self.shape)
        self._chk(self._L.oracle3d_set_populations(self.h, _ptr(a)))

    def get_populations(self):
        a = np.empty((2, 19) + self.shape)
        self._chk(self._L.oracle3d_get_populations(self.h, _ptr(a)))
        return a

    def step(self, n=1):
        self._chk(self._L.oracle3d_step(self.h, int(n)))

    @property
    def time(self):
        return self._L.oracle3d_time(self.h)

    def get_fields(self):
        out = [np.empty(self.shape) for _ in range(5)]
        self._chk(self._L.oracle3d_get_fields(self.h, *[_ptr(a) for a in out]))
        return out

    def reduce(self):
        out = np.empty(9)
        self._chk(self._L.oracle3d_reduce(self.h, _ptr(out)))
        return out

    def node_forces(self, x, y, z):
        out = np.empty(18)
        self._chk(self._L.oracle3d_node_forces(self.h, x, y, z, _ptr(out)))
        return out.reshape(6, 3)

    def adhesion_vector(self, x, y, z):
        out = np.empty(3)
        self._chk(self._L.oracle3d_adhesion_vector(self.h, x, y, z, _ptr(out)))
        return out

    def interface_points(self, wall_kind, wall):
        w = np.ascontiguousarray(wall, dtype=np.float64)
        n = ctypes.c_int()
        self._chk(self._L.oracle3d_interface_points(self.h, wall_kind, _ptr(w), None, None, None, 0,
                                                    ctypes.byref(n)))
        p = [np.empty(n.value) for _ in range(3)]
        self._chk(self._L.oracle3d_interface_points(self.h, wall_kind, _ptr(w), *[_ptr(a) for a in p],
                                                    n.value, ctypes.byref(n)))
        return p

    def contact_angle(self, wall_kind, wall):
        w = np.ascontiguousarray(wall, dtype=np.float64)
        th = ctypes.c_double()
        self._chk(self._L.oracle3d_contact_angle(self.h, wall_kind, _ptr(w), ctypes.byref(th)))
        return th.value


def d3q19():
    L = lib()
    ex, ey, ez, opp = (np.empty(19, dtype=np.int32) for _ in range(4))
    w = np.empty(19)
    L.oracle3d_d3q19(_ptr(ex), _ptr(ey), _ptr(ez), _ptr(w), _ptr(opp))
    return ex, ey, ez, w, opp


def stencil3d():
    L = lib()
    ex, ey, ez, cp = (np.empty(92, dtype=np.int32) for _ in range(4))
    W = np.empty(92)
    n = L.oracle3d_stencil(_ptr(ex), _ptr(ey), _ptr(ez), _ptr(W), _ptr(cp))
    return ex[:n], ey[:n], ez[:n], W[:n], cp[:n]


def equilibrium3d(rho, u):
    uu = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty(19)
    lib().oracle3d_equilibrium(float(rho), _ptr(uu), _ptr(out))
    return out


def forcing3d(F, u):
    FF = np.ascontiguousarray(F, dtype=np.float64)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty(19)
    lib().oracle3d_forcing(_ptr(FF), _ptr(uu), _ptr(out))
    return out


def sphere_fit(px, py, pz):
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (px, py, pz)]
    out = np.empty(4)
    rc = lib().oracle3d_sphere_fit(*[_ptr(v) for v in a], len(a[0]), _ptr(out))
    if rc:
        raise OracleError(rc, "sphere fit failed")
    return out
