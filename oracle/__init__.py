"""ctypes wrapper of the CPU oracle (``orc.cpp``).

TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow, independent CPU
implementation of the particle step used to check the GPU library.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg may import this
module; the product package never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "orc.cpp")
HDR = os.path.join(HERE, "orc.h")
# ORC_LIB: another build of the oracle (the mutation sweep's planted-mistake copies)
LIB = os.environ.get("ORC_LIB") or os.path.join(HERE, "liborc.so")

CFLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-Wall", "-Wextra"]

NSTAT_2 = 31
NSTAT_4 = 86
AV_STEPS, AV_N, AV_MEAN, AV_M2, AV_HIST = 0, 1, 2, 6, 16
ST_N, ST_MEAN, ST_M2, ST_BINN, ST_BINM, ST_M3, ST_M4 = 0, 1, 5, 15, 23, 31, 51


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no contraction, no fast math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(SRC),
                                                                         os.path.getmtime(HDR)):
        tmp = LIB + ".tmp"
        subprocess.run(["g++", *CFLAGS, "-o", tmp, SRC], check=True)
        os.replace(tmp, LIB)
    return LIB


class _Params(ctypes.Structure):
    _fields_ = [("f32_state", ctypes.c_int32), ("model", ctypes.c_int32), ("moments", ctypes.c_int32),
                ("hist_bins", ctypes.c_int32), ("mix", ctypes.c_int32), ("psi_init", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("omega", ctypes.c_int32), ("vbins", ctypes.c_int32),
                ("pad_", ctypes.c_int32),
                ("dt", ctypes.c_double), ("nu", ctypes.c_double), ("C0", ctypes.c_double),
                ("CT", ctypes.c_double), ("Cs", ctypes.c_double), ("Ct", ctypes.c_double),
                ("Cmu", ctypes.c_double), ("kappa", ctypes.c_double), ("Ewall", ctypes.c_double),
                ("yp", ctypes.c_double), ("Lx", ctypes.c_double), ("Ly", ctypes.c_double),
                ("C3", ctypes.c_double), ("C4", ctypes.c_double), ("Cw1", ctypes.c_double),
                ("Cw2", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.environ.get("ORC_LIB") and (not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build(force=True)
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER
        d, i32, i64, u32, u64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
        vp = ctypes.c_void_p
        L.orc_create.restype = vp
        L.orc_create.argtypes = [P(_Params), i32, vp, i32, vp, vp, vp, vp]
        L.orc_destroy.argtypes = [vp]
        L.orc_add_ensemble.restype = i32
        L.orc_add_ensemble.argtypes = [vp, vp, u64, d, d, d]
        L.orc_nstat.restype = i32
        L.orc_nstat.argtypes = [vp]
        L.orc_count.restype = i64
        L.orc_count.argtypes = [vp, i32]
        L.orc_step.restype = i32
        L.orc_step.argtypes = [vp, i32]
        L.orc_stats.restype = i32
        L.orc_stats.argtypes = [vp, i32, vp]
        L.orc_get_state.restype = i32
        L.orc_get_state.argtypes = [vp, i32] + [vp] * 7
        L.orc_set_state.restype = i32
        L.orc_set_state.argtypes = [vp, i32] + [vp] * 7
        L.orc_get_step.restype = i64
        L.orc_get_step.argtypes = [vp]
        L.orc_set_step.argtypes = [vp, i64]
        L.orc_set_threads.argtypes = [i32]
        L.orc_set_cond_means.argtypes = [vp, i32, vp]
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_normals.argtypes = [u64, u32, u32, u32, i32, vp]
        L.orc_normals_batch.argtypes = [u64, i64, u32, u32, i32, vp]
        L.orc_log64.restype = d
        L.orc_log64.argtypes = [d]
        L.orc_log32.restype = ctypes.c_float
        L.orc_log32.argtypes = [ctypes.c_float]
        L.orc_sincos2pi64.argtypes = [d, P(d), P(d)]
        L.orc_sincos2pi32.argtypes = [ctypes.c_float, P(ctypes.c_float), P(ctypes.c_float)]
        L.orc_cbrt64.restype = d
        L.orc_cbrt64.argtypes = [d]
        L.orc_coefficients.argtypes = [vp, vp]
        L.orc_set_drift.argtypes = [vp, vp]
        L.orc_set_pressure_gradient.argtypes = [vp, vp]
        L.orc_mix_rate.argtypes = [vp, i32, vp]
        L.orc_wall_alpha.argtypes = [vp, vp]
        L.orc_exp64.restype = d
        L.orc_exp64.argtypes = [d]
        L.orc_get_omega.restype = i32
        L.orc_get_omega.argtypes = [vp, i32, vp]
        L.orc_set_omega.restype = i32
        L.orc_set_omega.argtypes = [vp, i32, vp]
        L.orc_omega_fields.argtypes = [vp, vp, vp, vp]
        L.orc_navg.restype = i32
        L.orc_navg.argtypes = [vp]
        L.orc_average_start.argtypes = [vp]
        L.orc_average_stop.argtypes = [vp]
        L.orc_average.restype = i32
        L.orc_average.argtypes = [vp, i32, vp]
        L.orc_locate.restype = i32
        L.orc_locate.argtypes = [vp, d, d]
        L.orc_wallfn_hits.restype = i64
        L.orc_wallfn_hits.argtypes = [vp]
        L.orc_walk.restype = i32
        L.orc_walk.argtypes = [vp, i32, d, d, P(d), P(d), vp, P(i32), P(d)]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def params_of(wl) -> _Params:
    c = wl.constants
    return _Params(f32_state=1 if wl.precision == "f32" else 0, model=int(wl.model), moments=int(wl.moments),
                   hist_bins=int(wl.hist_bins), mix=1 if wl.mix else 0, psi_init=int(wl.psi_init),
                   flags=int(getattr(wl, 'flags', 15)),
                   dt=wl.dt, nu=wl.nu, C0=wl.C0, CT=c["CT"], Cs=c["Cs"], Ct=c["Ct"], Cmu=c["Cmu"],
                   kappa=c["kappa"], Ewall=c["Ewall"], yp=wl.yp, Lx=wl.mesh.Lx, Ly=wl.mesh.Ly,
                   omega=1 if getattr(wl, "omega", False) else 0, vbins=int(getattr(wl, "vbins", 2)),
                   C3=c.get("C3", 5.0),
                   C4=c.get("C4", 0.25), Cw1=c.get("Cw1", 0.5), Cw2=c.get("Cw2", 0.73))


class Oracle:
    """The oracle run of one workload (all its ensembles)."""

    def __init__(self, wl, ensembles: Optional[list] = None, threads: Optional[int] = None):
        L = lib()
        if threads is not None:
            L.orc_set_threads(int(threads))
        self.wl = wl
        m = wl.mesh
        self._keep = [np.ascontiguousarray(m.vtx, np.float64), np.ascontiguousarray(m.tri, np.int32),
                      np.ascontiguousarray(m.nbr, np.int32), np.ascontiguousarray(m.ekind, np.int32),
                      np.ascontiguousarray(wl.fields, np.float64)]
        self._p = params_of(wl)
        self.ctx = L.orc_create(ctypes.byref(self._p), m.nvert, _ptr(self._keep[0]), m.nelem,
                                _ptr(self._keep[1]), _ptr(self._keep[2]), _ptr(self._keep[3]),
                                _ptr(self._keep[4]))
        if not self.ctx:
            raise RuntimeError("orc_create failed")
        self.nstat = L.orc_nstat(self.ctx)
        ens = wl.ensembles if ensembles is None else ensembles
        for en in ens:
            counts = np.ascontiguousarray(en.counts, np.int64)
            L.orc_add_ensemble(self.ctx, _ptr(counts), int(en.seed), float(en.x0[0]), float(en.x0[1]),
                               float(en.r0))
        self.nens = len(ens)

    def __del__(self):
        if getattr(self, "ctx", None):
            lib().orc_destroy(self.ctx)
            self.ctx = None

    def step(self, n: int = 1) -> None:
        r = lib().orc_step(self.ctx, int(n))
        if r != 0:
            raise RuntimeError(f"oracle step failed with status {r}")

    @property
    def step_index(self) -> int:
        return int(lib().orc_get_step(self.ctx))

    @step_index.setter
    def step_index(self, s: int) -> None:
        lib().orc_set_step(self.ctx, int(s))

    def count(self, ens: int = 0) -> int:
        return int(lib().orc_count(self.ctx, ens))

    def stats(self, ens: int = 0) -> np.ndarray:
        out = np.zeros((self.wl.mesh.nelem, self.nstat))
        lib().orc_stats(self.ctx, ens, _ptr(out))
        return out

    def state(self, ens: int = 0) -> dict:
        n = self.count(ens)
        arr = {k: np.zeros(n) for k in ("x", "y", "u", "v", "w", "psi")}
        arr["elem"] = np.zeros(n, np.int32)
        lib().orc_get_state(self.ctx, ens, *(_ptr(arr[k]) for k in ("x", "y", "u", "v", "w", "psi", "elem")))
        return arr

    def set_state(self, st: dict, ens: int = 0) -> None:
        a = {k: np.ascontiguousarray(st[k], np.float64) for k in ("x", "y", "u", "v", "w", "psi")}
        a["elem"] = np.ascontiguousarray(st["elem"], np.int32)
        lib().orc_set_state(self.ctx, ens, *(_ptr(a[k]) for k in ("x", "y", "u", "v", "w", "psi", "elem")))

    def omega(self, ens: int = 0) -> np.ndarray:
        """Turbulent frequency per particle, id order."""
        out = np.zeros(self.count(ens))
        if lib().orc_get_omega(self.ctx, ens, _ptr(out)) != 0:
            raise RuntimeError("the workload carries no turbulent frequency")
        return out

    def set_omega(self, om, ens: int = 0) -> None:
        a = np.ascontiguousarray(om, np.float64)
        if lib().orc_set_omega(self.ctx, ens, _ptr(a)) != 0:
            raise RuntimeError("the workload carries no turbulent frequency")

    def omega_fields(self):
        """(<omega> at each centroid, S_omega per element, <omega> at each
        wall-function edge midpoint (nelem x 3, 0 elsewhere))."""
        ne = self.wl.mesh.nelem
        om0, sw, omw = np.zeros(ne), np.zeros(ne), np.zeros((ne, 3))
        lib().orc_omega_fields(self.ctx, _ptr(om0), _ptr(sw), _ptr(omw))
        return om0, sw, omw

    def average_start(self) -> None:
        """Average the statistics of every following step (restarts the average)."""
        lib().orc_average_start(self.ctx)

    def average_stop(self) -> None:
        lib().orc_average_stop(self.ctx)

    def average(self, ens: int = 0) -> np.ndarray:
        """Time-averaged records (nelem x navg), layout of ORC_AV_*."""
        L = lib()
        out = np.zeros((self.wl.mesh.nelem, L.orc_navg(self.ctx)))
        L.orc_average(self.ctx, ens, _ptr(out))
        return out

    def locate(self, x: float, y: float) -> int:
        return int(lib().orc_locate(self.ctx, float(x), float(y)))

    def wallfn_hits(self) -> int:
        """Particle steps so far whose frequency a wall-function reflection changed."""
        return int(lib().orc_wallfn_hits(self.ctx))

    def set_cond_means(self, cm, ens: int = 0) -> None:
        """IECM toward the given conditional means (nelem x 8) instead of the
        binned estimate, until called with None."""
        if cm is None:
            lib().orc_set_cond_means(self.ctx, ens, None)
            return
        a = np.ascontiguousarray(cm, np.float64).reshape(self.wl.mesh.nelem, 8)
        lib().orc_set_cond_means(self.ctx, ens, _ptr(a))

    def coefficients(self) -> np.ndarray:
        out = np.zeros((self.wl.mesh.nvert, 16))
        lib().orc_coefficients(self.ctx, _ptr(out))
        return out

    def set_drift(self, g6) -> None:
        """Replace G_11 G_12 G_21 G_22 G_33 C0 eps of every vertex (nvert x 6)."""
        a = np.ascontiguousarray(g6, np.float64).reshape(self.wl.mesh.nvert, 6)
        lib().orc_set_drift(self.ctx, _ptr(a))

    def set_pressure_gradient(self, g2) -> None:
        """Replace d<P>/dx and d<P>/dy of every vertex (nvert x 2)."""
        a = np.ascontiguousarray(g2, np.float64).reshape(self.wl.mesh.nvert, 2)
        lib().orc_set_pressure_gradient(self.ctx, _ptr(a))

    def mix_rate(self, ens: int = 0) -> np.ndarray:
        out = np.zeros(self.wl.mesh.nelem)
        lib().orc_mix_rate(self.ctx, ens, _ptr(out))
        return out

    def wall_alpha(self) -> np.ndarray:
        out = np.zeros((self.wl.mesh.nelem, 3))
        lib().orc_wall_alpha(self.ctx, _ptr(out))
        return out

    def walk(self, e: int, s, t, vel, om: Optional[float] = None):
        """One walk (see orc_walk); with om given, also returns the frequency
        after the wall conditions."""
        tx = ctypes.c_double(float(t[0]))
        ty = ctypes.c_double(float(t[1]))
        v = np.ascontiguousarray(vel, np.float64).copy()
        nref = ctypes.c_int32(0)
        o = None if om is None else ctypes.c_double(float(om))
        r = lib().orc_walk(self.ctx, int(e), float(s[0]), float(s[1]), ctypes.byref(tx), ctypes.byref(ty),
                           _ptr(v), ctypes.byref(nref), None if o is None else ctypes.byref(o))
        if o is not None:
            return r, (tx.value, ty.value), v, nref.value, o.value
        return r, (tx.value, ty.value), v, nref.value


# ---------------------------------------------------------------------------
# unit-level helpers


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def normals(seed: int, pid: int, step: int, ens: int, f32: bool) -> np.ndarray:
    out = np.zeros(8)
    lib().orc_normals(seed, pid, step, ens, 1 if f32 else 0, _ptr(out))
    return out


def normals_batch(seed: int, n: int, step: int, ens: int, f32: bool) -> np.ndarray:
    out = np.zeros((n, 8))
    lib().orc_normals_batch(seed, n, step, ens, 1 if f32 else 0, _ptr(out))
    return out


def exp64(x: float) -> float:
    return lib().orc_exp64(x)


def log64(x: float) -> float:
    return lib().orc_log64(x)


def log32(x: float) -> float:
    return lib().orc_log32(x)


def sincos2pi64(t: float):
    s, c = ctypes.c_double(), ctypes.c_double()
    lib().orc_sincos2pi64(t, ctypes.byref(s), ctypes.byref(c))
    return s.value, c.value


def sincos2pi32(t: float):
    s, c = ctypes.c_float(), ctypes.c_float()
    lib().orc_sincos2pi32(t, ctypes.byref(s), ctypes.byref(c))
    return s.value, c.value


def cbrt64(x: float) -> float:
    return lib().orc_cbrt64(x)
