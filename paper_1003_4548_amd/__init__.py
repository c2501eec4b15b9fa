"""Python binding of the pdfpic C ABI (``include/pdfpic.h``).

Argument marshalling only: every step of the particle method runs in the HIP
kernels of ``libpdfpic.so``.  PyTorch supplies the device arena and the HIP
stream.  Importing this module does not need a GPU; creating a
:class:`Simulation` does, and it raises if the library was not built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdfpic.so")

PDF_OK = 0
STATUS = {0: "PDF_OK", -1: "PDF_E_ARG", -2: "PDF_E_MESH", -3: "PDF_E_SIZE", -4: "PDF_E_HIP",
          -5: "PDF_E_LOST", -6: "PDF_E_NAN", -7: "PDF_E_CAPACITY", -8: "PDF_E_STATE"}

ST_N, ST_MEAN, ST_M2, ST_BINN, ST_BINM, ST_M3, ST_M4 = 0, 1, 5, 15, 23, 31, 51
NSTAT_2, NSTAT_4 = 31, 86
NFIELD = 20

# exported entry points (the declarations of include/pdfpic.h)
ENTRY_POINTS = ("pdf_create", "pdf_query_sizes", "pdf_init_mesh", "pdf_seed_particles", "pdf_step",
                "pdf_step_graph", "pdf_step_timed", "pdf_autotune", "pdf_set_launch", "pdf_repack", "pdf_repack_count",
                "pdf_estimate_statistics", "pdf_elliptic_relaxation", "pdf_pressure_projection", "pdf_relaxation_size", "pdf_nstat", "pdf_sync", "pdf_metrics",
                "pdf_mlp_work_floats", "pdf_mlp_dataset", "pdf_mlp_forward", "pdf_mlp_grad", "pdf_mlp_grad_noalloc", "pdf_mlp_train",
                "pdf_mlp_norm", "pdf_mlp_round", "pdf_mlp_infer", "pdf_mlp_attach",
                "pdf_get_state", "pdf_set_state", "pdf_set_step", "pdf_get_omega", "pdf_omega_fields", "pdf_navg", "pdf_average_attach",
                "pdf_locate", "pdf_average_probe", "pdf_count", "pdf_steps_done", "pdf_error_string", "pdf_destroy")


class PdfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class PdfParams(ctypes.Structure):
    _fields_ = [("f32_state", ctypes.c_int32), ("model", ctypes.c_int32), ("moments", ctypes.c_int32),
                ("hist_bins", ctypes.c_int32), ("mix", ctypes.c_int32), ("psi_init", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("omega", ctypes.c_int32), ("vbins", ctypes.c_int32),
                ("reserved", ctypes.c_int32),
                ("dt", ctypes.c_double), ("nu", ctypes.c_double), ("C0", ctypes.c_double),
                ("CT", ctypes.c_double), ("Cs", ctypes.c_double), ("Ct", ctypes.c_double),
                ("Cmu", ctypes.c_double), ("kappa", ctypes.c_double), ("Ewall", ctypes.c_double),
                ("yp", ctypes.c_double), ("Lx", ctypes.c_double), ("Ly", ctypes.c_double),
                ("slack", ctypes.c_double), ("C3", ctypes.c_double), ("C4", ctypes.c_double),
                ("Cw1", ctypes.c_double), ("Cw2", ctypes.c_double)]


class PdfMesh(ctypes.Structure):
    _fields_ = [("nvert", ctypes.c_int32), ("nelem", ctypes.c_int32), ("vtx", ctypes.c_void_p),
                ("tri", ctypes.c_void_p), ("nbr", ctypes.c_void_p), ("ekind", ctypes.c_void_p),
                ("fields", ctypes.c_void_p)]


class PdfSizes(ctypes.Structure):
    _fields_ = [("nvert", ctypes.c_int32), ("nelem", ctypes.c_int32), ("nens", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("nparticles", ctypes.c_int64),
                ("arena_bytes", ctypes.c_int64), ("slots", ctypes.c_int64)]


_lib = None


def library_path() -> str:
    return LIB_PATH


def load_library():
    """Load libpdfpic.so; raise if it was not built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1003_4548_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.pdf_create.restype = i32
    L.pdf_create.argtypes = [P(PdfParams), vp, P(vp)]
    L.pdf_query_sizes.restype = i32
    L.pdf_query_sizes.argtypes = [vp, P(PdfSizes)]
    L.pdf_init_mesh.restype = i32
    L.pdf_init_mesh.argtypes = [vp, P(PdfMesh), vp, i64]
    L.pdf_seed_particles.restype = i32
    L.pdf_seed_particles.argtypes = [vp, i32, vp, vp, vp]
    L.pdf_step.restype = i32
    L.pdf_step.argtypes = [vp, i32]
    L.pdf_step_graph.restype = i32
    L.pdf_step_graph.argtypes = [vp, i32]
    L.pdf_step_timed.restype = i32
    L.pdf_step_timed.argtypes = [vp, i32, P(ctypes.c_double)]
    L.pdf_autotune.restype = i32
    L.pdf_autotune.argtypes = [vp, i32, P(i32), P(i32)]
    L.pdf_set_launch.restype = i32
    L.pdf_set_launch.argtypes = [vp, i32, i32]
    u32, u64, f32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float
    L.pdf_mlp_work_floats.restype = i64
    L.pdf_mlp_work_floats.argtypes = [i32]
    L.pdf_mlp_dataset.restype = i32
    L.pdf_mlp_dataset.argtypes = [vp, i32, u64, u32, vp]
    L.pdf_mlp_forward.restype = i32
    L.pdf_mlp_forward.argtypes = [vp, i64, i32, vp, vp, vp, vp]
    L.pdf_mlp_grad.restype = i32
    L.pdf_mlp_grad.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    L.pdf_mlp_grad_noalloc.restype = i32
    L.pdf_mlp_grad_noalloc.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    L.pdf_mlp_train.restype = i32
    L.pdf_mlp_train.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, i32, i32, f32, u64, i64, vp]
    L.pdf_mlp_norm.restype = i32
    L.pdf_mlp_norm.argtypes = [vp, i64, vp, vp]
    L.pdf_mlp_round.restype = i32
    L.pdf_mlp_round.argtypes = [vp, vp, vp]
    L.pdf_mlp_infer.restype = i32
    L.pdf_mlp_infer.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp]
    L.pdf_mlp_attach.restype = i32
    L.pdf_mlp_attach.argtypes = [vp, vp, vp, vp, vp]
    L.pdf_repack.restype = i32
    L.pdf_repack.argtypes = [vp]
    L.pdf_repack_count.restype = i64
    L.pdf_repack_count.argtypes = [vp]
    L.pdf_estimate_statistics.restype = i32
    L.pdf_estimate_statistics.argtypes = [vp, vp, i32]
    L.pdf_elliptic_relaxation.restype = i32
    L.pdf_elliptic_relaxation.argtypes = [vp, i32, ctypes.c_double, vp, vp, vp, vp]
    L.pdf_pressure_projection.restype = i32
    L.pdf_pressure_projection.argtypes = [vp, i32, ctypes.c_double, vp, vp, vp, vp]
    L.pdf_relaxation_size.restype = i32
    L.pdf_relaxation_size.argtypes = [vp, vp]
    L.pdf_nstat.restype = i32
    L.pdf_nstat.argtypes = [vp]
    L.pdf_sync.restype = i32
    L.pdf_sync.argtypes = [vp]
    L.pdf_get_state.restype = i32
    L.pdf_get_state.argtypes = [vp, i32, vp, vp]
    L.pdf_metrics.restype = i32
    L.pdf_metrics.argtypes = [vp, vp]
    L.pdf_set_state.restype = i32
    L.pdf_set_state.argtypes = [vp, i32, vp, vp, vp]
    L.pdf_set_step.restype = i32
    L.pdf_set_step.argtypes = [vp, i64]
    L.pdf_get_omega.restype = i32
    L.pdf_get_omega.argtypes = [vp, i32, vp, vp, vp]
    L.pdf_omega_fields.restype = i32
    L.pdf_omega_fields.argtypes = [vp, vp, vp, vp]
    L.pdf_navg.restype = i32
    L.pdf_navg.argtypes = [vp]
    L.pdf_average_attach.restype = i32
    L.pdf_average_attach.argtypes = [vp, vp]
    L.pdf_locate.restype = i32
    L.pdf_locate.argtypes = [vp, vp, i32, vp]
    L.pdf_average_probe.restype = i32
    L.pdf_average_probe.argtypes = [vp, vp, i32, vp, i32, vp]
    L.pdf_count.restype = i64
    L.pdf_count.argtypes = [vp, i32]
    L.pdf_steps_done.restype = i64
    L.pdf_steps_done.argtypes = [vp]
    L.pdf_error_string.restype = ctypes.c_char_p
    L.pdf_error_string.argtypes = [vp]
    L.pdf_destroy.restype = None
    L.pdf_destroy.argtypes = [vp]
    _lib = L
    return L


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Simulation:
    """One set of ensembles on one mesh, advanced by the HIP library.

    mesh arrays are host numpy arrays in the layout of ``include/pdfpic.h``;
    ``counts`` is a list (one per ensemble) of per-element particle counts.
    """

    def __init__(self, *, vtx, tri, nbr, ekind, fields, counts: Sequence[np.ndarray],
                 seeds: Sequence[int], sources: Sequence[Sequence[float]], precision: str = "f32",
                 model: int = 1, moments: int = 2, hist_bins: int = 0, mix: bool = True,
                 psi_init: int = 0, flags: int = 15, dt: float = 1e-3, nu: float = 0.0,
                 C0: float = 2.1, CT: float = 6.0, Cs: float = 0.02, Ct: float = 0.7,
                 Cmu: float = 0.09, kappa: float = 0.41, Ewall: float = 8.5, yp: float = 0.0,
                 Lx: float = 1.0, Ly: float = 1.0, slack: float = 2.0, omega: bool = False, vbins: int = 2,
                 C3: float = 5.0, C4: float = 0.25, Cw1: float = 0.5, Cw2: float = 0.73,
                 device: str = "cuda:0", stream=None):
        import torch

        self.torch = torch
        L = load_library()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.params = PdfParams(f32_state=1 if precision == "f32" else 0, model=int(model), moments=int(moments),
                                hist_bins=int(hist_bins), mix=1 if mix else 0, psi_init=int(psi_init),
                                flags=int(flags), omega=1 if omega else 0, vbins=int(vbins), reserved=0,
                                dt=dt, nu=nu, C0=C0, CT=CT, Cs=Cs,
                                Ct=Ct, Cmu=Cmu, kappa=kappa, Ewall=Ewall, yp=yp, Lx=Lx, Ly=Ly, slack=slack,
                                C3=C3, C4=C4, Cw1=Cw1, Cw2=Cw2)
        self.ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            self._check(L.pdf_create(ctypes.byref(self.params), ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.byref(self.ctx)), "pdf_create")
        self._host = dict(vtx=np.ascontiguousarray(vtx, np.float64), tri=np.ascontiguousarray(tri, np.int32),
                          nbr=np.ascontiguousarray(nbr, np.int32), ekind=np.ascontiguousarray(ekind, np.int32),
                          fields=np.ascontiguousarray(fields, np.float64))
        self.nvert = int(self._host["vtx"].shape[0])
        self.nelem = int(self._host["tri"].shape[0])
        self.nens = len(counts)
        cnt = np.ascontiguousarray(np.stack([np.asarray(c, np.int64) for c in counts]), np.int64)
        self.counts = cnt
        sz = PdfSizes(nvert=self.nvert, nelem=self.nelem, nens=self.nens, reserved=0,
                      nparticles=int(cnt.sum()), arena_bytes=0, slots=0)
        self._check(L.pdf_query_sizes(self.ctx, ctypes.byref(sz)), "pdf_query_sizes")
        self.arena_bytes = int(sz.arena_bytes)
        self.slots = int(sz.slots)
        self.arena = torch.empty(self.arena_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.arena.data_ptr()
        self._arena_ptr = (base + 255) // 256 * 256
        h = self._host
        mesh = PdfMesh(nvert=self.nvert, nelem=self.nelem, vtx=_ptr(h["vtx"]).value, tri=_ptr(h["tri"]).value,
                       nbr=_ptr(h["nbr"]).value, ekind=_ptr(h["ekind"]).value, fields=_ptr(h["fields"]).value)
        with torch.cuda.device(self.device):
            self._check(L.pdf_init_mesh(self.ctx, ctypes.byref(mesh), ctypes.c_void_p(self._arena_ptr),
                                        self.arena_bytes), "pdf_init_mesh")
            self._seeds = np.ascontiguousarray(np.asarray(seeds, np.uint64))
            self._src = np.ascontiguousarray(np.asarray(sources, np.float64).reshape(self.nens, 3))
            self._check(L.pdf_seed_particles(self.ctx, self.nens, _ptr(cnt), _ptr(self._seeds), _ptr(self._src)),
                        "pdf_seed_particles")
        self.nstat = int(L.pdf_nstat(self.ctx))

    @classmethod
    def from_workload(cls, wl, device: str = "cuda:0", ensembles=None, **kw):
        """Build from a workload description (mesh, fields, ensembles, model)."""
        m = wl.mesh
        ens = wl.ensembles if ensembles is None else ensembles
        c = wl.constants
        args = dict(vtx=m.vtx, tri=m.tri, nbr=m.nbr, ekind=m.ekind, fields=wl.fields,
                    counts=[e.counts for e in ens], seeds=[e.seed for e in ens],
                    sources=[(e.x0[0], e.x0[1], e.r0) for e in ens], precision=wl.precision,
                    model=wl.model, moments=wl.moments, hist_bins=wl.hist_bins, mix=wl.mix,
                    psi_init=wl.psi_init, flags=getattr(wl, "flags", 15), dt=wl.dt, nu=wl.nu, C0=wl.C0,
                    CT=c["CT"], Cs=c["Cs"], Ct=c["Ct"], Cmu=c["Cmu"], kappa=c["kappa"], Ewall=c["Ewall"],
                    yp=wl.yp, Lx=m.Lx, Ly=m.Ly, omega=bool(getattr(wl, "omega", False)),
                    vbins=int(getattr(wl, "vbins", 2)),
                    C3=c.get("C3", 5.0), C4=c.get("C4", 0.25), Cw1=c.get("Cw1", 0.5), Cw2=c.get("Cw2", 0.73),
                    device=device)
        args.update(kw)
        return cls(**args)

    # -- helpers -----------------------------------------------------------------
    def _check(self, status: int, what: str) -> None:
        if status != PDF_OK:
            msg = ""
            if self.ctx:
                raw = load_library().pdf_error_string(self.ctx)
                msg = raw.decode() if raw else ""
            raise PdfError(int(status), f"{what}: {msg}")

    def close(self) -> None:
        if getattr(self, "ctx", None) and self.ctx.value:
            load_library().pdf_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the C ABI, call for call -------------------------------------------------
    def step(self, n: int = 1) -> None:
        self._check(load_library().pdf_step(self.ctx, int(n)), "pdf_step")

    def step_timed(self, n: int = 1) -> float:
        """As step(), returning the summed HIP-event time of the n steps'
        kernels in milliseconds (waits)."""
        ms = ctypes.c_double(0.0)
        self._check(load_library().pdf_step_timed(self.ctx, int(n), ctypes.byref(ms)), "pdf_step_timed")
        return ms.value

    def step_graph(self, n: int = 1) -> None:
        """As step(), replaying a HIP graph of six steps."""
        self._check(load_library().pdf_step_graph(self.ctx, int(n)), "pdf_step_graph")

    def autotune(self, steps_per_trial: int = 5):
        """Pick the launch shape by timing real steps; returns (group, persist)."""
        g, pe = ctypes.c_int32(), ctypes.c_int32()
        self._check(load_library().pdf_autotune(self.ctx, int(steps_per_trial), ctypes.byref(g), ctypes.byref(pe)),
                    "pdf_autotune")
        return int(g.value), int(pe.value)

    def set_launch(self, group: int, persist: int = 0) -> None:
        self._check(load_library().pdf_set_launch(self.ctx, int(group), int(persist)), "pdf_set_launch")

    def repack(self) -> None:
        """Re-lay out the element segments from the current counts now."""
        self._check(load_library().pdf_repack(self.ctx), "pdf_repack")

    def repacks(self) -> int:
        """Repacks done since seeding (waits for the stream)."""
        n = int(load_library().pdf_repack_count(self.ctx))
        if n < 0:
            raise PdfError(-4, "pdf_repack_count failed")
        return n

    def sync(self) -> None:
        self._check(load_library().pdf_sync(self.ctx), "pdf_sync")

    def steps_done(self) -> int:
        return int(load_library().pdf_steps_done(self.ctx))

    def count(self, ens: int = 0) -> int:
        return int(load_library().pdf_count(self.ctx, int(ens)))

    def statistics_device(self):
        """Statistics of the current state as a device tensor (nens, nelem, nstat)."""
        out = self.torch.empty((self.nens, self.nelem, self.nstat), dtype=self.torch.float64, device=self.device)
        self._check(load_library().pdf_estimate_statistics(self.ctx, ctypes.c_void_p(out.data_ptr()), 0),
                    "pdf_estimate_statistics")
        return out

    def statistics(self) -> np.ndarray:
        out = np.zeros((self.nens, self.nelem, self.nstat))
        self._check(load_library().pdf_estimate_statistics(self.ctx, _ptr(out), 1), "pdf_estimate_statistics")
        return out

    def elliptic_relaxation(self, max_iters: int = 4000, tol: float = 1e-10, outputs: bool = True) -> dict:
        """Solve the elliptic relaxation from the statistics of the current
        state and write G and C0 eps into the coefficient table (waits).
        Returns iterations, converged, clamped (vertices whose C0 was
        negative), from_stats (elements whose stresses came from the
        particles), resid (||r|| / ||b|| per component) and, with outputs,
        wp (nvert x 5) and coef (nvert x 6) as numpy arrays."""
        info = np.zeros(4, np.int32)
        resid = np.zeros(5)
        wp = coef = None
        if outputs:
            wp = self.torch.empty((self.nvert, 5), dtype=self.torch.float64, device=self.device)
            coef = self.torch.empty((self.nvert, 6), dtype=self.torch.float64, device=self.device)
        self._check(load_library().pdf_elliptic_relaxation(
            self.ctx, int(max_iters), float(tol), ctypes.c_void_p(wp.data_ptr() if outputs else 0),
            ctypes.c_void_p(coef.data_ptr() if outputs else 0), _ptr(info), _ptr(resid)), "pdf_elliptic_relaxation")
        out = dict(iterations=int(info[0]), converged=bool(info[1]), clamped=int(info[2]), from_stats=int(info[3]),
                   resid=resid)
        if outputs:
            out["wp"] = wp.cpu().numpy()
            out["coef"] = coef.cpu().numpy()
        return out

    def pressure_projection(self, max_iters: int = 20000, tol: float = 1e-10, outputs: bool = True) -> dict:
        """Project the particles' mean velocity (one ensemble): solve for the
        pressure increment, add its gradient to the mean pressure gradient and
        correct every particle's velocity (waits).  The correction covers the
        steps since the previous applied projection (since seeding for the
        first), so it may be called every n steps.  Returns iterations,
        converged, applied, from_stats, resid and, with outputs, phi (nvert,
        up to a constant) and grad (nvert x 2) as numpy arrays."""
        info = np.zeros(4, np.int32)
        resid = np.zeros(5)
        phi = grad = None
        if outputs:
            phi = self.torch.empty((self.nvert,), dtype=self.torch.float64, device=self.device)
            grad = self.torch.empty((self.nvert, 2), dtype=self.torch.float64, device=self.device)
        self._check(load_library().pdf_pressure_projection(
            self.ctx, int(max_iters), float(tol), ctypes.c_void_p(phi.data_ptr() if outputs else 0),
            ctypes.c_void_p(grad.data_ptr() if outputs else 0), _ptr(info), _ptr(resid)), "pdf_pressure_projection")
        out = dict(iterations=int(info[0]), converged=bool(info[1]), applied=bool(info[2]), from_stats=int(info[3]),
                   resid=resid)
        if outputs:
            out["phi"] = phi.cpu().numpy()
            out["grad"] = grad.cpu().numpy()
        return out

    def relaxation_size(self) -> dict:
        """Unknowns, nonzeros and the padded row length of the relaxation
        system, and the aggregates of the projection's coarse space."""
        out = np.zeros(4, np.int64)
        self._check(load_library().pdf_relaxation_size(self.ctx, _ptr(out)), "pdf_relaxation_size")
        return dict(unknowns=int(out[0]), nonzeros=int(out[1]), row_width=int(out[2]), aggregates=int(out[3]))

    def state_device(self, ens: int = 0):
        n = self.count(ens)
        vals = self.torch.empty((6, n), dtype=self.torch.float64, device=self.device)
        elem = self.torch.empty((n,), dtype=self.torch.int32, device=self.device)
        self._check(load_library().pdf_get_state(self.ctx, int(ens), ctypes.c_void_p(vals.data_ptr()),
                                                 ctypes.c_void_p(elem.data_ptr())), "pdf_get_state")
        return vals, elem

    def state(self, ens: int = 0) -> dict:
        """State in id order; with the turbulent frequency also "omega"."""
        if self.params.omega:
            n = self.count(ens)
            vals = self.torch.empty((6, n), dtype=self.torch.float64, device=self.device)
            elem = self.torch.empty((n,), dtype=self.torch.int32, device=self.device)
            om = self.torch.empty((n,), dtype=self.torch.float64, device=self.device)
            self._check(load_library().pdf_get_omega(self.ctx, int(ens), ctypes.c_void_p(vals.data_ptr()),
                                                     ctypes.c_void_p(elem.data_ptr()),
                                                     ctypes.c_void_p(om.data_ptr())), "pdf_get_omega")
        else:
            vals, elem = self.state_device(ens)
        self.stream.synchronize()
        v = vals.cpu().numpy()
        out = dict(x=v[0], y=v[1], u=v[2], v=v[3], w=v[4], psi=v[5], elem=elem.cpu().numpy())
        if self.params.omega:
            out["omega"] = om.cpu().numpy()
        return out

    # -- time averaging and probes ---------------------------------------------
    def average_attach(self):
        """Start (or restart) time averaging; returns the accumulator tensor
        (nens, nelem, navg) that every following step merges into."""
        navg = int(load_library().pdf_navg(self.ctx))
        self._avg = self.torch.empty((self.nens, self.nelem, navg), dtype=self.torch.float64, device=self.device)
        self._check(load_library().pdf_average_attach(self.ctx, ctypes.c_void_p(self._avg.data_ptr())),
                    "pdf_average_attach")
        return self._avg

    def average_detach(self) -> None:
        self._check(load_library().pdf_average_attach(self.ctx, None), "pdf_average_attach")

    def average(self) -> np.ndarray:
        """The time-averaged records so far (waits for the stream)."""
        self.stream.synchronize()
        return self._avg.cpu().numpy()

    def locate(self, points) -> np.ndarray:
        """Element containing each point (lowest index; -1 outside)."""
        xy = self.torch.tensor(np.asarray(points, np.float64).reshape(-1, 2), device=self.device)
        out = self.torch.empty((xy.shape[0],), dtype=self.torch.int32, device=self.device)
        self._check(load_library().pdf_locate(self.ctx, ctypes.c_void_p(xy.data_ptr()), int(xy.shape[0]),
                                              ctypes.c_void_p(out.data_ptr())), "pdf_locate")
        self.stream.synchronize()
        return out.cpu().numpy()

    def probe(self, elems, ens: int = 0) -> np.ndarray:
        """Probe rows (steps, count per step, <psi>, <psi'^2>, CDF at the bin
        edges) of the current time average at the given elements."""
        el = self.torch.tensor(np.asarray(elems, np.int32), device=self.device)
        hist = int(self.params.hist_bins)
        out = self.torch.empty((el.shape[0], 4 + hist), dtype=self.torch.float64, device=self.device)
        self._check(load_library().pdf_average_probe(self.ctx, ctypes.c_void_p(self._avg.data_ptr()), int(ens),
                                                     ctypes.c_void_p(el.data_ptr()), int(el.shape[0]),
                                                     ctypes.c_void_p(out.data_ptr())), "pdf_average_probe")
        self.stream.synchronize()
        return out.cpu().numpy()

    def set_state(self, st: dict, ens: int = 0) -> None:
        """Replace ensemble ens's state with st (x y u v w psi elem, and omega
        when carried), particle i becoming id i (checkpoint restore)."""
        t = self.torch
        vals = t.tensor(np.stack([np.asarray(st[k], np.float64) for k in ("x", "y", "u", "v", "w", "psi")]),
                        device=self.device)
        elem = t.tensor(np.asarray(st["elem"], np.int32), device=self.device)
        om = None
        if self.params.omega:
            om = t.tensor(np.asarray(st["omega"], np.float64), device=self.device)
        self.stream.synchronize()
        self._check(load_library().pdf_set_state(self.ctx, int(ens), ctypes.c_void_p(vals.data_ptr()),
                                                 ctypes.c_void_p(elem.data_ptr()),
                                                 None if om is None else ctypes.c_void_p(om.data_ptr())),
                    "pdf_set_state")

    def metrics(self) -> dict:
        """Counters of the current state (see pdf_metrics)."""
        out = np.zeros(8, np.int64)
        self._check(load_library().pdf_metrics(self.ctx, _ptr(out)), "pdf_metrics")
        keys = ("particles", "arrivals_last_step", "min_per_cell", "max_per_cell", "cells_over_three_quarters",
                "repacks", "error_word", "steps_done")
        return {k: int(v) for k, v in zip(keys, out)}

    def set_step(self, step: int) -> None:
        """Philox step word of the next step (resume from a checkpoint)."""
        self._check(load_library().pdf_set_step(self.ctx, int(step)), "pdf_set_step")

    def omega_fields(self):
        """(<omega> per centroid, S_omega per element, <omega> per wall-function
        edge midpoint (nelem x 3))."""
        om0, sw, omw = np.zeros(self.nelem), np.zeros(self.nelem), np.zeros((self.nelem, 3))
        self._check(load_library().pdf_omega_fields(self.ctx, _ptr(om0), _ptr(sw), _ptr(omw)), "pdf_omega_fields")
        return om0, sw, omw
