"""Workload presets: mesh + frozen fields + model parameters + particle layout.

Each preset is a synthetic stand-in for one of the measured configurations
(the paper's street canyon of section 3, whose meshes, converged fields and
wind-tunnel data are not available).  Particle counts per element follow the
paper's uniform-weight particle-in-cell picture: density proportional to the
fluid volume, so an element receives a share of the N particles proportional
to its area (largest-remainder rounding, ties to the lower element index).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from functools import lru_cache
from typing import List

import numpy as np

from .fields import uniform_fields, canyon_fields
from .mesh import Mesh, canyon_mesh, unit_square_mesh, doubly_periodic_box

# model kinds
SLM = 0   # simplified Langevin model, eq. (19): G_ij = -(1/2 + 3/4 C0)<omega> delta_ij
GLM = 1   # drift tensor and C0 from the elliptic-relaxation tensor, eqs. (12)-(13)

# initial scalar rules
PSI_ZERO = 0
PSI_LEFT_QUARTER = 1   # psi = 1 where x < 0.25, else 0

H_SOURCE_DIAMETER = 0.01   # source diameter in units of h = H/2 (section 3)


@dataclass
class Ensemble:
    counts: np.ndarray          # (E,) int64 particles per element
    seed: int
    x0: tuple = (1.0, 0.0)      # source centre
    r0: float = 0.0             # source radius (0: no source)

    @property
    def n(self) -> int:
        return int(self.counts.sum())


@dataclass
class Workload:
    name: str
    mesh: Mesh
    fields: np.ndarray
    ensembles: List[Ensemble]
    precision: str = "f32"          # particle state type: "f64" or "f32"
    model: int = GLM
    dt: float = 1e-3
    nu: float = 1.0 / 12000.0
    C0: float = 2.1                 # SLM constant
    moments: int = 2                # highest central moment order estimated (2 or 4)
    hist_bins: int = 0              # scalar histogram bins per element (0: none)
    mix: bool = True                # IECM on
    psi_init: int = PSI_ZERO
    flags: int = 15                 # sub-steps: 1 velocity, 2 position/tracking, 4 IECM, 8 source
    steps: int = 100
    yp: float = 0.0                 # wall-function distance of the stripped walls
    omega: bool = False             # stochastic turbulent frequency per particle, eqs. (9)-(10)
    vbins: int = 2                  # velocity bins per component for <phi|V>: 2 (signs) or 5
    constants: dict = field(default_factory=lambda: dict(CT=6.0, Cs=0.02, Ct=0.7, Cmu=0.09,
                                                         kappa=0.41, Ewall=8.5, C3=5.0, C4=0.25,
                                                         Cw1=0.5, Cw2=0.73))

    @property
    def n_total(self) -> int:
        return sum(e.n for e in self.ensembles)

    @property
    def nens(self) -> int:
        return len(self.ensembles)

    def describe(self) -> dict:
        return dict(workload=self.name, mesh=self.mesh.name, elements=self.mesh.nelem,
                    vertices=self.mesh.nvert, particles=self.n_total, ensembles=self.nens,
                    precision=self.precision, model=("SLM" if self.model == SLM else "GLM"),
                    dt=self.dt, steps=self.steps, moments=self.moments, hist_bins=self.hist_bins,
                    omega=self.omega, vbins=self.vbins)


def apportion(areas: np.ndarray, n: int) -> np.ndarray:
    """Largest-remainder split of n particles proportional to element area."""
    q = n * areas / areas.sum()
    base = np.floor(q).astype(np.int64)
    rem = n - int(base.sum())
    frac = q - base
    order = np.lexsort((np.arange(len(q)), -frac))
    base[order[:rem]] += 1
    return base


def uniform_counts(mesh: Mesh, ppe: int) -> np.ndarray:
    return np.full(mesh.nelem, ppe, dtype=np.int64)


@lru_cache(maxsize=8)
def _canyon(target: int, wallfn: bool):
    m = canyon_mesh(target, wallfn=wallfn)
    return m, canyon_fields(m)


# ----------------------------------------------------------------------------
# the five measured configurations


def config1(steps: int = 100) -> Workload:
    """Plain method, small: 20x20x2 unit square, 50 particles/element, FP64, SLM."""
    m = unit_square_mesh(20)
    f = uniform_fields(m.nvert, U=(1.0, 0.0), k=1.0, eps=1.0)
    ens = [Ensemble(counts=uniform_counts(m, 50), seed=0)]
    return Workload(name="plain_square_800e_40k_f64", mesh=m, fields=f, ensembles=ens,
                    precision="f64", model=SLM, dt=0.01, nu=0.0, C0=2.1, moments=2,
                    psi_init=PSI_LEFT_QUARTER, steps=steps)


def _source_radius(H: float = 1.0) -> float:
    h = H / 2.0
    return 0.5 * H_SOURCE_DIAMETER * h


def config2(steps: int = 500, n: int = 1_000_000, seed: int = 0, target: int = 10000) -> Workload:
    """Street canyon, ~10k elements, 1M particles, GLM, no-slip walls, FP32 state."""
    m, f = _canyon(target, False)
    ens = [Ensemble(counts=apportion(m.areas(), n), seed=seed, x0=(1.0, 0.0), r0=_source_radius())]
    return Workload(name=f"canyon_{m.nelem}e_{n // 1000}k_glm_f32", mesh=m, fields=f, ensembles=ens,
                    precision="f32", model=GLM, dt=1e-3, nu=1.0 / 12000.0, moments=2, steps=steps)


def config3(steps: int = 1000, n: int = 10_000_000, seed: int = 0, target: int = 50000) -> Workload:
    """Large canyon with wall functions: ~50k elements, 10M particles, SLM C0=3.5,
    moments to 4th order and 32-bin scalar histograms."""
    yp = 13.0 / 256.0
    m, f = _canyon(target, True)
    ens = [Ensemble(counts=apportion(m.areas(), n), seed=seed, x0=(1.0, yp), r0=_source_radius())]
    return Workload(name=f"canyon_wf_{m.nelem}e_{n // 1_000_000}M_slm_f32", mesh=m, fields=f,
                    ensembles=ens, precision="f32", model=SLM, dt=1e-3, nu=1.0 / 12000.0, C0=3.5,
                    moments=4, hist_bins=32, steps=steps, yp=yp)


def config3w(steps: int = 1000, n: int = 10_000_000, seed: int = 0, target: int = 50000) -> Workload:
    """The large wall-function canyon with the stochastic turbulent frequency
    carried by every particle (eqs. 8-10 and the wall condition on omega)."""
    wl = config3(steps=steps, n=n, seed=seed, target=target)
    wl.omega = True
    wl.name = wl.name + "_omega"
    return wl


def config3b(steps: int = 1000, n: int = 10_000_000, seed: int = 0, target: int = 50000) -> Workload:
    """The large wall-function canyon with <phi|V> on 5 x 5 x 5 velocity bins
    (the bin structure of section 3)."""
    wl = config3(steps=steps, n=n, seed=seed, target=target)
    wl.vbins = 5
    wl.name = wl.name + "_bins5"
    return wl


def config4(steps: int = 100, nens: int = 64, target: int = 10000) -> Workload:
    """64 independent canyon runs of uneven size on the 10k-element mesh."""
    m, f = _canyon(target, False)
    rng = np.random.Generator(np.random.Philox(12345))
    sizes = np.rint(np.exp(rng.uniform(math.log(1e4), math.log(1e6), size=nens))).astype(np.int64)
    xs = rng.uniform(0.5, 1.5, size=nens)
    ens = [Ensemble(counts=apportion(m.areas(), int(sizes[i])), seed=1000 + i,
                    x0=(float(xs[i]), 0.0), r0=_source_radius()) for i in range(nens)]
    return Workload(name=f"canyon_{m.nelem}e_batched{nens}", mesh=m, fields=f, ensembles=ens,
                    precision="f32", model=GLM, dt=1e-3, nu=1.0 / 12000.0, moments=2, steps=steps)


def config5(ppe: int = 20, seed: int = 101, steps: int = 500, target: int = 10000) -> Workload:
    """Canyon run at a given particles/element for the learned conditional mean."""
    m, f = _canyon(target, False)
    n = ppe * m.nelem
    ens = [Ensemble(counts=apportion(m.areas(), n), seed=seed, x0=(1.0, 0.0), r0=_source_radius())]
    return Workload(name=f"canyon_{m.nelem}e_{ppe}ppe", mesh=m, fields=f, ensembles=ens,
                    precision="f32", model=GLM, dt=1e-3, nu=1.0 / 12000.0, moments=2, steps=steps)


# ----------------------------------------------------------------------------
# small cases for parity tests


def small_canyon(target: int = 2000, ppe: int = 40, seed: int = 7, wallfn: bool = False,
                 precision: str = "f32", moments: int = 2, hist_bins: int = 0, nens: int = 1,
                 steps: int = 20, omega: bool = False, vbins: int = 2) -> Workload:
    m, f = _canyon(target, wallfn)
    yp = 13.0 / 256.0 if wallfn else 0.0
    n = ppe * m.nelem
    ens = []
    for i in range(nens):
        ni = n if nens == 1 else max(1, n * (i + 1) // (2 * nens))
        ens.append(Ensemble(counts=apportion(m.areas(), ni), seed=seed + i,
                            x0=(0.75 + 0.5 * i / max(1, nens), yp),
                            r0=0.05))
    return Workload(name=f"small_canyon_{m.nelem}e", mesh=m, fields=f, ensembles=ens,
                    precision=precision, model=(SLM if wallfn else GLM), dt=1e-3,
                    nu=1.0 / 12000.0, C0=(3.5 if wallfn else 2.1), moments=moments,
                    hist_bins=hist_bins, steps=steps, yp=yp, omega=omega, vbins=vbins)


def tiny_canyon(**kw) -> Workload:
    kw.setdefault("target", 600)
    kw.setdefault("ppe", 20)
    return small_canyon(**kw)


def square_box(n: int = 8, ppe: int = 50, periodic_y: bool = True, precision: str = "f64",
               seed: int = 3, model: int = SLM, dt: float = 0.01, fields=None, C0: float = 2.1,
               steps: int = 10) -> Workload:
    m = doubly_periodic_box(n) if periodic_y else unit_square_mesh(n)
    f = uniform_fields(m.nvert) if fields is None else fields(m)
    ens = [Ensemble(counts=uniform_counts(m, ppe), seed=seed)]
    return Workload(name=f"box{n}", mesh=m, fields=f, ensembles=ens, precision=precision,
                    model=model, dt=dt, nu=0.0, C0=C0, moments=2, psi_init=PSI_LEFT_QUARTER,
                    steps=steps)
