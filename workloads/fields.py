"""Frozen synthetic Eulerian fields at mesh vertices.

In the paper the mean velocity, mean pressure, Reynolds stresses, dissipation
and the elliptic-relaxation tensor come from Eulerian finite-element solves
(section 2.1, eq. (14); the closing summary of section 2.2).  Those solvers are outside the
particle step, so every workload here freezes smooth synthetic fields instead.
The particle method reads them at vertices and interpolates linearly.

Per-vertex layout, float64, column order ``FIELD_NAMES``:

    U, V            mean velocity <U>, <V> (W = 0, d/dz = 0)
    dUdx .. dVdy    mean velocity gradient
    lapU, lapV      Laplacian of the mean velocity
    dPdx, dPdy      mean pressure gradient (density 1)
    R11 R22 R33 R12 Reynolds stresses (R13 = R23 = 0)
    eps             dissipation rate
    P11 P12 P21 P22 P33   elliptic-relaxation tensor (wp_ij), zero off the
                    listed components

The canyon recipe:

* stream function: a channel profile above roof level plus a clockwise canyon
  vortex, both vanishing to second order at the street and the side walls,
  so the mean velocity is divergence free;
* k peaks in the shear layer at roof level and is damped toward the walls;
* anisotropy of magnitude below 0.15, so the stresses are realizable;
* eps = k^(3/2) / max(kappa d, 0.02), d the distance to the nearest no-slip
  wall;
* wp_ij is the local right-hand side of eq. (14) with the L^2 term dropped,
  using eqs. (15)-(17) and Table 2's constants, with the shear part damped
  where needed so that the drift tensor of eq. (12) stays stable (real parts
  of its eigenvalues below -0.2 <omega>) and C0 of eq. (13) stays >= 0.1;
* the mean pressure gradient closes the steady mean momentum balance,
  -dP/dx_i = <U_j> d<U_i>/dx_j + dR_ij/dx_j - nu lap <U_i>.
"""
from __future__ import annotations

import numpy as np
import sympy as sp

FIELD_NAMES = ("U", "V", "dUdx", "dUdy", "dVdx", "dVdy", "lapU", "lapV", "dPdx", "dPdy",
               "R11", "R22", "R33", "R12", "eps", "P11", "P12", "P21", "P22", "P33")
NFIELD = len(FIELD_NAMES)
F = {n: i for i, n in enumerate(FIELD_NAMES)}

# Table 2 of the paper (constants used by the synthetic wp recipe only)
TABLE2 = dict(C1=1.85, C2=0.63, C3=5.0, C4=0.25, CT=6.0, CL=0.134, Ceta=72.0, Cv=1.4,
              gamma5=0.1, Comega1=0.5, Comega2=0.73, Cs=0.02, Ct=0.7)


def uniform_fields(nvert: int, U=(1.0, 0.0), k: float = 1.0, eps: float = 1.0) -> np.ndarray:
    """Homogeneous isotropic turbulence in a uniform stream (no gradients)."""
    f = np.zeros((nvert, NFIELD))
    f[:, F["U"]] = U[0]
    f[:, F["V"]] = U[1]
    r = 2.0 * k / 3.0
    f[:, F["R11"]] = r
    f[:, F["R22"]] = r
    f[:, F["R33"]] = r
    f[:, F["eps"]] = eps
    return f


# ----------------------------------------------------------------------------
# canyon


def _velocity_functions(U0=1.0, delta=0.1, A=20.0, sq=0.6, xl=0.5, xr=1.5, ys=0.0, yr=1.0,
                        slip_floor=0.0):
    """Channel profile above y = yr plus a clockwise vortex in xl < x < xr.

    With slip_floor = 0 both parts vanish to second order on the walls (no
    slip); with slip_floor > 0 (wall functions) the stream function vanishes
    to first order on the walls: no flow through them, a finite tangential
    velocity along them."""
    x, y = sp.symbols("x y", real=True)
    s = y - yr
    if slip_floor > 0.0:
        S_ch = slip_floor * s + (1.0 - slip_floor) * (s - delta * sp.tanh(s / delta))
        X = (x - xl) * (xr - x)
        yy = y - ys
        q = yy * sp.exp(-(yy / sq) ** 2)
        Psi_v = -A * 0.25 * X * q
    else:
        S_ch = s - delta * sp.tanh(s / delta)          # dS/dy = tanh^2(s/delta), 0 for y < yr
        X = (x - xl) * (xr - x)
        q = y ** 2 * sp.exp(-(y / sq) ** 2)
        Psi_v = -A * X ** 2 * q
    out = {}
    for name, psi in (("ch", U0 * S_ch), ("v", Psi_v)):
        U = sp.diff(psi, y)
        V = -sp.diff(psi, x)
        exprs = [U, V, sp.diff(U, x), sp.diff(U, y), sp.diff(V, x), sp.diff(V, y),
                 sp.diff(U, x, 2) + sp.diff(U, y, 2), sp.diff(V, x, 2) + sp.diff(V, y, 2)]
        out[name] = sp.lambdify((x, y), exprs, "numpy")
    return out


def _mean_velocity(xy, g):
    fn = _velocity_functions(xl=g["x_l"], xr=g["x_r"], ys=g["y_street"], yr=g["y_roof"],
                             slip_floor=g.get("slip_floor", 0.0))
    x, y = xy[:, 0], xy[:, 1]
    res = np.zeros((len(x), 8))
    ch = np.array([np.broadcast_to(v, x.shape) for v in fn["ch"](x, y)]).T
    res += np.where((y >= g["y_roof"])[:, None], ch, 0.0)
    v = np.array([np.broadcast_to(v, x.shape) for v in fn["v"](x, y)]).T
    inside = (x >= g["x_l"]) & (x <= g["x_r"])
    res += np.where(inside[:, None], v, 0.0)
    return res


def _wall_distance(x, y, g):
    """Distance to the nearest no-slip wall of the full-resolution canyon."""
    def seg(px, py, ax, ay, bx, by):
        dx, dy = bx - ax, by - ay
        t = np.clip(((px - ax) * dx + (py - ay) * dy) / (dx * dx + dy * dy), 0.0, 1.0)
        return np.hypot(px - (ax + t * dx), py - (ay + t * dy))
    Lx = g["Lx"]
    d = np.full(x.shape, np.inf)
    for sh in (-Lx, 0.0, Lx):
        xs = x + sh
        d = np.minimum(d, seg(xs, y, g["x_l"], 0.0, g["x_r"], 0.0))
        d = np.minimum(d, seg(xs, y, g["x_l"], 0.0, g["x_l"], 1.0))
        d = np.minimum(d, seg(xs, y, g["x_r"], 0.0, g["x_r"], 1.0))
        d = np.minimum(d, seg(xs, y, 0.0, 1.0, g["x_l"], 1.0))
        d = np.minimum(d, seg(xs, y, g["x_r"], 1.0, Lx, 1.0))
    return d


def _stresses(x, y, dUdy, g, k0=0.002, k1=0.02, sk=0.25):
    d = _wall_distance(x, y, g)
    k = (k0 + k1 * np.exp(-((y - 1.0) / sk) ** 2)) * (0.25 + 0.75 * np.tanh(d / 0.05))
    b11 = 0.08
    b22 = -0.06
    b33 = -0.02
    b12 = -0.10 * np.tanh(0.2 * dUdy)
    R11 = 2.0 * k * (b11 + 1.0 / 3.0)
    R22 = 2.0 * k * (b22 + 1.0 / 3.0)
    R33 = 2.0 * k * (b33 + 1.0 / 3.0)
    R12 = 2.0 * k * b12
    eps = k ** 1.5 / np.maximum(0.41 * d, 0.02)
    return R11, R22, R33, R12, eps, k


# near-wall recipe of the wall-function canyon
WALL_BLEND = 0.05          # distance over which the wall statistics take over
LOG_KAPPA, LOG_E, LOG_CMU = 0.41, 8.5, 0.09


def _log_law_uhat(Ut, yp, nu):
    """u_hat with |Ut| = (u_hat / kappa) ln(E yp u_hat / nu), by bisection on
    ln u_hat (the right-hand side grows with u_hat above nu / (E yp));
    floored where |Ut| is too small for a root."""
    lo = np.full(Ut.shape, np.log(1.001 * nu / (LOG_E * yp)))
    hi = np.full(Ut.shape, np.log(10.0))
    target = np.abs(Ut)
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        u = np.exp(mid)
        f = u / LOG_KAPPA * np.log(LOG_E * yp * u / nu)
        lo = np.where(f < target, mid, lo)
        hi = np.where(f < target, hi, mid)
    return np.exp(0.5 * (lo + hi))


def _stripped_walls(geo):
    """The wall-function walls of a stripped canyon: (a, b, inward normal)."""
    yp_r = geo.y_roof
    return [((geo.x_l, geo.y_street), (geo.x_r, geo.y_street), (0.0, 1.0)),
            ((geo.x_l, geo.y_street), (geo.x_l, yp_r), (1.0, 0.0)),
            ((geo.x_r, geo.y_street), (geo.x_r, yp_r), (-1.0, 0.0)),
            ((0.0, yp_r), (geo.x_l, yp_r), (0.0, 1.0)),
            ((geo.x_r, yp_r), (geo.Lx, yp_r), (0.0, 1.0))]


def _wall_stresses(px, py, vel_at, base, geo, yp, nu):
    """Stresses blended toward log-law equilibrium at the stripped walls.

    At a wall-function wall the statistics at y_p should be those of an
    equilibrium log layer: with the tangential mean velocity U_t at the
    nearest point of the wall,
    u_hat from the log law, k = u_hat^2 / C_mu^(1/2), wall-normal variance
    u_hat^2 (so that alpha of the wall condition is 2 in the absence of a
    pressure-gradient correction), shear stress -tanh(U_t / 0.05) C_mu^(1/2) k;
    u_hat is at least half the base flow's C_mu^(1/4) k^(1/2).
    Each wall i contributes its target with weight (1 - s_i / WALL_BLEND)^2
    (s_i the distance to it); the base stresses keep the remaining weight
    (targets only, normalised, where the weights sum past 1)."""
    R11, R22, R33, R12 = base
    acc = np.zeros((4, len(px)))
    wsum = np.zeros(len(px))
    for (ax, ay), (bx, by), (nx, ny) in _stripped_walls(geo):
        for sh in (-geo.Lx, 0.0, geo.Lx):
            qx = px + sh
            dx, dy = bx - ax, by - ay
            t = np.clip(((qx - ax) * dx + (py - ay) * dy) / (dx * dx + dy * dy), 0.0, 1.0)
            s = np.hypot(qx - (ax + t * dx), py - (ay + t * dy))
            w = np.maximum(0.0, 1.0 - s / WALL_BLEND) ** 2
            if not (w > 0).any():
                continue
            tx, ty = ny, -nx                       # wall tangent
            # the tangential mean velocity at the wall point nearest to p
            U, V = vel_at(ax + t * dx - sh, ay + t * dy)
            Ut = U * tx + V * ty
            # where the tangential velocity is too small for a log layer
            # (corners) u_hat keeps half the base flow's value: alpha < 2 there
            uh = np.maximum(_log_law_uhat(Ut, yp, nu), LOG_CMU ** 0.25 * np.sqrt(0.5 * (R11 + R22 + R33)))
            k = uh * uh / np.sqrt(LOG_CMU)
            Rnn = uh * uh
            Rzz = 0.55 * k
            Rtt = 2.0 * k - Rnn - Rzz
            # a smooth sign: the mean pressure gradient differentiates the stresses
            Rtn = -np.tanh(Ut / 0.05) * np.sqrt(LOG_CMU) * k
            # back to (x, y): R = Rtt t t^T + Rnn n n^T + Rtn (t n^T + n t^T)
            r11 = Rtt * tx * tx + Rnn * nx * nx + 2 * Rtn * tx * nx
            r22 = Rtt * ty * ty + Rnn * ny * ny + 2 * Rtn * ty * ny
            r12 = Rtt * tx * ty + Rnn * nx * ny + Rtn * (tx * ny + nx * ty)
            acc += w * np.stack([r11, r22, Rzz, r12])
            wsum += w
    keep = np.maximum(0.0, 1.0 - wsum)
    norm = np.maximum(1.0, wsum)
    out = [(keep * b + a) / norm for b, a in zip((R11, R22, R33, R12), acc)]
    return out


def canyon_fields(mesh, nu: float = 1.0 / 12000.0, with_stats: bool = False):
    """Synthetic frozen fields for a street-canyon mesh (full or stripped)."""
    g = dict(Lx=2.0, x_l=0.5, x_r=1.5, y_street=0.0, y_roof=1.0)
    geo = getattr(mesh, "geometry", None)
    flow = dict(g)
    if geo is not None and geo.wallfn:
        # mean flow built on the stripped walls: no flow through them
        flow.update(x_l=geo.x_l, x_r=geo.x_r, y_street=geo.y_street, y_roof=geo.y_roof, slip_floor=0.3)
    xy = mesh.vtx
    x, y = xy[:, 0], xy[:, 1]
    mv = _mean_velocity(xy, flow)
    U, V, dUdx, dUdy, dVdx, dVdy, lapU, lapV = mv.T

    wallfn = geo is not None and geo.wallfn

    def stress_at(px, py):
        m = _mean_velocity(np.stack([px, py], axis=1), flow)
        R11, R22, R33, R12, eps, k = _stresses(px, py, m[:, 3], g)
        if wallfn:
            # log-law equilibrium at the wall-function walls; eps from the new k
            def vel_at(qx, qy):
                w = _mean_velocity(np.stack([qx, qy], axis=1), flow)
                return w[:, 0], w[:, 1]
            R11, R22, R33, R12 = _wall_stresses(px, py, vel_at, (R11, R22, R33, R12), geo, geo.y_street, nu)
            k = 0.5 * (R11 + R22 + R33)
            eps = k ** 1.5 / np.maximum(0.41 * _wall_distance(px, py, g), 0.02)
        return R11, R22, R33, R12, eps, k

    R11, R22, R33, R12, eps, k = stress_at(x, y)
    h = 1e-6
    dR11dx = (stress_at(x + h, y)[0] - stress_at(x - h, y)[0]) / (2 * h)
    dR12dx = (stress_at(x + h, y)[3] - stress_at(x - h, y)[3]) / (2 * h)
    dR12dy = (stress_at(x, y + h)[3] - stress_at(x, y - h)[3]) / (2 * h)
    dR22dy = (stress_at(x, y + h)[1] - stress_at(x, y - h)[1]) / (2 * h)
    dPdx = -(U * dUdx + V * dUdy + dR11dx + dR12dy - nu * lapU)
    dPdy = -(U * dVdx + V * dVdy + dR12dx + dR22dy - nu * lapV)

    # elliptic-relaxation tensor: local right-hand side of eq. (14)
    c = TABLE2
    CT = c["CT"]
    omega = 2.0 * eps / (k + np.sqrt(k * k + 4.0 * nu * CT * CT * eps))   # eq. (8) solved for <omega>
    nV = len(x)
    Rm = np.zeros((nV, 3, 3))
    Rm[:, 0, 0], Rm[:, 1, 1], Rm[:, 2, 2] = R11, R22, R33
    Rm[:, 0, 1] = Rm[:, 1, 0] = R12
    gradU = np.zeros((nV, 3, 3))            # gradU[k, l] = d<U_k>/dx_l
    gradU[:, 0, 0], gradU[:, 0, 1], gradU[:, 1, 0], gradU[:, 1, 1] = dUdx, dUdy, dVdx, dVdy
    tr = R11 + R22 + R33
    bt = Rm / tr[:, None, None] - np.eye(3)[None] / 3.0
    Av = np.minimum(1.0, c["Cv"] * (2.0 * k / 3.0) ** -3 * np.linalg.det(Rm))
    g5 = c["gamma5"]
    I3 = np.eye(3)
    H = ((c["C2"] * Av + g5 / 3.0)[:, None, None, None, None] * np.einsum("ik,jl->ijkl", I3, I3)[None]
         - g5 / 3.0 * np.einsum("il,jk->ijkl", I3, I3)[None]
         + g5 * np.einsum("nik,jl->nijkl", bt, I3)
         - g5 * np.einsum("nil,jk->nijkl", bt, I3))
    rapid = k[:, None, None] * np.einsum("nijkl,nkl->nij", H, gradU)
    slow = (0.5 * (1.0 - c["C1"]) * k * omega)[:, None, None] * I3[None]
    # damp the rapid part where the drift tensor would lose stability
    scale = np.ones(nV)
    n_damped = 0
    for it in range(60):
        wp = slow + scale[:, None, None] * rapid
        G = (2.0 * wp - eps[:, None, None] * I3[None]) / (2.0 * k)[:, None, None]
        ev = np.linalg.eigvals(G[:, :2, :2]).real.max(axis=1)
        C0 = -2.0 * np.einsum("nij,nij->n", wp, Rm) / (3.0 * k * eps)
        bad = (ev > -0.2 * omega) | (C0 < 0.1) | (G[:, 2, 2] > -0.2 * omega)
        if not bad.any():
            break
        if it == 0:
            n_damped = int(bad.sum())
        scale = np.where(bad, scale * 0.8, scale)
    else:
        raise ValueError("synthetic wp: could not stabilise the drift tensor")

    f = np.zeros((nV, NFIELD))
    for name, arr in (("U", U), ("V", V), ("dUdx", dUdx), ("dUdy", dUdy), ("dVdx", dVdx), ("dVdy", dVdy),
                      ("lapU", lapU), ("lapV", lapV), ("dPdx", dPdx), ("dPdy", dPdy),
                      ("R11", R11), ("R22", R22), ("R33", R33), ("R12", R12), ("eps", eps),
                      ("P11", wp[:, 0, 0]), ("P12", wp[:, 0, 1]), ("P21", wp[:, 1, 0]),
                      ("P22", wp[:, 1, 1]), ("P33", wp[:, 2, 2])):
        f[:, F[name]] = arr
    if not np.all(np.isfinite(f)):
        raise ValueError("non-finite synthetic field")
    ev = np.linalg.eigvalsh(Rm)
    if ev.min() <= 0:
        raise ValueError("synthetic Reynolds stress not realizable")
    if with_stats:
        return f, dict(n_damped=n_damped, min_stress_eig=float(ev.min()))
    return f
