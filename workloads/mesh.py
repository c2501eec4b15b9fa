"""Triangular meshes for the particle step.

Conventions shared by every consumer (oracle and GPU library read the same
arrays):

* ``vtx``   (V, 2) float64 vertex coordinates.
* ``tri``   (E, 3) int32 vertex ids, counter-clockwise.
* ``nbr``   (E, 3) int32.  Edge k of element e joins ``tri[e,k]`` and
  ``tri[e,(k+1)%3]``.  ``nbr[e,k]`` is the element on the other side of that
  edge: the interior neighbour, or the periodic partner for a periodic edge,
  or -1 on a wall.
* ``ekind`` (E, 3) int32 edge kind, one of :class:`EDGE`.

The paper tracks particles on one unstructured triangular grid that also
carries the statistics (section 2.2, last paragraph; section 3).  Its Gmsh
meshes are not available; these generators build seeded stand-ins of the same
kind: Delaunay triangulations of jittered points, refined toward the no-slip
walls.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.spatial import Delaunay


class EDGE:
    INTERIOR = 0
    NOSLIP = 1        # resolved no-slip wall
    SLIP = 2          # free-slip (specular) wall
    WALLFN = 3        # wall-function wall (stripped domain)
    PERIODIC_XP = 4   # crossing this edge adds +Lx to x
    PERIODIC_XM = 5   # crossing this edge adds -Lx to x
    PERIODIC_YP = 6   # crossing this edge adds +Ly to y
    PERIODIC_YM = 7   # crossing this edge adds -Ly to y


@dataclass
class Mesh:
    name: str
    vtx: np.ndarray
    tri: np.ndarray
    nbr: np.ndarray
    ekind: np.ndarray
    Lx: float
    Ly: float

    @property
    def nelem(self) -> int:
        return int(self.tri.shape[0])

    @property
    def nvert(self) -> int:
        return int(self.vtx.shape[0])

    def areas(self) -> np.ndarray:
        a = self.vtx[self.tri[:, 0]]
        b = self.vtx[self.tri[:, 1]]
        c = self.vtx[self.tri[:, 2]]
        return 0.5 * ((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))

    def centroids(self) -> np.ndarray:
        return self.vtx[self.tri].mean(axis=1)

    def boundary_edges(self, kind: int):
        """(element, local edge) pairs of the given kind."""
        e, k = np.nonzero(self.ekind == kind)
        return e, k

    def locate_brute(self, p) -> int:
        """Index of an element containing point p (closed triangles), or -1.

        Brute force over all elements, exact enough for test points that are
        not within rounding distance of an edge.
        """
        a = self.vtx[self.tri[:, 0]]
        b = self.vtx[self.tri[:, 1]]
        c = self.vtx[self.tri[:, 2]]
        def o(u, v):
            return (v[:, 0] - u[:, 0]) * (p[1] - u[:, 1]) - (v[:, 1] - u[:, 1]) * (p[0] - u[:, 0])
        inside = (o(a, b) >= 0) & (o(b, c) >= 0) & (o(c, a) >= 0)
        idx = np.nonzero(inside)[0]
        return int(idx[0]) if idx.size else -1


# ----------------------------------------------------------------------------
# topology


def _morton(cx: np.ndarray, cy: np.ndarray) -> np.ndarray:
    """Interleaved-bit (Z-order) key of points scaled to a 2^16 grid."""
    def spread(v):
        v = v.astype(np.uint64)
        v = (v | (v << np.uint64(8))) & np.uint64(0x00FF00FF)
        v = (v | (v << np.uint64(4))) & np.uint64(0x0F0F0F0F)
        v = (v | (v << np.uint64(2))) & np.uint64(0x33333333)
        v = (v | (v << np.uint64(1))) & np.uint64(0x55555555)
        return v
    x0, x1 = cx.min(), cx.max()
    y0, y1 = cy.min(), cy.max()
    s = max(x1 - x0, y1 - y0)
    ix = np.clip(((cx - x0) / s * 65535.0).astype(np.int64), 0, 65535)
    iy = np.clip(((cy - y0) / s * 65535.0).astype(np.int64), 0, 65535)
    return spread(ix) | (spread(iy) << np.uint64(1))


def build_mesh(name, vtx, tri, classify, Lx, Ly, reorder=True) -> Mesh:
    """Orient, reorder and connect a triangulation.

    ``classify(ax, ay, bx, by)`` returns the EDGE kind of a boundary edge.
    Elements are renumbered in Z-order of their centroids and vertices in
    order of first use, so that neighbouring elements sit close in memory.
    """
    vtx = np.ascontiguousarray(vtx, dtype=np.float64)
    tri = np.array(tri, dtype=np.int64)
    a, b, c = vtx[tri[:, 0]], vtx[tri[:, 1]], vtx[tri[:, 2]]
    cr = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    if np.any(np.abs(cr) < 1e-14):
        raise ValueError(f"{name}: degenerate triangle")
    flip = cr < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    if reorder:
        cen = vtx[tri].mean(axis=1)
        order = np.argsort(_morton(cen[:, 0], cen[:, 1]), kind="stable")
        tri = tri[order]
        # vertices in order of first use
        first = np.full(len(vtx), -1, dtype=np.int64)
        flat = tri.reshape(-1)
        seen_order = []
        for v in flat:
            if first[v] < 0:
                first[v] = len(seen_order)
                seen_order.append(v)
        if len(seen_order) != len(vtx):
            raise ValueError(f"{name}: unused vertices")
        vtx = vtx[np.array(seen_order)]
        tri = first[tri]
    E = len(tri)
    V = len(vtx)
    # edges
    ea = tri.reshape(-1)
    eb = tri[:, [1, 2, 0]].reshape(-1)
    key = np.minimum(ea, eb) * V + np.maximum(ea, eb)
    order = np.argsort(key, kind="stable")
    ks = key[order]
    nbr = -np.ones(E * 3, dtype=np.int64)
    ekind = np.zeros(E * 3, dtype=np.int64)
    i = 0
    n = len(ks)
    boundary = []
    while i < n:
        if i + 1 < n and ks[i + 1] == ks[i]:
            if i + 2 < n and ks[i + 2] == ks[i]:
                raise ValueError(f"{name}: non-manifold edge")
            p, q = order[i], order[i + 1]
            nbr[p] = q // 3
            nbr[q] = p // 3
            i += 2
        else:
            boundary.append(order[i])
            i += 1
    # classify boundary edges
    pend = {}
    for slot in boundary:
        e, k = divmod(int(slot), 3)
        va, vb = tri[e, k], tri[e, (k + 1) % 3]
        kind = classify(vtx[va, 0], vtx[va, 1], vtx[vb, 0], vtx[vb, 1])
        ekind[slot] = kind
        if kind >= EDGE.PERIODIC_XP:
            if kind in (EDGE.PERIODIC_XP, EDGE.PERIODIC_XM):
                ys = tuple(sorted((vtx[va, 1], vtx[vb, 1])))
                pend.setdefault(("x", ys), []).append(slot)
            else:
                xs = tuple(sorted((vtx[va, 0], vtx[vb, 0])))
                pend.setdefault(("y", xs), []).append(slot)
    for key2, slots in pend.items():
        if len(slots) != 2:
            raise ValueError(f"{name}: unmatched periodic edge {key2}")
        p, q = slots
        kp, kq = ekind[p], ekind[q]
        if {int(kp), int(kq)} not in ({EDGE.PERIODIC_XP, EDGE.PERIODIC_XM}, {EDGE.PERIODIC_YP, EDGE.PERIODIC_YM}):
            raise ValueError(f"{name}: periodic edge paired with wrong kind")
        nbr[p] = q // 3
        nbr[q] = p // 3
    m = Mesh(name=name, vtx=vtx, tri=tri.astype(np.int32),
             nbr=nbr.reshape(E, 3).astype(np.int32),
             ekind=ekind.reshape(E, 3).astype(np.int32), Lx=float(Lx), Ly=float(Ly))
    return m


# ----------------------------------------------------------------------------
# structured unit square


def unit_square_mesh(n: int = 20, periodic_y: bool = False) -> Mesh:
    """n x n squares on [0,1]^2, each cut by the (i,j)-(i+1,j+1) diagonal.

    Periodic in x; the walls y=0 and y=1 are free-slip, or periodic too when
    ``periodic_y`` is set (the doubly periodic box of the constant-drift
    tests).
    """
    xs = np.linspace(0.0, 1.0, n + 1)
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    vtx = np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)
    vid = lambda i, j: j * (n + 1) + i
    tri = []
    for j in range(n):
        for i in range(n):
            tri.append((vid(i, j), vid(i + 1, j), vid(i + 1, j + 1)))
            tri.append((vid(i, j), vid(i + 1, j + 1), vid(i, j + 1)))

    def classify(ax, ay, bx, by):
        if ax == 0.0 and bx == 0.0:
            return EDGE.PERIODIC_XP
        if ax == 1.0 and bx == 1.0:
            return EDGE.PERIODIC_XM
        if ay == 0.0 and by == 0.0:
            return EDGE.PERIODIC_YP if periodic_y else EDGE.SLIP
        if ay == 1.0 and by == 1.0:
            return EDGE.PERIODIC_YM if periodic_y else EDGE.SLIP
        raise ValueError("unexpected boundary edge")

    name = f"square{n}" + ("_pp" if periodic_y else "")
    return build_mesh(name, vtx, np.array(tri), classify, 1.0, 1.0, reorder=False)


def doubly_periodic_box(n: int = 8) -> Mesh:
    return unit_square_mesh(n, periodic_y=True)


# ----------------------------------------------------------------------------
# street canyon


@dataclass
class CanyonGeometry:
    """Building/canyon outline in units of the building height H.

    The full-resolution domain is ([0,Lx] x [y_roof,y_top]) U ([x_l,x_r] x
    [y_street,y_roof]).  The wall-function variant strips a layer of
    thickness yp off every no-slip wall (section 2.2 and the wall-function
    mesh of section 3, which excludes y+ < 30).
    """
    Lx: float = 2.0
    x_l: float = 0.5
    x_r: float = 1.5
    y_street: float = 0.0
    y_roof: float = 1.0
    y_top: float = 2.0
    wallfn: bool = False

    @staticmethod
    def stripped(yp: float) -> "CanyonGeometry":
        return CanyonGeometry(x_l=0.5 + yp, x_r=1.5 - yp, y_street=yp, y_roof=1.0 + yp, wallfn=True)

    def area(self) -> float:
        return self.Lx * (self.y_top - self.y_roof) + (self.x_r - self.x_l) * (self.y_roof - self.y_street)


def _graded(a: float, b: float, h_of) -> np.ndarray:
    """Points from a to b (both included) whose spacing follows h_of(x)."""
    xs = np.linspace(a, b, 40001)
    g = 1.0 / h_of(xs)
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (g[1:] + g[:-1]) * np.diff(xs))])
    n = max(2, int(round(cum[-1])))
    pts = np.interp(np.linspace(0.0, cum[-1], n + 1), cum, xs)
    pts[0], pts[-1] = a, b
    return pts


def _spacing(h_max: float, ratio: float, d_ref: float):
    h_min = h_max * ratio

    def h(d):
        return h_min + (h_max - h_min) * np.minimum(1.0, np.maximum(d, 0.0) / d_ref)
    return h


def _block_points(xg: np.ndarray, yg: np.ndarray, rng: np.random.Generator, jitter: float) -> np.ndarray:
    """Tensor grid with interior points jittered by +-jitter*local spacing."""
    X, Y = np.meshgrid(xg, yg, indexing="ij")
    X = X.copy()
    Y = Y.copy()
    dx = np.minimum(np.diff(xg)[:-1], np.diff(xg)[1:])
    dy = np.minimum(np.diff(yg)[:-1], np.diff(yg)[1:])
    jx = rng.uniform(-jitter, jitter, size=(len(xg) - 2, len(yg) - 2))
    jy = rng.uniform(-jitter, jitter, size=(len(xg) - 2, len(yg) - 2))
    X[1:-1, 1:-1] += jx * dx[:, None]
    Y[1:-1, 1:-1] += jy * dy[None, :]
    return np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)


def _triangulate_block(pts: np.ndarray, area: float):
    d = Delaunay(pts)
    if len(d.coplanar):
        raise ValueError("Delaunay dropped points")
    t = d.simplices
    a, b, c = pts[t[:, 0]], pts[t[:, 1]], pts[t[:, 2]]
    ar = 0.5 * np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))
    if abs(ar.sum() - area) > 1e-9 * area or ar.min() < 1e-12:
        raise ValueError("block triangulation does not tile the block")
    return t


def _canyon_raw(geo: CanyonGeometry, h_max: float, ratio: float, d_ref: float, seed: int):
    h = _spacing(h_max, ratio, d_ref)
    x_can = _graded(geo.x_l, geo.x_r, lambda x: h(np.minimum(x - geo.x_l, geo.x_r - x)))
    x_left = _graded(0.0, geo.x_l, lambda x: h(geo.x_l - x))
    x_right = _graded(geo.x_r, geo.Lx, lambda x: h(x - geo.x_r))
    x_ch = np.concatenate([x_left[:-1], x_can, x_right[1:]])
    y_can = _graded(geo.y_street, geo.y_roof, lambda y: h(np.minimum(y - geo.y_street, geo.y_roof - y)))
    y_ch = _graded(geo.y_roof, geo.y_top, lambda y: h(y - geo.y_roof))
    rng = np.random.default_rng(seed)
    p_can = _block_points(x_can, y_can, rng, 0.25)
    p_ch = _block_points(x_ch, y_ch, rng, 0.25)
    t_can = _triangulate_block(p_can, (geo.x_r - geo.x_l) * (geo.y_roof - geo.y_street))
    t_ch = _triangulate_block(p_ch, geo.Lx * (geo.y_top - geo.y_roof))
    # merge: the canyon's top row coincides with the channel's opening points
    allp = np.concatenate([p_can, p_ch])
    vtx, inv = np.unique(allp, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    tri = np.concatenate([inv[t_can], inv[len(p_can) + t_ch]])
    return vtx, tri


def canyon_mesh(target_elems: int = 10000, wallfn: bool = False, yp: float = 13.0 / 256.0,
                ratio: float = 1.0 / 3.0, d_ref: float = 0.15, seed: int = 0, tol: float = 0.03) -> Mesh:
    """Seeded street-canyon mesh with about ``target_elems`` triangles.

    Square canyon (H = W = 1) under a channel of height 1, periodic in x over
    one building period Lx = 2; spacing grows linearly from ratio*h_max at the
    no-slip walls to h_max at distance d_ref.  With ``wallfn`` the domain is
    stripped by yp on every no-slip wall and those walls carry the
    wall-function condition.
    """
    geo = CanyonGeometry.stripped(yp) if wallfn else CanyonGeometry()
    # bisection on h_max for the element count
    lo, hi = 0.002, 0.2
    best = None
    for _ in range(40):
        hm = np.sqrt(lo * hi)
        vtx, tri = _canyon_raw(geo, hm, ratio, d_ref, seed)
        ne = len(tri)
        if best is None or abs(ne - target_elems) < abs(best[2] - target_elems):
            best = (vtx, tri, ne, hm)
        if abs(ne - target_elems) <= tol * target_elems:
            break
        if ne > target_elems:
            lo = hm
        else:
            hi = hm
    vtx, tri, ne, hm = best
    if abs(ne - target_elems) > tol * target_elems:
        raise ValueError(f"canyon mesh: could not reach {target_elems} elements (got {ne})")
    wall = EDGE.WALLFN if wallfn else EDGE.NOSLIP

    def classify(ax, ay, bx, by):
        if ay == geo.y_top and by == geo.y_top:
            return EDGE.SLIP
        if ax == 0.0 and bx == 0.0:
            return EDGE.PERIODIC_XP
        if ax == geo.Lx and bx == geo.Lx:
            return EDGE.PERIODIC_XM
        on_wall = ((ay == by) and (ay in (geo.y_street, geo.y_roof))) or ((ax == bx) and (ax in (geo.x_l, geo.x_r)))
        if not on_wall:
            raise ValueError(f"unexpected boundary edge ({ax},{ay})-({bx},{by})")
        return wall

    name = ("canyon_wf" if wallfn else "canyon") + f"_{ne}"
    m = build_mesh(name, vtx, tri, classify, geo.Lx, geo.y_top)
    if abs(m.areas().sum() - geo.area()) > 1e-12 * max(1.0, geo.area()) * 10:
        raise ValueError("canyon mesh area mismatch")
    m.geometry = geo  # type: ignore[attr-defined]
    return m
