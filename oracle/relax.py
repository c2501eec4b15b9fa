"""Oracle of the elliptic-relaxation solve (section 2.1, eqs. 12-18).

TEST INFRASTRUCTURE ONLY: a plain CPU implementation, with scipy's sparse
matrices and direct solver, of what the library's relaxation entry point
computes.  Only the tests, the smoke check and the benchmark's CPU leg use it.

The tensor wp_ij solves eq. (14),

    wp_ij - L^2 lap wp_ij = 1/2 (1 - C1) k <omega> delta_ij + k H_ijkl d<U_k>/dx_l,

with H of eq. (15), A_v of eq. (16), the anisotropy b of eq. (17) and the
length scale L of eq. (18); G_ij and C0 then follow from eqs. (12)-(13).
Readings (the design notes list them):
* per element: the Reynolds stress from the particle statistics (second
  central moments of u, v, w; <u'w'> and <v'w'> are zero in the statistically
  two-dimensional flow and not used), the frozen stress where the element
  holds fewer than N_MIN particles; k = tr R / 2; eps and d<U>/dx the frozen
  fields at the centroid (vertex average); <omega> the positive root of
  eq. (8);
* C_xi = 1 + 1.3 n.n with n a unit vector is 2.3;
* Galerkin P1 finite elements on the mesh's vertices, the two vertices of a
  periodic seam being one unknown; L^2 and the right-hand side constant per
  element; natural (homogeneous Neumann) conditions on every wall, the
  paper's wall conditions for wp being in a work that is not available;
* the components solved are wp_11, wp_12, wp_21, wp_22 and wp_33 (the others
  vanish in the two-dimensional flow);
* per vertex, k and R are the area-weighted averages over the elements
  around it, eps the frozen value; C0 below zero is set to zero (a negative
  diffusion coefficient has no meaning) and counted.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# Table 2
C1, C2, CT, CL, CETA, CV, GAMMA5 = 1.85, 0.63, 6.0, 0.134, 72.0, 1.4, 0.1
C_XI = 2.3
N_MIN = 10
COMPONENTS = ((0, 0), (0, 1), (1, 0), (1, 1), (2, 2))   # wp_11 wp_12 wp_21 wp_22 wp_33

# record offsets (oracle/orc.h)
ST_N, ST_M2 = 0, 5
# field columns (workloads/fields.py order)
F_U, F_DUDX, F_R11, F_EPS = 0, 2, 10, 14


def canonical_vertices(mesh):
    """Map each vertex to one unknown: the two copies of a vertex on a
    periodic seam (equal coordinates up to one period) share it."""
    vtx = mesh.vtx
    V = len(vtx)
    parent = np.arange(V)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    shift = {4: (mesh.Lx, 0.0), 5: (-mesh.Lx, 0.0), 6: (0.0, mesh.Ly), 7: (0.0, -mesh.Ly)}
    for e in range(mesh.nelem):
        for k in range(3):
            kind = int(mesh.ekind[e, k])
            if kind not in shift:
                continue
            nb = int(mesh.nbr[e, k])
            sx, sy = shift[kind]
            for v in (mesh.tri[e, k], mesh.tri[e, (k + 1) % 3]):
                p = vtx[v] + (sx, sy)
                for w in mesh.tri[nb]:
                    if vtx[w][0] == p[0] and vtx[w][1] == p[1]:
                        ra, rb = find(v), find(w)
                        if ra != rb:
                            parent[max(ra, rb)] = min(ra, rb)
    roots = np.array([find(v) for v in range(V)])
    uniq, canon = np.unique(roots, return_inverse=True)
    return canon, len(uniq)


def element_geometry(mesh):
    """Area and the P1 shape-function gradients of every element."""
    p = mesh.vtx[mesh.tri]                       # E x 3 x 2
    x, y = p[:, :, 0], p[:, :, 1]
    area2 = (x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0])
    # grad phi_a = (y_{a+1} - y_{a+2}, x_{a+2} - x_{a+1}) / (2A)
    gx = np.stack([y[:, (a + 1) % 3] - y[:, (a + 2) % 3] for a in range(3)], axis=1) / area2[:, None]
    gy = np.stack([x[:, (a + 2) % 3] - x[:, (a + 1) % 3] for a in range(3)], axis=1) / area2[:, None]
    return 0.5 * area2, gx, gy


def assemble(mesh, L2):
    """Mass matrix M and the L^2-weighted stiffness matrix of the P1 Galerkin
    form of eq. (14), over the canonical unknowns."""
    canon, nc = canonical_vertices(mesh)
    area, gx, gy = element_geometry(mesh)
    rows, cols, mvals, kvals = [], [], [], []
    for a in range(3):
        for b in range(3):
            rows.append(canon[mesh.tri[:, a]])
            cols.append(canon[mesh.tri[:, b]])
            mvals.append(area / 12.0 * (2.0 if a == b else 1.0))
            kvals.append(L2 * area * (gx[:, a] * gx[:, b] + gy[:, a] * gy[:, b]))
    r, c = np.concatenate(rows), np.concatenate(cols)
    M = sp.csr_matrix((np.concatenate(mvals), (r, c)), shape=(nc, nc))
    K = sp.csr_matrix((np.concatenate(kvals), (r, c)), shape=(nc, nc))
    return M, K, canon, nc, area


def mean_omega(k, eps, nu):
    """<omega> of eq. (8), eps = <omega>(k + nu C_T^2 <omega>), positive root."""
    return 2.0 * eps / (k + np.sqrt(k * k + 4.0 * nu * CT * CT * eps))


def rhs_tensor(k, R, om, grad):
    """Right-hand side of eq. (14) per element (3 x 3 tensor), with H from
    eqs. (15)-(17).  R: E x 3 x 3, grad: E x 3 x 3 with grad[k, l] = d<U_k>/dx_l."""
    E = len(k)
    I = np.eye(3)
    b = R / np.trace(R, axis1=1, axis2=2)[:, None, None] - I / 3.0
    Av = np.minimum(1.0, CV * (2.0 * k / 3.0) ** -3 * np.linalg.det(R))
    S = np.zeros((E, 3, 3))
    for i in range(3):
        for j in range(3):
            acc = np.zeros(E)
            for kk in range(3):
                for ll in range(3):
                    H = ((C2 * Av + GAMMA5 / 3.0) * I[i, kk] * I[j, ll] - GAMMA5 / 3.0 * I[i, ll] * I[j, kk]
                         + GAMMA5 * b[:, i, kk] * I[j, ll] - GAMMA5 * b[:, i, ll] * I[j, kk])
                    acc = acc + H * grad[:, kk, ll]
            S[:, i, j] = k * acc + (0.5 * (1.0 - C1) * k * om if i == j else 0.0)
    return S


def element_inputs(mesh, fields, stats, nu):
    """k, R, eps, <omega>, L^2 and the right-hand side per element."""
    tri = mesh.tri
    fc = fields[tri].mean(axis=1)                # centroid values of the frozen fields
    E = mesh.nelem
    R = np.zeros((E, 3, 3))
    frozen = np.zeros((E, 3, 3))
    frozen[:, 0, 0], frozen[:, 1, 1], frozen[:, 2, 2] = fc[:, F_R11], fc[:, F_R11 + 1], fc[:, F_R11 + 2]
    frozen[:, 0, 1] = frozen[:, 1, 0] = fc[:, F_R11 + 3]
    m2 = stats[:, ST_M2:ST_M2 + 10]              # pairs a <= b of (u, v, w, psi)
    est = np.zeros((E, 3, 3))
    est[:, 0, 0], est[:, 0, 1], est[:, 1, 1], est[:, 2, 2] = m2[:, 0], m2[:, 1], m2[:, 4], m2[:, 7]
    est[:, 1, 0] = est[:, 0, 1]
    use = stats[:, ST_N] >= N_MIN
    R[use] = est[use]
    R[~use] = frozen[~use]
    k = 0.5 * np.trace(R, axis1=1, axis2=2)
    eps = fc[:, F_EPS]
    om = mean_omega(k, eps, nu)
    grad = np.zeros((E, 3, 3))
    grad[:, 0, 0], grad[:, 0, 1], grad[:, 1, 0], grad[:, 1, 1] = (fc[:, F_DUDX], fc[:, F_DUDX + 1],
                                                                  fc[:, F_DUDX + 2], fc[:, F_DUDX + 3])
    S = rhs_tensor(k, R, om, grad)
    L = CL * np.maximum(C_XI * k ** 1.5 / eps, CETA * (nu ** 3 / eps) ** 0.25)
    return dict(k=k, R=R, eps=eps, omega=om, L2=L * L, S=S)


def solve_with(mesh, L2, S):
    """The Galerkin solution of w - L^2 lap w = s with L2 and s constant per
    element (S: E x m), at the canonical unknowns (nc x m): the load of
    unknown i is the sum over its elements of s_e times a third of the area."""
    M, K, canon, nc, area = assemble(mesh, L2)
    lu = spla.splu((M + K).tocsc())
    S = np.asarray(S, np.float64).reshape(mesh.nelem, -1)
    out = np.zeros((nc, S.shape[1]))
    for c in range(S.shape[1]):
        rhs = np.zeros(nc)
        np.add.at(rhs, canon[mesh.tri].ravel(), np.repeat(S[:, c] * area / 3.0, 3))
        out[:, c] = lu.solve(rhs)
    return out, dict(M=M, K=K, canon=canon, nc=nc, area=area)


def solve(mesh, fields, stats, nu):
    """wp at the canonical unknowns (nc x 5, COMPONENTS order) and the pieces
    that produced it."""
    ins = element_inputs(mesh, fields, stats, nu)
    S = np.stack([ins["S"][:, i, j] for i, j in COMPONENTS], axis=1)
    wp, parts = solve_with(mesh, ins["L2"], S)
    return wp, dict(ins, **parts)


def vertex_coefficients(mesh, fields, wp, parts):
    """G_11 G_12 G_21 G_22 G_33 and C0 eps per mesh vertex (eqs. 12-13), from
    wp at the canonical unknowns; returns (V x 6, number of vertices whose C0
    was negative)."""
    canon, nc, area = parts["canon"], parts["nc"], parts["area"]
    R = parts["R"]
    wsum = np.zeros(nc)
    Rs = np.zeros((nc, 3, 3))
    for a in range(3):
        np.add.at(wsum, canon[mesh.tri[:, a]], area)
        np.add.at(Rs, canon[mesh.tri[:, a]], area[:, None, None] * R)
    Rv = Rs / wsum[:, None, None]
    kv = 0.5 * np.trace(Rv, axis1=1, axis2=2)
    out = np.zeros((mesh.nvert, 6))
    neg = 0
    for v in range(mesh.nvert):
        c = canon[v]
        w = np.zeros((3, 3))
        for q, (i, j) in enumerate(COMPONENTS):
            w[i, j] = wp[c, q]
        eps = fields[v, F_EPS]
        k = kv[c]
        G = (2.0 * w - eps * np.eye(3)) / (2.0 * k)
        C0 = -2.0 * np.sum(w * Rv[c]) / (3.0 * k * eps)
        if C0 < 0.0:
            C0 = 0.0
            neg += 1
        out[v] = [G[0, 0], G[0, 1], G[1, 0], G[1, 1], G[2, 2], C0 * eps]
    return out, neg
