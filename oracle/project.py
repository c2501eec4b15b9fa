"""Oracle of the mean-pressure projection (closing summary of section 2.2;
section 3: the mean-pressure Poisson equation on the Eulerian grid by finite
elements).

TEST INFRASTRUCTURE ONLY: a plain CPU implementation, with scipy's sparse
matrices and direct solver, of what the library's projection entry point
computes.  Only the tests, the smoke check and the benchmark's CPU leg use it.

The paper obtains the mean pressure of eq. (6) by a projection scheme whose
details are in a work that is not available.  The reading taken here (the
design notes list it) is the incremental projection of the particles' mean
velocity onto weakly divergence-free fields:

* per element, the mean velocity (U_e, V_e) of its particles (the frozen
  mean velocity at the centroid where the element holds fewer than N_MIN
  particles);
* the pressure increment phi solves lap(phi) = div<U> / dt with the wall
  condition d(phi)/dn = <U>.n / dt (the corrected velocity has no normal
  component at walls), in Galerkin P1 form on the mesh's vertices (periodic
  seam copies one unknown):

      sum_e int_e grad(phi) . grad(psi_i) = (1/dt) sum_e area_e <U>_e . grad(psi_i)|_e

  for every shape function psi_i; the right-hand side sums to zero (the
  shape functions sum to one), the constants are the null space, and phi is
  taken with zero mean over the unknowns;
* grad(phi) is constant per element; per vertex it is the area-weighted
  average over the elements around it;
* the mean pressure gradient at every vertex gains the vertex gradient
  (<P> becomes <P> + phi), and every particle's velocity loses dt times the
  gradient of its element, computed in double and rounded to the state type.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import relax as R

N_MIN = 10
F_U = 0
ST_N, ST_MEAN = 0, 1


def shape_gradients(mesh):
    """Area and the gradients of the three P1 shape functions of every element."""
    return R.element_geometry(mesh)


def element_velocity(mesh, fields, stats):
    """(E x 2) mean velocity per element: the particles' where the element
    holds N_MIN or more, the frozen field at the centroid otherwise."""
    fc = fields[mesh.tri].mean(axis=1)
    U = fc[:, F_U:F_U + 2].copy()
    use = stats[:, ST_N] >= N_MIN
    U[use] = stats[use, ST_MEAN:ST_MEAN + 2]
    return U


def load(mesh, U, dt, canon, nc):
    """(1/dt) sum_e area_e U_e . grad(psi_i)|_e at the canonical unknowns."""
    area, gx, gy = shape_gradients(mesh)
    b = np.zeros(nc)
    for a in range(3):
        np.add.at(b, canon[mesh.tri[:, a]], area * (U[:, 0] * gx[:, a] + U[:, 1] * gy[:, a]) / dt)
    return b


def solve_poisson(mesh, b):
    """The zero-mean solution of K phi = b (K the P1 stiffness matrix, seams
    joined), by a direct solve of the system bordered with the constraint
    sum(phi) = 0."""
    M, K, canon, nc, area = R.assemble(mesh, np.ones(mesh.nelem))
    one = sp.csr_matrix(np.ones((1, nc)))
    A = sp.bmat([[K, one.T], [one, None]]).tocsc()
    sol = spla.spsolve(A, np.concatenate([b, [0.0]]))
    return sol[:nc], sol[nc], dict(K=K, canon=canon, nc=nc, area=area)


def element_gradient(mesh, phi_v):
    """grad(phi) per element (E x 2) from the values at the mesh vertices."""
    area, gx, gy = shape_gradients(mesh)
    p = phi_v[mesh.tri]
    return np.stack([(p * gx).sum(axis=1), (p * gy).sum(axis=1)], axis=1)


def vertex_gradient(mesh, ge):
    """Area-weighted average of the element gradients around each vertex
    (copies of a seam vertex averaged over all their elements)."""
    canon, nc = R.canonical_vertices(mesh)
    area = shape_gradients(mesh)[0]
    ws = np.zeros(nc)
    gs = np.zeros((nc, 2))
    for a in range(3):
        np.add.at(ws, canon[mesh.tri[:, a]], area)
        np.add.at(gs, canon[mesh.tri[:, a]], area[:, None] * ge)
    return (gs / ws[:, None])[canon]


def project(mesh, fields, stats, dt):
    """phi at the mesh vertices, grad(phi) per element and per vertex, and
    the pieces that produced them."""
    canon, nc = R.canonical_vertices(mesh)
    U = element_velocity(mesh, fields, stats)
    b = load(mesh, U, dt, canon, nc)
    phi, lam, parts = solve_poisson(mesh, b)
    phi_v = phi[canon]
    ge = element_gradient(mesh, phi_v)
    gv = vertex_gradient(mesh, ge)
    return dict(phi=phi_v, grad_elem=ge, grad_vertex=gv, U=U, b=b, lam=lam, **parts)


def correct_state(state, ge, dt, f32):
    """Particle velocities less dt grad(phi) of their element (double, then
    rounded to the state type)."""
    out = dict(state)
    e = state["elem"]
    for q, k in ((0, "u"), (1, "v")):
        v = np.asarray(state[k], np.float64) - dt * ge[e, q]
        out[k] = v.astype(np.float32).astype(np.float64) if f32 else v
    return out
