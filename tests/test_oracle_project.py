"""Pins of the mean-pressure projection oracle (oracle/project.py).

* A gradient field is removed entirely: element velocities U_e = dt grad(chi)
  of a P1 function chi (periodic seams continuous) give phi = chi minus its
  mean, and U - dt grad(phi) = 0, to the direct solver's rounding.  This is
  the discrete Helmholtz decomposition: the Galerkin equations make phi the
  P1 function whose gradient is the projection of U / dt onto P1 gradients.
* The corrected field is weakly divergence free: its load against every
  shape function vanishes (to rounding relative to the uncorrected load),
  for random element velocities on the canyon with walls.
* A uniform flow in the doubly periodic box is divergence free: phi = 0.
* A linear pressure increment on the square periodic in x (phi = c y) has the
  same gradient at every element and every vertex.
* The load sums to zero (the shape functions sum to one) and the bordering
  multiplier vanishes.
* Elements with fewer than ten particles take the frozen velocity at the
  centroid (ten or more: the particles' mean).
* The lumped-mass integral of the vertex gradients equals the integral of
  the element gradients, and seam copies share their value.
"""
import numpy as np

import oracle.project as P
import oracle.relax as R
import workloads as W
from workloads.fields import uniform_fields
from workloads.mesh import doubly_periodic_box, unit_square_mesh


def _stats_with_means(U, n=20):
    st = np.zeros((len(U), 31))
    st[:, 0] = n
    st[:, 1:3] = U
    return st


def _p1_gradient(mesh, chi_v):
    area, gx, gy = R.element_geometry(mesh)
    p = chi_v[mesh.tri]
    return np.stack([(p * gx).sum(axis=1), (p * gy).sum(axis=1)], axis=1)


def test_gradient_field_is_removed():
    dt = 1e-3
    for mesh in (W.tiny_canyon().mesh, doubly_periodic_box(7), unit_square_mesh(6)):
        canon, nc = R.canonical_vertices(mesh)
        chi = np.random.default_rng(3).normal(size=nc)
        chi_v = chi[canon]
        U = dt * _p1_gradient(mesh, chi_v)
        f = uniform_fields(mesh.nvert)
        r = P.project(mesh, f, _stats_with_means(U), dt)
        np.testing.assert_allclose(r["phi"], chi_v - chi.mean(), rtol=0, atol=1e-9 * np.abs(chi).max())
        np.testing.assert_allclose(U - dt * r["grad_elem"], 0.0, atol=1e-9 * np.abs(U).max())


def test_corrected_field_is_weakly_divergence_free():
    dt = 1e-3
    wl = W.tiny_canyon()
    mesh = wl.mesh
    rng = np.random.default_rng(4)
    U = rng.normal(size=(mesh.nelem, 2))
    r = P.project(mesh, wl.fields, _stats_with_means(U), dt)
    canon, nc = R.canonical_vertices(mesh)
    b0 = P.load(mesh, U, dt, canon, nc)
    b1 = P.load(mesh, U - dt * r["grad_elem"], dt, canon, nc)
    assert np.abs(b0).max() > 1.0
    assert np.abs(b1).max() <= 1e-10 * np.abs(b0).max()
    # orthogonal to every P1 gradient
    chi_v = rng.normal(size=nc)[canon]
    area = R.element_geometry(mesh)[0]
    g = _p1_gradient(mesh, chi_v)
    Uc = U - dt * r["grad_elem"]
    assert abs((area[:, None] * Uc * g).sum()) <= 1e-10 * (area[:, None] * np.abs(U) * np.abs(g)).sum()
    # the load sums to zero and the bordering multiplier vanishes
    assert abs(b0.sum()) <= 1e-12 * np.abs(b0).sum()
    assert abs(r["lam"]) <= 1e-12 * np.abs(b0).max()


def test_uniform_flow_in_the_periodic_box_is_left_alone():
    mesh = doubly_periodic_box(8)
    U = np.tile([[0.8, -0.3]], (mesh.nelem, 1))
    r = P.project(mesh, uniform_fields(mesh.nvert), _stats_with_means(U), 1e-3)
    assert np.abs(r["b"]).max() <= 1e-12
    assert np.abs(r["phi"]).max() <= 1e-12 and np.abs(r["grad_vertex"]).max() <= 1e-9


def test_linear_increment_has_one_gradient_everywhere():
    mesh = unit_square_mesh(9)          # periodic in x, walls at y = 0 and 1
    dt, c = 2e-3, 0.7
    U = np.tile([[0.0, dt * c]], (mesh.nelem, 1))
    r = P.project(mesh, uniform_fields(mesh.nvert), _stats_with_means(U), dt)
    np.testing.assert_allclose(r["grad_elem"], np.tile([[0.0, c]], (mesh.nelem, 1)), atol=1e-10)
    np.testing.assert_allclose(r["grad_vertex"], np.tile([[0.0, c]], (mesh.nvert, 1)), atol=1e-10)
    y = mesh.vtx[:, 1]
    canon, nc = R.canonical_vertices(mesh)
    ref = c * y - (np.bincount(canon, c * y, nc) / np.bincount(canon, minlength=nc)).mean()
    np.testing.assert_allclose(r["phi"], ref, atol=1e-10)


def test_sparse_elements_take_the_frozen_velocity():
    wl = W.tiny_canyon()
    mesh = wl.mesh
    st = _stats_with_means(np.full((mesh.nelem, 2), 5.0), n=20)
    st[::3, 0] = 9
    st[1::3, 0] = 10      # ten particles: the particles' mean
    U = P.element_velocity(mesh, wl.fields, st)
    fc = wl.fields[mesh.tri].mean(axis=1)
    np.testing.assert_array_equal(U[::3], fc[::3, 0:2])
    keep = np.ones(mesh.nelem, bool)
    keep[::3] = False
    assert np.all(U[keep] == 5.0)


def test_vertex_gradients_conserve_the_integral():
    # the lumped-mass integral of the vertex gradients equals the integral of
    # the element gradients (each element's area splits equally among its
    # three vertices), on a graded mesh with periodic seams
    mesh = W.tiny_canyon().mesh
    canon, nc = R.canonical_vertices(mesh)
    rng = np.random.default_rng(6)
    ge = rng.normal(size=(mesh.nelem, 2))
    gv = P.vertex_gradient(mesh, ge)
    area = R.element_geometry(mesh)[0]
    mass = np.zeros(nc)
    for a in range(3):
        np.add.at(mass, canon[mesh.tri[:, a]], area / 3.0)
    rep = np.array([np.flatnonzero(canon == i)[0] for i in range(nc)])
    np.testing.assert_allclose((mass[:, None] * gv[rep]).sum(axis=0), (area[:, None] * ge).sum(axis=0),
                               rtol=1e-12)
    # the copies of a seam vertex hold one value
    for i in range(nc):
        v = np.flatnonzero(canon == i)
        assert np.all(gv[v] == gv[v[0]])


def test_state_correction_is_per_element():
    ge = np.array([[1.0, -2.0], [0.5, 0.25]])
    st = {"u": np.array([1.0, 1.0, 2.0]), "v": np.array([0.0, 1.0, 0.0]), "elem": np.array([0, 1, 1]),
          "x": np.zeros(3), "y": np.zeros(3), "w": np.zeros(3), "psi": np.zeros(3)}
    out = P.correct_state(st, ge, 0.1, f32=False)
    np.testing.assert_array_equal(out["u"], [0.9, 0.95, 1.95])
    np.testing.assert_array_equal(out["v"], [0.2, 0.975, -0.025])
