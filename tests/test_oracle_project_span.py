"""The span a mean-pressure projection covers, on the CPU oracle.

The projection adds grad(phi) to the mean pressure gradient and takes
T grad(phi) off the particles' velocities, with T the time since the
previous projection (n steps of dt).  In a linear picture: let e be the
gradient part of the forcing the mean pressure gradient has not yet
balanced.  Over n steps the mean velocity gains the divergent part n dt e;
the projection finds grad(phi) = n dt e / T and the remaining imbalance is
e - grad(phi).  With T = n dt that is zero: the gradient settles after one
call, up to the statistical noise of the particle means.  With T = dt it is
(1 - n) e: projecting every six steps multiplies the imbalance by -5 per
call.  Both runs below step the oracle's particles between projections
(the doubly periodic box and the small canyon with walls); the span-covering
one stays at the noise level with bounded velocities, the one-step one
grows by orders of magnitude.
"""
import numpy as np
import pytest

import oracle as O
import oracle.project as P
import workloads as W


def _cycles(wl, span_steps, every=6, cycles=6):
    orc = O.Oracle(wl)
    orc.step(every)
    u0 = np.abs(orc.state()["u"]).max()
    G = wl.fields[:, 8:10].copy()
    g = []
    for _ in range(cycles):
        T = span_steps * wl.dt
        ref = P.project(wl.mesh, wl.fields, orc.stats(), T)
        corrected = P.correct_state(orc.state(), ref["grad_elem"], T, wl.precision == "f32")
        s = orc.step_index
        orc.set_state(corrected)
        orc.step_index = s
        G = G + ref["grad_vertex"]
        orc.set_pressure_gradient(G)
        g.append(np.abs(ref["grad_vertex"]).max())
        orc.step(every)
    return np.array(g), u0, np.abs(orc.state()["u"]).max()


@pytest.mark.parametrize("case", ["periodic_box", "canyon"])
def test_projection_over_its_span_settles_and_over_one_step_does_not(case):
    wl = (W.square_box(n=8, ppe=30, periodic_y=True, precision="f64", dt=1e-3, steps=6) if case == "periodic_box"
          else W.small_canyon(target=600, ppe=30, steps=6, precision="f64"))
    g6, u0, u6 = _cycles(wl, span_steps=6)
    g1, _, u1 = _cycles(wl, span_steps=1)
    print(f"{case}: span 6 dt {np.round(g6, 3)} max|u| {u0:.3g} -> {u6:.3g}; "
          f"span dt {np.round(g1, 3)} max|u| -> {u1:.3g}")
    assert g6[2:].max() <= 4 * g6[:2].max()
    assert u6 <= 2 * u0
    assert g1[-1] >= 100 * g1[0]
    assert u1 >= 10 * u0
