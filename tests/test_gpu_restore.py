"""Checkpoint restore and the device error paths, forced from the host through
pdf_set_state (every kernel still exits normally).

* A run restored from a checkpoint (state of every ensemble in id order plus
  the Philox step word) continues with the same trajectories as the
  uninterrupted run: position, velocity and element bit-exact; the scalar
  and the turbulent frequency within the parity tolerance (the restored
  segments hold the particles in another order, so element sums round
  differently).
* Rejected restores leave the state unchanged: an element index out of
  range (PDF_E_ARG), more particles in an element than its segment holds
  (PDF_E_CAPACITY).
* A non-finite velocity raises PDF_E_NAN at the next sync; a particle placed
  far outside the domain cannot be tracked and raises PDF_E_LOST (the oracle
  loses it too); a later restore clears the error and the run continues.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

from test_gpu_parity import assert_state_parity
from test_gpu_omega import assert_omega_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_4548_amd as P
    P.load_library()
    return P


def _label(wl, extra=""):
    print(f"[case] restore {wl.name} n={wl.n_total} ens={wl.nens} {wl.precision} {extra}", flush=True)


CASES = {
    "three_ensembles": lambda: W.tiny_canyon(precision="f32", nens=3),
    "wallfn_omega": lambda: W.small_canyon(target=600, ppe=30, wallfn=True, moments=4, hist_bins=32, omega=True),
    "double": lambda: W.tiny_canyon(precision="f64"),
}


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("case", list(CASES))
def test_resume_from_checkpoint(gpu, case, graph):
    wl = CASES[case]()
    _label(wl, f"graph={graph}")
    a = gpu.Simulation.from_workload(wl)
    b = gpu.Simulation.from_workload(wl)
    run_a = a.step_graph if graph else a.step
    run_b = b.step_graph if graph else b.step
    run_a(9)
    a.sync()
    ckpt = [a.state(en) for en in range(wl.nens)]
    run_b(4)                        # a different state, overwritten below
    for en in range(wl.nens):
        b.set_state(ckpt[en], en)
    b.set_step(9)
    run_a(7)
    run_b(7)
    a.sync()
    b.sync()
    orc = O.Oracle(wl)
    orc.step(16)
    for en in range(wl.nens):
        ga, gb = a.state(en), b.state(en)
        assert_state_parity(gb, ga, what=f"{case} resumed vs uninterrupted ens {en}")
        assert_state_parity(gb, orc.state(en), what=f"{case} resumed vs oracle ens {en}")
        if wl.omega:
            assert_omega_parity(gb, orc.omega(en), what=f"{case} omega ens {en}")


def test_rejected_restores_leave_the_state(gpu):
    wl = W.tiny_canyon(precision="f32")
    _label(wl, "rejected")
    sim = gpu.Simulation.from_workload(wl)
    sim.step(3)
    sim.sync()
    before = sim.state()
    bad = dict(before)
    bad["elem"] = before["elem"].copy()
    bad["elem"][17] = wl.mesh.nelem
    with pytest.raises(gpu.PdfError) as ei:
        sim.set_state(bad)
    assert ei.value.code == -1
    full = dict(before)
    full["elem"] = np.zeros_like(before["elem"])       # every particle in element 0
    with pytest.raises(gpu.PdfError) as ei:
        sim.set_state(full)
    assert ei.value.code == -7
    after = sim.state()
    for k in ("x", "y", "u", "v", "w", "psi", "elem"):
        np.testing.assert_array_equal(after[k], before[k])
    sim.step(2)
    sim.sync()


def test_nan_and_lost_particles_raise_and_recover(gpu):
    wl = W.tiny_canyon(precision="f32")
    _label(wl, "fault paths")
    sim = gpu.Simulation.from_workload(wl)
    sim.step(2)
    sim.sync()
    good = sim.state()
    # a non-finite spanwise velocity: the particle stays in its element
    st = {k: v.copy() for k, v in good.items()}
    st["w"][5] = np.nan
    sim.set_state(st)
    sim.step(1)
    with pytest.raises(gpu.PdfError) as ei:
        sim.sync()
    assert ei.value.code == -6
    # a particle far outside the domain: the walk gives up
    st = {k: v.copy() for k, v in good.items()}
    st["x"][0], st["y"][0] = 5.0, 5.0
    orc = O.Oracle(wl)
    orc.set_state(st)
    with pytest.raises(RuntimeError, match="-5"):
        orc.step(1)
    sim.set_state(st)
    sim.step(1)
    with pytest.raises(gpu.PdfError) as ei:
        sim.sync()
    assert ei.value.code == -5
    # restoring the good state clears the error; the run goes on
    sim.set_state(good)
    sim.set_step(2)
    sim.step(3)
    sim.sync()
    ref = O.Oracle(wl)
    ref.step(5)
    assert_state_parity(sim.state(), ref.state(), what="after recovery")


@pytest.mark.parametrize("launch", [(64, 0), (16, 1)])
def test_restore_after_an_error_inside_a_multistep_call(gpu, launch):
    """A non-finite velocity in one ensemble raises the error in the first of
    five steps; the other four return at once, leaving every ensemble's
    counters and the persistent scheduler's work counters stale.  Restoring
    one ensemble keeps the error (the others are void too); restoring all of
    them lets the run go on, trajectories bit-exact against the oracle."""
    wl = W.small_canyon(target=2000, ppe=20, nens=3)
    _label(wl, f"error inside step(5), launch={launch}")
    sim = gpu.Simulation.from_workload(wl)
    sim.set_launch(*launch)
    sim.step(4)
    sim.sync()
    good = [sim.state(en) for en in range(wl.nens)]
    bad = {k: v.copy() for k, v in good[1].items()}
    bad["w"][123] = np.nan
    sim.set_state(bad, 1)
    sim.step(5)
    with pytest.raises(gpu.PdfError) as ei:
        sim.sync()
    assert ei.value.code == -6
    sim.set_state(good[0], 0)
    with pytest.raises(gpu.PdfError):
        sim.sync()                      # ensembles 1 and 2 are still void
    sim.set_state(good[2], 2)
    sim.set_state(good[1], 1)
    sim.sync()
    sim.set_step(4)
    sim.step(7)
    sim.sync()
    m = sim.metrics()
    assert m["error_word"] == 0 and m["particles"] == wl.n_total
    orc = O.Oracle(wl)
    orc.step(11)
    for en in range(wl.nens):
        assert_state_parity(sim.state(en), orc.state(en), what=f"after restore ens {en}")
