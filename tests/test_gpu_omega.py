"""Parity of the stochastic turbulent frequency (eqs. 8-10 and the
wall-function condition) between the HIP library and the CPU oracle.

Bar, as for the rest of the step: position, velocity and element index stay
bit-exact (omega does not feed back into them); the frozen frequency fields,
the seeded omega and omega after every step are bit-exact (eq. 9 takes the
frozen <omega>, so both sides perform the same operations); the record's
estimates (<omega>, <omega'^2>, eps) within 1e-5, because they are sums over
the element's particles added in a different order on the two sides.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

from test_gpu_parity import TOL, assert_state_parity, assert_stats_parity

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
    print(f"[case] omega {wl.name} n={wl.n_total} ens={wl.nens} {wl.precision} {extra}", flush=True)


CASES = {
    "wallfn_m4_hist_f32": lambda: W.small_canyon(target=600, ppe=30, wallfn=True, moments=4, hist_bins=32,
                                                 steps=30, omega=True),
    "glm_f32": lambda: W.tiny_canyon(precision="f32", steps=30, omega=True),
    "glm_f64": lambda: W.tiny_canyon(precision="f64", steps=15, omega=True),
    "three_ensembles_f32": lambda: W.tiny_canyon(precision="f32", nens=3, steps=15, omega=True),
}


def assert_omega_parity(g, o, what=""):
    a, b = g["omega"], o
    assert a.shape == b.shape, what
    assert (a >= 0).all(), what
    bad = a != b
    if bad.any():
        i = int(np.argmax(bad))
        raise AssertionError(f"{what}: omega differs at {bad.sum()} particles, first id {i}: "
                             f"gpu {a[i]!r} oracle {b[i]!r}")


def assert_omega_record(sg, so, what=""):
    """The last three record entries: <omega>, <omega'^2>, eps."""
    mg, vg, eg = sg[:, -3], sg[:, -2], sg[:, -1]
    mo, vo, eo = so[:, -3], so[:, -2], so[:, -1]
    sd = np.sqrt(np.maximum(vo, 0.0))
    np.testing.assert_array_less(np.abs(mg - mo), TOL * np.maximum(np.abs(mo), sd) + 1e-300, err_msg=what)
    np.testing.assert_array_less(np.abs(vg - vo), TOL * np.maximum(vo, mo * mo * 1e-3) + 1e-300, err_msg=what)
    np.testing.assert_array_less(np.abs(eg - eo), TOL * np.abs(eo) + 1e-300, err_msg=what)


@pytest.mark.parametrize("case", ["wallfn_m4_hist_f32", "glm_f64"])
def test_frozen_frequency_fields_bit_exact(gpu, case):
    wl = CASES[case]()
    _label(wl, "fields")
    sim = gpu.Simulation.from_workload(wl)
    orc = O.Oracle(wl, ensembles=[])
    for a, b, name in zip(sim.omega_fields(), orc.omega_fields(), ("om0", "somega", "omw")):
        np.testing.assert_array_equal(a, b, err_msg=name)


@pytest.mark.parametrize("case", list(CASES))
def test_seeded_frequency_bit_exact(gpu, case):
    wl = CASES[case]()
    _label(wl, "seeding")
    sim = gpu.Simulation.from_workload(wl)
    sim.sync()
    orc = O.Oracle(wl)
    for en in range(wl.nens):
        g = sim.state(en)
        assert_state_parity(g, orc.state(en), psi_exact=True, what=f"{case} seed ens {en}")
        np.testing.assert_array_equal(g["omega"], orc.omega(en))


@pytest.mark.parametrize("case", list(CASES))
def test_frequency_trajectory_parity(gpu, case):
    wl = CASES[case]()
    _label(wl, "trajectory")
    sim = gpu.Simulation.from_workload(wl)
    orc = O.Oracle(wl)
    done = 0
    for cp in sorted({1, 2, wl.steps // 3, wl.steps}):
        sim.step(cp - done)
        orc.step(cp - done)
        done = cp
        sim.sync()
        for en in range(wl.nens):
            g = sim.state(en)
            assert_state_parity(g, orc.state(en), what=f"{case} step {done} ens {en}")
            assert_omega_parity(g, orc.omega(en), what=f"{case} step {done} ens {en}")
    sg = sim.statistics()
    assert sg.shape[2] == orc.nstat
    for en in range(wl.nens):
        so = orc.stats(en)
        assert_stats_parity(sg[en], so, wl.moments, wl.hist_bins, what=f"{case} ens {en}")
        assert_omega_record(sg[en], so, what=f"{case} ens {en}")
    if wl.yp > 0:
        # the run exercised the wall condition on omega
        assert orc.wallfn_hits() > 20


@pytest.mark.parametrize("shape", [(16, 0), (32, 1), (64, 1), (16, 1), (8, 0), (8, 1)])
def test_frequency_launch_shapes(gpu, shape):
    wl = CASES["wallfn_m4_hist_f32"]()
    wl.steps = 8
    _label(wl, f"shape={shape}")
    sim = gpu.Simulation.from_workload(wl)
    sim.set_launch(*shape)
    orc = O.Oracle(wl)
    sim.step(wl.steps)
    orc.step(wl.steps)
    sim.sync()
    g = sim.state()
    assert_state_parity(g, orc.state(), what=f"{shape}")
    assert_omega_parity(g, orc.omega(), what=f"{shape}")
    so = orc.stats()
    sg = sim.statistics()[0]
    assert_stats_parity(sg, so, wl.moments, wl.hist_bins, what=f"{shape}")
    assert_omega_record(sg, so, what=f"{shape}")


def test_frequency_statistics_of_gpu_state(gpu):
    """Estimation alone: the oracle's record of the GPU's own state."""
    wl = CASES["wallfn_m4_hist_f32"]()
    _label(wl, "stats on gpu state")
    sim = gpu.Simulation.from_workload(wl)
    sim.step(9)
    sim.sync()
    g = sim.state()
    orc = O.Oracle(wl)
    orc.set_state(g)
    orc.set_omega(g["omega"])
    so = orc.stats()
    sg = sim.statistics()[0]
    assert_stats_parity(sg, so, wl.moments, wl.hist_bins, what="gpu state")
    assert_omega_record(sg, so, what="gpu state")


@pytest.mark.parametrize("graph", [False, True])
def test_frequency_with_graphs_and_repacks(gpu, graph):
    """Graph replays and segment repacks move omega with the particle."""
    wl = CASES["wallfn_m4_hist_f32"]()
    _label(wl, f"repack graph={graph}")
    sim = gpu.Simulation.from_workload(wl, slack=1.0)
    sim.set_launch(32, 0)
    orc = O.Oracle(wl)
    run = sim.step_graph if graph else sim.step
    for n in (7, 12, 11):
        run(n)
        orc.step(n)
        sim.sync()
        g = sim.state()
        assert_state_parity(g, orc.state(), what=f"graph={graph} step {orc.step_index}")
        assert_omega_parity(g, orc.omega(), what=f"graph={graph} step {orc.step_index}")
        if n == 7:
            sim.repack()
    assert sim.repacks() >= 2


def test_frequency_entry_points_without_frequency(gpu):
    wl = W.tiny_canyon(precision="f32", steps=1)
    sim = gpu.Simulation.from_workload(wl)
    assert sim.nstat == O.NSTAT_2
    with pytest.raises(gpu.PdfError) as ei:
        sim.omega_fields()
    assert ei.value.code == -8
    assert "omega" not in sim.state()
