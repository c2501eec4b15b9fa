"""Parity of the 5 x 5 x 5 velocity bins for <phi|V> (section 3) between the
HIP library and the CPU oracle.

Bar: position, velocity and element bit-exact (the bins only steer the
scalar); the 125 bin counts per element exact; the bin means and the scalar
within 1e-5 (scale-aware, the element's scalar standard deviation), because
the element moments that place the bin edges and the per-bin sums are added
in a different order on the two sides.
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
    print(f"[case] bins5 {wl.name} n={wl.n_total} ens={wl.nens} {wl.precision} {extra}", flush=True)


def _glm():
    wl = W.small_canyon(target=600, ppe=60, precision="f32", vbins=5, steps=20)
    wl.psi_init = W.PSI_LEFT_QUARTER
    return wl


def _wallfn():
    wl = W.small_canyon(target=600, ppe=60, precision="f32", vbins=5, moments=4, hist_bins=32, wallfn=True,
                        steps=20)
    wl.psi_init = W.PSI_LEFT_QUARTER
    return wl


CASES = {"glm": _glm, "wallfn_m4_hist": _wallfn}


def assert_fine_parity(sg, so, off, what=""):
    np.testing.assert_array_equal(sg[:, off:off + 125], so[:, off:off + 125], err_msg=what)
    sig = np.sqrt(np.maximum(so[:, O.ST_M2 + 9], 0.0))[:, None]
    b = so[:, off + 125:off + 250]
    err = np.abs(sg[:, off + 125:off + 250] - b)
    lim = TOL * np.maximum(np.abs(b), np.maximum(sig, 1e-30))
    assert (err <= lim).all(), f"{what}: fine-bin means, worst {np.max(err / lim)}"


def _offset(wl):
    return (O.NSTAT_4 if wl.moments >= 4 else O.NSTAT_2) + wl.hist_bins


@pytest.mark.parametrize("case", list(CASES))
def test_fine_bin_trajectory_and_statistics(gpu, case):
    wl = CASES[case]()
    _label(wl, "trajectory")
    sim = gpu.Simulation.from_workload(wl)
    orc = O.Oracle(wl)
    assert sim.nstat == orc.nstat == _offset(wl) + 250
    done = 0
    for cp in (1, 5, wl.steps):
        sim.step(cp - done)
        orc.step(cp - done)
        done = cp
        sim.sync()
        assert_state_parity(sim.state(), orc.state(), what=f"{case} step {done}")
    sg, so = sim.statistics()[0], orc.stats()
    assert_stats_parity(sg, so, wl.moments, wl.hist_bins, what=case)
    assert_fine_parity(sg, so, _offset(wl), what=case)
    # the fine bins are populated
    assert (np.count_nonzero(so[:, _offset(wl):_offset(wl) + 125], axis=1) > 8).mean() > 0.5


@pytest.mark.parametrize("shape", [(16, 0), (32, 1), (64, 1), (16, 1), (8, 0)])
def test_fine_bin_launch_shapes(gpu, shape):
    wl = _wallfn()
    wl.steps = 6
    _label(wl, f"shape={shape}")
    sim = gpu.Simulation.from_workload(wl)
    sim.set_launch(*shape)
    orc = O.Oracle(wl)
    sim.step(6)
    orc.step(6)
    sim.sync()
    assert_state_parity(sim.state(), orc.state(), what=f"{shape}")
    sg, so = sim.statistics()[0], orc.stats()
    assert_stats_parity(sg, so, wl.moments, wl.hist_bins, what=f"{shape}")
    assert_fine_parity(sg, so, _offset(wl), what=f"{shape}")


def test_fine_bins_with_graphs_repacks_and_averaging(gpu):
    wl = _glm()
    _label(wl, "graph+repack+average")
    sim = gpu.Simulation.from_workload(wl, slack=1.0)
    sim.set_launch(32, 0)
    orc = O.Oracle(wl)
    sim.average_attach()
    orc.average_start()
    for n in (7, 12, 5):
        sim.step_graph(n)
        orc.step(n)
        sim.sync()
        assert_state_parity(sim.state(), orc.state(), what=f"graph step {orc.step_index}")
        if n == 7:
            sim.repack()
    assert sim.repacks() >= 1
    ag, ao = sim.average()[0], orc.average()
    np.testing.assert_array_equal(ag[:, O.AV_N], ao[:, O.AV_N])
    np.testing.assert_allclose(ag[:, O.AV_MEAN + 3], ao[:, O.AV_MEAN + 3], rtol=TOL,
                               atol=TOL * np.sqrt(np.maximum(ao[:, O.AV_M2 + 9], 0)).max() + 1e-300)


def test_fine_bins_refuse_the_network(gpu):
    import ctypes
    import torch
    from paper_1003_4548_amd import mlp as PM
    wl = _glm()
    sim = gpu.Simulation.from_workload(wl)
    w = torch.zeros(PM.NPARAM, dtype=torch.int16, device="cuda:0")
    norm = torch.zeros(4 * 32, dtype=torch.float32, device="cuda:0")
    cm = torch.zeros(wl.mesh.nelem * 8, dtype=torch.float64, device="cuda:0")
    r = gpu.load_library().pdf_mlp_attach(sim.ctx, ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(norm.data_ptr()),
                                          ctypes.c_void_p(cm.data_ptr()), None)
    assert r == -8
