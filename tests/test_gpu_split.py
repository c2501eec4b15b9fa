"""Split orders for every model variant with kernels of its own: three
ensembles of uneven size, whose cells of at most eight particles at seeding
step in a launch of their own at 4 lanes per cell (16 cells per wavefront),
with fourth moments and histograms, with the 5 x 5 x 5 velocity bins and with
the turbulent frequency (section 2, section 3).

Bars as in the other parity tests: position, velocity and element bit-exact
for every ensemble; the statistics of the GPU's own state within 1e-5
(scale-aware), counts, histograms and fine-bin counts exact.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

from test_gpu_bins import _offset, assert_fine_parity
from test_gpu_omega import assert_omega_parity, assert_omega_record
from test_gpu_parity import assert_state_parity, assert_stats_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_4548_amd as P
    P.load_library()
    return P


CASES = {
    "wallfn_m4_hist": lambda: W.tiny_canyon(nens=3, wallfn=True, moments=4, hist_bins=32, steps=12),
    "glm_bins5": lambda: W.tiny_canyon(nens=3, vbins=5, steps=12),
    "wallfn_omega": lambda: W.tiny_canyon(nens=3, wallfn=True, omega=True, steps=12),
}


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("case", list(CASES))
def test_split_order_parity(gpu, case, graph):
    wl = CASES[case]()
    counts = np.concatenate([np.asarray(e.counts) for e in wl.ensembles])
    small = int((counts <= 8).sum())
    assert 8 * small >= counts.size and 8 * (counts.size - small) >= counts.size   # the order splits
    print(f"[case] split order {case} {wl.name} n={wl.n_total} graph={graph}", flush=True)
    sim = gpu.Simulation.from_workload(wl)
    run = sim.step_graph if graph else sim.step
    orc = O.Oracle(wl)
    for n in (1, 11):
        run(n)
        orc.step(n)
        sim.sync()
        for en in range(wl.nens):
            what = f"{case} graph={graph} step {orc.step_index} ens {en}"
            assert_state_parity(sim.state(en), orc.state(en), what=what)
            if wl.omega:
                assert_omega_parity(sim.state(en), orc.omega(en), what=what)
    sg = sim.statistics()
    for en in range(wl.nens):
        what = f"{case} graph={graph} statistics ens {en}"
        g = sim.state(en)
        orc.set_state(g, en)
        if wl.omega:
            orc.set_omega(g["omega"], en)
        so = orc.stats(en)
        assert_stats_parity(sg[en], so, wl.moments, wl.hist_bins, what=what)
        if wl.vbins == 5:
            assert_fine_parity(sg[en], so, _offset(wl), what=what)
        if wl.omega:
            assert_omega_record(sg[en], so, what=what)
