"""Parity at the sizes and launch shapes the benchmark times, over longer runs.

* The 10M-particle wall-function canyon (moments to fourth order, 32-bin
  histograms) over 102 steps at the tuned shape, with a repack requested from
  the host at step 50 besides the automatic ones: trajectories bit-exact
  against the float oracle, the statistics of the GPU state within the
  scale-aware 1e-5 bar, counts and histograms exact.
* The learned conditional means inside the step at the size the benchmark
  times them (20 particles per element on the 50k-element resolved-wall
  canyon, 1M particles, one-item-per-wavefront shape from the autotuner):
  every step bit-exact against the oracle fed the same means.
* Two identical runs: trajectories and the scalar bit for bit (the scalar
  takes its bin means rounded to float), the statistics records within
  1e-12 (sums over a cell follow the order in which particles arrived from
  other wavefronts, which is not fixed).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import mlp as M

from test_gpu_parity import assert_state_parity, assert_stats_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_4548_amd as P
    from paper_1003_4548_amd import mlp as PM
    P.load_library()
    return P, PM, torch


def _label(wl, extra=""):
    print(f"[case] {wl.name} n={wl.n_total} ens={wl.nens} {wl.precision} {extra}", flush=True)


def test_config3_hundred_steps_with_repacks(gpu):
    P, _, _ = gpu
    wl = W.config3(steps=102)
    _label(wl, "102 steps, repacks")
    sim = P.Simulation.from_workload(wl)
    shape = sim.autotune(steps_per_trial=1)
    print(f"[case] tuned shape {shape}, {sim.steps_done()} tuning steps", flush=True)
    tuned = sim.steps_done()
    assert tuned < 50
    sim.step_graph(50 - tuned)
    sim.repack()
    sim.step_graph(52)
    sim.sync()
    assert sim.repacks() >= 1
    done = sim.steps_done()
    assert done >= 102
    orc = O.Oracle(wl)
    orc.step(done)
    g = sim.state()
    assert_state_parity(g, orc.state(), what=f"config3 after {done} steps")
    orc.set_state(g)
    assert_stats_parity(sim.statistics()[0], orc.stats(), wl.moments, wl.hist_bins, what="config3 stats")


def test_config5_in_step_inference_at_benchmark_size(gpu):
    P, PM, torch = gpu
    wl = W.config5(ppe=20, seed=101, target=50000)
    wl.psi_init = W.PSI_LEFT_QUARTER      # scalar spread in many elements from the start
    _label(wl, "learned means in the step")
    sim = P.Simulation.from_workload(wl)
    shape = sim.autotune(steps_per_trial=1)
    if shape[1]:
        sim.set_launch(shape[0], 0)       # the learned means run inside one-item-per-wavefront steps
    print(f"[case] launch shape: {shape[0]} lanes per cell, one item per wavefront", flush=True)
    sim.step(6)
    sim.sync()
    stats = sim.statistics()[0]
    feat = M.features_from_stats(stats)
    norm = M.feature_norm(feat[stats[:, O.ST_N] > 0])
    net = PM.ConditionalMeanNet()
    p = M.init_params(9)
    wo, bo, o, i = M.LAYOUT[3]
    p[wo:wo + o * i] *= 0.05
    net.set_master(np.asarray(p, np.float32))
    net.norm.copy_(torch.as_tensor(np.asarray(norm, np.float32)).reshape(4, 32).to(net.device))
    lm = net.attach(sim)
    s0 = sim.state()
    orc = O.Oracle(wl)
    for k in range(3):
        sim.step(1)
        sim.sync()
        cm = lm.cm.cpu().numpy()
        orc.set_state(s0)
        orc.step_index = sim.steps_done() - 1
        orc.set_cond_means(cm)
        orc.step(1)
        s1, o1 = sim.state(), orc.state()
        for q in ("x", "y", "u", "v", "w", "psi", "elem"):
            np.testing.assert_array_equal(s1[q], o1[q], err_msg=f"step {k} {q}")
        s0 = s1
    served = int(lm.served.cpu()[0])
    print(f"[case] cells served by the network over 3 steps: {served}", flush=True)
    assert served > 1000
    lm.detach()


@pytest.mark.parametrize("graph", [False, True])
def test_two_identical_runs(gpu, graph):
    P, _, _ = gpu
    wl = W.small_canyon(target=2000, ppe=40, steps=30, wallfn=True, moments=4, hist_bins=32)
    _label(wl, f"repeat graph={graph}")
    runs = []
    for _ in range(2):
        sim = P.Simulation.from_workload(wl)
        (sim.step_graph if graph else sim.step)(wl.steps)
        sim.sync()
        runs.append((sim.state(), sim.statistics()[0]))
        sim.close()
    (a, ra), (b, rb) = runs
    for q in ("x", "y", "u", "v", "w", "psi", "elem"):
        np.testing.assert_array_equal(a[q], b[q], err_msg=q)
    np.testing.assert_array_equal(ra[:, O.ST_N], rb[:, O.ST_N])
    np.testing.assert_array_equal(ra[:, O.NSTAT_4:O.NSTAT_4 + 32], rb[:, O.NSTAT_4:O.NSTAT_4 + 32])
    np.testing.assert_allclose(ra, rb, rtol=1e-12, atol=1e-15)
