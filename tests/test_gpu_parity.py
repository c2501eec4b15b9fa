"""Parity of the HIP library (through its C ABI) with the CPU oracle.

Bar:
* particle position, velocity and element index: bit-exact over the whole run
  (they do not depend on the statistics, and both sides perform the same IEEE
  operations in the same order);
* scalar and statistics: within 1e-5 of the oracle, scale-aware
  (|a - b| <= 1e-5 max(|b|, s), s the element's standard deviation to the
  moment's order), because sums over an element's particles are added in a
  different order on the two sides;
* counts and histograms: exact.
"""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_4548_amd as P
    P.load_library()
    return P


def _label(wl, extra=""):
    print(f"[case] {wl.name} n={wl.n_total} ens={wl.nens} {wl.precision} {extra}", flush=True)


def assert_state_parity(g, o, psi_exact=False, what=""):
    for k in ("x", "y", "u", "v", "w", "elem"):
        if not np.array_equal(g[k], o[k]):
            bad = np.nonzero(g[k] != o[k])[0]
            raise AssertionError(f"{what}: {k} differs at {bad.size} particles, first id {bad[0]}: "
                                 f"gpu {g[k][bad[0]]!r} oracle {o[k][bad[0]]!r}")
    if psi_exact:
        np.testing.assert_array_equal(g["psi"], o["psi"])
    else:
        np.testing.assert_allclose(g["psi"], o["psi"], rtol=TOL, atol=1e-6, err_msg=what)


def assert_stats_parity(sg, so, moments, hist_bins, what=""):
    """Scale-aware comparison of statistics records (nelem x nstat)."""
    np.testing.assert_array_equal(sg[:, O.ST_N], so[:, O.ST_N], err_msg=what)
    m2 = so[:, O.ST_M2:O.ST_M2 + 10]
    diag = m2[:, [0, 4, 7, 9]]                              # uu vv ww psipsi
    sig = np.sqrt(np.maximum(diag, 0.0))
    tiny = 1e-30

    def close(a, b, scale, name):
        err = np.abs(a - b)
        lim = TOL * np.maximum(np.abs(b), np.maximum(scale, tiny))
        bad = err > lim
        if bad.any():
            i = np.argwhere(bad)[0]
            raise AssertionError(f"{what}: {name} differs at {tuple(i)}: gpu {a[tuple(i)]!r} "
                                 f"oracle {b[tuple(i)]!r} (scale {np.broadcast_to(scale, a.shape)[tuple(i)]!r})")

    close(sg[:, O.ST_MEAN:O.ST_MEAN + 4], so[:, O.ST_MEAN:O.ST_MEAN + 4], sig, "means")
    pairs = [(a, b) for a in range(4) for b in range(a, 4)]
    sc2 = np.stack([sig[:, a] * sig[:, b] for a, b in pairs], axis=1)
    close(sg[:, O.ST_M2:O.ST_M2 + 10], m2, sc2, "second moments")
    np.testing.assert_array_equal(sg[:, O.ST_BINN:O.ST_BINN + 8], so[:, O.ST_BINN:O.ST_BINN + 8], err_msg=what)
    close(sg[:, O.ST_BINM:O.ST_BINM + 8], so[:, O.ST_BINM:O.ST_BINM + 8], sig[:, 3:4], "bin means")
    off = O.NSTAT_2
    if moments >= 4:
        trip = [(a, b, c) for a in range(4) for b in range(a, 4) for c in range(b, 4)]
        quad = [(a, b, c, d) for a in range(4) for b in range(a, 4) for c in range(b, 4) for d in range(c, 4)]
        sc3 = np.stack([sig[:, a] * sig[:, b] * sig[:, c] for a, b, c in trip], axis=1)
        sc4 = np.stack([sig[:, a] * sig[:, b] * sig[:, c] * sig[:, d] for a, b, c, d in quad], axis=1)
        close(sg[:, O.ST_M3:O.ST_M3 + 20], so[:, O.ST_M3:O.ST_M3 + 20], sc3, "third moments")
        close(sg[:, O.ST_M4:O.ST_M4 + 35], so[:, O.ST_M4:O.ST_M4 + 35], sc4, "fourth moments")
        off = O.NSTAT_4
    if hist_bins:
        np.testing.assert_array_equal(sg[:, off:off + hist_bins], so[:, off:off + hist_bins], err_msg=what)


CASES = {
    "config1_f64": lambda: W.config1(),
    "tiny_canyon_glm_f32": lambda: W.tiny_canyon(precision="f32", steps=40),
    "tiny_canyon_glm_f64": lambda: W.tiny_canyon(precision="f64", steps=20),
    "small_canyon_wallfn_m4_hist": lambda: W.small_canyon(target=600, ppe=30, wallfn=True, moments=4,
                                                          hist_bins=32, steps=30),
    "tiny_canyon_3_ensembles": lambda: W.tiny_canyon(precision="f32", nens=3, steps=20),
}


@pytest.mark.parametrize("case", list(CASES))
def test_seeding_bit_exact(gpu, case):
    wl = CASES[case]()
    _label(wl, "seeding")
    sim = gpu.Simulation.from_workload(wl)
    sim.sync()
    orc = O.Oracle(wl)
    for en in range(wl.nens):
        assert_state_parity(sim.state(en), orc.state(en), psi_exact=True, what=f"{case} seed ens {en}")


@pytest.mark.parametrize("case", list(CASES))
def test_trajectory_parity(gpu, case):
    wl = CASES[case]()
    _label(wl, "trajectory")
    sim = gpu.Simulation.from_workload(wl)
    orc = O.Oracle(wl)
    done = 0
    checkpoints = sorted({1, 2, max(1, wl.steps // 4), wl.steps})
    for cp in checkpoints:
        sim.step(cp - done)
        orc.step(cp - done)
        done = cp
        sim.sync()
        assert sim.steps_done() == done
        for en in range(wl.nens):
            assert_state_parity(sim.state(en), orc.state(en), what=f"{case} step {done} ens {en}")
    sg = sim.statistics()
    for en in range(wl.nens):
        assert_stats_parity(sg[en], orc.stats(en), wl.moments, wl.hist_bins, what=f"{case} ens {en}")


@pytest.mark.parametrize("case", ["config1_f64", "tiny_canyon_glm_f32", "small_canyon_wallfn_m4_hist"])
def test_statistics_on_gpu_state(gpu, case):
    """Estimation alone: the oracle's statistics of the GPU's own state."""
    wl = CASES[case]()
    _label(wl, "stats on gpu state")
    sim = gpu.Simulation.from_workload(wl)
    sim.step(7)
    sim.sync()
    orc = O.Oracle(wl)
    g = sim.state()
    orc.set_state(g)
    assert_stats_parity(sim.statistics()[0], orc.stats(), wl.moments, wl.hist_bins, what=case)


@pytest.mark.parametrize("case", ["config1_f64", "tiny_canyon_glm_f32"])
def test_one_step_from_gpu_state(gpu, case):
    """The scalar after one step from the GPU's own state (IECM with the GPU's
    statistics order) and the full state, step by step."""
    wl = CASES[case]()
    _label(wl, "per-step")
    sim = gpu.Simulation.from_workload(wl)
    orc = O.Oracle(wl)
    for n in range(5):
        g0 = sim.state()
        orc.set_state(g0)
        orc.step_index = n
        orc.step(1)
        sim.step(1)
        sim.sync()
        assert_state_parity(sim.state(), orc.state(), what=f"{case} step {n}")


@pytest.mark.parametrize("flags", [4, 1, 2, 8 | 2])
def test_substeps(gpu, flags):
    wl = W.tiny_canyon(precision="f32", steps=3)
    wl.flags = flags
    _label(wl, f"flags={flags}")
    sim = gpu.Simulation.from_workload(wl)
    orc = O.Oracle(wl)
    sim.step(3)
    orc.step(3)
    sim.sync()
    assert_state_parity(sim.state(), orc.state(), what=f"flags {flags}")


def test_counts_and_invariants_config1(gpu):
    wl = W.config1()
    _label(wl, "invariants")
    sim = gpu.Simulation.from_workload(wl)
    psi0 = sim.state()["psi"].sum()
    sim.step(100)
    sim.sync()
    st = sim.statistics()[0]
    assert st[:, O.ST_N].sum() == 40000
    s = sim.state()
    assert s["psi"].min() >= 0 and s["psi"].max() <= 1
    assert abs(s["psi"].sum() - psi0) < 40000 * 1e-13


def test_config2_full_size_parity(gpu):
    """The 1M-particle canyon in the launch configuration the benchmark times."""
    wl = W.config2(steps=3)
    _label(wl, "full size")
    sim = gpu.Simulation.from_workload(wl)
    orc = O.Oracle(wl)
    shape = sim.autotune(steps_per_trial=1)     # the benchmark tunes the same way
    print(f"[case] tuned shape {shape}", flush=True)
    sim.step(3)
    orc.step(sim.steps_done())
    sim.sync()
    assert_state_parity(sim.state(), orc.state(), what="config2")
    g = sim.state()
    orc.set_state(g)
    assert_stats_parity(sim.statistics()[0], orc.stats(), wl.moments, wl.hist_bins, what="config2 stats")


SHAPES = [(64, 0), (64, 1), (32, 0), (32, 1), (16, 0), (16, 1), (8, 0), (8, 1)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("case", ["tiny_canyon_glm_f32", "small_canyon_wallfn_m4_hist", "tiny_canyon_3_ensembles"])
def test_launch_shapes_give_the_same_trajectories(gpu, case, shape):
    """Lanes per cell and the persistent scheduler change how work is laid out,
    never the particle trajectories; statistics stay within the tolerance."""
    wl = CASES[case]()
    wl.steps = 6
    _label(wl, f"shape={shape}")
    sim = gpu.Simulation.from_workload(wl)
    sim.set_launch(*shape)
    orc = O.Oracle(wl)
    sim.step(wl.steps)
    orc.step(wl.steps)
    sim.sync()
    sg = sim.statistics()
    for en in range(wl.nens):
        assert_state_parity(sim.state(en), orc.state(en), what=f"{case} {shape} ens {en}")
        assert_stats_parity(sg[en], orc.stats(en), wl.moments, wl.hist_bins, what=f"{case} {shape} ens {en}")


def test_autotune_keeps_parity(gpu):
    wl = W.tiny_canyon(precision="f32", steps=4)
    _label(wl, "autotune")
    sim = gpu.Simulation.from_workload(wl)
    shape = sim.autotune(steps_per_trial=2)
    assert shape[0] in (8, 16, 32, 64) and shape[1] in (0, 1)
    done = sim.steps_done()
    assert done == 2 * 8 * 3      # two rounds of eight candidates, 1 + 2 steps each
    orc = O.Oracle(wl)
    orc.step(done)
    sim.sync()
    assert_state_parity(sim.state(), orc.state(), what="after autotune")


@pytest.mark.parametrize("shape", [(64, 0), (32, 1), (8, 0)])
def test_graph_replay_matches_eager(gpu, shape):
    """Six-step graph replays, with eager work and synchronisation between
    them, against a run launched step by step."""
    wl = W.tiny_canyon(precision="f32", steps=0)
    _label(wl, f"graph {shape}")
    eager = gpu.Simulation.from_workload(wl)
    graph = gpu.Simulation.from_workload(wl)
    eager.set_launch(*shape)
    graph.set_launch(*shape)
    orc = O.Oracle(wl)
    for rep, n in enumerate([6, 6, 7, 12, 5]):
        graph.step_graph(n)
        eager.step(n)
        orc.step(n)
        graph.sync()
        eager.sync()
        assert graph.steps_done() == eager.steps_done() == orc.step_index
        g, e = graph.state(), eager.state()
        assert_state_parity(g, orc.state(), what=f"graph replay {rep}")
        assert_state_parity(e, orc.state(), what=f"eager {rep}")
        np.testing.assert_allclose(g["psi"], e["psi"], rtol=1e-6, atol=1e-7)
        _ = graph.statistics()          # eager work between replays


def test_split_launch_graph_and_eager(gpu):
    """Batched ensembles whose cells of at most eight particles and the others
    each make up an eighth of the cells or more: their steps take two launches
    that run side by side (a parallel graph branch; a second stream when
    stepping eagerly).  Graph replays and eager steps, each against the
    oracle, bit for bit in every ensemble."""
    wl = W.config4(steps=0, nens=8, target=2000)
    counts = np.concatenate([e.counts for e in wl.ensembles])
    small = int((counts <= 8).sum())
    assert 8 * small >= len(counts) and 8 * (len(counts) - small) >= len(counts)
    _label(wl, "split launch")
    eager = gpu.Simulation.from_workload(wl)
    graph = gpu.Simulation.from_workload(wl)
    for s in (eager, graph):
        s.set_launch(16, 0)
    orc = O.Oracle(wl)
    for rep, n in enumerate([6, 7, 5]):
        graph.step_graph(n)
        eager.step(n)
        orc.step(n)
        graph.sync()
        eager.sync()
        for en in range(wl.nens):
            o = orc.state(en)
            assert_state_parity(graph.state(en), o, what=f"graph {rep} ens {en}")
            assert_state_parity(eager.state(en), o, what=f"eager {rep} ens {en}")
    eager.close()
    graph.close()


@pytest.mark.parametrize("graph", [False, True])
def test_repack_keeps_parity(gpu, graph):
    """Segments sized with no slack run short of room within a few steps, so
    the device-side repack runs repeatedly (plus one requested from the host
    at an odd step count); trajectories stay bit-exact and the statistics
    within tolerance."""
    wl = W.small_canyon(target=600, ppe=30, wallfn=True, moments=4, hist_bins=32, steps=0)
    _label(wl, f"repack graph={graph}")
    sim = gpu.Simulation.from_workload(wl, slack=1.0)
    orc = O.Oracle(wl)
    run = sim.step_graph if graph else sim.step
    for n in (7, 12, 17):
        run(n)
        orc.step(n)
        sim.sync()
        assert_state_parity(sim.state(), orc.state(), what=f"repack graph={graph} step {orc.step_index}")
        if n == 7:
            sim.repack()
    assert sim.repacks() >= 2
    sim.sync()
    assert_stats_parity(sim.statistics()[0], orc.stats(), wl.moments, wl.hist_bins, what="after repacks")


def test_repack_is_idle_with_room(gpu):
    """With the default slack a short run needs no repack."""
    wl = W.tiny_canyon(precision="f32", steps=12)
    _label(wl, "no repack")
    sim = gpu.Simulation.from_workload(wl)
    sim.step(12)
    sim.sync()
    assert sim.repacks() == 0


def test_config3_full_size_parity(gpu):
    """The 10M-particle wall-function canyon (moments to 4th order, histograms)
    at the benchmark's tuned launch shape: whole trajectories bit-exact, the
    statistics of the GPU state against the oracle's."""
    wl = W.config3(steps=2)
    _label(wl, "full size")
    sim = gpu.Simulation.from_workload(wl)
    shape = sim.autotune(steps_per_trial=1)
    print(f"[case] tuned shape {shape}", flush=True)
    sim.step(2)
    sim.sync()
    orc = O.Oracle(wl)
    orc.step(sim.steps_done())
    g = sim.state()
    assert_state_parity(g, orc.state(), what="config3")
    orc.set_state(g)
    assert_stats_parity(sim.statistics()[0], orc.stats(), wl.moments, wl.hist_bins, what="config3 stats")


def test_config4_full_size_parity(gpu):
    """64 batched ensembles of uneven size (12M particles) at the tuned shape:
    every ensemble bit-exact, each one as if run alone."""
    wl = W.config4(steps=2)
    _label(wl, "full size")
    sim = gpu.Simulation.from_workload(wl)
    shape = sim.autotune(steps_per_trial=1)
    print(f"[case] tuned shape {shape}", flush=True)
    sim.step(2)
    sim.sync()
    orc = O.Oracle(wl)
    orc.step(sim.steps_done())
    sg = sim.statistics()
    for en in range(wl.nens):
        assert_state_parity(sim.state(en), orc.state(en), what=f"config4 ens {en}")
    for en in (0, 17, 63):
        orc_one = O.Oracle(wl, ensembles=[wl.ensembles[en]])
        orc_one.set_state(sim.state(en))
        assert_stats_parity(sg[en], orc_one.stats(), wl.moments, wl.hist_bins, what=f"config4 stats ens {en}")


def test_empty_ensemble_and_empty_cells(gpu):
    """An ensemble with no particles at all next to a normal one."""
    wl = W.tiny_canyon(precision="f32", nens=2, steps=5)
    wl.ensembles[1].counts = np.zeros_like(wl.ensembles[1].counts)
    _label(wl, "empty ensemble")
    sim = gpu.Simulation.from_workload(wl)
    orc = O.Oracle(wl)
    sim.step(5)
    orc.step(5)
    sim.sync()
    assert sim.count(1) == 0
    assert_state_parity(sim.state(0), orc.state(0), what="non-empty ensemble")
    sg = sim.statistics()
    assert not sg[1].any()
    assert_stats_parity(sg[0], orc.stats(0), wl.moments, wl.hist_bins, what="non-empty ensemble")


def test_host_rejects_bad_input(gpu):
    """Argument and mesh errors come back as status codes, before any kernel
    touches the data."""
    wl = W.tiny_canyon(precision="f32", steps=1)
    # clockwise element
    tri = wl.mesh.tri.copy()
    tri[0] = tri[0][::-1]
    with pytest.raises(gpu.PdfError) as ex:
        gpu.Simulation.from_workload(wl, tri=tri)
    assert ex.value.code == -2
    # a vertex id out of range
    tri = wl.mesh.tri.copy()
    tri[3, 1] = wl.mesh.nvert + 5
    with pytest.raises(gpu.PdfError) as ex:
        gpu.Simulation.from_workload(wl, tri=tri)
    assert ex.value.code == -2
    # unsupported statistics shape
    with pytest.raises(gpu.PdfError) as ex:
        gpu.Simulation.from_workload(wl, moments=3)
    assert ex.value.code == -1
    sim = gpu.Simulation.from_workload(wl)
    with pytest.raises(gpu.PdfError) as ex:
        sim.set_launch(48, 0)
    assert ex.value.code == -1


@pytest.mark.parametrize("cfg", ["config3", "config2"])
def test_long_run_keeps_every_particle(gpu, cfg):
    """1200 graph steps at full size and the tuned shape: the segments keep
    room for every step's arrivals (repacks as needed), no particle is lost
    and the state stays finite."""
    wl = getattr(W, cfg)(steps=1200)
    _label(wl, "long run")
    sim = gpu.Simulation.from_workload(wl)
    shape = sim.autotune(steps_per_trial=1)
    print(f"[case] tuned shape {shape}", flush=True)
    for _ in range(4):
        sim.step_graph(300)
        sim.sync()
        m = sim.metrics()
        print(f"[case] {m}", flush=True)
        assert m["particles"] == wl.n_total and m["error_word"] == 0
    assert sim.repacks() >= 1 or cfg == "config2"
