"""Learned conditional means: the HIP kernels (through the C ABI) against the
oracle network, and the gain of the trained network over the binned estimate.

Bars: forward outputs and gradients within the rounding of bfloat16
activations (the oracle rounds at the same points; float32 against float64
accumulation can move a value across a rounding boundary, 2^-8 relative);
exact where every operation is exact (selection weights); dataset rows with
the same subsample decisions and float32-rounded statistics; IECM with the
network's conditional means bit-exact against the oracle fed the same means.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import mlp as M

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


def _label(what):
    print(f"[case] {what}", flush=True)


def _net(PM, torch, params, norm):
    net = PM.ConditionalMeanNet()
    net.set_master(np.asarray(params, np.float32))
    net.norm.copy_(torch.as_tensor(np.asarray(norm, np.float32)).reshape(4, 32).to(net.device))
    return net


def _unit_norm():
    return np.stack([np.zeros(32), np.ones(32), np.full(32, -3e38), np.full(32, 3e38)]).astype(np.float32)


def _bf16_exact(rng, shape, scale=4.0):
    return M.bf16(rng.uniform(-scale, scale, size=shape)).astype(np.float32)


def test_forward_with_selection_weights_is_exact(gpu):
    """Selection weights make every product and sum exact, so any slip in the
    operand or output lane layout of the matrix-core tiles shows as a wrong
    element."""
    P, PM, torch = gpu
    _label("mlp selection forward")
    p = np.zeros(M.NPARAM)
    (l1, l2, l3, l4) = M.LAYOUT
    pi1 = [(7 * u + 3) % 32 for u in range(32)]
    W1 = np.zeros((64, 32)); W1[np.arange(32), pi1] = 1.0
    W4 = np.zeros((8, 64)); perm = [5, 0, 31, 7, 12, 3, 20, 9]; W4[np.arange(8), perm] = 1.0
    p[l1[0]:l1[0] + 2048] = W1.ravel()
    p[l2[0]:l2[0] + 4096] = np.eye(64).ravel()
    p[l3[0]:l3[0] + 4096] = np.eye(64).ravel()
    p[l4[0]:l4[0] + 512] = W4.ravel()
    p[l4[1]:l4[1] + 8] = np.arange(8) * 0.25
    rng = np.random.default_rng(0)
    rows = np.zeros((37, 64), np.float32)          # 37: a ragged last tile
    rows[:, :32] = _bf16_exact(rng, (37, 32))
    net = _net(PM, torch, p, _unit_norm())
    y = net.forward(torch.as_tensor(rows).cuda()).cpu().numpy()
    x = rows[:, :32].astype(np.float64)
    expect = np.maximum(x[:, pi1][:, perm], 0.0) + np.arange(8) * 0.25
    np.testing.assert_array_equal(y, expect)


def test_forward_matches_oracle(gpu):
    P, PM, torch = gpu
    _label("mlp forward")
    rng = np.random.default_rng(1)
    params = M.init_params(3)
    rows = np.zeros((1000, 64), np.float32)
    rows[:, :32] = rng.normal(size=(1000, 32))
    norm = M.feature_norm(rows[:, :32])
    net = _net(PM, torch, params, norm)
    y = net.forward(torch.as_tensor(rows).cuda()).cpu().numpy().astype(np.float64)
    yo, _ = M.forward(params, M.normalise(rows[:, :32], norm), emulate=True)
    scale = np.abs(yo).max()
    err = np.abs(y - yo)
    assert err.max() <= 3e-2 * scale, err.max() / scale
    assert np.sqrt((err ** 2).mean()) <= 2e-3 * scale


def _rows(rng, B, frac_untrained=0.1):
    rows = np.zeros((B, 64), np.float32)
    rows[:, :32] = rng.normal(size=(B, 32))
    rows[:, 32:40] = rng.normal(size=(B, 8))
    lw = rng.random(size=(B, 8))
    lw /= lw.sum(axis=1, keepdims=True)
    lw[rng.random(B) < frac_untrained] = 0.0
    rows[:, 40:48] = lw
    return rows


def test_gradient_matches_oracle(gpu):
    P, PM, torch = gpu
    _label("mlp gradient")
    rng = np.random.default_rng(2)
    B = 203
    rows = _rows(rng, B)
    params = M.init_params(4)
    norm = M.feature_norm(rows[:, :32])
    net = _net(PM, torch, params, norm)
    loss, g = net.grad(torch.as_tensor(rows).cuda())
    loss = float(loss.cpu()[0])
    g = g.cpu().numpy().astype(np.float64)
    lo, go = M.loss_and_grad(params.astype(np.float64), M.normalise(rows[:, :32], norm),
                             rows[:, 32:40], rows[:, 40:48], emulate=True)
    assert abs(loss - lo) <= 1e-3 * abs(lo)
    cos = float(g @ go / (np.linalg.norm(g) * np.linalg.norm(go)))
    assert cos > 0.9999, cos
    for (wo, bo, o, i) in M.LAYOUT:
        for sl in (slice(wo, wo + o * i), slice(bo, bo + o)):
            ref = go[sl]
            np.testing.assert_allclose(g[sl], ref, rtol=0, atol=2e-2 * np.abs(ref).max() + 1e-9)


def test_training_steps_match_oracle(gpu):
    """Three Adam steps on Philox-drawn batches, replayed by the oracle."""
    P, PM, torch = gpu
    _label("mlp train")
    rng = np.random.default_rng(3)
    nrows, B, lr, seed = 500, 64, 1e-3, 0x1234_5678_9ABC
    rows = _rows(rng, nrows)
    params = M.init_params(5)
    norm = M.feature_norm(rows[:, :32])
    net = _net(PM, torch, params, norm)
    losses = net.train(torch.as_tensor(rows).cuda(), iters=3, batch=B, lr=lr, seed=seed).cpu().numpy()
    th = params.astype(np.float64)
    m = np.zeros(M.NPARAM)
    v = np.zeros(M.NPARAM)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    xh = M.normalise(rows[:, :32], norm)
    for t in range(1, 4):
        idx = [int(O.philox4x32_10([j, t, 0x7A11, 0], key)[0]) % nrows for j in range(B)]
        lo, g = M.loss_and_grad(th, xh[idx], rows[idx, 32:40], rows[idx, 40:48], emulate=True)
        assert abs(losses[t - 1] - lo) <= 2e-3 * lo, (t, losses[t - 1], lo)
        th, m, v = M.adam(th.astype(np.float32).astype(np.float64), m, v, g, t, lr)
    got = net.master.cpu().numpy().astype(np.float64)
    d = np.abs(got - th)
    # Adam moves every parameter by about lr per step; a gradient component
    # near zero can change sign between the two sides
    assert np.mean(d > 0.05 * lr) < 0.01, np.mean(d > 0.05 * lr)
    assert d.max() <= 6.5 * lr


def _scalar_canyon(ppe, target=600, steps=8, seed=11):
    wl = W.small_canyon(target=target, ppe=ppe, steps=steps, seed=seed)
    wl.psi_init = W.PSI_LEFT_QUARTER
    return wl


def test_dataset_rows_match_oracle(gpu):
    P, PM, torch = gpu
    wl = _scalar_canyon(ppe=120)
    _label(f"mlp dataset {wl.name} n={wl.n_total}")
    sim = P.Simulation.from_workload(wl)
    sim.step(wl.steps)
    sim.sync()
    rows = PM.dataset(sim, target=20, key=777, draw=5).cpu().numpy()
    ro = M.dataset_rows(sim.state(), wl.mesh.nelem, 20, 777, 5)
    np.testing.assert_array_equal(rows[:, 0], ro[:, 0])                       # same subsamples
    np.testing.assert_array_equal(rows[:, 56:64], ro[:, 56:64])               # reference counts
    np.testing.assert_array_equal(rows[:, 15:23], ro[:, 15:23])               # bin fractions
    np.testing.assert_allclose(rows[:, :32], ro[:, :32], rtol=2e-6, atol=1e-9)
    np.testing.assert_allclose(rows[:, 40:48], ro[:, 40:48], rtol=1e-6, atol=0)
    np.testing.assert_allclose(rows[:, 48:56], ro[:, 48:56], rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(rows[:, 32:40], ro[:, 32:40], rtol=1e-4, atol=1e-4)
    trained = rows[:, 40:48].sum(axis=1) > 0
    assert trained.sum() > 20
    # normalisation kernel against the oracle's on the training rows
    net = PM.ConditionalMeanNet()
    net.fit_norm(torch.as_tensor(rows).cuda())
    no = M.feature_norm(rows[trained, :32])
    ng = net.norm.cpu().numpy()
    np.testing.assert_allclose(ng[0], no[0], rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(ng[1], no[1], rtol=1e-4)
    np.testing.assert_array_equal(ng[2:], no[2:])


def _small_output(params, s=0.05):
    p = params.copy()
    wo, bo, o, i = M.LAYOUT[3]
    p[wo:wo + o * i] *= s
    return p


def test_inference_matches_oracle(gpu):
    P, PM, torch = gpu
    wl = _scalar_canyon(ppe=20)
    _label(f"mlp infer {wl.name}")
    sim = P.Simulation.from_workload(wl)
    sim.step(wl.steps)
    sim.sync()
    stats = sim.statistics()[0]
    feat = M.features_from_stats(stats)
    live = stats[:, O.ST_N] > 0
    norm = M.feature_norm(feat[live])
    params = _small_output(M.init_params(6))
    net = _net(PM, torch, params, norm)
    cm, served = net.infer(torch.as_tensor(stats).cuda())
    cm = cm.cpu().numpy()
    cmo, oko, mo = M.infer(stats, params, norm)
    sig = np.sqrt(np.maximum(stats[:, O.ST_M2 + 9], 0.0))
    took = np.any(cm != stats[:, O.ST_BINM:O.ST_BINM + 8], axis=1)
    both = took & oko
    assert both.sum() > 20
    err = np.abs(cm[both] - cmo[both])
    assert np.all(err <= 2e-2 * sig[both, None] + 1e-12), err.max()
    # a decision may differ only where an estimate is within the tolerance of the [0, 1] bounds
    edge = (mo.min(axis=1) < 2e-2 * sig) | (mo.max(axis=1) > 1.0 - 2e-2 * sig)
    differ = took != oko
    assert np.all(edge[differ])
    assert abs(int(served.cpu()[0]) - int(oko.sum())) <= int(edge.sum())


@pytest.mark.parametrize("shape", [(64, 0), (16, 0), (32, 1), (8, 0)])
def test_step_with_learned_means_matches_oracle(gpu, shape):
    """IECM toward the network's conditional means: the oracle, given the same
    means, reproduces the step bit for bit (inside the step kernel for the
    one-item-per-wavefront shapes, a separate pass for the persistent one)."""
    P, PM, torch = gpu
    wl = _scalar_canyon(ppe=20, steps=4)
    _label(f"mlp step {wl.name} shape {shape}")
    sim = P.Simulation.from_workload(wl)
    sim.set_launch(*shape)
    sim.step(wl.steps)
    sim.sync()
    stats = sim.statistics()[0]
    feat = M.features_from_stats(stats)
    norm = M.feature_norm(feat[stats[:, O.ST_N] > 0])
    net = _net(PM, torch, _small_output(M.init_params(7)), norm)
    lm = net.attach(sim)
    s0 = sim.state()
    orc = O.Oracle(wl)
    for k in range(3):
        sim.step(1)
        sim.sync()
        cm = lm.cm.cpu().numpy()
        orc.set_state(s0)
        orc.step_index = wl.steps + k
        orc.set_cond_means(cm)
        orc.step(1)
        s1 = sim.state()
        o1 = orc.state()
        for q in ("x", "y", "u", "v", "w", "psi", "elem"):
            np.testing.assert_array_equal(s1[q], o1[q], err_msg=f"step {k} {q}")
        s0 = s1
    assert int(lm.served.cpu()[0]) > 0
    lm.detach()
    # detached: the binned means again
    orc.set_cond_means(None)
    orc.set_state(s0)
    orc.step_index = wl.steps + 3
    sim.step(1)
    orc.step(1)
    sim.sync()
    s1, o1 = sim.state(), orc.state()
    np.testing.assert_array_equal(s1["x"], o1["x"])
    np.testing.assert_allclose(s1["psi"], o1["psi"], rtol=1e-5, atol=1e-6)


def test_trained_network_beats_the_binned_estimate(gpu):
    """Trained on subsamples of 20 particles per element drawn from a run with
    many, the network's conditional means (with the fallback) are closer to
    the whole-population values than the binned means of the same subsamples,
    on draws it was not trained on."""
    P, PM, torch = gpu
    wl = _scalar_canyon(ppe=300, target=1500, steps=0)
    _label(f"mlp gain {wl.name} n={wl.n_total}")
    sim = P.Simulation.from_workload(wl)
    train, test = [], []
    for snap in range(8):
        sim.step(15)
        for d in range(6):
            train.append(PM.dataset(sim, target=20, key=1001, draw=100 * snap + d))
        test.append(PM.dataset(sim, target=20, key=2002, draw=snap).cpu().numpy())
    sim.sync()
    rows = torch.cat(train)
    net = PM.ConditionalMeanNet(seed=1)
    net.fit_norm(rows)
    loss = net.train(rows, iters=1500, batch=1024, lr=2e-3, seed=5).cpu().numpy()
    assert loss[-100:].mean() < 0.8 * loss[:20].mean()
    params = M.bf16_value(net.weights_bf16())
    norm = net.norm.cpu().numpy()
    ep, el, served = M.plain_and_learned_error(np.concatenate(test), params, norm)
    print(f"[case] plain@20 {ep:.4g} learned@20 {el:.4g} served {served:.3f}", flush=True)
    assert served > 0.3
    assert el < 0.8 * ep


def test_learned_means_same_in_step_and_in_separate_pass(gpu):
    """The means computed inside the step kernel equal those of the separate
    inference kernel on the same statistics, bit for bit, with graph replays
    and direct launches alike."""
    P, PM, torch = gpu
    wl = _scalar_canyon(ppe=20, steps=6)
    _label(f"mlp fused vs separate {wl.name}")
    sim = P.Simulation.from_workload(wl)
    sim.set_launch(16, 0)          # statistics summed in the same order as in the step below
    sim.step(wl.steps)
    sim.sync()
    stats = sim.statistics()[0]
    feat = M.features_from_stats(stats)
    norm = M.feature_norm(feat[stats[:, O.ST_N] > 0])
    net = _net(PM, torch, _small_output(M.init_params(8)), norm)
    ref, _ = net.infer(sim.statistics_device()[0])
    lm = net.attach(sim)
    sim.step(1)
    sim.sync()
    np.testing.assert_array_equal(lm.cm.cpu().numpy(), ref.cpu().numpy())
    # the graph path with the network attached, against direct launches of
    # the same sequence
    other = P.Simulation.from_workload(wl)
    other.set_launch(16, 0)
    other.step(wl.steps)
    lm3 = net.attach(other)
    other.step(1)
    sim.step_graph(12)
    other.step(12)
    sim.sync()
    other.sync()
    s1, s2 = sim.state(), other.state()
    for q in ("x", "y", "u", "v", "w", "elem"):
        np.testing.assert_array_equal(s1[q], s2[q])
    np.testing.assert_allclose(s1["psi"], s2["psi"], rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(lm.cm.cpu().numpy(), lm3.cm.cpu().numpy(), rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("graph", [False, True])
def test_network_over_a_split_order(gpu, graph):
    """Three ensembles of uneven size, whose cells of at most eight particles
    step in a launch of their own at 4 lanes per cell: with a network attached
    every cell steps in one launch, and after detaching the two launches
    resume.  Positions, velocities and elements do not depend on the scalar's
    means and stay bit-exact with the oracle for every ensemble."""
    P, PM, torch = gpu
    wl = W.tiny_canyon(precision="f32", nens=3, steps=2)
    counts = np.concatenate([np.asarray(e.counts) for e in wl.ensembles])
    small = int((counts <= 8).sum())
    assert 8 * small >= counts.size and 8 * (counts.size - small) >= counts.size   # the order splits
    _label(f"mlp over a split order {wl.name} graph={graph}")
    sim = P.Simulation.from_workload(wl)
    run = sim.step_graph if graph else sim.step
    run(2)
    sim.sync()
    stats = sim.statistics()[2]
    feat = M.features_from_stats(stats)
    norm = M.feature_norm(feat[stats[:, O.ST_N] > 0])
    net = _net(PM, torch, _small_output(M.init_params(7)), norm)
    lm = net.attach(sim)
    run(4)
    sim.sync()
    lm.detach()
    run(6)
    sim.sync()
    orc = O.Oracle(wl)
    orc.step(12)
    for en in range(wl.nens):
        g, o = sim.state(en), orc.state(en)
        for q in ("x", "y", "u", "v", "w", "elem"):
            np.testing.assert_array_equal(g[q], o[q], err_msg=f"ensemble {en} {q}")
