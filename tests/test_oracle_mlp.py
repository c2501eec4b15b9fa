"""Pins of the learned conditional-mean oracle against definitions that do not
use it: finite differences, closed forms, invariants and brute force."""
import numpy as np
import pytest

import oracle as O
from oracle import mlp as M


def test_bf16_rounding_matches_an_independent_definition():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-6, 6, size=4000),
                        [1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 3.0e-5]])
    x32 = x.astype(np.float32).astype(np.float64)
    m, e = np.frexp(x32)                       # x = m 2^e, 0.5 <= |m| < 1
    ref = np.round(m * 2.0 ** 8) * 2.0 ** (e - 8)   # 8 significant bits, ties to even
    np.testing.assert_array_equal(M.bf16(x), ref)
    assert M.bf16_bits([1.0])[0] == 0x3F80
    assert M.bf16([1.0 + 2.0 ** -8])[0] == 1.0            # tie to even
    assert M.bf16([1.0 + 3 * 2.0 ** -8])[0] == 1.0 + 2.0 ** -6


def test_forward_with_selection_weights_is_a_permuted_relu():
    """W1 copies the 32 inputs to the first 32 units, W2 and W3 are identities and
    W4 picks 8 units in a fixed non-symmetric order: y_b = relu(x_perm(b)) + b4_b."""
    p = np.zeros(M.NPARAM)
    (w1, b1), (w2, b2), (w3, b3), (w4, b4) = [(slice(wo, wo + o * i), slice(bo, bo + o))
                                              for (wo, bo, o, i) in M.LAYOUT]
    W1 = np.zeros((64, 32)); W1[np.arange(32), np.arange(32)] = 1.0
    p[w1] = W1.ravel()
    p[w2] = np.eye(64).ravel()
    p[w3] = np.eye(64).ravel()
    perm = [5, 0, 31, 7, 12, 3, 20, 9]
    W4 = np.zeros((8, 64)); W4[np.arange(8), perm] = 1.0
    p[w4] = W4.ravel()
    p[b4] = np.arange(8) * 0.25
    x = np.random.default_rng(2).normal(size=(6, 32))
    y, _ = M.forward(p, x, emulate=False)
    np.testing.assert_allclose(y, np.maximum(x[:, perm], 0.0) + np.arange(8) * 0.25, rtol=0, atol=0)


def _problem(seed, B=7):
    rng = np.random.default_rng(seed)
    params = rng.normal(size=M.NPARAM) * 0.2
    x = rng.normal(size=(B, 32))
    t = rng.normal(size=(B, 8))
    lw = rng.random(size=(B, 8))
    lw[0, 3] = 0.0
    lw /= lw.sum(axis=1, keepdims=True)
    return params, x, t, lw


def test_gradient_matches_central_differences():
    params, x, t, lw = _problem(3)
    _, g = M.loss_and_grad(params, x, t, lw, emulate=False)
    rng = np.random.default_rng(4)
    idx = np.concatenate([rng.choice(M.NPARAM, 300, replace=False),
                          [lay[1] for lay in M.LAYOUT], [M.NPARAM - 1]])
    h = 1e-6
    for k in idx:
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        fd = (M.loss_and_grad(pp, x, t, lw, emulate=False)[0] - M.loss_and_grad(pm, x, t, lw, emulate=False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (k, fd, g[k])


def test_projection_conserves_the_element_scalar():
    rng = np.random.default_rng(5)
    y = rng.normal(size=(50, 8))
    nb = rng.integers(0, 6, size=(50, 8)).astype(float)
    nb[:, 0] += 1
    n = nb.sum(axis=1, keepdims=True)
    p = M.project(y, nb / n)
    np.testing.assert_allclose((nb / n * p).sum(axis=1), 0.0, atol=1e-13)
    mean, sig = rng.random(size=(50, 1)), rng.random(size=(50, 1))
    m = mean + sig * p
    np.testing.assert_allclose((nb * m).sum(axis=1), (n * mean)[:, 0], rtol=1e-13)


def test_adam_first_step_is_a_signed_step():
    g = np.array([3.0, -0.5, 1e-3, -7.0])
    th, m, v = M.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, lr=0.01)
    np.testing.assert_allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def _record(n, mean, m2, nb, bm):
    r = np.zeros((1, 31))
    r[0, O.ST_N] = n
    r[0, O.ST_MEAN:O.ST_MEAN + 4] = mean
    r[0, O.ST_M2:O.ST_M2 + 10] = m2
    r[0, O.ST_BINN:O.ST_BINN + 8] = nb
    r[0, O.ST_BINM:O.ST_BINM + 8] = bm
    return r


def test_features_of_a_hand_made_record():
    m2 = np.arange(10) * 0.01 + 0.01
    m2[9] = 0.0625
    nb = np.array([2, 3, 0, 5, 1, 4, 3, 2], float)
    bm = np.linspace(0.1, 0.8, 8)
    f = M.features_from_stats(_record(20, [1.0, -0.5, 0.25, 0.3], m2, nb, bm))[0]
    assert f.dtype == np.float32
    np.testing.assert_array_equal(f[0], np.float32(20 / 64))
    np.testing.assert_array_equal(f[1:5], np.float32([1.0, -0.5, 0.25, 0.3]))
    np.testing.assert_array_equal(f[5:15], m2.astype(np.float32))
    np.testing.assert_array_equal(f[15:23], (nb / 20).astype(np.float32))
    np.testing.assert_array_equal(f[23:31], bm.astype(np.float32))
    assert f[31] == np.float32(0.25)


def test_inference_fallback_rules():
    rng = np.random.default_rng(6)
    params = M.init_params(0)
    nb = np.array([3, 2, 4, 1, 2, 3, 2, 3], float)
    base = dict(mean=[1.0, 0.0, 0.0, 0.5], m2=np.full(10, 0.01), nb=nb, bm=np.full(8, 0.5))
    recs = np.concatenate([_record(20, **base), _record(5, **base), _record(80, **base)])
    feat = M.features_from_stats(recs)
    norm = np.stack([np.zeros(32), np.ones(32), feat.min(axis=0) - 1.0, feat.max(axis=0) + 1.0]).astype(np.float32)
    # tiny output weights keep every estimate near the mean, inside [0, 1]
    p = params.copy()
    wo, bo, o, i = M.LAYOUT[3]
    p[wo:wo + o * i] *= 1e-3
    cm, ok, m = M.infer(recs, p, norm)
    assert ok.tolist() == [True, False, False]            # 8 <= n <= 64
    np.testing.assert_array_equal(cm[1], recs[1, O.ST_BINM:O.ST_BINM + 8])
    # a feature outside the training range
    norm2 = norm.copy()
    norm2[3, 5] = feat[0, 5] - 1e-3
    assert not M.infer(recs[:1], p, norm2)[1][0]
    # an estimate outside [0, 1]
    p3 = p.copy()
    p3[bo:bo + o] = np.array([400.0, -400.0, 0, 0, 0, 0, 0, 0])
    cm3, ok3, m3 = M.infer(recs[:1], p3, norm)
    assert not ok3[0] and (m3.min() < 0.0 or m3.max() > 1.0)
    np.testing.assert_array_equal(cm3[0], recs[0, O.ST_BINM:O.ST_BINM + 8])


def _tiny_state(rng, nelem=6, per=(30, 12, 200, 0, 5, 64)):
    elem = np.concatenate([np.full(k, e) for e, k in enumerate(per)]).astype(np.int32)
    rng.shuffle(elem)
    n = len(elem)
    return {"elem": elem, "u": rng.normal(size=n), "v": rng.normal(size=n), "w": rng.normal(size=n),
            "psi": rng.random(size=n)}


def test_dataset_rows_with_the_whole_population_reduce_to_the_binned_estimate():
    rng = np.random.default_rng(7)
    st = _tiny_state(rng)
    rows = M.dataset_rows(st, 6, target=10 ** 6, key=99, draw=0)
    for e in range(6):
        sel = st["elem"] == e
        n = sel.sum()
        r = rows[e]
        if n == 0:
            assert not r.any()
            continue
        assert r[0] == np.float32(n / 64)
        u, v, w, s = (st[k][sel] for k in ("u", "v", "w", "psi"))
        b = (u > u.mean()) * 1 + (v > v.mean()) * 2 + (w > w.mean()) * 4
        for q in range(8):
            assert r[56 + q] == (b == q).sum()
            if (b == q).any():
                np.testing.assert_allclose(r[48 + q], s[b == q].mean(), rtol=1e-6)
                np.testing.assert_allclose(r[23 + q], s[b == q].mean(), rtol=1e-6)
        # reference means conserve the element's scalar
        np.testing.assert_allclose((r[56:64] * r[48:56]).sum(), s.sum(), rtol=1e-5)


def test_dataset_subsample_is_a_bernoulli_draw_of_the_target_size():
    rng = np.random.default_rng(8)
    nelem, per = 40, 500
    elem = np.repeat(np.arange(nelem), per).astype(np.int32)
    st = {"elem": elem, "u": rng.normal(size=elem.size), "v": rng.normal(size=elem.size),
          "w": rng.normal(size=elem.size), "psi": rng.random(size=elem.size)}
    rows = M.dataset_rows(st, nelem, target=20, key=1234, draw=3)
    ns = rows[:, 0] * 64
    # binomial(500, 0.04): mean 20, sd 4.38; the mean of 40 draws within 4 sd of the mean
    assert abs(ns.mean() - 20.0) < 4 * 4.38 / np.sqrt(nelem)
    # reference counts cover the whole element
    np.testing.assert_array_equal(rows[:, 56:64].sum(axis=1), per)
    # the decision uses the documented Philox counter
    u = M.subsample_uniform(1234, [0, 1, 2], 3, 0)
    r = O.philox4x32_10([0, 3, M.SUB_BLOCK, 0], [1234, 0])
    assert u[0] == float(r[0]) * 2.0 ** -32 + 2.0 ** -33


def test_training_the_oracle_network_reduces_the_loss():
    """A few hundred Adam steps on a smooth synthetic regression."""
    rng = np.random.default_rng(9)
    B = 256
    x = rng.normal(size=(B, 32))
    lw = np.full((B, 8), 1 / 8)
    t = np.tanh(x[:, :8] - x[:, 8:16])
    t -= t.mean(axis=1, keepdims=True)
    p = M.init_params(1).astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = M.loss_and_grad(p, x, t, lw, emulate=False)[0]
    for it in range(1, 301):
        loss, g = M.loss_and_grad(p, x, t, lw, emulate=False)
        p, m, v = M.adam(p, m, v, g, it, lr=3e-3)
    assert loss < 0.2 * l0
