"""Oracle of the learned conditional-mean estimator (numpy, float64).

TEST INFRASTRUCTURE ONLY: used by the tests and the benchmark to check the
GPU library's MLP kernels; the product package never imports it.

What is computed.  IECM, eq. (7), relaxes each particle's scalar toward
<phi|V>, the mean scalar of the particles whose velocity falls in the same
velocity bin of its element (2 x 2 x 2 bins by the sign of each velocity
fluctuation).  With few particles per element the binned estimate is noisy.
The learned estimator maps per-element statistics of those few particles to
the eight conditional means:

* features (32, float32) from one element's statistics record: count / 64,
  the means of (u, v, w, psi), the ten central second moments, the eight bin
  fractions n_b / n, the eight binned means (the element mean for an empty
  bin) and the scalar standard deviation;
* normalised features (f - mu) * inv_s, rounded to bfloat16;
* a multilayer perceptron 32 -> 64 -> 64 -> 64 -> 8 with ReLU, bfloat16
  weights and biases, float32 accumulation, hidden activations rounded to
  bfloat16 (10952 parameters);
* outputs y_b read as standardised conditional means and projected so that
  the bin-population-weighted sum is zero: p_b = y_b - sum_c w_c y_c with
  w_c = n_c / n.  The estimate m_b = <psi> + sigma_psi p_b then conserves the
  element's scalar under IECM: sum_b n_b m_b = n <psi>;
* fallback to the binned means unless 8 <= n <= 64, every feature lies in
  the training range and every m_b lies in [0, 1].

Training data come from runs with many particles per element: in each
element a Bernoulli subsample (probability target / n, drawn with Philox)
plays the few-particle estimator; the targets are the conditional means of
all the element's particles in the bins split at the subsample's means.

BF16 emulation: with ``emulate=True`` every value the GPU rounds to bfloat16
(normalised inputs, hidden activations, back-propagated pre-activation
gradients) is rounded here at the same point (float64 -> float32 -> bfloat16,
round to nearest even); everything else is float64.  ``emulate=False`` is the
plain float64 network used for the finite-difference gradient check.
"""
from __future__ import annotations

import numpy as np

from . import ST_N, ST_MEAN, ST_M2, ST_BINN, ST_BINM, philox4x32_10

NFEAT, NHID, NOUT = 32, 64, 8
SIZES = [(NHID, NFEAT), (NHID, NHID), (NHID, NHID), (NOUT, NHID)]   # (out, in) per layer
ROW = 64            # dataset row: features 32, targets 8, loss weights 8, reference means 8, reference counts 8


def _layout():
    off, lay = 0, []
    for (o, i) in SIZES:
        lay.append((off, off + o * i, o, i))   # weight offset, bias offset
        off += o * i + o
    return lay, off


LAYOUT, NPARAM = _layout()
assert NPARAM == 10952

N_MIN, N_MAX = 8, 64          # element counts the learned estimator serves
SIGMA_MIN = 1e-4              # rows with a smaller subsample scalar std are not trained on
T_CLIP = 8.0                  # standardised targets are clipped to +-T_CLIP
SUB_BLOCK = 0x5EED            # Philox block word of the subsample draw


# ---------------------------------------------------------------------------
# bfloat16


def bf16_bits(x) -> np.ndarray:
    """Round to bfloat16 (float64 -> float32 -> bfloat16, nearest even); the 16-bit codes."""
    f = np.ascontiguousarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = u + 0x7FFF + ((u >> 16) & 1)
    return ((u >> 16) & 0xFFFF).astype(np.uint16)


def bf16_value(bits) -> np.ndarray:
    b = np.ascontiguousarray(bits, np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def bf16(x) -> np.ndarray:
    return bf16_value(bf16_bits(x))


# ---------------------------------------------------------------------------
# parameters


def unpack(params):
    """(W, b) per layer, float64 views of a flat parameter vector."""
    p = np.asarray(params, np.float64)
    out = []
    for (wo, bo, o, i) in LAYOUT:
        out.append((p[wo:wo + o * i].reshape(o, i), p[bo:bo + o]))
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases (float32 master copy)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM, np.float32)
    for li, (wo, bo, o, i) in enumerate(LAYOUT):
        lim = np.sqrt(6.0 / i) if li < 3 else np.sqrt(3.0 / i)
        p[wo:wo + o * i] = rng.uniform(-lim, lim, size=o * i).astype(np.float32)
    return p


# ---------------------------------------------------------------------------
# features


def features_from_stats(rec) -> np.ndarray:
    """Feature vectors (ncell x 32, float32) from statistics records (ncell x nstat)."""
    rec = np.asarray(rec, np.float64)
    n = rec[:, ST_N]
    f = np.zeros((rec.shape[0], NFEAT))
    f[:, 0] = n / 64.0
    f[:, 1:5] = rec[:, ST_MEAN:ST_MEAN + 4]
    f[:, 5:15] = rec[:, ST_M2:ST_M2 + 10]
    with np.errstate(invalid="ignore", divide="ignore"):
        frac = np.where(n[:, None] > 0, rec[:, ST_BINN:ST_BINN + 8] / n[:, None], 0.0)
    f[:, 15:23] = frac
    f[:, 23:31] = rec[:, ST_BINM:ST_BINM + 8]
    f[:, 31] = np.sqrt(np.maximum(rec[:, ST_M2 + 9], 0.0))
    return f.astype(np.float32)


def normalise(feat, norm) -> np.ndarray:
    """bfloat16 of (f - mu) * inv_s computed in float32; norm = [mu, inv_s, fmin, fmax] x 32."""
    nm = np.asarray(norm, np.float32).reshape(4, NFEAT)
    x = (np.asarray(feat, np.float32) - nm[0]) * nm[1]
    return bf16(x)


def feature_norm(feat) -> np.ndarray:
    """Normalisation and training range of a feature set: [mu, inv_s, fmin, fmax] (float32, 4 x 32)."""
    f = np.asarray(feat, np.float64)
    mu = f.mean(axis=0)
    sd = f.std(axis=0)
    inv = np.where(sd > 1e-12, 1.0 / np.maximum(sd, 1e-12), 1.0)
    return np.stack([mu, inv, f.min(axis=0), f.max(axis=0)]).astype(np.float32)


# ---------------------------------------------------------------------------
# network


def forward(params, xhat, emulate: bool = True):
    """y (B x 8) and the hidden activations of the network at inputs xhat (B x 32)."""
    layers = unpack(bf16(params) if emulate else params)
    h = np.asarray(xhat, np.float64)
    acts = [h]
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        if li < 3:
            h = np.maximum(z, 0.0)
            if emulate:
                h = bf16(h)
            acts.append(h)
        else:
            h = z
    return h, acts


def project(y, w):
    """p_b = y_b - sum_c w_c y_c."""
    y = np.asarray(y, np.float64)
    return y - (np.asarray(w, np.float64) * y).sum(axis=1, keepdims=True)


def loss_and_grad(params, xhat, target, lw, emulate: bool = True):
    """Batch loss (1/B) sum_i sum_b lw_ib (p_ib - t_ib)^2 and its gradient (NPARAM, float64)."""
    B = xhat.shape[0]
    y, acts = forward(params, xhat, emulate)
    lw = np.asarray(lw, np.float64)
    p = project(y, lw)
    r = p - np.asarray(target, np.float64)
    loss = float((lw * r * r).sum() / B)
    g = 2.0 * lw * r / B
    dz = g - lw * g.sum(axis=1, keepdims=True)
    layers = unpack(bf16(params) if emulate else params)
    grad = np.zeros(NPARAM)
    for li in range(3, -1, -1):
        if emulate:
            dz = bf16(dz)
        wo, bo, o, i = LAYOUT[li]
        hin = acts[li]
        grad[wo:wo + o * i] = (dz.T @ hin).reshape(-1)
        grad[bo:bo + o] = dz.sum(axis=0)
        if li > 0:
            dh = dz @ layers[li][0]
            dz = dh * (acts[li] > 0.0)
    return loss, grad


def adam(master, m, v, grad, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (t counts from 1); returns new (master, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return master - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# estimator


def infer(rec, params, norm):
    """Conditional means per cell (ncell x 8) and the mask of cells that took the
    learned value, from statistics records with the learned estimator."""
    rec = np.asarray(rec, np.float64)
    nm = np.asarray(norm, np.float32).reshape(4, NFEAT)
    feat = features_from_stats(rec)
    y, _ = forward(params, normalise(feat, norm), emulate=True)
    y = y.astype(np.float32).astype(np.float64)
    n = rec[:, ST_N]
    with np.errstate(invalid="ignore", divide="ignore"):
        w = np.where(n[:, None] > 0, rec[:, ST_BINN:ST_BINN + 8] / n[:, None], 0.0)
    p = project(y, w)
    sig = np.sqrt(np.maximum(rec[:, ST_M2 + 9], 0.0))
    m = rec[:, ST_MEAN + 3:ST_MEAN + 4] + sig[:, None] * p
    inbox = np.all((feat >= nm[2]) & (feat <= nm[3]), axis=1)
    ok = (n >= N_MIN) & (n <= N_MAX) & inbox & (sig > 0.0) & np.all((m >= 0.0) & (m <= 1.0), axis=1)
    cm = np.where(ok[:, None], m, rec[:, ST_BINM:ST_BINM + 8])
    return cm, ok, m


# ---------------------------------------------------------------------------
# training data


def subsample_uniform(key: int, ids, draw: int, ens: int) -> np.ndarray:
    """The Philox uniform in (0, 1) that decides each particle's subsample membership."""
    out = np.empty(len(ids))
    k = [key & 0xFFFFFFFF, (key >> 32) & 0xFFFFFFFF]
    for j, pid in enumerate(ids):
        r = philox4x32_10([int(pid), draw & 0xFFFFFFFF, SUB_BLOCK, ens], k)
        out[j] = float(r[0]) * 2.0 ** -32 + 2.0 ** -33
    return out


def dataset_rows(state, nelem: int, target: int, key: int, draw: int, ens: int = 0) -> np.ndarray:
    """One training row per element (nelem x 64, float32) from a particle state in id order."""
    elem = np.asarray(state["elem"])
    val = np.stack([state["u"], state["v"], state["w"], state["psi"]], axis=1).astype(np.float64)
    ids = np.arange(len(elem))
    uni = subsample_uniform(key, ids, draw, ens)
    rows = np.zeros((nelem, ROW), np.float32)
    order = np.argsort(elem, kind="stable")
    bounds = np.searchsorted(elem[order], np.arange(nelem + 1))
    for e in range(nelem):
        idx = order[bounds[e]:bounds[e + 1]]
        n = len(idx)
        if n == 0:
            continue
        p = float(target) / float(n)
        sel = idx[uni[idx] < p]
        ns = len(sel)
        if ns == 0:
            continue
        vs = val[sel]
        mean = vs.sum(axis=0) / ns
        d = vs - mean
        m2 = np.array([(d[:, a] * d[:, b]).sum() / ns for a in range(4) for b in range(a, 4)])
        bins_s = (vs[:, 0] > mean[0]) * 1 + (vs[:, 1] > mean[1]) * 2 + (vs[:, 2] > mean[2]) * 4
        nb = np.array([(bins_s == b).sum() for b in range(8)], np.float64)
        bm = np.array([vs[bins_s == b, 3].sum() / nb[b] if nb[b] > 0 else mean[3] for b in range(8)])
        rec = np.zeros(31)
        rec[ST_N] = ns
        rec[ST_MEAN:ST_MEAN + 4] = mean
        rec[ST_M2:ST_M2 + 10] = m2
        rec[ST_BINN:ST_BINN + 8] = nb
        rec[ST_BINM:ST_BINM + 8] = bm
        rows[e, :32] = features_from_stats(rec[None, :])[0]
        va = val[idx]
        bins_a = (va[:, 0] > mean[0]) * 1 + (va[:, 1] > mean[1]) * 2 + (va[:, 2] > mean[2]) * 4
        na = np.array([(bins_a == b).sum() for b in range(8)], np.float64)
        mall = va[:, 3].sum() / n
        mref = np.array([va[bins_a == b, 3].sum() / na[b] if na[b] > 0 else mall for b in range(8)])
        sig = np.sqrt(max(m2[9], 0.0))
        if ns >= 2 and sig > SIGMA_MIN:
            rows[e, 32:40] = np.clip((mref - mean[3]) / sig, -T_CLIP, T_CLIP)
            rows[e, 40:48] = nb / ns
        rows[e, 48:56] = mref
        rows[e, 56:64] = na
    return rows


def plain_and_learned_error(rows, params, norm):
    """Population-weighted RMS error of the binned and of the learned estimate
    against the reference conditional means of dataset rows (the learned one
    with its fallback).  Returns (plain, learned, fraction of the rows in the
    trained domain, subsample scalar spread above SIGMA_MIN, that took the
    learned value)."""
    rows = np.asarray(rows, np.float64)
    feat = rows[:, :32]
    n = feat[:, 0] * 64.0
    plain = feat[:, 23:31]
    rec = np.zeros((rows.shape[0], 31))
    rec[:, ST_N] = np.rint(n)
    rec[:, ST_MEAN:ST_MEAN + 4] = feat[:, 1:5]
    rec[:, ST_M2:ST_M2 + 10] = feat[:, 5:15]
    rec[:, ST_BINN:ST_BINN + 8] = np.rint(feat[:, 15:23] * rec[:, ST_N:ST_N + 1])
    rec[:, ST_BINM:ST_BINM + 8] = plain
    cm, ok, _ = infer(rec, params, norm)
    wgt = rows[:, 56:64] * (n[:, None] > 0)
    ref = rows[:, 48:56]
    den = wgt.sum()
    ep = np.sqrt((wgt * (plain - ref) ** 2).sum() / den)
    el = np.sqrt((wgt * (cm - ref) ** 2).sum() / den)
    varies = (n > 0) & (feat[:, 31] > SIGMA_MIN)
    return float(ep), float(el), float(ok[varies].mean() if varies.any() else 0.0)
