"""Precision report: the float-state GPU path against the double-precision
oracle (the truth), same seeds, 20 steps, on the 1M-particle canyon (second
moments) and the 10M-particle wall-function canyon (moments to fourth order,
32-bin scalar histograms).

The float path is bit-exact against the oracle's float mirror (the parity
tests); this states how far it is from the double-precision result, for
every statistic of the record, as the maximum and RMS difference in units of
the Monte Carlo standard error of that statistic in its element:
* means: sqrt(var / n);
* central moments of order 2 to 4 (every index combination): the standard
  deviation of the per-particle product over sqrt(n);
* velocity-binned conditional means <phi|V>: the scalar's standard deviation
  in the bin over sqrt(n_bin);
* bin counts and histogram counts: sqrt(n p (1 - p)).
Standard errors come from the double-precision state.  Float rounding moves
a few particles (those within rounding distance of an edge) into the
neighbouring element; each shifts its elements' statistics by about
1/sqrt(n) standard errors, and the rest of the difference is far below the
sampling noise.  The table is written to gpurun_out/precision_<case>.md.
"""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_4548_amd as P
    P.load_library()
    return P


PAIRS = [(a, b) for a in range(4) for b in range(a, 4)]
TRIPS = [(a, b, c) for a in range(4) for b in range(a, 4) for c in range(b, 4)]
QUADS = [(a, b, c, d) for a in range(4) for b in range(a, 4) for c in range(b, 4) for d in range(c, 4)]
NAMES = "uvwp"


def _standard_errors(st, ne, moments, hist):
    """Per element and statistic, from the double-precision particles."""
    e = st["elem"]
    n = np.bincount(e, minlength=ne).astype(np.float64)
    nn = np.maximum(n, 1.0)
    X = np.stack([st["u"], st["v"], st["w"], st["psi"]], axis=1)
    mean = np.stack([np.bincount(e, X[:, q], ne) for q in range(4)], axis=1) / nn[:, None]
    D = X - mean[e]

    def se_of(prod):
        m1 = np.bincount(e, prod, ne) / nn
        m2 = np.bincount(e, prod * prod, ne) / nn
        return np.sqrt(np.maximum(m2 - m1 * m1, 0.0) / nn)

    out = {"mean": np.stack([se_of(X[:, q]) for q in range(4)], axis=1),
           "m2": np.stack([se_of(D[:, a] * D[:, b]) for a, b in PAIRS], axis=1)}
    if moments >= 4:
        out["m3"] = np.stack([se_of(D[:, a] * D[:, b] * D[:, c]) for a, b, c in TRIPS], axis=1)
        out["m4"] = np.stack([se_of(D[:, a] * D[:, b] * D[:, c] * D[:, d]) for a, b, c, d in QUADS], axis=1)
    b = (D[:, 0] > 0).astype(int) + 2 * (D[:, 1] > 0) + 4 * (D[:, 2] > 0)
    key = e * 8 + b
    nb = np.bincount(key, minlength=8 * ne).astype(np.float64)
    nbb = np.maximum(nb, 1.0)
    s1 = np.bincount(key, X[:, 3], 8 * ne) / nbb
    s2 = np.bincount(key, X[:, 3] ** 2, 8 * ne) / nbb
    out["binm"] = np.sqrt(np.maximum(s2 - s1 * s1, 0.0) / nbb).reshape(ne, 8)
    p = (nb / np.repeat(nn, 8)).reshape(ne, 8)
    out["binn"] = np.sqrt(np.maximum(n[:, None] * p * (1 - p), 0.0))
    if hist:
        hb = np.clip(np.floor(X[:, 3] * hist), 0, hist - 1).astype(int)
        cnt = np.bincount(e * hist + hb, minlength=hist * ne).reshape(ne, hist)
        ph = cnt / nn[:, None]
        out["hist"] = np.sqrt(np.maximum(n[:, None] * ph * (1 - ph), 0.0))
    return n, out


def _report(case, sg, so, n, se, moments, hist):
    ok = n >= 20
    rows = []

    def add(name, g, o, s):
        z = (g - o) / np.where(s > 0, s, np.inf)
        z = z[ok][(s[ok] > 1e-12 * np.maximum(1.0, np.abs(o[ok])))]
        if z.size == 0:
            return
        rows.append((name, z.size, float(np.abs(z).max()), float(np.sqrt((z ** 2).mean()))))

    for q in range(4):
        add(f"<{NAMES[q]}>", sg[:, O.ST_MEAN + q], so[:, O.ST_MEAN + q], se["mean"][:, q])
    for t, (a, b) in enumerate(PAIRS):
        add(f"<{NAMES[a]}'{NAMES[b]}'>", sg[:, O.ST_M2 + t], so[:, O.ST_M2 + t], se["m2"][:, t])
    for q in range(8):
        add(f"<phi|V> bin {q}", sg[:, O.ST_BINM + q], so[:, O.ST_BINM + q], se["binm"][:, q])
        add(f"count bin {q}", sg[:, O.ST_BINN + q], so[:, O.ST_BINN + q], se["binn"][:, q])
    if moments >= 4:
        for t, (a, b, c) in enumerate(TRIPS):
            add(f"<{NAMES[a]}'{NAMES[b]}'{NAMES[c]}'>", sg[:, O.ST_M3 + t], so[:, O.ST_M3 + t], se["m3"][:, t])
        for t, q4 in enumerate(QUADS):
            add("<" + "".join(NAMES[i] + "'" for i in q4) + ">", sg[:, O.ST_M4 + t], so[:, O.ST_M4 + t],
                se["m4"][:, t])
    if hist:
        off = O.NSTAT_4 if moments >= 4 else O.NSTAT_2
        for h in range(hist):
            add(f"histogram bin {h}", sg[:, off + h], so[:, off + h], se["hist"][:, h])
    lines = [f"| statistic | elements | max (standard errors) | RMS (standard errors) |", "|---|---|---|---|"]
    lines += [f"| {r[0]} | {r[1]} | {r[2]:.2e} | {r[3]:.2e} |" for r in rows]
    txt = "\n".join(lines)
    os.makedirs(os.path.join(ROOT, "gpurun_out"), exist_ok=True)
    with open(os.path.join(ROOT, "gpurun_out", f"precision_{case}.md"), "w") as f:
        f.write(txt + "\n")
    print(txt, flush=True)
    return rows


CASES = {"canyon1m": lambda steps: W.config2(steps=steps), "canyon10m": lambda steps: W.config3(steps=steps)}


@pytest.mark.parametrize("case", list(CASES))
def test_float_path_against_double_oracle(gpu, case):
    steps = 20
    wl32 = CASES[case](steps)
    wl64 = CASES[case](steps)
    wl64.precision = "f64"
    print(f"[case] precision report {wl32.name} n={wl32.n_total} steps={steps}", flush=True)
    sim = gpu.Simulation.from_workload(wl32)
    sim.step(steps)
    sim.sync()
    sg = sim.statistics()[0]
    sim.close()
    orc = O.Oracle(wl64)
    orc.step(steps)
    so = orc.stats()
    st = orc.state()
    del orc
    n, se = _standard_errors(st, wl64.mesh.nelem, wl64.moments, wl64.hist_bins)
    np.testing.assert_array_equal(so[:, O.ST_N], n)
    assert (n >= 20).mean() > 0.9
    moved = np.abs(sg[:, O.ST_N] - n).sum()
    print(f"[report] {case}: element-count differences (particles): {moved:.0f} of {wl32.n_total}", flush=True)
    assert moved <= 1e-4 * wl32.n_total
    rows = _report(case, sg, so, n, se, wl64.moments, wl64.hist_bins)
    expected = 4 + 10 + 16 + (55 if wl64.moments >= 4 else 0) + wl64.hist_bins
    assert len(rows) >= expected - 2          # a histogram bin may be empty everywhere
    worst_rms = max(r[3] for r in rows)
    worst_max = max(r[2] for r in rows)
    print(f"[report] {case}: worst RMS {worst_rms:.3g}, worst max {worst_max:.3g} standard errors", flush=True)
    assert worst_rms < 0.1 and worst_max < 6.0
