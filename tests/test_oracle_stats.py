"""Pin of the oracle's particle-in-cell estimation (ensemble averages per
element, section 2 and section 3) against numpy / math.fsum on the same state."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _numpy_stats(st, nelem, moments, hist_bins):
    e = st["elem"]
    vals = np.stack([st["u"], st["v"], st["w"], st["psi"]], axis=1)
    out = []
    for el in range(nelem):
        sel = e == el
        n = int(sel.sum())
        rec = {"n": n}
        if n == 0:
            out.append(rec)
            continue
        x = vals[sel]
        mean = np.array([math.fsum(x[:, q]) / n for q in range(4)])
        d = x - mean
        rec["mean"] = mean
        rec["m2"] = np.array([np.mean(d[:, a] * d[:, b]) for a, b in itertools.combinations_with_replacement(range(4), 2)])
        if moments >= 4:
            rec["m3"] = np.array([np.mean(d[:, a] * d[:, b] * d[:, c])
                                  for a, b, c in itertools.combinations_with_replacement(range(4), 3)])
            rec["m4"] = np.array([np.mean(d[:, a] * d[:, b] * d[:, c] * d[:, g])
                                  for a, b, c, g in itertools.combinations_with_replacement(range(4), 4)])
        b = (x[:, 0] > mean[0]) * 1 + (x[:, 1] > mean[1]) * 2 + (x[:, 2] > mean[2]) * 4
        cnt = np.bincount(b, minlength=8)
        s = np.bincount(b, weights=x[:, 3], minlength=8)
        rec["binn"] = cnt
        rec["binm"] = np.where(cnt > 0, s / np.maximum(cnt, 1), mean[3])
        if hist_bins:
            rec["hist"] = np.histogram(np.clip(x[:, 3], 0, 1), bins=hist_bins, range=(0.0, 1.0))[0]
        out.append(rec)
    return out


@pytest.mark.parametrize("case", ["config1", "canyon_m4"])
def test_statistics_match_numpy(case):
    if case == "config1":
        wl = W.config1()
        steps = 5
    else:
        wl = W.small_canyon(target=600, ppe=30, precision="f32", moments=4, hist_bins=32, wallfn=True)
        steps = 30
    orc = O.Oracle(wl)
    orc.step(steps)
    st = orc.state()
    got = orc.stats()
    ref = _numpy_stats(st, wl.mesh.nelem, wl.moments, wl.hist_bins)
    for el, r in enumerate(ref):
        g = got[el]
        assert g[O.ST_N] == r["n"]
        if r["n"] == 0:
            assert (g == 0).all()
            continue
        np.testing.assert_allclose(g[O.ST_MEAN:O.ST_MEAN + 4], r["mean"], rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(g[O.ST_M2:O.ST_M2 + 10], r["m2"], rtol=1e-11, atol=1e-16)
        np.testing.assert_array_equal(g[O.ST_BINN:O.ST_BINN + 8], r["binn"])
        np.testing.assert_allclose(g[O.ST_BINM:O.ST_BINM + 8], r["binm"], rtol=1e-13, atol=1e-15)
        if wl.moments >= 4:
            np.testing.assert_allclose(g[O.ST_M3:O.ST_M3 + 20], r["m3"], rtol=1e-10, atol=1e-17)
            np.testing.assert_allclose(g[O.ST_M4:O.ST_M4 + 35], r["m4"], rtol=1e-10, atol=1e-18)
            np.testing.assert_array_equal(g[O.NSTAT_4:O.NSTAT_4 + 32], r["hist"])
    # totals
    assert got[:, O.ST_N].sum() == len(st["x"])
