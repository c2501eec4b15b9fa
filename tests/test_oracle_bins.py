"""Pins of the oracle's 5 x 5 x 5 velocity bins for <phi|V> (section 3 uses
a (5 x 5 x 5) bin structure for the conditional scalar mean of eq. 7).

Reading: per velocity component five bins of width 1.2 sigma over
[-3 sigma, 3 sigma] about the element mean (edges at +-0.6 and +-1.8 sigma),
the outermost bins open, sigma from the element's central second moments;
bin = k_u + 5 k_v + 25 k_w; sigma = 0 puts every particle in the middle bin.

* Counts and conditional means against numpy's digitize on the same state
  (independent of the oracle's division-based bin formula), empty bins
  reporting the element mean.
* IECM with the fine bins conserves the scalar sum of every (element, bin)
  and contracts its centred sum of squares by (1 - r)^2 exactly as eq. (7)
  with the bin mean.
* Elements whose particles share one velocity reduce IECM to IEM (one bin).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from workloads.fields import F, uniform_fields

EDGES = np.array([-1.8, -0.6, 0.6, 1.8])


def _fine_keys(st, rec):
    e = st["elem"]
    k = np.zeros(len(e), np.int64)
    mult = 1
    for q, (name, t) in enumerate((("u", 0), ("v", 4), ("w", 7))):
        m = rec[e, O.ST_MEAN + q]
        sd = np.sqrt(rec[e, O.ST_M2 + t])
        z_edges = m[:, None] + sd[:, None] * EDGES[None, :]
        kq = (st[name][:, None] >= z_edges).sum(axis=1)
        kq = np.where(sd > 0, kq, 2)
        k += mult * kq
        mult *= 5
    return k


def _wl(**kw):
    wl = W.small_canyon(target=600, ppe=60, precision="f64", vbins=5, **kw)
    return wl


def test_fine_bin_counts_and_means():
    wl = _wl()
    orc = O.Oracle(wl)
    orc.step(4)
    st, rec = orc.state(), orc.stats()
    assert rec.shape[1] == O.NSTAT_2 + 250
    k = _fine_keys(st, rec)
    e = st["elem"]
    ne = wl.mesh.nelem
    key = e * 125 + k
    cnt = np.bincount(key, minlength=125 * ne).reshape(ne, 125)
    np.testing.assert_array_equal(rec[:, O.NSTAT_2:O.NSTAT_2 + 125], cnt)
    s = np.bincount(key, weights=st["psi"], minlength=125 * ne).reshape(ne, 125)
    mean = np.where(cnt > 0, s / np.maximum(cnt, 1), rec[:, O.ST_MEAN + 3][:, None])
    np.testing.assert_allclose(rec[:, O.NSTAT_2 + 125:], mean, rtol=1e-13, atol=1e-15)
    # the bins are used: more than the eight sign bins' worth per element
    assert (np.count_nonzero(cnt, axis=1) > 8).mean() > 0.9


def test_fine_bins_with_histograms_and_frequency():
    wl = W.small_canyon(target=600, ppe=60, precision="f32", vbins=5, moments=4, hist_bins=32, wallfn=True,
                        omega=True)
    orc = O.Oracle(wl)
    orc.step(3)
    st, rec = orc.state(), orc.stats()
    off = O.NSTAT_4 + 32 + 3
    assert rec.shape[1] == off + 250
    k = _fine_keys(st, rec)
    cnt = np.bincount(st["elem"] * 125 + k, minlength=125 * wl.mesh.nelem).reshape(-1, 125)
    np.testing.assert_array_equal(rec[:, off:off + 125], cnt)


def test_iecm_with_fine_bins_conserves_and_contracts():
    wl = _wl()
    wl.psi_init = W.PSI_LEFT_QUARTER
    orc = O.Oracle(wl)
    orc.step(3)
    wl.flags = 4
    orc2 = O.Oracle(wl)
    orc2.set_state(orc.state())
    st0, rec0 = orc2.state(), orc2.stats()
    orc2.step(1)
    st1 = orc2.state()
    for q in ("x", "y", "u", "v", "w", "elem"):
        np.testing.assert_array_equal(st0[q], st1[q])
    e = st0["elem"]
    key = e * 125 + _fine_keys(st0, rec0)
    n = 125 * wl.mesh.nelem
    r = orc2.mix_rate()[e]
    s0 = np.bincount(key, weights=st0["psi"], minlength=n)
    s1 = np.bincount(key, weights=st1["psi"], minlength=n)
    np.testing.assert_allclose(s1, s0, rtol=0, atol=1e-12)
    cnt = np.bincount(key, minlength=n)
    m0 = np.divide(s0, cnt, out=np.zeros_like(s0), where=cnt > 0)[key]
    c0 = (st0["psi"] - m0) ** 2
    c1 = (st1["psi"] - m0) ** 2
    np.testing.assert_allclose(c1, (1 - r) ** 2 * c0, rtol=1e-9, atol=1e-15)
    assert (s0 > 0).sum() > 500


def test_one_velocity_is_one_bin():
    wl = W.configs.square_box(n=4, ppe=30, precision="f64")
    wl.vbins = 5
    wl.flags = 4
    orc = O.Oracle(wl)
    st = orc.state()
    st["u"][:] = 1.0
    st["v"][:] = 0.0
    st["w"][:] = 0.0
    orc.set_state(st)
    rec = orc.stats()
    np.testing.assert_array_equal(rec[:, O.NSTAT_2 + 62], rec[:, O.ST_N])       # the middle bin
    np.testing.assert_allclose(rec[:, O.NSTAT_2 + 125 + 62], rec[:, O.ST_MEAN + 3], rtol=1e-15)
    orc.step(1)
    psi1 = orc.state()["psi"]
    r = orc.mix_rate()[st["elem"]]
    m = rec[st["elem"], O.ST_MEAN + 3]
    np.testing.assert_allclose(psi1, st["psi"] - r * (st["psi"] - m), rtol=1e-15, atol=1e-15)
