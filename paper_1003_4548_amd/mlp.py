"""Python binding of the learned conditional means (``include/pdfmlp.h``).

Argument marshalling only: dataset extraction, normalisation, training,
inference and the use inside the particle step run in the HIP kernels of
``libpdfpic.so``; PyTorch holds the device buffers and the stream.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import PdfError, load_library

NPARAM = 10952
NFEAT = 32
NOUT = 8
ROW = 64
NOALLOC_MAX_BATCH = 1024   # largest batch of pdf_mlp_grad_noalloc
# (out, in) of the four layers, in parameter order: W then b
LAYERS = ((64, 32), (64, 64), (64, 64), (8, 64))


def _vp(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def _check(status: int, what: str) -> None:
    if status != 0:
        raise PdfError(status, what)


def he_uniform(seed: int = 0) -> np.ndarray:
    """Initial parameters: uniform weights with variance 2 / fan-in in the hidden
    layers and 1 / fan-in in the output layer, zero biases (float32)."""
    rng = np.random.default_rng(seed)
    out = []
    for li, (o, i) in enumerate(LAYERS):
        lim = np.sqrt((6.0 if li < 3 else 3.0) / i)
        out.append(rng.uniform(-lim, lim, size=o * i))
        out.append(np.zeros(o))
    p = np.concatenate(out).astype(np.float32)
    assert p.size == NPARAM
    return p


class ConditionalMeanNet:
    """The network, its optimiser state and its normalisation, on one device."""

    def __init__(self, device: str = "cuda:0", seed: int = 0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        load_library()
        self.master = torch.from_numpy(he_uniform(seed)).to(self.device)
        self.adam_m = torch.zeros(NPARAM, dtype=torch.float32, device=self.device)
        self.adam_v = torch.zeros(NPARAM, dtype=torch.float32, device=self.device)
        self.w = torch.zeros(NPARAM, dtype=torch.int16, device=self.device)
        self.norm = torch.zeros((4, NFEAT), dtype=torch.float32, device=self.device)
        self.norm[1] = 1.0
        self.norm[2] = -3.0e38
        self.norm[3] = 3.0e38
        self.t = 0
        self._work = None
        self._work_batch = 0
        self.round()

    # -- helpers ---------------------------------------------------------------
    @property
    def _s(self) -> ctypes.c_void_p:
        return ctypes.c_void_p(self.stream.cuda_stream)

    def _workspace(self, batch: int):
        if self._work is None or batch > self._work_batch:
            n = int(load_library().pdf_mlp_work_floats(int(batch)))
            self._work = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
            self._work_batch = batch
        return self._work

    def set_master(self, params) -> None:
        self.master.copy_(self.torch.as_tensor(np.asarray(params, np.float32)).to(self.device))
        self.round()

    def round(self) -> None:
        _check(load_library().pdf_mlp_round(_vp(self.master), _vp(self.w), self._s), "pdf_mlp_round")

    def weights_bf16(self) -> np.ndarray:
        self.stream.synchronize()
        return self.w.cpu().numpy().view(np.uint16).copy()

    # -- the C ABI ---------------------------------------------------------------
    def fit_norm(self, rows) -> None:
        """Normalisation and training range from the rows with nonzero loss weights."""
        _check(load_library().pdf_mlp_norm(_vp(rows), int(rows.shape[0]), _vp(self.norm), self._s), "pdf_mlp_norm")

    def train(self, rows, iters: int, batch: int = 1024, lr: float = 1e-3, seed: int = 0):
        """iters Adam steps on batches drawn from rows; returns the loss per step (device)."""
        loss = self.torch.empty(int(iters), dtype=self.torch.float32, device=self.device)
        work = self._workspace(batch)
        _check(load_library().pdf_mlp_train(_vp(rows), int(rows.shape[0]), _vp(self.norm), _vp(self.master),
                                            _vp(self.adam_m), _vp(self.adam_v), _vp(self.w), _vp(work),
                                            _vp(loss), int(iters), int(batch), float(lr), int(seed),
                                            int(self.t), self._s), "pdf_mlp_train")
        self.t += int(iters)
        return loss

    def grad(self, rows, batch: Optional[int] = None):
        """(loss, gradient) over the first batch rows (device tensors)."""
        b = int(rows.shape[0] if batch is None else batch)
        work = self._workspace(b)
        g = self.torch.empty(NPARAM, dtype=self.torch.float32, device=self.device)
        loss = self.torch.empty(1, dtype=self.torch.float32, device=self.device)
        _check(load_library().pdf_mlp_grad(_vp(rows), b, _vp(self.norm), _vp(self.w), _vp(work), _vp(g), _vp(loss),
                                           self._s), "pdf_mlp_grad")
        return loss, g

    def grad_noalloc(self, rows, batch: Optional[int] = None, out=None):
        """grad() through the entry point without a workspace (the library's
        static scratch; batch <= NOALLOC_MAX_BATCH).  out: optional (loss,
        gradient) device tensors to fill, so that the call allocates nothing."""
        b = int(rows.shape[0] if batch is None else batch)
        if out is None:
            out = (self.torch.empty(1, dtype=self.torch.float32, device=self.device),
                   self.torch.empty(NPARAM, dtype=self.torch.float32, device=self.device))
        loss, g = out
        _check(load_library().pdf_mlp_grad_noalloc(_vp(rows), b, _vp(self.norm), _vp(self.w), _vp(g), _vp(loss),
                                                   self._s), "pdf_mlp_grad_noalloc")
        return loss, g

    def forward(self, rows):
        """Unprojected outputs (nrows x 8) of the features in the rows' first 32 columns."""
        rows = rows.contiguous()
        y = self.torch.empty((rows.shape[0], NOUT), dtype=self.torch.float32, device=self.device)
        _check(load_library().pdf_mlp_forward(_vp(rows), int(rows.shape[0]), int(rows.shape[1]), _vp(self.norm),
                                              _vp(self.w), _vp(y), self._s), "pdf_mlp_forward")
        return y

    def infer(self, stats):
        """Conditional means (ncell x 8) from statistics records (ncell x nstat) and
        the number of cells that took the network's value."""
        stats = stats.reshape(-1, stats.shape[-1]).contiguous()
        cm = self.torch.empty((stats.shape[0], NOUT), dtype=self.torch.float64, device=self.device)
        served = self.torch.zeros(1, dtype=self.torch.int32, device=self.device)
        _check(load_library().pdf_mlp_infer(_vp(stats), int(stats.shape[1]), int(stats.shape[0]), _vp(self.w),
                                            _vp(self.norm), _vp(cm), _vp(served), self._s), "pdf_mlp_infer")
        return cm, served

    def attach(self, sim) -> "LearnedMeans":
        """Use the network in sim's steps; returns the handle holding the outputs."""
        return LearnedMeans(self, sim)


class LearnedMeans:
    """The device buffers of an attached network: the conditional means of the
    last step (ncell x 8) and the count of cells served since attaching."""

    def __init__(self, net: ConditionalMeanNet, sim):
        torch = net.torch
        self.net, self.sim = net, sim
        self.cm = torch.zeros((sim.nens * sim.nelem, NOUT), dtype=torch.float64, device=net.device)
        self.served = torch.zeros(1, dtype=torch.int32, device=net.device)
        sim._check(load_library().pdf_mlp_attach(sim.ctx, _vp(net.w), _vp(net.norm), _vp(self.cm), _vp(self.served)),
                   "pdf_mlp_attach")

    def detach(self) -> None:
        self.sim._check(load_library().pdf_mlp_attach(self.sim.ctx, None, None, None, None), "pdf_mlp_attach")


def dataset(sim, target: int, key: int, draw: int):
    """Training rows (nens*nelem x 64, float32, device) of sim's current state."""
    torch = sim.torch
    rows = torch.empty((sim.nens * sim.nelem, ROW), dtype=torch.float32, device=sim.device)
    sim._check(load_library().pdf_mlp_dataset(sim.ctx, int(target), int(key), int(draw) & 0xFFFFFFFF, _vp(rows)),
               "pdf_mlp_dataset")
    return rows


def records_from_rows(rows):
    """Statistics records (nrows x 31 doubles) carried by dataset rows: the
    subsample's count, means, second moments, bin counts and binned means."""
    torch = rows.torch if hasattr(rows, "torch") else __import__("torch")
    f = rows[:, :32].double()
    rec = torch.zeros((rows.shape[0], 31), dtype=torch.float64, device=rows.device)
    n = torch.round(f[:, 0] * 64.0)
    rec[:, 0] = n
    rec[:, 1:5] = f[:, 1:5]
    rec[:, 5:15] = f[:, 5:15]
    rec[:, 15:23] = torch.round(f[:, 15:23] * n[:, None])
    rec[:, 23:31] = f[:, 23:31]
    return rec


def estimate_error(rows, cm=None) -> float:
    """Population-weighted RMS difference between an estimate of the eight
    conditional means (cm, nrows x 8; None: the subsample's binned means) and
    the whole-population values carried by dataset rows."""
    n = rows[:, 0] * 64.0
    est = rows[:, 23:31].double() if cm is None else cm.double()
    ref = rows[:, 48:56].double()
    wgt = rows[:, 56:64].double() * (n > 0).double()[:, None]
    return float((((est - ref) ** 2) * wgt).sum() / wgt.sum()) ** 0.5
