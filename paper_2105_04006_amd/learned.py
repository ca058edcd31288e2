"""Learned band proposal: the network, its training step and its inference.

The network takes a per-object feature vector (a 1,024-bin coarse periodogram
and 64 sampling-window features, scaled) and proposes which of 64 equal-width
frequency bands hold the periodogram's peak.  The bands refined per object
are the network's most probable ones followed by the bands whose coarse power
peaks highest; objects whose proposal or refined peak is weak are re-run on
the whole grid.  Every arithmetic step runs in the library's kernels (BF16
matrix-core GEMMs with FP32 accumulation, softmax cross-entropy, Adam, the
feature, selection and periodogram kernels); this module owns the device
buffers and calls the kernels in order.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import lsp

DIMS = (1088, 512, 256, 64)


def _p(x):
    return ctypes.c_void_p(x.data_ptr()) if x is not None else None


def _s(stream=None):
    return lsp._stream_handle(stream)


def _ok(st, what):
    if st != lsp.OK:
        raise lsp.LspError(st, what)


def gemm(A, B, M, N, K, sam, sak, sbk, sbn, C=None, C_bf16=None, bias=None, mask=None,
         relu=False, ldc=None, stream=None):
    """C = A.B through lsp_gemm_bf16 (A, B: int16 tensors holding BF16 bits)."""
    _ok(lsp.lib().lsp_gemm_bf16(int(M), int(N), int(K), _p(A), int(sam), int(sak), _p(B),
                                int(sbk), int(sbn), _p(bias), _p(mask), int(bool(relu)), _p(C),
                                _p(C_bf16), int(ldc if ldc is not None else N), _s(stream)),
        "lsp_gemm_bf16")


def to_bf16(x, out=None, stream=None):
    """FP32 device tensor -> BF16 bits (int16 tensor) via lsp_cast_bf16."""
    out = torch.empty(x.shape, dtype=torch.int16, device=x.device) if out is None else out
    _ok(lsp.lib().lsp_cast_bf16(_p(x), x.numel(), _p(out), _s(stream)), "lsp_cast_bf16")
    return out


def bf16_to_f32(h):
    """BF16 bits (int16 tensor) -> float32 tensor (exact widening)."""
    return (h.to(torch.int32) << 16).view(torch.float32)


def he_init(seed, dims=DIMS):
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for a, b in zip(dims[:-1], dims[1:]):
        params.append(rng.normal(0.0, np.sqrt(2.0 / a), size=(a, b)))
        params.append(np.zeros(b))
    return params


def banded_init(seed, dims=DIMS, coarse=lsp.FEAT_COARSE, per_band=4,
                thresholds=(-0.5, 0.5, 1.5, 3.0), noise=0.05):
    """He initialisation with a band-detector path written into part of it.

    The coarse features come in n_bands groups of coarse / n_bands columns,
    one group per output band.  Hidden layer 1 gets `per_band` units per band
    that average their group's standardised columns and subtract a threshold
    (a piecewise-linear, increasing response to the band's strength), hidden
    layer 2 one unit per band that adds them, and the output layer reads that
    unit into the band's logit.  The initial network therefore ranks bands by
    their coarse power; training adjusts every weight from there, including
    the remaining randomly initialised units.
    """
    rng = np.random.default_rng(seed)
    d0, d1, d2, d3 = dims
    n_bands = d3
    group = coarse // n_bands
    W1, b1, W2, b2, W3, b3 = he_init(seed, dims)
    k1 = n_bands * per_band
    assert k1 <= d1 and n_bands <= d2 and len(thresholds) == per_band
    W1[:, :k1] *= noise
    W2[:k1, :] *= noise
    W2[:, :n_bands] *= noise
    W3 *= noise
    for b in range(n_bands):
        for s_, th in enumerate(thresholds):
            u = b * per_band + s_
            W1[b * group:(b + 1) * group, u] += 1.0 / group
            b1[u] = -th
            W2[u, b] += 1.0
        W3[b, b] += 1.0
    return [W1, b1, W2, b2, W3, b3]


class BandNet:
    """1088 -> 512 -> 256 -> 64 ReLU network with FP32 master weights, BF16 copies
    for the GEMMs, and Adam state, all on one device."""

    def __init__(self, device, seed=0, dims=DIMS, params=None, init="banded", row_norm=True):
        self.dims = tuple(dims)
        self.device = device
        self.row_norm = bool(row_norm)
        if params is None:
            params = (banded_init(seed, self.dims) if init == "banded"
                      else he_init(seed, self.dims))
        self.master = [torch.as_tensor(np.asarray(p, np.float32), device=device).contiguous()
                       for p in params]
        self.w_bf16 = [to_bf16(self.master[2 * l]) for l in range(3)]
        self.m = [torch.zeros_like(p) for p in self.master]
        self.v = [torch.zeros_like(p) for p in self.master]
        self.step = 0
        self.mean = None
        self.inv_std = None
        self._bufs = {}
        # the library's view of the network (lsp_mlp) and of its Adam moments;
        # the tensors behind the pointers live as long as this object
        self.c_net = lsp.Mlp()
        self.c_net.dims[:] = list(self.dims)
        for l in range(3):
            self.c_net.w[l] = self.master[2 * l].data_ptr()
            self.c_net.b[l] = self.master[2 * l + 1].data_ptr()
            self.c_net.w_bf16[l] = self.w_bf16[l].data_ptr()
        self.c_m, self.c_v = self._c_grads(self.m), self._c_grads(self.v)
        self.grads = [torch.empty_like(p) for p in self.master]
        self.c_grads = self._c_grads(self.grads)

    @staticmethod
    def _c_grads(arrays):
        g = lsp.MlpGrads()
        for l in range(3):
            g.w[l] = arrays[2 * l].data_ptr()
            g.b[l] = arrays[2 * l + 1].data_ptr()
        return g

    # ------------------------------------------------------------- buffers
    def _buf(self, name, shape, dtype):
        b = self._bufs.get(name)
        if b is None or tuple(b.shape) != tuple(shape) or b.dtype != dtype:
            b = torch.empty(shape, dtype=dtype, device=self.device)
            self._bufs[name] = b
        return b

    # ------------------------------------------------------- standardising
    def normalize_rows(self, feats, stream=None):
        """In place: standardise each row's coarse block (lsp_row_normalize),
        if this network was built with row_norm.  Applied to every feature
        matrix before the column standardiser, in training and inference."""
        if self.row_norm:
            n, d = feats.shape
            _ok(lsp.lib().lsp_row_normalize(_p(feats), n, d, 0, lsp.FEAT_COARSE, _s(stream)),
                "lsp_row_normalize")
        return feats

    def fit_standardizer(self, feats, pool=lsp.FEAT_COARSE, stream=None):
        """Column means and scales from a training set; the first `pool`
        columns (the coarse spectrum, whose columns are shifted copies of each
        other) share one mean and scale."""
        n, d = feats.shape
        self.mean = torch.empty(d, dtype=torch.float32, device=self.device)
        self.inv_std = torch.empty(d, dtype=torch.float32, device=self.device)
        _ok(lsp.lib().lsp_col_stats(_p(feats), n, d, _p(self.mean), _p(self.inv_std),
                                    _s(stream)), "lsp_col_stats")
        if pool:
            _ok(lsp.lib().lsp_pool_stats(_p(self.mean), _p(self.inv_std), 0, int(pool),
                                         _s(stream)), "lsp_pool_stats")

    def standardize(self, feats, out=None, stream=None):
        n, d = feats.shape
        out = torch.empty((n, d), dtype=torch.int16, device=self.device) if out is None else out
        _ok(lsp.lib().lsp_standardize_bf16(_p(feats), n, d, _p(self.mean), _p(self.inv_std),
                                           _p(out), _s(stream)), "lsp_standardize_bf16")
        return out

    # ------------------------------------------------------------ forward
    def forward(self, x_bf16, logits=None, stream=None):
        """x_bf16: [n, 1088] int16 (BF16 bits).  Returns FP32 logits [n, 64]
        (lsp_mlp_forward; the hidden activations stay in this object's
        buffers for gradients)."""
        n = x_bf16.shape[0]
        d0, d1, d2, d3 = self.dims
        h1 = self._buf("h1", (n, d1), torch.int16)
        h2 = self._buf("h2", (n, d2), torch.int16)
        logits = torch.empty((n, d3), dtype=torch.float32, device=self.device) \
            if logits is None else logits
        _ok(lsp.lib().lsp_mlp_forward(ctypes.byref(self.c_net), _p(x_bf16), n, _p(h1), _p(h2),
                                      _p(logits), _s(stream)), "lsp_mlp_forward")
        return logits

    # ----------------------------------------------------------- training
    def gradients(self, x_bf16, labels, stream=None):
        """Forward + backward on one batch (lsp_mlp_forward, lsp_mlp_backward:
        the mean softmax cross-entropy over the batch); returns (loss rows,
        [dW1, db1, dW2, db2, dW3, db3])."""
        n = x_bf16.shape[0]
        logits = self.forward(x_bf16, stream=stream)
        h1, h2 = self._bufs["h1"], self._bufs["h2"]
        loss_rows = self._buf("loss", (n,), torch.float32)
        nb = int(lsp.lib().lsp_mlp_workspace_bytes(ctypes.byref(self.c_net), n))
        ws = self._buf("mlp_ws", (nb,), torch.uint8)
        _ok(lsp.lib().lsp_mlp_backward(ctypes.byref(self.c_net), _p(x_bf16), _p(labels), n,
                                       _p(h1), _p(h2), _p(logits), ctypes.c_float(1.0 / n),
                                       ctypes.byref(self.c_grads), _p(loss_rows), _p(ws), nb,
                                       _s(stream)), "lsp_mlp_backward")
        return loss_rows, self.grads

    def scratch_views(self, n):
        """Named views of the last lsp_mlp_backward workspace for n rows, in
        its documented layout: dlogits, dlogits_bf16, dz2, dz2b, dz1, dz1b."""
        ws = self._bufs["mlp_ws"]
        views, at = {}, 0
        for name, low, c in (("dlogits", "dlogits_bf16", self.dims[3]),
                             ("dz2", "dz2b", self.dims[2]), ("dz1", "dz1b", self.dims[1])):
            views[name] = ws[at:at + n * c * 4].view(torch.float32).view(n, c)
            at += -(-n * c * 4 // 256) * 256
            views[low] = ws[at:at + n * c * 2].view(torch.int16).view(n, c)
            at += -(-n * c * 2 // 256) * 256
        return views

    def train_step(self, x_bf16, labels, lr=1e-3, stream=None):
        loss_rows, _ = self.gradients(x_bf16, labels, stream=stream)
        self.step += 1
        _ok(lsp.lib().lsp_mlp_adam(ctypes.byref(self.c_net), ctypes.byref(self.c_grads),
                                   ctypes.byref(self.c_m), ctypes.byref(self.c_v), self.step,
                                   ctypes.c_float(lr), ctypes.c_float(0.9), ctypes.c_float(0.999),
                                   ctypes.c_float(1e-8), _s(stream)), "lsp_mlp_adam")
        return loss_rows

    def params_numpy(self):
        return [p.detach().cpu().numpy().astype(np.float64) for p in self.master]


def top_bands(logits, k=8, stream=None):
    """Indices of the k highest logits per row (decreasing) and their softmax mass."""
    n, c = logits.shape
    idx = torch.empty((n, k), dtype=torch.int32, device=logits.device)
    mass = torch.empty(n, dtype=torch.float32, device=logits.device)
    _ok(lsp.lib().lsp_top_k(_p(logits), n, c, k, _p(idx), _p(mass), _s(stream)), "lsp_top_k")
    return idx, mass


def peak_bands(peaks_raw, n, band_bins, n_bands, out=None, stream=None):
    """Training labels (band of each full-grid peak, -1 if none) via lsp_peak_bands."""
    out = torch.empty(n, dtype=torch.int32, device=peaks_raw.device) if out is None else out
    _ok(lsp.lib().lsp_peak_bands(_p(peaks_raw), int(n), int(band_bins), int(n_bands), _p(out),
                                 _s(stream)), "lsp_peak_bands")
    return out


def trim_bands(idx, n_net, logits, score, tau, alpha, out=None, kept_mass=None, stream=None):
    """lsp_trim_bands: per row of proposed bands idx [n x top], keep network
    slots (the first n_net) while the kept softmax mass is below tau and
    coarse slots whose band score reaches alpha times the row's largest;
    the others become -1 in out.  Returns (out, kept_mass)."""
    n, top = idx.shape
    c = (logits if logits is not None else score).shape[1]
    out = torch.empty_like(idx) if out is None else out
    _ok(lsp.lib().lsp_trim_bands(_p(idx), int(n), int(top), int(n_net), _p(logits), _p(score),
                                 int(c), ctypes.c_float(tau), ctypes.c_float(alpha), _p(out),
                                 _p(kept_mass), _s(stream)), "lsp_trim_bands")
    return out, kept_mass


def select_fallback(peaks_raw, mass, n, mass_min, power_min, objects, count, stream=None):
    """Objects to re-run on the whole grid (lsp_select_fallback); fills objects[:count]."""
    _ok(lsp.lib().lsp_select_fallback(_p(peaks_raw), _p(mass), int(n), ctypes.c_float(mass_min),
                                      ctypes.c_float(power_min), _p(objects), _p(count),
                                      _s(stream)), "lsp_select_fallback")


class BandGeometry:
    """n_bands equal bands of ceil(n_f / n_bands) bins (the last one may be shorter)."""

    def __init__(self, n_f, n_bands=64):
        self.n_f = int(n_f)
        self.n_bands = int(n_bands)
        self.band_bins = -(-self.n_f // self.n_bands)


class LearnedPeriodogram:
    """Peaks of a CSR batch from proposed bands (Section 3.4's batch peaks,
    computed on a fraction of the grid).

    For each object: features -> standardise -> network -> the `top` bands to
    refine (see propose), of which only the confident ones are kept (network
    bands until their softmax mass reaches tau, coarse-power bands whose
    score reaches alpha times the object's largest; lsp_trim_bands) -> the
    FP32 batch kernels on those bands only (row mode) -> objects whose
    proposal is uncertain (softmax mass of the refined network bands below
    mass_min) or whose refined peak is weak (power below power_min) are
    re-run on the whole grid.  Every step is a library kernel; the host only
    reads the number of fallback objects to size the last launch.
    ``method="generalized"`` refines (and falls back) with the generalized
    periodogram and errors ``dy`` (Section 4.11); the features are the same.
    """

    def __init__(self, net, geometry, offsets, t, y, f_min, f_max, unit=lsp.CYCLES, top=8,
                 mass_min=0.0, power_min=0.0, k=0, waves=0, proposal="hybrid", top_net=4,
                 method="standard", dy=None, alpha=0.0, tau=2.0):
        if proposal not in ("network", "coarse", "hybrid"):
            raise ValueError("proposal must be 'network', 'coarse' or 'hybrid'")
        self.net, self.geo, self.top = net, geometry, int(top)
        self.proposal = proposal
        self.top_net = int(top) if proposal == "network" else int(top_net)
        self.offsets, self.t, self.y = offsets, t, y
        self.n_obj = int(offsets.numel()) - 1
        self.mass_min, self.power_min = float(mass_min), float(power_min)
        self.alpha, self.tau = float(alpha), float(tau)
        dev = t.device
        self.feat = lsp.Features(offsets, t, y, f_min, f_max, unit=unit)
        self.x = torch.empty((self.n_obj, net.dims[0]), dtype=torch.int16, device=dev)
        self.logits = torch.empty((self.n_obj, net.dims[-1]), dtype=torch.float32, device=dev)
        self.idx = torch.empty((self.n_obj, self.top), dtype=torch.int32, device=dev)
        self.rows = torch.empty((self.n_obj, self.top), dtype=torch.int32, device=dev)
        self.idx_net = torch.empty((self.n_obj, self.top_net), dtype=torch.int32, device=dev)
        self.idx_coarse = torch.empty((self.n_obj, self.top), dtype=torch.int32, device=dev)
        self.band_score = torch.empty((self.n_obj, geometry.n_bands), dtype=torch.float32,
                                      device=dev)
        self.mass = torch.empty(self.n_obj, dtype=torch.float32, device=dev)
        self.peaks_raw = torch.empty(self.n_obj * lsp.PEAK_BYTES, dtype=torch.uint8, device=dev)
        self.objects = torch.empty(self.n_obj, dtype=torch.int32, device=dev)
        self.count = torch.zeros(1, dtype=torch.int32, device=dev)
        self.refine = lsp.Rows(offsets, t, y, f_min, f_max, geometry.n_f, None,
                               self.rows.view(-1), geometry.band_bins, self.top, unit=unit,
                               form=lsp.FORM_FP32P, peaks=self.peaks_raw, k=k, waves=waves,
                               method=method, dy=dy)
        self.full = lsp.Rows(offsets, t, y, f_min, f_max, geometry.n_f, self.objects, None, 0, 1,
                             unit=unit, form=lsp.FORM_FP32P, peaks=self.peaks_raw, k=k,
                             waves=waves, max_rows=self.n_obj, method=method, dy=dy)
        self.n_fallback = 0

    def propose(self, stream=None):
        """Features, network and top bands; fills self.idx (the `top`
        proposed bands), self.rows (those kept, -1 for the others) and
        self.mass (the network's softmax mass on its kept picks).

        proposal="network": the network's `top` most probable bands.
        proposal="coarse": the `top` bands whose pooled coarse power peaks
        highest (no network).  proposal="hybrid": the network's `top_net`
        bands, then coarse-power bands not already taken, up to `top`."""
        L = lsp.lib()
        n, nb = self.n_obj, self.geo.n_bands
        feats = self.net.normalize_rows(self.feat(stream), stream=stream)
        net = self.proposal != "coarse"  # "coarse": the method without the network
        if net:
            self.net.standardize(feats, out=self.x, stream=stream)
            self.net.forward(self.x, logits=self.logits, stream=stream)
            first = self.idx if self.proposal == "network" else self.idx_net
            _ok(L.lsp_top_k(_p(self.logits), n, nb, self.top_net, _p(first), None,
                            _s(stream)), "lsp_top_k")
        if self.proposal != "network":
            # row normalisation is increasing within a row, so band maxima of
            # the normalised coarse block rank bands as the raw power does
            _ok(L.lsp_band_max(_p(feats), n, feats.shape[1], 0, nb, lsp.FEAT_COARSE // nb,
                               _p(self.band_score), _s(stream)), "lsp_band_max")
            target = self.idx if self.proposal == "coarse" else self.idx_coarse
            _ok(L.lsp_top_k(_p(self.band_score), n, nb, self.top, _p(target), None, _s(stream)),
                "lsp_top_k")
        if self.proposal == "hybrid":
            _ok(L.lsp_merge_bands(_p(self.idx_net), self.top_net, _p(self.idx_coarse), self.top,
                                  n, self.top, _p(self.idx), _s(stream)), "lsp_merge_bands")
        self.trim(self.alpha, self.tau, stream)

    @property
    def n_net(self):
        """Proposed slots that come from the network (the first ones)."""
        return {"network": self.top, "coarse": 0, "hybrid": self.top_net}[self.proposal]

    def trim(self, alpha, tau, stream=None):
        """Keep the confident proposed bands (lsp_trim_bands) in self.rows."""
        net = self.proposal != "coarse"
        trim_bands(self.idx, self.n_net, self.logits if net else None,
                   self.band_score if self.proposal != "network" else None, tau, alpha,
                   out=self.rows, kept_mass=self.mass if net else None, stream=stream)

    def refine_only(self, stream=None):
        self.propose(stream)
        self.refine(stream)
        return self

    def __call__(self, stream=None):
        self.refine_only(stream)
        # the coarse rule has no proposal mass: only the refined power decides
        mass = None if self.proposal == "coarse" else self.mass
        select_fallback(self.peaks_raw, mass, self.n_obj, self.mass_min, self.power_min,
                        self.objects, self.count, stream)
        n = int(self.count.item())  # synchronises: sizes the fallback launch
        self.n_fallback = n
        if n:
            self.full.set_rows(self.objects[:n])
            self.full(stream)
        return self

    def peaks(self):
        return self.peaks_raw.cpu().numpy().view(lsp.PEAK_DTYPE).copy()


def shift_bands(x, labels, shifts, n_bands, out=None, out_labels=None, stream=None):
    """lsp_shift_bands on BF16 rows: move the coarse spectrum by shifts[i] bands."""
    n, d = x.shape
    out = torch.empty_like(x) if out is None else out
    out_labels = torch.empty_like(labels) if out_labels is None else out_labels
    group = lsp.FEAT_COARSE // n_bands
    _ok(lsp.lib().lsp_shift_bands(_p(x), _p(labels), _p(shifts), n, d, lsp.FEAT_COARSE, group,
                                  n_bands, ctypes.c_float(0.0), _p(out), _p(out_labels),
                                  _s(stream)), "lsp_shift_bands")
    return out, out_labels


def train_proposer(net, feats, labels, epochs=20, batch=1024, lr=1e-3, lr_final=1e-4,
                   augment=0.5, seed=0, log=None, stream=None):
    """Adam on softmax cross-entropy over contiguous minibatches (the synthetic
    training objects are drawn independently, so their order is already random);
    the learning rate decays geometrically from lr to lr_final.  Fits the
    standardiser first (the coarse spectrum pooled to one scale, which is
    what makes shifted copies comparable).

    With augment > 0, that fraction of each minibatch has its coarse spectrum
    moved so that its label becomes a band drawn uniformly (lsp_shift_bands;
    the draws come from a seeded host generator).  `feats` is row-normalised
    in place first when the network uses row normalisation.  Returns the mean loss of
    each epoch."""
    n = feats.shape[0]
    n_bands = net.dims[-1]
    net.normalize_rows(feats, stream=stream)  # in place
    net.fit_standardizer(feats, stream=stream)
    x = net.standardize(feats, stream=stream)
    steps = max(1, (n // batch)) * epochs
    decay = (lr_final / lr) ** (1.0 / max(1, steps - 1))
    rate = lr
    rng = np.random.default_rng(seed)
    lab_host = labels.cpu().numpy()
    xa = torch.empty((batch, x.shape[1]), dtype=x.dtype, device=x.device)
    la = torch.empty(batch, dtype=torch.int32, device=x.device)
    hist = []
    for ep in range(epochs):
        tot = torch.zeros((), dtype=torch.float32, device=feats.device)
        nb = 0
        for b0 in range(0, n - batch + 1, batch):
            xb, lb = x[b0:b0 + batch], labels[b0:b0 + batch]
            if augment > 0:
                lab = lab_host[b0:b0 + batch]
                target = rng.integers(0, n_bands, batch)
                move = (rng.random(batch) < augment) & (lab >= 0)
                sh = np.where(move, target - lab, 0).astype(np.int32)
                shifts = torch.as_tensor(sh, device=x.device)
                xb, lb = shift_bands(xb, lb, shifts, n_bands, out=xa, out_labels=la,
                                     stream=stream)
            loss_rows = net.train_step(xb, lb, lr=rate, stream=stream)
            tot += loss_rows.sum()
            nb += 1
            rate *= decay
        hist.append(float(tot.item()) / max(1, nb * batch))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4f}")
    return hist


def calibrate(refined, full, mass, target=0.999, weights=None):
    """Thresholds (mass_min, power_min) that keep the recovery rate on a
    validation set at or above `target` with the fewest fallbacks (or, with
    `weights`, the least total weight of fallback objects -- e.g. their
    observation counts, to which a whole-grid re-run is proportional).
    Returns (mass_min, power_min, number of fallbacks).

    refined, full: peak arrays (refine only, whole grid); mass: proposal mass
    (None for a rule that has none).
    An object is recovered if its refined peak is within one bin of the
    whole-grid peak; a fallback object is recovered by construction."""
    mm, pm, n_fb, _ = _calibrate(refined, full, mass, target, weights)
    return mm, pm, n_fb


def _calibrate(refined, full, mass, target, weights, n_quantiles=101):
    """calibrate, also returning the fallback weight.  For each mass
    threshold, every power threshold is scored at once: the misses are the
    unrecovered objects at or above it, the fallbacks those below it."""
    ok = full["status"] == 0
    hit = ok & (np.abs(refined["index"] - full["index"]) <= 1)
    n = int(ok.sum())
    if n == 0:
        return 0.0, 0.0, 0, 0.0
    allowed = int(np.floor((1.0 - target) * n))
    pw = np.where(np.isfinite(refined["power"]), refined["power"], -1.0)
    w = np.ones(len(refined)) if weights is None else np.asarray(weights, np.float64)
    q = np.linspace(0.0, 1.0, n_quantiles)
    if mass is None:  # a rule without proposal mass: only the power threshold
        mass = np.ones(len(refined), np.float32)
        m_grid = np.zeros(1)
    else:
        m_grid = np.unique(np.concatenate([[0.0], np.quantile(mass[ok], q), [2.0]]))
    p_grid = np.unique(np.concatenate([[0.0], np.quantile(pw[ok], q), [2.0]]))
    best = (2.0, 2.0, n + 1, np.inf)
    for mm in m_grid:
        base = ok & ((mass < mm) | (refined["index"] < 0))  # fall back whatever the power
        cand = ok & ~base                                    # fall back iff power < pm
        miss_pw = np.sort(pw[cand & ~hit])
        miss = len(miss_pw) - np.searchsorted(miss_pw, p_grid, side="left")
        order = np.argsort(pw[cand], kind="stable")
        cand_pw = pw[cand][order]
        cum_w = np.concatenate([[0.0], np.cumsum(w[cand][order])])
        below = np.searchsorted(cand_pw, p_grid, side="left")
        fb_w = float(w[base].sum()) + cum_w[below]
        key = np.where(miss <= allowed, fb_w, np.inf)
        j = int(np.argmin(key))
        if key[j] < best[3]:
            best = (float(mm), float(p_grid[j]), int(base.sum() + below[j]), float(key[j]))
    return best


def _group_peaks(index, power, kept):
    """Peak of each object over its kept slots: highest power, lowest bin on
    ties (the order the row-mode kernels merge a group's rows in)."""
    pw = np.where(kept & (index >= 0), power, -np.inf)
    m = pw.max(axis=1)
    at_max = (pw == m[:, None]) & np.isfinite(m)[:, None]
    idx = np.where(at_max, index, np.iinfo(np.int64).max).min(axis=1)
    out = np.zeros(len(index), lsp.PEAK_DTYPE)
    out["index"] = np.where(np.isfinite(m), idx, -1)
    out["power"] = np.where(np.isfinite(m), m, np.nan)
    return out


ALPHAS = (0.0, 0.3, 0.5, 0.6, 0.7, 0.8, 0.85, 0.9, 0.95, 0.98, 1.0)
TAUS = (2.0, 0.999, 0.99, 0.98, 0.95, 0.9, 0.8, 0.7, 0.6, 0.5)


def calibrate_bands(lp, full, n_t, target=0.999, alphas=ALPHAS, taus=TAUS, log=None):
    """Band trimming and fallback thresholds for one proposal rule, chosen on
    a validation set: the (alpha, tau, mass_min, power_min) that evaluate the
    fewest (observation, bin) terms -- kept bands of every object plus the
    whole grid of every fallback object -- with at least `target` of the
    objects recovering their whole-grid peak within one bin.

    lp: a LearnedPeriodogram over the validation objects (its proposals are
    computed here); full: their whole-grid peaks; n_t: their observation
    counts.  Every proposed slot's band is refined on its own once (row mode,
    one row per object); each candidate trimming then picks its objects'
    peaks from those, with the kernels' own keep decisions (lsp_trim_bands).
    Returns ((mass_min, power_min, fallbacks, alpha, tau), evaluated fraction
    of the whole grid)."""
    geo = lp.geo
    lp.propose()
    n, top = lp.idx.shape
    slot_index = np.full((n, top), -1, np.int64)
    slot_power = np.full((n, top), -np.inf)
    for r in range(top):
        col = lp.idx[:, r].contiguous()
        rows = lsp.Rows(lp.offsets, lp.t, lp.y, lp.refine.grid.f_min, lp.refine.grid.f_max,
                        geo.n_f, None, col, geo.band_bins, 1, unit=lp.refine.grid.unit,
                        form=lsp.FORM_FP32P, method="generalized" if lp.refine.gen else "standard",
                        dy=lp.refine.dy)
        rows()
        pk = rows.peaks()
        slot_index[:, r] = pk["index"]
        slot_power[:, r] = np.where(np.isfinite(pk["power"]), pk["power"], -np.inf)
        del rows
    idx = lp.idx.cpu().numpy().astype(np.int64)
    bins = np.where(idx >= 0, np.minimum(geo.band_bins, geo.n_f - idx * geo.band_bins), 0)
    n_t = np.asarray(n_t, np.float64)
    whole = float(n_t.sum()) * geo.n_f
    net = lp.proposal != "coarse"
    a_grid = alphas if lp.proposal != "network" else (0.0,)
    t_grid = taus if net else (2.0,)
    best = None
    for a in a_grid:
        for tau in t_grid:
            lp.trim(a, tau)
            kept = lp.rows.cpu().numpy() >= 0
            mass = lp.mass.cpu().numpy() if net else None
            refined = _group_peaks(slot_index, slot_power, kept)
            refine_terms = float(np.sum(n_t * np.sum(kept * bins, axis=1)))
            mm, pm, n_fb, fb_w = _calibrate(refined, full, mass, target, n_t, n_quantiles=51)
            total = refine_terms + fb_w * geo.n_f
            if best is None or total < best[0]:
                best = (total, (mm, pm, n_fb, float(a), float(tau)))
    lp.trim(best[1][3], best[1][4])
    if log:
        mm, pm, n_fb, a, tau = best[1]
        log(f"calibrated {lp.proposal}: alpha={a} tau={tau} mass_min={mm:.4f} "
            f"power_min={pm:.4f}, {n_fb}/{n} validation fallbacks, evaluated "
            f"{best[0] / whole:.4f} of the grid")
    return best[1], best[0] / whole


def _tensors(w, device):
    return (torch.as_tensor(w.offsets, device=device), torch.as_tensor(w.t, device=device),
            torch.as_tensor(w.y, device=device))


def _errors(w, device, method):
    return torch.as_tensor(w.dy, device=device) if method == "generalized" else None


def whole_grid_peaks(w, tensors, method="standard", dy=None):
    """Peaks of a whole CSR batch on its full grid (FP32 form): the labels of
    training and the reference of calibration."""
    off, t, y = tensors
    p = lsp.Periodogram(t, y, w.f_min, w.f_max, w.n_f, offsets=off, form=lsp.FORM_FP32P,
                        pgram=False, unit=w.unit, method=method, dy=dy)
    p()
    return p


class Proposer:
    """A trained band-proposal network with its band geometry and the fallback
    thresholds calibrated for each proposal rule (see fit_proposer)."""

    def __init__(self, net, geometry, thresholds, history, train_seconds, n_train, n_val):
        self.net, self.geo = net, geometry
        # proposal -> (mass_min, power_min, validation fallbacks, alpha, tau)
        self.thresholds = thresholds
        self.history = history
        self.train_seconds = train_seconds
        self.n_train, self.n_val = n_train, n_val

    def periodogram(self, offsets, t, y, f_min, f_max, unit=lsp.CYCLES, proposal="hybrid",
                    method="standard", dy=None, **kw):
        mass_min, power_min, _, alpha, tau = self.thresholds[proposal]
        return LearnedPeriodogram(self.net, self.geo, offsets, t, y, f_min, f_max, unit=unit,
                                  mass_min=mass_min, power_min=power_min, proposal=proposal,
                                  method=method, dy=dy, alpha=alpha, tau=tau, **kw)


def fit_proposer(make, device, n_train=40000, n_val=20000, seed_train=None, seed_val=None,
                 n_bands=64, method="standard", proposals=("hybrid",), epochs=30, batch=512,
                 target=0.999, net_seed=7, log=None, adaptive=True):
    """Train the proposal network on objects the method itself labels, then
    calibrate the fallback thresholds on independent objects.

    make(n_obj, seed) returns a synthetic Workload of the target population
    (its grid is the grid the proposals are for).  Training labels are the
    bands of the whole-grid FP32 peaks of n_train objects; for every rule in
    `proposals` the thresholds are chosen on n_val other objects so that at
    least `target` of them recover the whole-grid peak within one bin: with
    `adaptive`, jointly with the band trimming, for the fewest evaluated
    terms (calibrate_bands); otherwise for all `top` bands and the fewest
    fallbacks (calibrate)."""
    import time

    wtr = make(n_train, seed_train)
    geo = BandGeometry(wtr.n_f, n_bands)
    ttr = _tensors(wtr, device)
    feats = lsp.Features(*ttr, wtr.f_min, wtr.f_max, unit=wtr.unit)()
    ptr = whole_grid_peaks(wtr, ttr, method, _errors(wtr, device, method))
    labels = peak_bands(ptr.peaks_raw, wtr.n_obj, geo.band_bins, geo.n_bands)
    net = BandNet(device, seed=net_seed, dims=DIMS[:-1] + (n_bands,))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = train_proposer(net, feats, labels, epochs=epochs, batch=batch, lr=1e-3,
                          lr_final=3e-5, augment=0.9)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    if log:
        log(f"trained on {wtr.n_obj} objects in {train_s:.1f} s, loss {hist[0]:.3f} -> "
            f"{hist[-1]:.3f}")
    del feats, ptr, ttr, labels
    wva = make(n_val, seed_val)
    tva = _tensors(wva, device)
    dva = _errors(wva, device, method)
    full = whole_grid_peaks(wva, tva, method, dva).peaks()
    n_t = np.diff(wva.offsets)
    thresholds = {}
    for prop in proposals:
        lpv = LearnedPeriodogram(net, geo, *tva, wva.f_min, wva.f_max, unit=wva.unit,
                                 proposal=prop, method=method, dy=dva)
        if adaptive:
            thresholds[prop], _ = calibrate_bands(lpv, full, n_t, target=target, log=log)
        else:
            lpv.refine_only()
            mass = None if prop == "coarse" else lpv.mass.cpu().numpy()
            thresholds[prop] = calibrate(lpv.peaks(), full, mass, target=target) + (0.0, 2.0)
            if log:
                mm, pm, nfb = thresholds[prop][:3]
                log(f"calibrated {prop}: mass_min={mm:.4f} power_min={pm:.4f}, "
                    f"{nfb}/{wva.n_obj} validation fallbacks")
        del lpv
    return Proposer(net, geo, thresholds, hist, train_s, wtr.n_obj, wva.n_obj)
