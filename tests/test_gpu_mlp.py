"""Band-proposal network kernels vs the CPU reference (needs an MI355X)."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mlp_ref  # noqa: E402
from paper_2105_04006_amd import learned, lsp  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


U32 = 2.0 ** -24  # FP32 unit roundoff


def gamma(k):
    """Bound factor of a k-term FP32 sum in any order (products exact)."""
    return k * U32 / (1.0 - k * U32)


def bits(a, dev):
    return torch.as_tensor(mlp_ref.bf16_bits(a).view(np.int16), device=dev)


@pytest.mark.parametrize("M,N,K", [(64, 64, 32), (200, 130, 100), (37, 70, 1088), (1, 5, 3)])
def test_gemm_plain_and_transposed(dev, M, N, K):
    rng = np.random.default_rng(M * 1000 + N)
    A = mlp_ref.bf16_round(rng.normal(size=(M, K)))
    B = mlp_ref.bf16_round(rng.normal(size=(K, N)))
    ref = A @ B
    # BF16 products are exact in FP32; the K-term FP32 accumulation, in any
    # order, is within gamma(K) sum |a||b| of the exact sum
    tol = gamma(K) * (np.abs(A) @ np.abs(B))
    C = torch.empty((M, N), dtype=torch.float32, device=dev)
    say(f"gemm {M}x{N}x{K}")
    learned.gemm(bits(A, dev), bits(B, dev), M, N, K, K, 1, N, 1, C=C)
    torch.cuda.synchronize()
    assert np.all(np.abs(C.cpu().numpy() - ref) <= tol)
    # the same product from transposed storage of both operands
    At, Bt = bits(np.ascontiguousarray(A.T), dev), bits(np.ascontiguousarray(B.T), dev)
    C2 = torch.empty((M, N), dtype=torch.float32, device=dev)
    learned.gemm(At, Bt, M, N, K, 1, M, 1, K, C=C2)
    torch.cuda.synchronize()
    assert np.all(np.abs(C2.cpu().numpy() - ref) <= tol)


def test_gemm_epilogues(dev):
    rng = np.random.default_rng(7)
    M, N, K = 150, 96, 64
    A = mlp_ref.bf16_round(rng.normal(size=(M, K)))
    B = mlp_ref.bf16_round(rng.normal(size=(K, N)))
    bias = rng.normal(size=N).astype(np.float32)
    mask = mlp_ref.bf16_round(rng.normal(size=(M, N)))
    Cf = torch.empty((M, N), dtype=torch.float32, device=dev)
    Cb = torch.empty((M, N), dtype=torch.int16, device=dev)
    learned.gemm(bits(A, dev), bits(B, dev), M, N, K, K, 1, N, 1, C=Cf, C_bf16=Cb,
                 bias=torch.as_tensor(bias, device=dev), relu=True)
    torch.cuda.synchronize()
    ref = np.maximum(A @ B + bias, 0.0)
    # K products and the bias in FP32; ReLU does not enlarge the error
    tol = gamma(K + 1) * (np.abs(A) @ np.abs(B) + np.abs(bias))
    assert np.all(np.abs(Cf.cpu().numpy() - ref) <= tol)
    cb = mlp_ref.from_bf16_bits(Cb.cpu().numpy().view(np.uint16))
    assert np.array_equal(cb, mlp_ref.bf16_round(Cf.cpu().numpy()))
    learned.gemm(bits(A, dev), bits(B, dev), M, N, K, K, 1, N, 1, C=Cf, mask=bits(mask, dev))
    torch.cuda.synchronize()
    ref = (A @ B) * (mask > 0)
    assert np.all(np.abs(Cf.cpu().numpy() - ref) <= gamma(K) * (np.abs(A) @ np.abs(B)))


def test_small_kernels(dev):
    rng = np.random.default_rng(11)
    n, c = 37, 64
    z = rng.normal(size=(n, c)).astype(np.float32) * 3
    lab = rng.integers(0, c, size=n).astype(np.int32)
    lab[[3, 17]] = -1      # ignored rows
    lab[30] = c
    zt = torch.as_tensor(z, device=dev)
    g = torch.empty_like(zt)
    loss = torch.empty(n, dtype=torch.float32, device=dev)
    L = lsp.lib()
    p = learned._p
    assert L.lsp_softmax_xent(p(zt), p(torch.as_tensor(lab, device=dev)), n, c,
                              ctypes.c_float(1.0 / n), p(g), None, p(loss), None) == 0
    ref_loss, ref_g = mlp_ref.softmax_xent(z.astype(np.float64), lab)
    torch.cuda.synchronize()
    # FP32 softmax of exact FP32 logits: expf of z - max ((|z - max| + 1) u),
    # the 64-term sum and the division (72 u in all, relative to p), the
    # subtraction at the label and the scaling by 1/n; the loss row's
    # logarithm and additions (70 + 3 |loss|) u
    zz = z.astype(np.float64) - z.max(axis=1, keepdims=True)
    pr = np.exp(zz)
    pr /= pr.sum(axis=1, keepdims=True)
    keep = (lab >= 0) & (lab < c)
    rows = np.arange(n)[keep]
    loss_rows = np.zeros(n)
    loss_rows[rows] = -np.log(pr[rows, lab[keep]])
    assert np.all(np.abs(loss.cpu().numpy() - loss_rows) <= U32 * (70.0 + 3.0 * loss_rows))
    e_g = ((np.abs(zz) + 72.0) * U32 * pr + 2.0 * U32 + U32 * np.abs(ref_g * n)) / n
    assert np.all(np.abs(g.cpu().numpy() - ref_g) <= np.where(keep[:, None], e_g, 0.0))
    cs = torch.empty(c, dtype=torch.float32, device=dev)
    assert L.lsp_col_sums(p(zt), n, c, p(cs), None) == 0
    torch.cuda.synchronize()
    # FP32 column sums, any order
    assert np.all(np.abs(cs.cpu().numpy() - z.astype(np.float64).sum(axis=0))
                  <= gamma(n) * np.abs(z).astype(np.float64).sum(axis=0))
    mean = torch.empty(c, dtype=torch.float32, device=dev)
    inv = torch.empty(c, dtype=torch.float32, device=dev)
    assert L.lsp_col_stats(p(zt), n, c, p(mean), p(inv), None) == 0
    torch.cuda.synchronize()
    # FP64 two-pass statistics rounded once to FP32: half an FP32 ulp, plus
    # the FP64 sums' own error (n 2^-53 relative, far below it)
    zd = z.astype(np.float64)
    assert np.all(np.abs(mean.cpu().numpy() - zd.mean(axis=0))
                  <= U32 * np.abs(zd.mean(axis=0)) + n * 2.0 ** -53 * np.abs(zd).mean(axis=0))
    want_inv = 1.0 / zd.std(axis=0)
    assert np.all(np.abs(inv.cpu().numpy() - want_inv) <= (U32 + (n + 4) * 2.0 ** -53) * want_inv)
    idx, mass = learned.top_bands(zt, k=8)
    torch.cuda.synchronize()
    order = np.argsort(-z, axis=1, kind="stable")[:, :8]
    assert np.array_equal(idx.cpu().numpy(), order)
    e = np.exp(z - z.max(axis=1, keepdims=True))
    pm = e / e.sum(axis=1, keepdims=True)
    # 8 FP32 softmax probabilities (as above) and their FP32 sum
    want_mass = np.take_along_axis(pm, order, 1).sum(1)
    e_mass = (np.abs(z - z.max(axis=1, keepdims=True)).max(axis=1) + 80.0) * U32 * want_mass
    assert np.all(np.abs(mass.cpu().numpy() - want_mass) <= e_mass)


def bf16_of(h):
    """BF16 bits (int16 tensor) -> float64 numpy values."""
    return mlp_ref.from_bf16_bits(h.cpu().numpy().view(np.uint16))


def check_store(got, z, e, what):
    """A BF16 store of an FP32 result: got must be a round-to-nearest BF16 value
    of some number within e of the FP64 value z, so |got - z| <= e + half a
    BF16 ulp of (|z| + e), i.e. <= e + 2^-8 (|z| + e); where z is not within e
    of a rounding boundary the two must agree exactly (counted, not asserted)."""
    lim = e + 2.0 ** -8 * (np.abs(z) + e)
    err = np.abs(got - z)
    same = float(np.mean(got == mlp_ref.bf16_round(z)))
    say(f"  {what}: max |d| / bound {np.max(err / np.maximum(lim, 1e-300)):.3g}, "
        f"equal to the rounded FP64 value: {same:.4f}")
    assert np.all(err <= lim), what


def check_sum(got, z, e, what):
    err = np.abs(got - z)
    say(f"  {what}: max |d| / bound {np.max(err / np.maximum(e, 1e-300)):.3g}")
    assert np.all(err <= e), what


def test_training_step_matches_reference(dev):
    """One forward/backward step of the full-size network, checked stage by
    stage: every GEMM, softmax and column sum against FP64 arithmetic on the
    exact BF16/FP32 operands the GPU itself stored for that stage.

    Bounds, per element (u = 2^-24): a K-term product (plus bias) accumulated
    in FP32 is within gamma(K + 1) (|A| |B| + |bias|) of its FP64 value, the
    BF16 operands' products being exact in FP32; a BF16 store of such a result
    adds at most half a BF16 ulp (check_store); conversions of the GPU's own
    FP32 values to BF16 are exact roundings; softmax gradients move by at
    most 2 p_i max_k |dz_k| / n under logit errors dz, plus FP32 rounding
    of exp(z - max) (u |z - max| for the argument, 1 ulp for expf), of the
    64-term sum and of the division ((|z - max| + 72) u p_i / n), and of the
    subtraction and scaling (u |p - onehot| + 2u at the label); the loss row,
    log-sum-exp minus the label's logit, by at most 2 max_k |dz_k| plus
    (70 + 3 |loss|) u.  Then one Adam step moves every parameter by at most
    lr."""
    rng = np.random.default_rng(5)
    n = 96
    d0, d1, d2, d3 = mlp_ref.DIMS
    params = mlp_ref.init_params(9)
    for pp in params[1::2]:
        pp += rng.normal(0, 0.05, size=pp.shape)
    x = mlp_ref.bf16_round(rng.normal(size=(n, d0)))
    labels = rng.integers(0, d3, size=n).astype(np.int32)
    net = learned.BandNet(dev, params=params)
    xb = bits(x, dev)
    lab = torch.as_tensor(labels, device=dev)
    loss_rows, grads = net.gradients(xb, lab)
    torch.cuda.synchronize()
    B = dict(net._bufs)
    B.update(net.scratch_views(n))
    W1, W2, W3 = (bf16_of(w) for w in net.w_bf16)
    b1, b2, b3 = (net.master[i].double().cpu().numpy() for i in (1, 3, 5))
    a = np.abs
    # forward
    h1 = bf16_of(B["h1"])
    z1 = x @ W1 + b1
    check_store(h1, np.maximum(z1, 0.0), gamma(d0 + 1) * (a(x) @ a(W1) + a(b1)), "h1")
    h2 = bf16_of(B["h2"])
    z2 = h1 @ W2 + b2
    check_store(h2, np.maximum(z2, 0.0), gamma(d1 + 1) * (a(h1) @ a(W2) + a(b2)), "h2")
    z3 = h2 @ W3 + b3
    e3 = gamma(d2 + 1) * (a(h2) @ a(W3) + a(b3))
    zz = z3 - z3.max(axis=1, keepdims=True)
    p = np.exp(zz)
    p /= p.sum(axis=1, keepdims=True)
    emax = e3.max(axis=1, keepdims=True)
    ref_rows = np.log(np.exp(zz).sum(axis=1)) - zz[np.arange(n), labels]
    check_sum(loss_rows.double().cpu().numpy(), ref_rows,
              2.0 * emax[:, 0] + U32 * (70.0 + 3.0 * a(ref_rows)), "loss rows")
    g3 = B["dlogits"].double().cpu().numpy()
    onehot = np.zeros((n, d3))
    onehot[np.arange(n), labels] = 1.0
    e_p = 2.0 * p * emax + (a(zz) + 72.0) * U32 * p  # logits error; expf, 64-term sum, divide
    check_sum(g3, (p - onehot) / n, (e_p + 2.0 * U32 * onehot + U32 * a(p - onehot)) / n,
              "softmax gradient")
    g3b = bf16_of(B["dlogits_bf16"])
    assert np.array_equal(g3b, mlp_ref.bf16_round(g3)), "g3 -> BF16"
    # backward: each gradient from the GPU's own stored operands
    dW1, db1, dW2, db2, dW3, db3 = (g.double().cpu().numpy() for g in grads)
    check_sum(dW3, h2.T @ g3b, gamma(n) * (a(h2).T @ a(g3b)), "dW3")
    check_sum(db3, g3.sum(axis=0), gamma(n) * a(g3).sum(axis=0), "db3")
    dz2 = B["dz2"].double().cpu().numpy()
    u2 = g3b @ W3.T
    check_sum(dz2, u2 * (h2 > 0), gamma(d3) * (a(g3b) @ a(W3.T)) * (h2 > 0), "dz2")
    dz2b = bf16_of(B["dz2b"])
    assert np.array_equal(dz2b, mlp_ref.bf16_round(dz2)), "dz2 -> BF16"
    check_sum(dW2, h1.T @ dz2b, gamma(n) * (a(h1).T @ a(dz2b)), "dW2")
    check_sum(db2, dz2.sum(axis=0), gamma(n) * a(dz2).sum(axis=0), "db2")
    dz1 = B["dz1"].double().cpu().numpy()
    u1 = dz2b @ W2.T
    check_sum(dz1, u1 * (h1 > 0), gamma(d2) * (a(dz2b) @ a(W2.T)) * (h1 > 0), "dz1")
    dz1b = bf16_of(B["dz1b"])
    assert np.array_equal(dz1b, mlp_ref.bf16_round(dz1)), "dz1 -> BF16"
    check_sum(dW1, x.T @ dz1b, gamma(n) * (a(x).T @ a(dz1b)), "dW1")
    check_sum(db1, dz1.sum(axis=0), gamma(n) * a(dz1).sum(axis=0), "db1")
    # the end-to-end distance to the BF16-emulated reference run of the same
    # step (informative: rounding choices may differ near BF16 boundaries)
    bparams = [mlp_ref.bf16_round(q) if i % 2 == 0 else q.astype(np.float32).astype(np.float64)
               for i, q in enumerate(params)]
    logits, cache = mlp_ref.forward(bparams, x, bf16=True)
    _, dl = mlp_ref.softmax_xent(logits, labels)
    for name, g, r in zip(["dW1", "db1", "dW2", "db2", "dW3", "db3"],
                          (dW1, db1, dW2, db2, dW3, db3),
                          mlp_ref.backward(bparams, cache, dl, bf16=True)):
        say(f"  end to end {name}: max |d| / max |ref| "
            f"{np.max(a(g - r)) / (np.max(a(r)) + 1e-12):.3g}")
    before = [q.clone() for q in net.master]
    net.train_step(xb, lab, lr=1e-3)
    torch.cuda.synchronize()
    for b, q in zip(before, net.master):
        d = (q - b).abs().max().item()
        assert 0.0 < d <= 1.01e-3  # the first Adam step moves each parameter by <= lr


def test_peak_bands_and_fallback_selection(dev):
    rng = np.random.default_rng(12)
    n = 5000
    pk = np.zeros(n, lsp.PEAK_DTYPE)
    pk["index"] = rng.integers(0, 6400, n)
    pk["power"] = rng.uniform(0, 1, n)
    pk["status"] = 0
    pk["status"][[5, 77, 4000]] = [1, 2, 3]
    pk["index"][[5, 77, 4000]] = -1
    pk["index"][[9, 11]] = -1          # no peak found although status OK
    pk["power"][13] = np.nan
    mass = rng.uniform(0, 1, n).astype(np.float32)
    raw = torch.as_tensor(pk.view(np.uint8), device=dev)
    mt = torch.as_tensor(mass, device=dev)
    L = lsp.lib()
    p = learned._p
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    assert L.lsp_peak_bands(p(raw), n, 100, 64, p(labels), None) == 0
    want = np.where((pk["status"] == 0) & (pk["index"] >= 0), pk["index"] // 100, -1)
    torch.cuda.synchronize()
    assert np.array_equal(labels.cpu().numpy(), want)
    objs = torch.full((n,), -5, dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    for mmin, pmin, use_mass in ((0.6, 0.3, True), (0.0, 0.0, False), (2.0, 0.0, True)):
        assert L.lsp_select_fallback(p(raw), p(mt) if use_mass else None, n,
                                     ctypes.c_float(mmin), ctypes.c_float(pmin), p(objs), p(cnt),
                                     None) == 0
        torch.cuda.synchronize()
        ok = pk["status"] == 0
        need = ok & ((pk["index"] < 0) | ~(pk["power"] >= np.float32(pmin)))
        if use_mass:
            need |= ok & ~(mass >= np.float32(mmin))
        sel = np.nonzero(need)[0]
        k = int(cnt.item())
        assert k == len(sel)
        assert np.array_equal(objs.cpu().numpy()[:k], sel)


def test_row_normalize_pool_stats_and_shift(dev):
    rng = np.random.default_rng(13)
    n, d = 300, 1088
    x = rng.gamma(2.0, 0.1, size=(n, d)).astype(np.float32)
    x[7, :1024] = 0.25  # a constant coarse block
    xt = torch.as_tensor(x, device=dev)
    L = lsp.lib()
    p = learned._p
    assert L.lsp_row_normalize(p(xt), n, d, 0, 1024, None) == 0
    torch.cuda.synchronize()
    c = x[:, :1024].astype(np.float64)
    sd = c.std(axis=1, keepdims=True)
    want = np.where(sd > 0, (c - c.mean(axis=1, keepdims=True)) / np.where(sd > 0, sd, 1), 0.0)
    got = xt.cpu().numpy()
    # FP64 statistics (one pass: relative error ~ count 2^-53 (1 + mean^2 /
    # var)) and one FP32 rounding of each output
    mu2 = c.mean(axis=1, keepdims=True) ** 2 / np.where(sd > 0, sd * sd, 1.0)
    e_rn = U32 * np.abs(want) + 1024 * 2.0 ** -52 * (1.0 + mu2) * (np.abs(want) + 1.0)
    assert np.all(np.abs(got[:, :1024] - want) <= e_rn)
    assert np.array_equal(got[:, 1024:], x[:, 1024:])
    # pooled column statistics over the coarse block
    mean = torch.empty(d, dtype=torch.float32, device=dev)
    inv = torch.empty(d, dtype=torch.float32, device=dev)
    assert L.lsp_col_stats(p(xt), n, d, p(mean), p(inv), None) == 0
    assert L.lsp_pool_stats(p(mean), p(inv), 0, 1024, None) == 0
    torch.cuda.synchronize()
    blk = got[:, :1024].astype(np.float64)
    # pooled from per-column FP32 statistics (each within half an FP32 ulp):
    # the pooled mean within 2 u |mean|-scale, the pooled 1/std within a few
    # u relative (the per-column values enter var_j + m_j^2 with relative
    # error <= 2 u each, then the difference with the squared mean, whose
    # cancellation is bounded by (mean^2 + E x^2) / var)
    bm, bv = blk.mean(), blk.var()
    amp = (bm * bm + (blk * blk).mean()) / bv
    assert abs(mean.cpu().numpy()[0] - bm) <= 4 * U32 * np.abs(blk).mean()
    assert np.all(np.abs(inv.cpu().numpy()[:1024] * np.sqrt(bv) - 1.0) <= 4 * U32 * amp + 2 * U32)
    oth = got[:, 1024:].astype(np.float64)
    w_inv = 1.0 / oth.std(0)
    assert np.all(np.abs(inv.cpu().numpy()[1024:] - w_inv) <= (U32 + (n + 4) * 2.0 ** -53) * w_inv)
    # shift augmentation on BF16 rows
    xb = torch.as_tensor(rng.integers(-2000, 2000, size=(n, d)).astype(np.int16), device=dev)
    lab = rng.integers(-1, 64, n).astype(np.int32)
    sh = rng.integers(-70, 70, n).astype(np.int32)
    out, out_lab = learned.shift_bands(xb, torch.as_tensor(lab, device=dev),
                                       torch.as_tensor(sh, device=dev), 64)
    torch.cuda.synchronize()
    xh, oh = xb.cpu().numpy(), out.cpu().numpy()
    for i in (0, 5, 77, 299):
        for j in (0, 15, 16, 500, 1023, 1024, 1087):
            src = j - 16 * sh[i]
            if j < 1024:
                want = xh[i, src] if 0 <= src < 1024 else 0
            else:
                want = xh[i, j]
            assert oh[i, j] == want, (i, j)
    nl = lab + sh
    want_lab = np.where((lab >= 0) & (nl >= 0) & (nl < 64), nl, -1)
    assert np.array_equal(out_lab.cpu().numpy(), want_lab)


def test_band_max_and_merge(dev):
    rng = np.random.default_rng(21)
    n, d = 257, 1088
    x = rng.normal(size=(n, d)).astype(np.float32)
    xt = torch.as_tensor(x, device=dev)
    out = torch.empty((n, 64), dtype=torch.float32, device=dev)
    L = lsp.lib()
    p = learned._p
    assert L.lsp_band_max(p(xt), n, d, 0, 64, 16, p(out), None) == 0
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), x[:, :1024].reshape(n, 64, 16).max(axis=2))
    a = rng.integers(-1, 64, size=(n, 4)).astype(np.int32)
    b = rng.integers(0, 64, size=(n, 8)).astype(np.int32)
    b[3] = a[3, 0]          # every entry of b already taken or repeated
    m = torch.empty((n, 8), dtype=torch.int32, device=dev)
    assert L.lsp_merge_bands(p(torch.as_tensor(a, device=dev)), 4,
                             p(torch.as_tensor(b, device=dev)), 8, n, 8, p(m), None) == 0
    torch.cuda.synchronize()
    got = m.cpu().numpy()
    for i in range(n):
        want = []
        for v in list(a[i]) + list(b[i]):
            if v >= 0 and v not in want and len(want) < 8:
                want.append(int(v))
        want += [-1] * (8 - len(want))
        assert list(got[i]) == want, i


TRIM_TOL = 1e-5


def _trim_reference(idx, n_net, logits, score, tau, alpha):
    """The keep rule in FP64: (kept bands, kept mass, per-slot distance of the
    decision from its threshold)."""
    n, top = idx.shape
    out = np.full_like(idx, -1)
    mass = np.zeros(n)
    margin = np.full(idx.shape, np.inf)
    for i in range(n):
        if logits is not None:
            z = logits[i].astype(np.float64)
            p = np.exp(z - z.max())
            p /= p.sum()
        smax = score[i].max() if score is not None else 0.0
        cum, any_net = 0.0, False
        for r in range(top):
            b = idx[i, r]
            if b < 0:
                continue
            if r < n_net:
                keep = (not any_net) or cum < tau
                if any_net:
                    margin[i, r] = abs(cum - tau)
                if keep:
                    any_net = True
                    cum += p[b]
            else:
                keep = (n_net == 0 and r == 0) or score is None or score[i, b] >= alpha * smax
                if score is not None and not (n_net == 0 and r == 0):
                    margin[i, r] = abs(float(score[i, b]) - alpha * float(smax))
            out[i, r] = b if keep else -1
        mass[i] = cum
    return out, mass, margin


def test_trim_bands(dev):
    """lsp_trim_bands against the keep rule in FP64: identical decisions
    except near a threshold, kept mass within TRIM_TOL.

    The kernel's probabilities are FP32: exp(z - max) (about 1 ulp and u |z -
    max| for the rounded argument, |z - max| < 16 here), the 64-term sum
    (64 u) and the division (1 u) leave each within 90 u (u = 2^-24) of its
    FP64 value relative to itself, so a sum of at most 8 kept probabilities
    (at most 1) is within 90 u = 5.4e-6 of the FP64 mass; a mass decision can
    differ only where the FP64 running mass is that close to tau.  A score
    decision compares FP32 values exactly except for the rounding of alpha *
    max (half an ulp of a number below 1).  TRIM_TOL = 1e-5 covers both."""
    rng = np.random.default_rng(22)
    n, c, top = 400, 64, 8
    logits = rng.normal(0, 2.0, (n, c)).astype(np.float32)
    score = rng.uniform(0, 1, (n, c)).astype(np.float32)
    idx = np.full((n, top), -1, np.int32)
    for i in range(n):
        net = list(np.argsort(-logits[i].astype(np.float64), kind="stable")[:4])
        rest = [b for b in np.argsort(-score[i].astype(np.float64), kind="stable") if b not in net]
        row = net + rest[: top - 4]
        if i % 10 == 0:
            row[-2:] = [-1, -1]
        idx[i] = row
    it = torch.as_tensor(idx, device=dev)
    lt = torch.as_tensor(logits, device=dev)
    st = torch.as_tensor(score, device=dev)
    cases = [(4, True, True, 2.0, 0.0), (4, True, True, 0.9, 0.5), (4, True, True, 0.5, 0.8),
             (4, True, True, 0.0, 1.0), (top, True, False, 0.95, 0.0),
             (0, False, True, 2.0, 0.6), (0, False, True, 0.0, 0.999)]
    for n_net, use_l, use_s, tau, alpha in cases:
        say(f"trim n_net={n_net} tau={tau} alpha={alpha}")
        km = torch.empty(n, dtype=torch.float32, device=dev)
        out, _ = learned.trim_bands(it, n_net, lt if use_l else None, st if use_s else None,
                                    tau, alpha, kept_mass=km if use_l else None)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        want, mass, margin = _trim_reference(idx, n_net, logits if use_l else None,
                                             score if use_s else None, tau, alpha)
        differ = got != want
        assert np.all(margin[differ] < TRIM_TOL), (n_net, tau, alpha)
        if use_l:
            assert np.all(np.abs(km.cpu().numpy() - mass) <= TRIM_TOL)
        # kept network slots form a prefix, and the first valid slot is kept
        for i in range(n):
            valid = idx[i] >= 0
            assert got[i][valid][0] == idx[i][valid][0]
            k = got[i, :n_net] >= 0
            assert not np.any(k[1:] & ~k[:-1]) or np.any(idx[i, :n_net] < 0)


def test_network_entry_points_equal_their_primitives(dev):
    """lsp_mlp_forward, lsp_mlp_backward and lsp_mlp_adam run the layer order
    that the primitives express (three GEMMs with bias and ReLU; softmax
    cross-entropy; per layer the weight GEMM, the bias column sums and the
    masked back-propagating GEMM; one Adam step per parameter array): their
    results are bitwise those of the same primitives called one by one."""
    rng = np.random.default_rng(8)
    n = 80
    d0, d1, d2, d3 = mlp_ref.DIMS
    params = mlp_ref.init_params(4)
    for pp in params[1::2]:
        pp += rng.normal(0, 0.05, size=pp.shape)
    x = bits(mlp_ref.bf16_round(rng.normal(size=(n, d0))), dev)
    labels = rng.integers(0, d3, size=n).astype(np.int32)
    labels[3] = -1  # ignored row
    lab = torch.as_tensor(labels, device=dev)
    net = learned.BandNet(dev, params=params)
    say("lsp_mlp_forward / backward / adam")
    loss, grads = net.gradients(x, lab)
    got_logits = net.forward(x).clone()
    got = [g.clone() for g in grads]
    got_loss = loss.clone()
    net.train_step(x, lab, lr=1e-3)
    torch.cuda.synchronize()
    got_params = [q.clone() for q in net.master] + [w.clone() for w in net.w_bf16]

    # the same step, primitive by primitive, on a fresh copy of the network
    ref = learned.BandNet(dev, params=params)
    L = lsp.lib()
    W1, W2, W3 = ref.w_bf16
    b1, b2, b3 = ref.master[1], ref.master[3], ref.master[5]
    h1 = torch.empty((n, d1), dtype=torch.int16, device=dev)
    h2 = torch.empty((n, d2), dtype=torch.int16, device=dev)
    z = torch.empty((n, d3), dtype=torch.float32, device=dev)
    learned.gemm(x, W1, n, d1, d0, d0, 1, d1, 1, C_bf16=h1, bias=b1, relu=True)
    learned.gemm(h1, W2, n, d2, d1, d1, 1, d2, 1, C_bf16=h2, bias=b2, relu=True)
    learned.gemm(h2, W3, n, d3, d2, d2, 1, d3, 1, C=z, bias=b3)
    g3 = torch.empty((n, d3), dtype=torch.float32, device=dev)
    g3b = torch.empty((n, d3), dtype=torch.int16, device=dev)
    rows = torch.empty(n, dtype=torch.float32, device=dev)
    assert L.lsp_softmax_xent(z.data_ptr(), lab.data_ptr(), n, d3, ctypes.c_float(1.0 / n),
                              g3.data_ptr(), g3b.data_ptr(), rows.data_ptr(), None) == lsp.OK
    g = [torch.empty_like(q) for q in ref.master]
    learned.gemm(h2, g3b, d2, d3, n, 1, d2, d3, 1, C=g[4])
    assert L.lsp_col_sums(g3.data_ptr(), n, d3, g[5].data_ptr(), None) == lsp.OK
    dz2 = torch.empty((n, d2), dtype=torch.float32, device=dev)
    dz2b = torch.empty((n, d2), dtype=torch.int16, device=dev)
    learned.gemm(g3b, W3, n, d2, d3, d3, 1, 1, d3, C=dz2, C_bf16=dz2b, mask=h2)
    learned.gemm(h1, dz2b, d1, d2, n, 1, d1, d2, 1, C=g[2])
    assert L.lsp_col_sums(dz2.data_ptr(), n, d2, g[3].data_ptr(), None) == lsp.OK
    dz1 = torch.empty((n, d1), dtype=torch.float32, device=dev)
    dz1b = torch.empty((n, d1), dtype=torch.int16, device=dev)
    learned.gemm(dz2b, W2, n, d1, d2, d2, 1, 1, d2, C=dz1, C_bf16=dz1b, mask=h1)
    learned.gemm(x, dz1b, d0, d1, n, 1, d0, d1, 1, C=g[0])
    assert L.lsp_col_sums(dz1.data_ptr(), n, d1, g[1].data_ptr(), None) == lsp.OK
    for i, (q, gi) in enumerate(zip(ref.master, g)):
        wb = ref.w_bf16[i // 2].data_ptr() if i % 2 == 0 else None
        assert L.lsp_adam(q.data_ptr(), gi.data_ptr(), ref.m[i].data_ptr(), ref.v[i].data_ptr(),
                          q.numel(), 1, ctypes.c_float(1e-3), ctypes.c_float(0.9),
                          ctypes.c_float(0.999), ctypes.c_float(1e-8), wb, None) == lsp.OK
    torch.cuda.synchronize()
    assert torch.equal(got_logits, z)
    assert torch.equal(got_loss, rows) and got_loss[3].item() == 0.0
    for name, a, b in zip(["dW1", "db1", "dW2", "db2", "dW3", "db3"], got, g):
        assert torch.equal(a, b), name
    for a, b in zip(got_params, list(ref.master) + list(ref.w_bf16)):
        assert torch.equal(a, b)


def test_gemm_large_tiles_all_load_modes(dev):
    """A product large enough for the 128 x 128 tiles (>= 256 workgroups),
    with ragged M, N and a K that is no multiple of the 32-deep k tile, read
    with 16-byte loads along k, with 16-byte loads along the rows transposed
    into LDS, and element by element (leading dimensions that are not
    multiples of 8): each within gamma(K) sum |a||b| of the FP64 product."""
    rng = np.random.default_rng(17)
    M, N, K = 6600, 520, 1000
    assert -(-M // 128) * -(-N // 128) >= 256
    A = mlp_ref.bf16_round(rng.normal(size=(M, K)))
    B = mlp_ref.bf16_round(rng.normal(size=(K, N)))
    ref = A @ B
    tol = gamma(K) * (np.abs(A) @ np.abs(B))
    C = torch.empty((M, N), dtype=torch.float32, device=dev)
    say("gemm 128x128 tiles: k-contiguous A, row-contiguous B")
    learned.gemm(bits(A, dev), bits(B, dev), M, N, K, K, 1, N, 1, C=C)
    torch.cuda.synchronize()
    assert np.all(np.abs(C.cpu().numpy() - ref) <= tol)
    say("gemm 128x128 tiles: row-contiguous A, k-contiguous B")
    At, Bt = bits(np.ascontiguousarray(A.T), dev), bits(np.ascontiguousarray(B.T), dev)
    learned.gemm(At, Bt, M, N, K, 1, M, 1, K, C=C)
    torch.cuda.synchronize()
    assert np.all(np.abs(C.cpu().numpy() - ref) <= tol)
    say("gemm 128x128 tiles: leading dimensions not multiples of 8")
    Ap = np.zeros((M, K + 3))
    Ap[:, :K] = A
    Bp = np.zeros((K, N + 5))
    Bp[:, :N] = B
    learned.gemm(bits(Ap, dev), bits(Bp, dev), M, N, K, K + 3, 1, N + 5, 1, C=C)
    torch.cuda.synchronize()
    assert np.all(np.abs(C.cpu().numpy() - ref) <= tol)
