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


def bits(a, dev):
    return torch.as_tensor(mlp_ref.bf16_bits(a).view(np.int16), device=dev)


@pytest.mark.parametrize("M,N,K", [(64, 64, 32), (200, 130, 100), (37, 70, 1088), (1, 5, 3)])
def test_gemm_plain_and_transposed(dev, M, N, K):
    rng = np.random.default_rng(M * 1000 + N)
    A = mlp_ref.bf16_round(rng.normal(size=(M, K)))
    B = mlp_ref.bf16_round(rng.normal(size=(K, N)))
    ref = A @ B
    tol = 1e-5 * np.sqrt(K) * np.abs(A).max() * np.abs(B).max() + 1e-6
    C = torch.empty((M, N), dtype=torch.float32, device=dev)
    say(f"gemm {M}x{N}x{K}")
    learned.gemm(bits(A, dev), bits(B, dev), M, N, K, K, 1, N, 1, C=C)
    torch.cuda.synchronize()
    assert np.max(np.abs(C.cpu().numpy() - ref)) <= tol
    # the same product from transposed storage of both operands
    At, Bt = bits(np.ascontiguousarray(A.T), dev), bits(np.ascontiguousarray(B.T), dev)
    C2 = torch.empty((M, N), dtype=torch.float32, device=dev)
    learned.gemm(At, Bt, M, N, K, 1, M, 1, K, C=C2)
    torch.cuda.synchronize()
    assert np.max(np.abs(C2.cpu().numpy() - ref)) <= tol


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
    assert np.max(np.abs(Cf.cpu().numpy() - ref)) <= 1e-4
    cb = mlp_ref.from_bf16_bits(Cb.cpu().numpy().view(np.uint16))
    assert np.array_equal(cb, mlp_ref.bf16_round(Cf.cpu().numpy()))
    learned.gemm(bits(A, dev), bits(B, dev), M, N, K, K, 1, N, 1, C=Cf, mask=bits(mask, dev))
    torch.cuda.synchronize()
    ref = (A @ B) * (mask > 0)
    assert np.max(np.abs(Cf.cpu().numpy() - ref)) <= 1e-4


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
    assert abs(loss.cpu().numpy().mean() - ref_loss) <= 1e-5
    assert np.max(np.abs(g.cpu().numpy() - ref_g)) <= 1e-6
    cs = torch.empty(c, dtype=torch.float32, device=dev)
    assert L.lsp_col_sums(p(zt), n, c, p(cs), None) == 0
    torch.cuda.synchronize()
    assert np.allclose(cs.cpu().numpy(), z.astype(np.float64).sum(axis=0), atol=1e-4)
    mean = torch.empty(c, dtype=torch.float32, device=dev)
    inv = torch.empty(c, dtype=torch.float32, device=dev)
    assert L.lsp_col_stats(p(zt), n, c, p(mean), p(inv), None) == 0
    torch.cuda.synchronize()
    assert np.allclose(mean.cpu().numpy(), z.mean(axis=0), atol=1e-5)
    assert np.allclose(inv.cpu().numpy(), 1.0 / z.astype(np.float64).std(axis=0), rtol=1e-5)
    idx, mass = learned.top_bands(zt, k=8)
    torch.cuda.synchronize()
    order = np.argsort(-z, axis=1, kind="stable")[:, :8]
    assert np.array_equal(idx.cpu().numpy(), order)
    e = np.exp(z - z.max(axis=1, keepdims=True))
    pm = e / e.sum(axis=1, keepdims=True)
    assert np.allclose(mass.cpu().numpy(), np.take_along_axis(pm, order, 1).sum(1), atol=1e-5)


def test_training_step_matches_reference(dev):
    """One forward/backward/Adam step of the full-size network on the GPU vs the
    BF16-emulated FP64 reference of the same arithmetic."""
    rng = np.random.default_rng(5)
    n = 96
    params = mlp_ref.init_params(9)
    for pp in params[1::2]:
        pp += rng.normal(0, 0.05, size=pp.shape)
    x = mlp_ref.bf16_round(rng.normal(size=(n, 1088)))
    labels = rng.integers(0, 64, size=n).astype(np.int32)
    net = learned.BandNet(dev, params=params)
    xb = bits(x, dev)
    lab = torch.as_tensor(labels, device=dev)
    loss_rows, grads = net.gradients(xb, lab)
    torch.cuda.synchronize()
    bparams = [mlp_ref.bf16_round(p) if i % 2 == 0 else p.astype(np.float32).astype(np.float64)
               for i, p in enumerate(params)]
    logits, cache = mlp_ref.forward(bparams, x, bf16=True)
    ref_loss, dl = mlp_ref.softmax_xent(logits, labels)
    ref_grads = mlp_ref.backward(bparams, cache, dl, bf16=True)
    assert abs(loss_rows.cpu().numpy().mean() - ref_loss) <= 2e-3 * max(1.0, ref_loss)
    for name, g, r in zip(["dW1", "db1", "dW2", "db2", "dW3", "db3"], grads, ref_grads):
        g = g.cpu().numpy()
        err = np.max(np.abs(g - r)) / (np.max(np.abs(r)) + 1e-12)
        say(f"  {name}: max rel err {err:.3g}")
        assert err <= 2e-2, name
    before = [p.clone() for p in net.master]
    net.train_step(xb, lab, lr=1e-3)
    torch.cuda.synchronize()
    for b, a in zip(before, net.master):
        d = (a - b).abs().max().item()
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
    assert np.max(np.abs(got[:, :1024] - want)) <= 1e-5
    assert np.array_equal(got[:, 1024:], x[:, 1024:])
    # pooled column statistics over the coarse block
    mean = torch.empty(d, dtype=torch.float32, device=dev)
    inv = torch.empty(d, dtype=torch.float32, device=dev)
    assert L.lsp_col_stats(p(xt), n, d, p(mean), p(inv), None) == 0
    assert L.lsp_pool_stats(p(mean), p(inv), 0, 1024, None) == 0
    torch.cuda.synchronize()
    blk = got[:, :1024].astype(np.float64)
    assert np.allclose(mean.cpu().numpy()[:1024], blk.mean(), atol=1e-6)
    assert np.allclose(inv.cpu().numpy()[:1024], 1.0 / blk.std(), rtol=1e-5)
    assert np.allclose(inv.cpu().numpy()[1024:], 1.0 / got[:, 1024:].astype(np.float64).std(0),
                       rtol=1e-5)
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
