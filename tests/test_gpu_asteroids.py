"""Period recovery on the asteroid-like population (Section 4.2's accuracy
study), on the paper's batch grid: 1,000 objects, [1.005, 150.796) rad/day,
N_f = 200,000 (needs an MI355X).

  - the FP32 and FP64 forms find the same peak bin for every object, for the
    standard and the generalized periodogram;
  - on a sample of objects the FP64 form's peaks are the oracle's (FP32 within
    one bin), whole periodograms computed on the CPU;
  - the study itself: twice the light-curve period at the peak matches the
    assigned rotation period within 0.1 h for most objects, more so with more
    observations, and the generalized periodogram (errors, floating mean)
    recovers at least as many as the standard one.  The thresholds sit just
    below the values this seeded population gives (standard 0.819 overall,
    0.969 with >= 300 points; generalized 0.861).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2105_04006_amd import lsp, synth  # noqa: E402
from test_gpu_parity import FP32_ATOL, cuda, dev, oracle, peak_ok, say  # noqa: E402,F401

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pop():
    return synth.make_workload("asteroids_1k")


def peaks(dev, w, form, method):
    say(f"  asteroids_1k form={form} {method}")
    p = lsp.Periodogram(cuda(w.t, dev), cuda(w.y, dev), w.f_min, w.f_max, w.n_f,
                        offsets=cuda(w.offsets, dev, torch.int64), unit=lsp.ANGULAR, form=form,
                        method=method, dy=cuda(w.dy, dev) if method == "generalized" else None,
                        pgram=False, peaks=True)
    p()
    torch.cuda.synchronize()
    return p.peaks()


def matched(w, pk, tol_h=0.1):
    return np.abs(2.0 * 24.0 * pk["period"] - w.p_rot_hours) <= tol_h


def test_recovery_study(dev, pop):
    w = pop
    n_t = np.diff(w.offsets)
    res = {}
    for method in ("standard", "generalized"):
        p32 = peaks(dev, w, lsp.FORM_FP32P, method)
        p64 = peaks(dev, w, lsp.FORM_FP64, method)
        assert np.all(np.abs(p32["index"] - p64["index"]) <= 1), method
        res[method] = matched(w, p32)
        say(f"    {method}: matched {res[method].mean():.4f}, N_t >= 300: "
            f"{res[method][n_t >= 300].mean():.4f}")
    std, gen = res["standard"], res["generalized"]
    assert std.mean() >= 0.80 and std[n_t >= 300].mean() >= 0.95
    assert std[n_t >= 50].mean() > std.mean()  # fewer points, fewer recoveries
    assert gen.mean() >= 0.85 and gen.mean() >= std.mean()


def test_recovery_peaks_against_oracle(dev, pop):
    rng = np.random.default_rng(37)
    n_t = np.diff(pop.offsets)
    pick = np.sort(rng.choice(np.nonzero(n_t <= 250)[0], 8, replace=False))
    sub_t, sub_y, sub_dy, lens = [], [], [], []
    for o in pick:
        a, b = pop.offsets[o], pop.offsets[o + 1]
        sub_t.append(pop.t[a:b]), sub_y.append(pop.y[a:b]), sub_dy.append(pop.dy[a:b])
        lens.append(b - a)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    t, y, dy = np.concatenate(sub_t), np.concatenate(sub_y), np.concatenate(sub_dy)
    w = pop
    ora_pg, ora_pk = oracle.batch(off, t, y, w.f_min, w.f_max, w.n_f, unit=1)
    gora_pg, gora_pk = oracle.gen_batch(off, t, y, dy, w.f_min, w.f_max, w.n_f, unit=1)
    for method, (opg, opk) in (("standard", (ora_pg, ora_pk)),
                               ("generalized", (gora_pg, gora_pk))):
        for form, tol, bins in ((lsp.FORM_FP64, 1e-9, 0), (lsp.FORM_FP32P, FP32_ATOL, 1)):
            p = lsp.Periodogram(cuda(t, dev), cuda(y, dev), w.f_min, w.f_max, w.n_f,
                                offsets=cuda(off, dev, torch.int64), unit=lsp.ANGULAR, form=form,
                                method=method,
                                dy=cuda(dy, dev) if method == "generalized" else None,
                                pgram=False, peaks=True)
            p()
            torch.cuda.synchronize()
            pk = p.peaks()
            for i in range(len(pick)):
                assert peak_ok(opg[i], opk["index"][i], pk["index"][i], tol, bins), \
                    (method, form, int(pick[i]))
