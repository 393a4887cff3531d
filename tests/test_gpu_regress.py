"""GPU parity of the regression kernel (esim_wlr_regress) and the log-brightness
kernel against the FP64 oracle, through the C ABI.

Tolerances: alpha within 1e-4 * max(1, |alpha|) (the contract); beta within
1e-4 * max(1, |beta|); R within 1e-6 absolute; kappa-hat (Hager's 1-norm
estimate) must not exceed the 1-norm condition number of the oracle's system
and must stay within a factor 5 of it."""
import numpy as np
import pytest
import torch

import oracle
from paper_2303_02608_amd import binding as B
from paper_2303_02608_amd import synth
from parity_util import oracle_clip, say, to_dev

pytestmark = pytest.mark.gpu


def _regress_all(E, feat, p: B.Params, t: int, lanes=None):
    y, fd = to_dev(E, feat)
    plan = B.Plan([y], [fd], [p])
    if lanes:
        plan.set_schedule(lanes, lanes, 4)
    HW = plan.npix
    a = torch.empty(HW, device="cuda")
    b = torch.empty((plan.D, HW), device="cuda")
    R = torch.empty(HW, device="cuda")
    K = torch.empty(HW, device="cuda")
    B.regress(plan, t, None, None, HW, a, b, R, K)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy(), R.cpu().numpy(), K.cpu().numpy()


def _oracle_all(E, feat, p: B.Params, t: int, kappa=True):
    clip = oracle_clip(E, feat)
    HW = clip.H * clip.W
    items = t * HW + np.arange(HW)
    op = oracle.Params(p.r, p.tr, p.C, p.h, p.b, p.ridge)
    return oracle.regress_items(clip, op, items, kappa=kappa)


def _check(a, b, R, K, ref, tag, unit_bandwidth=True, kappa1=None):
    th = ref["theta"]
    ea = np.abs(a - th[:, 0]) / np.maximum(1.0, np.abs(th[:, 0]))
    eb = np.abs(b.T - th[:, 1:]) / np.maximum(1.0, np.abs(th[:, 1:]))
    er = np.abs(R - ref["R"])
    say(f"{tag}: max rel err alpha {ea.max():.2e} beta {eb.max():.2e} R {er.max():.2e}")
    assert ea.max() <= 1e-4, tag
    assert eb.max() <= 1e-4, tag
    assert er.max() <= 1e-6, tag
    if kappa1 is not None and unit_bandwidth:
        # Hager's estimate is a lower bound of the 1-norm condition number and
        # in practice within a small factor of it (exact at most pixels here,
        # never below a tenth)
        idx, k1 = kappa1
        ratio = K[idx] / k1
        say(f"{tag}: kappa-hat / kappa_1 in [{ratio.min():.3f}, {ratio.max():.3f}], "
            f"median {np.median(ratio):.3f}")
        assert np.all(ratio <= 1 + 1e-3), tag
        assert np.all(ratio >= 0.1), tag
        assert np.median(ratio) >= 0.5, tag


def _equilibrated(A):
    s = 1.0 / np.sqrt(np.diag(A))
    return A * s[:, None] * s[None, :]


def _kappa1(E, feat, p: B.Params, t: int, n=150, seed=0):
    """1-norm condition numbers of the oracle's W-normalised systems scaled to
    unit diagonal, at sampled pixels (numpy's cond; the scaling also removes
    the bandwidths' column scaling, so both sides' matrices are the same)."""
    clip = oracle_clip(E, feat)
    HW = clip.H * clip.W
    idx = np.random.default_rng(seed).choice(HW, size=min(n, HW), replace=False)
    op = oracle.Params(p.r, p.tr, p.C, p.h, p.b, p.ridge)
    k1 = np.array([np.linalg.cond(_equilibrated(oracle.normal_equations(clip, op, t, i % clip.W,
                                                                        i // clip.W)[0]), 1)
                   for i in idx])
    return idx, k1


def test_log_brightness_matches_oracle():
    say("log_brightness n=100003")
    rng = np.random.default_rng(0)
    E = np.concatenate([[0.0, 1e-30, 1.0, 1e6], rng.exponential(0.5, 100003 - 4)]).astype(np.float32)
    y = B.log_brightness(torch.from_numpy(E).cuda()).cpu().numpy()
    ref = oracle.log_brightness(E)
    assert np.max(np.abs(y - ref) / np.maximum(1.0, np.abs(ref))) <= 2.5e-7
    # input 4 bytes off a 16-byte boundary: the one-value-per-lane kernel, the
    # same values bit for bit
    buf = torch.empty(E.size + 1, device="cuda")
    Eoff = buf[1:]
    Eoff.copy_(torch.from_numpy(E))
    assert Eoff.data_ptr() % 16 != 0
    y2 = B.log_brightness(Eoff).cpu().numpy()
    assert np.array_equal(y2.view(np.uint32), y.view(np.uint32))
    # lengths below and around one 16-byte vector (tail lanes only, or a few
    # vectors and a tail)
    for n in (1, 2, 3, 4, 5, 7):
        yn = B.log_brightness(torch.from_numpy(E[:n].copy()).cuda()).cpu().numpy()
        assert np.array_equal(yn.view(np.uint32), y[:n].view(np.uint32)), n
    assert B.log_brightness(torch.empty(0, device="cuda")).numel() == 0


@pytest.mark.parametrize("t", [0, 7, 15])
def test_dense_regress_small_workload(small_clip, t):
    cfg = small_clip["cfg"]
    p = B.Params(r=cfg["r"], tr=cfg["tr"], C=cfg["C"])
    say(f"dense regress small workload t={t}")
    out = _regress_all(small_clip["E"], small_clip["feat"], p, t)
    ref = _oracle_all(small_clip["E"], small_clip["feat"], p, t)
    _check(*out, ref, f"small t={t}", kappa1=_kappa1(small_clip["E"], small_clip["feat"], p, t))


@pytest.mark.parametrize("W,H,T,F,r,tr,t,ridge,seed", [
    (37, 23, 3, 1, 1, 0, 0, 1e-6, 1),
    (37, 23, 4, 3, 2, 1, 0, 1e-6, 2),
    (29, 31, 5, 7, 3, 2, 4, 1e-6, 3),
    (40, 17, 3, 10, 4, 1, 1, 1e-4, 4),
    (33, 35, 3, 12, 2, 1, 2, 0.0, 5),
    (45, 40, 3, 7, 9, 1, 1, 1e-6, 6),
    (20, 20, 2, 5, 12, 0, 1, 1e-6, 7),     # window larger than the image
])
def test_dense_regress_shapes(W, H, T, F, r, tr, t, ridge, seed):
    say(f"dense regress W={W} H={H} T={T} F={F} r={r} tr={tr} t={t} ridge={ridge}")
    d = synth.random_features_clip(W, H, T, F, seed)
    E, feat = d["E"].numpy(), d["feat"].numpy()
    p = B.Params(r=r, tr=tr, C=0.2, ridge=ridge)
    out = _regress_all(E, feat, p, t)
    ref = _oracle_all(E, feat, p, t)
    _check(*out, ref, f"shape {W}x{H} F={F} r={r}", kappa1=_kappa1(E, feat, p, t))


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16])
def test_lanes_per_item_variants(small_clip, lanes):
    cfg = small_clip["cfg"]
    p = B.Params(r=cfg["r"], tr=1, C=cfg["C"], h=1.3, b=[1.0, 0.8, 1.2, 1.1, 0.9, 1.0, 0.7, 1.5, 1.0])
    say(f"dense regress lanes={lanes}")
    out = _regress_all(small_clip["E"], small_clip["feat"], p, 3, lanes=lanes)
    ref = _oracle_all(small_clip["E"], small_clip["feat"], p, 3)
    _check(*out, ref, f"lanes={lanes}", unit_bandwidth=False)


@pytest.mark.parametrize("r", [3, 7])
def test_one_pass_instance(small_clip, r):
    """16 lanes per item with 2r + 1 <= 16 and no condition output selects the
    one-pass kernel instance (each lane owns one column)."""
    cfg = small_clip["cfg"]
    p = B.Params(r=r, tr=1, C=cfg["C"], h=1.1, b=[0.9, 1.2, 1.0, 1.1, 0.8, 1.0, 1.3, 0.9, 1.0])
    say(f"one-pass instance r={r}")
    y, fd = to_dev(small_clip["E"], small_clip["feat"])
    plan = B.Plan([y], [fd], [p])
    plan.set_schedule(16, 16, 2)
    HW = plan.npix
    a = torch.empty(HW, device="cuda")
    b = torch.empty((plan.D, HW), device="cuda")
    R = torch.empty(HW, device="cuda")
    B.regress(plan, 9, None, None, HW, a, b, R)
    torch.cuda.synchronize()
    ref = _oracle_all(small_clip["E"], small_clip["feat"], p, 9, kappa=False)
    _check(a.cpu().numpy(), b.cpu().numpy(), R.cpu().numpy(), None, ref, f"one-pass r={r}",
           unit_bandwidth=False)


@pytest.mark.parametrize("r,f16", [(3, False), (7, False), (5, True)])
def test_list_equals_dense_one_pass_bitwise(small_clip, r, f16):
    """A work list of every pixel and a dense launch, both with 16 lanes per
    item (the one-pass instance), give the same bits: same samples, same
    order, same sums; only the item mapping differs.  Two clips of different
    sizes, so that items of both clips share a wave at the clip boundary (the
    list launch's waterfall over clips)."""
    E, feat, cfg = small_clip["E"], small_clip["feat"], small_clip["cfg"]
    if f16:
        feat = feat.astype(np.float16)
    p = B.Params(r=r, tr=1, C=cfg["C"], h=1.1, b=[0.9, 1.2, 1.0, 1.1, 0.8, 1.0, 1.3, 0.9, 1.0])
    say(f"one-pass list vs dense r={r} f16={f16}")
    y1, fd1 = to_dev(E[:, 1:, 1:], feat[:, :, 1:, 1:])
    y2, fd2 = to_dev(E[:, 4:, 5:], feat[:, :, 4:, 5:])
    plan = B.Plan([y1, y2], [fd1, fd2], [p, p])
    plan.set_schedule(16, 16, 2)
    n = plan.npix
    hw1 = y1.shape[1] * y1.shape[2]
    hw2 = y2.shape[1] * y2.shape[2]
    items = np.concatenate([np.arange(hw1, dtype=np.int64), (np.int64(1) << 32) | np.arange(hw2, dtype=np.int64)])
    assert items.size == n and n % 16 != 0 and hw1 % 16 != 0
    wl = torch.from_numpy(items).cuda()
    cnt = torch.tensor([n, 0], dtype=torch.int32, device="cuda")
    for t in (0, 6):
        out = []
        for worklist in (None, wl):
            a = torch.full((n,), 7.0, device="cuda")
            b = torch.full((plan.D, n), 7.0, device="cuda")
            R = torch.full((n,), 7.0, device="cuda")
            B.regress(plan, t, worklist, None if worklist is None else cnt, n, a, b, R)
            torch.cuda.synchronize()
            out.append((a, b, R))
        for u, v in zip(*out):
            assert torch.equal(u, v), t
        assert torch.isfinite(out[0][0]).all()


def test_f16_features(small_clip):
    cfg = small_clip["cfg"]
    feat = small_clip["feat"].astype(np.float16)
    p = B.Params(r=cfg["r"], tr=1, C=cfg["C"])
    say("dense regress f16 features")
    out = _regress_all(small_clip["E"], feat, p, 2)
    ref = _oracle_all(small_clip["E"], feat, p, 2)
    _check(*out, ref, "f16")


def test_worklist_regress_with_padding_and_per_item_frames(small_clip):
    """Listed items in arbitrary order, -1 padding and out-of-range entries
    (skipped), with the frame carried by the item (t < 0)."""
    E, feat, cfg = small_clip["E"], small_clip["feat"], small_clip["cfg"]
    T, F, H, W = feat.shape
    HW = H * W
    rng = np.random.default_rng(5)
    n = 700
    tt = rng.integers(0, T, n)
    pix = rng.integers(0, HW, n)
    items = (tt.astype(np.int64) << 44) | pix.astype(np.int64)
    items[::37] = -1
    bad = np.array([(np.int64(T) << 44) | 5, (np.int64(1) << 32) | 3, HW + 10], np.int64)
    items = np.concatenate([items, bad])
    p = B.Params(r=cfg["r"], tr=1, C=cfg["C"])
    say("worklist regress, per-item frames")
    y, fd = to_dev(E, feat)
    plan = B.Plan([y], [fd], [p])
    wl = torch.from_numpy(items).cuda()
    cnt = torch.tensor([items.size, 0], dtype=torch.int32, device="cuda")
    nout = items.size
    a = torch.full((nout,), 123.0, device="cuda")
    b = torch.empty((plan.D, nout), device="cuda")
    B.regress(plan, -1, wl, cnt, nout, a, b)
    torch.cuda.synchronize()
    a = a.cpu().numpy()
    b = b.cpu().numpy()
    ok = items[:n] >= 0
    ref = oracle.regress_items(oracle_clip(E, feat), oracle.Params(p.r, p.tr, p.C),
                               (tt * HW + pix)[ok])
    th = ref["theta"]
    ea = np.abs(a[:n][ok] - th[:, 0]) / np.maximum(1, np.abs(th[:, 0]))
    eb = np.abs(b[:, :n][:, ok].T - th[:, 1:]) / np.maximum(1, np.abs(th[:, 1:]))
    assert ea.max() <= 1e-4 and eb.max() <= 1e-4
    # skipped entries keep their old value
    assert np.all(a[:n][~ok] == 123.0) and np.all(a[n:] == 123.0)


def test_regress_is_deterministic(small_clip):
    cfg = small_clip["cfg"]
    p = B.Params(r=cfg["r"], tr=1, C=cfg["C"])
    say("determinism")
    a1 = _regress_all(small_clip["E"], small_clip["feat"], p, 4)
    a2 = _regress_all(small_clip["E"], small_clip["feat"], p, 4)
    for u, v in zip(a1, a2):
        assert np.array_equal(u.view(np.uint32), v.view(np.uint32))

