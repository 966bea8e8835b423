"""Sub-cell peak refinement on the GPU against the FP64 oracle.

The start cells come from the oracle's own peak lists.  Both sides take the
same safeguarded Newton steps on the same continuous plane; the GPU evaluates
it in FP32, with an error of about 1e-6 of the plane's scale (its largest
|P|, often a masked border cell), which moves a maximum by about that error
divided by the curvature: far below the 2e-3 cell bound on the refined
position.  Values: within 2e-5 of the plane's scale: the plane's own FP32
error (max over cells about 3x its rms, ~3e-6 for the chirp-z path, whose
Bluestein transforms and the inverse x' DFT add FP32 stages) plus the sums
over x' and n2; a weak peak's own relative error is larger by the ratio of
the plane's maximum to it."""
import numpy as np
import pytest

from oracle import funnel_oracle as O
from paper_1904_09409_amd import funnel as F
from paper_1904_09409_amd import synth

pytestmark = pytest.mark.gpu
POS_TOL, VAL_TOL, ITERS = 2e-3, 2e-5, 4


def say(*a):
    print(*a, flush=True)


def oracle_lists(img, Np, K, spaces, kind):
    """Oracle peak lists per space: (records, count, name, g, max |P| of the plane)."""
    N, M = img.shape
    img = img.astype(np.float64)
    out = []
    for sp, name in ((0, "regular"), (1, "inverse")):
        if not spaces & (1 << sp):
            continue
        src = img if sp == 0 else img.T
        P = O.forward_regular(src, Np, kind)
        H, W = src.shape
        lst = O.peaks_list(np.abs(P), K, 0.0, 1, O.boundary_mask(H, W, Np), True)
        recs = np.zeros(K, dtype=F.PEAK_DTYPE)
        for i, idx in enumerate(lst):
            r, c = divmod(idx, W)
            k, b = O.peak_params(r, c, N, M, Np, name)
            recs[i] = (0, sp, r, c, abs(P[r, c]), np.float32(k), np.float32(b))
        out.append((recs, len(lst), name, O.resampled_rows(src, Np, kind), float(np.abs(P).max())))
    return out


def check(out, lists, b, Np):
    worst_p, worst_v = 0.0, 0.0
    for s, (recs, n, name, g, scale) in enumerate(lists):
        W = g.shape[1]
        for k in range(n):
            m, y, v = O.refine_peak(g, Np, int(recs[k]["row"]), int(recs[k]["col"]), ITERS)
            got = out[b, s, k]
            dm = abs(got["col"] - (m + W // 2))
            dy = abs(got["row"] - (y + Np // 2))
            dv = abs(got["value"] - v) / scale
            worst_p, worst_v = max(worst_p, dm, dy), max(worst_v, dv)
            assert max(dm, dy) <= POS_TOL and dv <= VAL_TOL, (b, name, k, got, (m, y, v))
            # Eq. 22 (or 24) at the refined cell
            k_exp = -2.0 * (got["col"] - W // 2) / W
            assert abs(got["slope"] - k_exp) <= 1e-6 * max(1.0, abs(k_exp))
        for k in range(n, len(recs)):
            assert all(v == 0 for v in out[b, s, k].tolist())
    return worst_p, worst_v


@pytest.mark.parametrize("B,N,M,Np,spaces,kind", [
    (3, 128, 128, 0, 3, "linear"),
    (2, 128, 256, 0, 3, "chirpz"),
    (2, 256, 128, 512, 2, "linear"),    # inverse space only, enlarged padding
])
def test_refine_matches_oracle(B, N, M, Np, spaces, kind):
    import torch
    K = 8
    say(f"refine {B} x {N}x{M} Np={Np} spaces={spaces} {kind}")
    imgs = [synth.mixed_lines(N, M, (2, 6), 0.1, np.random.default_rng([81, N, M, i])).image for i in range(B)]
    plan = F.FunnelPlan(B, N, M, Np, spaces, nvmt=kind)
    ns = plan.nspaces
    rec = np.zeros((B, ns, K), dtype=F.PEAK_DTYPE)
    cnt = np.zeros((B, ns), dtype=np.int32)
    lists = []
    for b in range(B):
        lb = oracle_lists(imgs[b], plan.Np, K, spaces, kind)
        for s, (recs, n, name, g, _) in enumerate(lb):
            recs["image"] = b
            rec[b, s], cnt[b, s] = recs, n
        lists.append(lb)
    x = torch.from_numpy(np.stack(imgs)).cuda()
    rec_t = torch.from_numpy(rec.view(np.int32).reshape(B, ns, K, F.PEAK_WORDS).copy()).cuda()
    out = F.refined_to_numpy(plan.refine(x, rec_t, torch.from_numpy(cnt).cuda(), ITERS))
    wp, wv = 0.0, 0.0
    for b in range(B):
        p, v = check(out, lists[b], b, plan.Np)
        wp, wv = max(wp, p), max(wv, v)
    say(f"  worst |position| {wp:.2e} cell, worst value error {wv:.2e} of the plane scale; "
        f"mean shift {out['shift'].mean():.3f}")


def test_refine_workload_1024():
    """The 32 x 1024^2 batch: refinement of the GPU's peak lists for all
    images, with the oracle's own lists substituted (and compared) on two
    sampled images."""
    import torch
    B, N, K = 32, 1024, 16
    say("refine 32 x 1024^2")
    imgs = synth.batch("grad", count=B, size=N, seed=0)
    x = torch.from_numpy(synth.stack(imgs)).cuda()
    plan = F.FunnelPlan(B, N, N)
    planes = plan.forward(x)
    rec, cnt = plan.peaks(planes, K=K)
    torch.cuda.synchronize()
    rec_h = rec.cpu().numpy().copy()
    cnt_h = cnt.cpu().numpy().copy()
    samples = (5, 26)
    lists = {}
    for b in samples:
        lb = oracle_lists(imgs[b].image, plan.Np, K, 3, "linear")
        for s, (recs, n, name, g, _) in enumerate(lb):
            recs["image"] = b
            rec_h[b, s] = recs.view(np.int32).reshape(K, F.PEAK_WORDS)
            cnt_h[b, s] = n
        lists[b] = lb
    out = F.refined_to_numpy(plan.refine(x, torch.from_numpy(rec_h).cuda(), torch.from_numpy(cnt_h).cuda(), ITERS))
    for b in samples:
        p, v = check(out, lists[b], b, plan.Np)
        say(f"  image {b}: worst |position| {p:.2e} cell, worst value error {v:.2e} of the plane scale")


def test_refine_accuracy_on_lines():
    """Eq. 19 with real-valued line parameters, on the GPU: long ridges in
    256^2 images; the refined slope bin and intercept are much closer to the
    line's continuous cell than the detected cell is."""
    import torch
    B, N = 6, 256
    rng = np.random.default_rng(85)
    lines, imgs = [], []
    for i in range(B):
        k = float(rng.uniform(-0.8, 0.8))
        b = float(rng.uniform(80, 176)) - k * N / 2
        ln = synth.Line("ridge", False, k, b, width=1.0)
        lines.append(ln)
        imgs.append(synth.render(N, N, [ln], 0.0, rng, bg=0.0).astype(np.float32))
    x = torch.from_numpy(np.stack(imgs)).cuda()
    plan = F.FunnelPlan(B, N, N, 0, F.FT_SPACE_REGULAR)
    planes = plan.forward(x)
    rec, cnt = plan.peaks(planes, K=1)
    out = F.refined_to_numpy(plan.refine(x, rec, cnt, ITERS))
    got = F.peaks_to_numpy(rec, cnt)
    Np = plan.Np
    e_cell, e_ref = [], []
    for i, ln in enumerate(lines):
        mt, yt = -ln.k * N / 2 + N // 2, ln.b + ln.k * N / 2 - N / 2 + Np // 2
        e_cell.append(np.hypot(int(got[i][0][0]["col"]) - mt, int(got[i][0][0]["row"]) - yt))
        e_ref.append(np.hypot(out[i, 0, 0]["col"] - mt, out[i, 0, 0]["row"] - yt))
    say(f"  cell error mean {np.mean(e_cell):.3f}, refined {np.mean(e_ref):.3f} (max {np.max(e_ref):.3f})")
    assert np.mean(e_ref) <= 0.05 and np.max(e_ref) <= 0.15 and np.mean(e_cell) > 0.2
