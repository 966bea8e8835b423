"""Full-size workloads checked against the FP64 oracle on sampled images:
the 32 x 1024^2 batch both with the tile variants the benchmark times
(bench.benchmark_variants: the counter table's set, else the autotuner's) and
with the plan defaults, its peak lists end to end, and the 64 x 512^2 batch;
the gradient of the peak loss against FP64 finite differences and the dense
operator."""
import numpy as np
import pytest

import pins
from helpers import peaks_match_on_decidable_prefix, rel_l2
from oracle import funnel_oracle as O
from paper_1904_09409_amd import funnel as F
from paper_1904_09409_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(*a):
    print(*a, flush=True)


def focus_cells(lines, N, M, Np):
    out = []
    for ln in lines:
        space, r, c = pins.expected_cell(ln, N, M, Np)
        out.append((0 if space == "regular" else 1, r, c))
    return out


def loss_gradient(plan, planes, imgs):
    """d/dP of sum over lines of |P| at the line's focus cell."""
    import torch
    dP = torch.zeros_like(planes)
    v, dv = plan.views(planes), plan.views(dP)
    for b, im in enumerate(imgs):
        for sp, r, c in focus_cells(im.lines, plan.N, plan.M, plan.Np):
            src = v.regular if sp == 0 else v.inverse
            dst = dv.regular if sp == 0 else dv.inverse
            dst[b, r, c] = torch.sign(src[b, r, c])
    return dP


def bench_plan(B, size):
    """A plan set up exactly as bench.py's default run sets up its plan."""
    import bench
    plan = F.FunnelPlan(B, size, size)
    src = bench.benchmark_variants(F, plan)
    say(f"  tile variants ({src}): {F.funnel_plan_variants(plan.handle)}")
    return plan


def check_peaks_end_to_end(plan, planes, refs, K=16, min_prefix=12):
    """GPU planes -> GPU peaks against oracle planes -> the literal list of
    Sec. 4.4 on the decidable prefix (helpers.peaks_match_on_decidable_prefix,
    with the stated 1e-5 bound checked cell by cell), at least min_prefix of
    the K peaks of every plane."""
    rec, cnt = plan.peaks(planes, K=K)
    got = F.peaks_to_numpy(rec, cnt)
    v = plan.views(planes)
    mask = O.boundary_mask(plan.N, plan.M, plan.Np)
    for b, ref in refs.items():
        decided = []
        for s, Pref in enumerate(ref):
            gp = (v.regular if s == 0 else v.inverse)[b].cpu().numpy()
            g = got[b][s]
            ids = [int(r) * Pref.shape[1] + int(c) for r, c in zip(g["row"], g["col"])]
            decided.append(peaks_match_on_decidable_prefix(O, ids, gp, Pref, TOL, mask, K, min_prefix))
        say(f"  image {b}: peaks identical to the oracle's on decidable prefixes {decided} of {K}")


def check_workload(config, B, size, samples, variants="default", peaks=False):
    import torch
    say(f"workload {config}: {B} x {size}^2 (samples {samples}), {variants} tile variants")
    imgs = synth.batch(config, count=B, size=size, seed=0)
    x = torch.from_numpy(synth.stack(imgs)).cuda()
    plan = bench_plan(B, size) if variants == "bench" else F.FunnelPlan(B, size, size)
    planes = plan.forward(x)
    dP = loss_gradient(plan, planes, imgs)
    dI = plan.adjoint(dP)
    torch.cuda.synchronize()
    v = plan.views(planes)
    Np = plan.Np
    dPh = dP.cpu().numpy()
    refs = {}
    for b in samples:
        img = imgs[b].image.astype(np.float64)
        ref_r, ref_i = O.forward(img, Np)
        refs[b] = (ref_r, ref_i)
        e_r = rel_l2(v.regular[b].cpu().numpy(), ref_r)
        e_i = rel_l2(v.inverse[b].cpu().numpy(), ref_i)
        ref_d = O.adjoint(dPh[b, :Np * size].reshape(Np, size).astype(np.float64),
                          dPh[b, Np * size:].reshape(Np, size).astype(np.float64), size, size, Np)
        e_d = rel_l2(dI[b].cpu().numpy(), ref_d)
        say(f"  image {b}: rel L2 regular {e_r:.2e} inverse {e_i:.2e} adjoint {e_d:.2e}")
        assert max(e_r, e_i, e_d) <= TOL
    if peaks:
        check_peaks_end_to_end(plan, planes, refs)


def test_grad_workload_1024_bench_variants():
    """32 x 1024^2, both spaces, forward + adjoint of the peak loss, in the
    launch configuration bench.py times (its tile variants), and the peak
    lists of two images end to end."""
    check_workload("grad", 32, 1024, samples=(0, 31), variants="bench", peaks=True)


def test_grad_workload_1024_default_variants():
    """The same batch with the plan's default tile variants."""
    check_workload("grad", 32, 1024, samples=(0, 31))


def test_plain_workload_512():
    """64 x 512^2, both spaces."""
    check_workload("plain", 64, 512, samples=(0, 33, 63))


def test_properties_at_full_size():
    """Linearity and the adjoint identity on the full 32 x 1024^2 batch,
    computed entirely by the library (no oracle needed at this size)."""
    import torch
    say("properties 32 x 1024^2")
    B = 32
    plan = F.FunnelPlan(B, 1024, 1024)
    g = torch.Generator(device="cuda").manual_seed(11)
    a = torch.rand((B, 1024, 1024), device="cuda", generator=g)
    b = torch.rand((B, 1024, 1024), device="cuda", generator=g)
    Pa = plan.forward(a).clone()
    Pb = plan.forward(b).clone()
    Pab = plan.forward(2 * a - b)
    err = (Pab - (2 * Pa - Pb)).norm() / Pab.norm()
    assert err.item() < 1e-5
    y = torch.randn(Pa.shape, device="cuda", generator=g)
    Aty = plan.adjoint(y)
    lhs = (Pa.double() * y.double()).sum().item()
    rhs = (a.double() * Aty.double()).sum().item()
    # <F a, y> = <a, F^T y>: the sums can cancel to a small value, so the
    # bound scales with the sums of absolute terms (the rounding of either
    # side is a tiny fraction of those); a missing or wrong term would be
    # of the order of the terms themselves
    scale = (Pa.double() * y.double()).abs().sum().item() + (a.double() * Aty.double()).abs().sum().item()
    say(f"  adjoint identity: lhs {lhs:.6e} rhs {rhs:.6e} |diff|/scale {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-8 * scale


def test_gradient_on_crops_fd_and_dense():
    """16x16 crops of the 1024^2 workload as standalone images (Np = 32): the
    library's gradient of L = sum |P| over the brightest cells equals FP64
    central finite differences (h = 1e-4) and the dense transposed operator."""
    import torch
    say("gradient on 16x16 crops")
    imgs = synth.batch("grad", count=2, size=1024, seed=0)
    crops = np.stack([imgs[0].image[500:516, 300:316], imgs[1].image[100:116, 700:716]]).astype(np.float32)
    B, N, M = 2, 16, 16
    plan = F.FunnelPlan(B, N, M)
    Np = plan.Np
    x = torch.from_numpy(crops).cuda()
    planes = plan.forward(x)
    P = planes.cpu().numpy()
    dP = np.zeros_like(P)
    sels = []
    for b in range(B):
        # brightest 4 cells per space, away from zero so |.| is smooth there
        sel = np.argsort(-np.abs(P[b]))[:8]
        dP[b, sel] = np.sign(P[b, sel])
        sels.append(sel)
    grad = plan.adjoint(torch.from_numpy(dP).cuda()).cpu().numpy()
    Fr = pins.dense_forward(O, N, M, "regular")
    Fi = pins.dense_forward(O, N, M, "inverse")
    Fd = np.concatenate([Fr, Fi], axis=0)            # plane layout: regular then inverse
    for b in range(B):
        img = crops[b].astype(np.float64)
        sel = sels[b]

        def loss(xx):
            pr, pi = O.forward(xx, Np)
            return np.abs(np.concatenate([pr.ravel(), pi.ravel()])[sel]).sum()

        h = 1e-4
        fd = np.zeros((N, M))
        for i in range(N):
            for j in range(M):
                e = np.zeros((N, M))
                e[i, j] = h
                fd[i, j] = (loss(img + e) - loss(img - e)) / (2 * h)
        dense = (Fd[sel].T @ dP[b, sel].astype(np.float64)).reshape(N, M)
        assert np.abs(fd - dense).max() <= 1e-7 * np.abs(dense).max()
        assert rel_l2(grad[b], fd) <= TOL
        assert rel_l2(grad[b], dense) <= TOL
