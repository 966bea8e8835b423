"""The band-limited (chirp-z) NVMT plans against the FP64 oracle.

Tolerance: rel L2 <= 1e-5 over each plane and gradient, as for the linear
NVMT.  The chirp-z row pass adds two FFTs of length 2W and three complex
products per element in FP32 (about 12 roundings of relative size 6e-8 along
each path, adding in quadrature) on top of the column passes, so the expected
error stays near 1e-6 (the chirp tables are FP64 values rounded once)."""
import numpy as np
import pytest

from helpers import rel_l2
from oracle import funnel_oracle as O
from paper_1904_09409_amd import funnel as F
from paper_1904_09409_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5
ROW_ROLES = (1, 4, 7, 10)     # fwd.regular.B, fwd.inverse.B, adj.regular.Bt, adj.inverse.Bt


def say(*a):
    print(*a, flush=True)


def split(flat, N, M, Np, spaces):
    out, off = [], 0
    if spaces & F.FT_SPACE_REGULAR:
        out.append(flat[off:off + Np * M].reshape(Np, M))
        off += Np * M
    if spaces & F.FT_SPACE_INVERSE:
        out.append(flat[off:off + Np * N].reshape(Np, N))
    return out


def oracle_pair(img, dflat, N, M, Np, spaces):
    """Oracle planes (list, in plan order) and image gradient."""
    img = img.astype(np.float64)
    planes, grad = [], np.zeros((N, M))
    parts = split(dflat.astype(np.float64), N, M, Np, spaces)
    k = 0
    if spaces & F.FT_SPACE_REGULAR:
        planes.append(O.forward_regular(img, Np, "chirpz"))
        grad += O.adjoint_regular(parts[k], N, M, Np, "chirpz")
        k += 1
    if spaces & F.FT_SPACE_INVERSE:
        planes.append(O.forward_inverse(img, Np, "chirpz"))
        grad += O.adjoint_inverse(parts[k], N, M, Np, "chirpz")
    return planes, grad


@pytest.mark.parametrize("B,N,M,Np,spaces", [
    (3, 64, 64, 0, 3),       # rows of 64: one block covers every image
    (9, 128, 64, 0, 3),      # Np 192; 9 images: several image groups and a ragged tail
    (3, 64, 256, 0, 3),      # Np 320 = 64 * 5
    (2, 256, 128, 512, 3),   # padded beyond N + M
    (3, 96, 64, 0, 1),       # regular space only (the inverse row length 96 has no chirp-z kernel)
    (2, 128, 512, 0, 2),     # inverse space only, Np 640
    (2, 512, 512, 0, 3),     # Np 1024, rows of 512
])
def test_every_chirpz_variant_matches_oracle(B, N, M, Np, spaces):
    import torch
    say(f"chirp-z {B} x {N}x{M} Np={Np} spaces={spaces}")
    imgs = [synth.mixed_lines(N, M, (2, 6), 0.1, np.random.default_rng([61, N, M, i])) for i in range(B)]
    x = torch.from_numpy(np.stack([im.image for im in imgs])).cuda()
    plan = F.FunnelPlan(B, N, M, Np, spaces, nvmt="chirpz")
    g = torch.Generator(device="cpu").manual_seed(N * 3 + M)
    dP = torch.randn((B, plan.plane_elems), generator=g, dtype=torch.float32)
    refs = [oracle_pair(imgs[b].image, dP[b].numpy(), N, M, plan.Np, spaces) for b in range(min(B, 3))]
    dPc = dP.cuda()
    defaults = F.funnel_plan_variants(plan.handle)
    tried = 0
    for v in range(12):
        roles = []
        for r in ROW_ROLES:
            if defaults[r] < 0:      # a role of the space this plan does not compute
                continue
            try:
                F.funnel_plan_set_variant(plan.handle, r, v)
                roles.append(r)
            except F.FunnelError:
                F.funnel_plan_set_variant(plan.handle, r, defaults[r])
        if not roles:
            continue
        tried += 1
        planes = plan.forward(x)
        dI = plan.adjoint(dPc)
        torch.cuda.synchronize()
        P, G = planes.cpu().numpy(), dI.cpu().numpy()
        worst = 0.0
        for b, (rp, rg) in enumerate(refs):
            errs = [rel_l2(got, exp) for got, exp in zip(split(P[b], N, M, plan.Np, spaces), rp)]
            errs.append(rel_l2(G[b], rg))
            worst = max(worst, *errs)
        say(f"  row variant {v} (roles {roles}): worst rel L2 {worst:.2e}")
        assert worst <= TOL, (v, worst)
    assert tried >= 2


# ---------------------------------------------------------------- 32 x 1024^2

def test_chirpz_workload_1024():
    """The benchmark shape (32 x 1024^2, both spaces) with an autotuned
    chirp-z plan.  Forward planes on sampled slope columns of two images; the
    adjoint of each space alone on sampled image columns (regular) and rows
    (inverse = columns of the transposed image); the adjoint identity over the
    whole batch."""
    import torch
    B, N = 32, 1024
    say("chirp-z workload 32 x 1024^2")
    imgs = synth.batch("grad", count=B, size=N, seed=0)
    x = torch.from_numpy(synth.stack(imgs)).cuda()
    plan = F.FunnelPlan(B, N, N, nvmt="chirpz")
    F.funnel_autotune(plan.handle)
    Np = plan.Np
    planes = plan.forward(x)
    v = plan.views(planes)
    rng = np.random.default_rng(5)
    cols = np.sort(rng.choice(N, 6, replace=False))
    for b in (0, 21):
        img = imgs[b].image.astype(np.float64)
        e_r = rel_l2(v.regular[b].cpu().numpy()[:, cols], O.forward_regular_columns(img, cols, Np, "chirpz"))
        e_i = rel_l2(v.inverse[b].cpu().numpy()[:, cols], O.forward_regular_columns(img.T, cols, Np, "chirpz"))
        say(f"  image {b}: sampled columns rel L2 regular {e_r:.2e} inverse {e_i:.2e}")
        assert max(e_r, e_i) <= TOL
    g = torch.Generator(device="cuda").manual_seed(13)
    y = torch.randn(planes.shape, device="cuda", generator=g)
    for space in ("regular", "inverse"):
        dP = y.clone()
        dv = plan.views(dP)
        (dv.inverse if space == "regular" else dv.regular).zero_()
        dI = plan.adjoint(dP)
        torch.cuda.synchronize()
        for b in (3, 30):
            d = (dv.regular if space == "regular" else dv.inverse)[b].cpu().numpy().astype(np.float64)
            if space == "regular":
                got = dI[b].cpu().numpy()[:, cols]
                exp = O.adjoint_regular_columns(d, N, N, cols, Np, "chirpz")
            else:
                got = dI[b].cpu().numpy()[cols, :].T
                exp = O.adjoint_regular_columns(d, N, N, cols, Np, "chirpz")
            e = rel_l2(got, exp)
            say(f"  adjoint {space} image {b}: sampled rel L2 {e:.2e}")
            assert e <= TOL
    Aty = plan.adjoint(y)
    lhs = (planes.double() * y.double()).sum().item()
    rhs = (x.double() * Aty.double()).sum().item()
    scale = (planes.double() * y.double()).abs().sum().item() + (x.double() * Aty.double()).abs().sum().item()
    say(f"  adjoint identity |diff|/scale {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-8 * scale


def test_chirpz_peaks_512():
    """Peaks of chirp-z planes (4 x 512^2, 6-10 lines): identical to the
    oracle's on every decidable prefix."""
    import torch
    from test_gpu_precision import check_peaks
    B, N = 4, 512
    say("chirp-z peaks 4 x 512^2")
    imgs = [synth.mixed_lines(N, N, (6, 10), 0.1, np.random.default_rng([67, i])) for i in range(B)]
    x = torch.from_numpy(np.stack([im.image for im in imgs])).cuda()
    plan = F.FunnelPlan(B, N, N, nvmt="chirpz")
    planes = plan.forward(x)
    rec, cnt = plan.peaks(planes, K=16)
    torch.cuda.synchronize()
    got = F.peaks_to_numpy(rec, cnt)
    v = plan.views(planes)
    mask = O.boundary_mask(N, N, plan.Np)
    decided = []
    for b in range(2):
        pr, pi = O.forward(imgs[b].image.astype(np.float64), plan.Np, "chirpz")
        gr, gi = v.regular[b].cpu().numpy(), v.inverse[b].cpu().numpy()
        assert max(rel_l2(gr, pr), rel_l2(gi, pi)) <= TOL
        decided += check_peaks(got, b, (gr, gi), (pr, pi), mask, (TOL, TOL))


def test_chirpz_graph_replays_match_eager():
    """A captured forward + adjoint of a chirp-z plan replays bitwise equal to
    the eager calls, with eager work in between."""
    import torch
    say("chirp-z graph replay")
    plan = F.FunnelPlan(5, 128, 256, nvmt="chirpz")
    x = torch.rand((5, 128, 256), device="cuda")
    planes = plan.new_planes()
    dP = torch.randn_like(planes)
    dI = torch.zeros_like(x)
    g = F.FunnelGraph(plan, F.FT_GRAPH_FORWARD | F.FT_GRAPH_ADJOINT, x, planes, dP, dI)
    ref_p = plan.forward(x).clone()
    ref_d = plan.adjoint(dP).clone()
    for rep in range(3):
        planes.zero_()
        dI.fill_(7.0)
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(planes, ref_p), rep
        assert torch.equal(dI, ref_d), rep
        plan.forward(x * 0.5)
        torch.cuda.synchronize()
