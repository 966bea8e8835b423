"""HIP path (through the C ABI) against the FP64 oracle, element by element.

Bar: relative L2 error <= 1e-5 per plane for the FP32 forward and adjoint;
peak indices identical (bitwise when both sides see the same FP32 plane, and
end to end wherever the oracle's own ordering margin is clear)."""
import numpy as np
import pytest

from helpers import rel_l2
from oracle import funnel_oracle as O
from paper_1904_09409_amd import funnel as F
from paper_1904_09409_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _torch():
    import torch
    return torch


def say(*a):
    print(*a, flush=True)


def run_forward(images, padded_len=0, spaces=F.FT_SPACE_BOTH):
    torch = _torch()
    B, N, M = images.shape
    plan = F.FunnelPlan(B, N, M, padded_len, spaces)
    x = torch.from_numpy(images).cuda()
    planes = plan.forward(x)
    torch.cuda.synchronize()
    return plan, planes


def oracle_planes(img, Np, spaces):
    out = []
    if spaces & F.FT_SPACE_REGULAR:
        out.append(O.forward_regular(img, Np))
    if spaces & F.FT_SPACE_INVERSE:
        out.append(O.forward_inverse(img, Np))
    return out


def gpu_planes(plan, planes, b):
    v = plan.views(planes)
    out = []
    if v.regular is not None:
        out.append(v.regular[b].cpu().numpy())
    if v.inverse is not None:
        out.append(v.inverse[b].cpu().numpy())
    return out


SMALL = [
    # (N, M, padded_len, spaces, batch)
    (8, 8, 0, 3, 2),
    (16, 16, 0, 3, 3),
    (40, 24, 0, 3, 2),       # mixed radix 8x3, 8x5; one partial column tile
    (80, 48, 0, 3, 2),       # several column tiles and a ragged tail
    (128, 128, 0, 3, 2),
    (96, 160, 0, 3, 1),
    (64, 64, 160, 1, 2),     # explicit padded length, regular space only
    (64, 64, 0, 2, 2),       # inverse space only
    (240, 320, 0, 3, 1),     # smallest ragged-workload size, Np = 560
]


@pytest.mark.parametrize("N,M,pad,spaces,B", SMALL)
def test_forward_matches_oracle(N, M, pad, spaces, B):
    say(f"forward parity N={N} M={M} pad={pad} spaces={spaces} B={B}")
    rng = np.random.default_rng(N * 1000 + M)
    images = rng.random((B, N, M)).astype(np.float32)
    plan, planes = run_forward(images, pad, spaces)
    for b in range(B):
        want = oracle_planes(images[b].astype(np.float64), plan.Np, spaces)
        got = gpu_planes(plan, planes, b)
        for g, w in zip(got, want):
            assert g.shape == w.shape
            e = rel_l2(g, w)
            assert e <= TOL, (b, e)


@pytest.mark.parametrize("N,M,pad,spaces,B", SMALL)
def test_adjoint_matches_oracle(N, M, pad, spaces, B):
    torch = _torch()
    say(f"adjoint parity N={N} M={M} pad={pad} spaces={spaces} B={B}")
    plan = F.FunnelPlan(B, N, M, pad, spaces)
    rng = np.random.default_rng(7 + N + M)
    dP = rng.standard_normal((B, plan.plane_elems)).astype(np.float32)
    dI = plan.adjoint(torch.from_numpy(dP).cuda())
    torch.cuda.synchronize()
    dI = dI.cpu().numpy()
    Np = plan.Np
    for b in range(B):
        off = 0
        want = np.zeros((N, M))
        if spaces & F.FT_SPACE_REGULAR:
            want += O.adjoint_regular(dP[b, off:off + Np * M].reshape(Np, M).astype(np.float64), N, M, Np)
            off += Np * M
        if spaces & F.FT_SPACE_INVERSE:
            want += O.adjoint_inverse(dP[b, off:off + Np * N].reshape(Np, N).astype(np.float64), N, M, Np)
        e = rel_l2(dI[b], want)
        assert e <= TOL, (b, e)


def test_adjoint_dot_product_on_gpu():
    """<F x, y> = <x, F^T y> with both sides computed by the library."""
    torch = _torch()
    say("gpu dot test 96x160")
    B, N, M = 2, 96, 160
    plan = F.FunnelPlan(B, N, M)
    g = torch.Generator(device="cuda").manual_seed(3)
    x = torch.rand((B, N, M), device="cuda", generator=g)
    y = torch.randn((B, plan.plane_elems), device="cuda", generator=g)
    lhs = (plan.forward(x).double() * y.double()).sum().item()
    rhs = (x.double() * plan.adjoint(y).double()).sum().item()
    assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), 1.0)


def test_run_to_run_bitwise():
    """No atomics: two runs give identical bits."""
    torch = _torch()
    say("bitwise determinism 128x128")
    rng = np.random.default_rng(5)
    images = rng.random((3, 128, 128)).astype(np.float32)
    plan = F.FunnelPlan(3, 128, 128)
    x = torch.from_numpy(images).cuda()
    a = plan.forward(x).clone()
    b = plan.forward(x)
    assert torch.equal(a, b)
    d1 = plan.adjoint(a).clone()
    d2 = plan.adjoint(a)
    assert torch.equal(d1, d2)
    r1, c1 = plan.peaks(a, K=8)
    r2, c2 = plan.peaks(a, K=8)
    assert torch.equal(c1, c2) and torch.equal(r1, r2)


def test_autograd_function():
    torch = _torch()
    say("autograd 64x64")
    plan = F.FunnelPlan(2, 64, 64)
    x = torch.rand((2, 64, 64), device="cuda", requires_grad=True)
    planes = F.funnel_transform(x, plan)
    w = torch.randn_like(planes)
    (planes * w).sum().backward()
    want = plan.adjoint(w)
    assert torch.allclose(x.grad, want)
