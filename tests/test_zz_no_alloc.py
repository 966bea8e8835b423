"""funnel_peaks_noalloc, the peak call that needs no workspace (its scratch
is a static device array), against funnel_peaks with a workspace: identical
lists on two calls in a row, the second on a smaller input, and a clear error
for a plan whose scratch need exceeds the static array."""
import ctypes

import numpy as np
import pytest

from paper_1904_09409_amd import funnel as F
from paper_1904_09409_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def noalloc(lib, plan, planes, K, thr, radius, flags, rec, cnt):
    return lib.funnel_peaks_noalloc(plan.handle, ctypes.c_void_p(planes.data_ptr()), K, thr, radius, flags,
                                    ctypes.c_void_p(rec.data_ptr()), ctypes.c_void_p(cnt.data_ptr()),
                                    ctypes.c_void_p(torch_stream()))


def torch_stream():
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("first,second", [
    ((8, 512, 512, 32, 0.0, 1, 0), (2, 128, 128, 8, 0.0, 2, F.FT_PEAK_CLAMP_BORDER)),
])
def test_noalloc_matches_workspace_call(first, second):
    import torch
    lib = F.load_library()
    for call, (B, N, M, K, thr, radius, flags) in enumerate((first, second)):
        say(f"  call {call}: {B} x {N}x{M}, K={K}, radius {radius}, flags {flags}")
        imgs = [synth.mixed_lines(N, M, (3, 8), 0.1, np.random.default_rng([71, call, i])).image for i in range(B)]
        plan = F.FunnelPlan(B, N, M)
        planes = plan.forward(torch.from_numpy(np.stack(imgs)).cuda())
        want_rec, want_cnt = plan.peaks(planes, K=K, threshold=thr, radius=radius, flags=flags)
        rec = torch.full_like(want_rec, -7)
        cnt = torch.full_like(want_cnt, -7)
        st = noalloc(lib, plan, planes, K, thr, radius, flags, rec, cnt)
        assert st == F.FT_OK, F.last_error()
        torch.cuda.synchronize()
        assert torch.equal(cnt, want_cnt)
        assert int(cnt.min()) >= 1
        for b in range(B):
            for s in range(plan.nspaces):
                n = int(cnt[b, s])
                assert torch.equal(rec[b, s, :n], want_rec[b, s, :n]), (call, b, s)
        # the binding's method (checks the buffers, then the same C call)
        rec2, cnt2 = torch.full_like(want_rec, -7), torch.full_like(want_cnt, -7)
        plan.peaks_noalloc(planes, rec2, cnt2, threshold=thr, radius=radius, flags=flags)
        torch.cuda.synchronize()
        assert torch.equal(cnt2, cnt) and torch.equal(rec2, rec)
        with pytest.raises(ValueError):
            plan.peaks_noalloc(planes, rec2[:, :, :, :3], cnt2)


def test_noalloc_rejects_beyond_scratch():
    import torch
    lib = F.load_library()
    plan = F.FunnelPlan(32, 1024, 1024)
    K = 256
    need = F.funnel_peaks_workspace_size(plan.handle, K)
    limit = 64 << 20
    assert need > limit
    planes = torch.zeros(16, device="cuda")
    rec = torch.full((4, F.PEAK_WORDS), -7, dtype=torch.int32, device="cuda")
    cnt = torch.full((4,), -7, dtype=torch.int32, device="cuda")
    st = noalloc(lib, plan, planes, K, 0.0, 1, 0, rec, cnt)
    assert st == F.FT_ERR_WORKSPACE_TOO_SMALL
    assert "scratch" in F.last_error()
    torch.cuda.synchronize()
    assert bool((rec == -7).all()) and bool((cnt == -7).all())
    # K = 16 on the same plan fits (17 MB)
    assert F.funnel_peaks_workspace_size(plan.handle, 16) <= limit
