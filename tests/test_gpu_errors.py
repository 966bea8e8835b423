"""The error contract of the hot calls on valid plans: every bad argument
gives its exact status code before any device work, and the caller's output
buffers keep their contents (sentinel-filled here).  Calls go straight
through the C ABI (ctypes), bypassing the binding's own checks."""
import ctypes
import math

import pytest

from paper_1904_09409_amd import funnel as F

pytestmark = pytest.mark.gpu

NAN = float("nan")
SENT = -12345


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    lib = F.load_library()
    plan = F.FunnelPlan(2, 64, 64)
    K = 8
    d = dict(
        lib=lib, plan=plan, K=K,
        images=torch.rand((2, 64, 64), device="cuda"),
        planes=torch.full((2, plan.plane_elems), float(SENT), device="cuda"),
        dimg=torch.full((2, 64, 64), float(SENT), device="cuda"),
        # 16 spare bytes so that ptr + 4 stays inside the allocation
        ws=torch.zeros(plan.ws.numel() + 64, dtype=torch.uint8, device="cuda"),
        pk_ws=torch.zeros(F.funnel_peaks_workspace_size(plan.handle, K) + 64, dtype=torch.uint8, device="cuda"),
        rf_ws=torch.zeros(F.funnel_refine_workspace_size(plan.handle, K) + 64, dtype=torch.uint8, device="cuda"),
        rec=torch.full((2, 2, K, F.PEAK_WORDS), SENT, dtype=torch.int32, device="cuda"),
        cnt=torch.full((2, 2), SENT, dtype=torch.int32, device="cuda"),
        chk=torch.full((2, 2, K, F.LINE_CHECK_WORDS), SENT, dtype=torch.int32, device="cuda"),
        ref=torch.full((2, 2, K, F.REFINED_WORDS), float(SENT), device="cuda"),
    )
    torch.cuda.synchronize()
    return d


def P(t, off=0):
    return ctypes.c_void_p(int(t.data_ptr()) + off)


def nbytes(t):
    return t.numel() * t.element_size()


def expect(code, st, *outs):
    import torch
    assert st == code, (F.status_string(st), F.last_error())
    assert F.last_error()
    torch.cuda.synchronize()
    for o in outs:
        if o.dtype == torch.int32:
            assert bool((o == SENT).all()), "an output was written by a rejected call"
        else:
            assert bool((o == float(SENT)).all()), "an output was written by a rejected call"


def test_forward_adjoint_errors(env):
    lib, plan, e = env["lib"], env["plan"], env
    h, need = plan.handle, F.funnel_workspace_size(plan.handle)
    img, pl, di, ws = e["images"], e["planes"], e["dimg"], e["ws"]
    for fn, src, dst in ((lib.funnel_forward, img, pl), (lib.funnel_adjoint, pl, di)):
        say(f"  {fn.__name__}")
        expect(F.FT_ERR_MISALIGNED, fn(h, P(src, 4), P(dst), P(ws), need, None), dst)
        expect(F.FT_ERR_MISALIGNED, fn(h, P(src), P(dst, 4), P(ws), need, None), dst)
        expect(F.FT_ERR_MISALIGNED, fn(h, P(src), P(dst), P(ws, 4), need, None), dst)
        expect(F.FT_ERR_MISALIGNED, fn(h, P(src), P(dst), P(ws, 8), need, None), dst)
        expect(F.FT_ERR_WORKSPACE_TOO_SMALL, fn(h, P(src), P(dst), P(ws), need - 1, None), dst)
        expect(F.FT_ERR_INVALID_ARG, fn(h, None, P(dst), P(ws), need, None), dst)
        expect(F.FT_ERR_INVALID_ARG, fn(h, P(src), None, P(ws), need, None), dst)
        expect(F.FT_ERR_INVALID_ARG, fn(h, P(src), P(dst), None, need, None), dst)
        expect(F.FT_ERR_INVALID_ARG, fn(None, P(src), P(dst), P(ws), need, None), dst)


def test_graph_errors(env):
    lib, plan, e = env["lib"], env["plan"], env
    h, need = plan.handle, F.funnel_workspace_size(plan.handle)
    g = ctypes.c_void_p(99)
    args = (P(e["images"]), P(e["planes"]), P(e["planes"]), P(e["dimg"]))
    for what in (0, 4, 0x80000001):
        expect(F.FT_ERR_INVALID_ARG, lib.funnel_graph_create(h, what, *args, P(e["ws"]), need, ctypes.byref(g)))
    expect(F.FT_ERR_MISALIGNED, lib.funnel_graph_create(h, F.FT_GRAPH_FORWARD, P(e["images"], 4), *args[1:],
                                                        P(e["ws"]), need, ctypes.byref(g)))
    expect(F.FT_ERR_WORKSPACE_TOO_SMALL, lib.funnel_graph_create(h, F.FT_GRAPH_ADJOINT, *args, P(e["ws"]), need - 1,
                                                                 ctypes.byref(g)))
    assert g.value is None


def test_peaks_errors(env):
    lib, plan, e = env["lib"], env["plan"], env
    h, K = plan.handle, env["K"]
    need = F.funnel_peaks_workspace_size(h, K)
    pl, rec, cnt, ws = e["planes"], e["rec"], e["cnt"], e["pk_ws"]

    def call(K=K, thr=0.0, radius=1, flags=0, planes=P(pl), r=P(rec), c=P(cnt), w=P(ws), n=need):
        return lib.funnel_peaks(h, planes, K, thr, radius, flags, r, c, w, n, None)

    for bad in (dict(K=0), dict(K=257), dict(K=-1), dict(radius=0), dict(radius=9), dict(thr=NAN),
                dict(flags=4), dict(flags=0x80000000), dict(planes=None), dict(r=None), dict(c=None),
                dict(w=None)):
        expect(F.FT_ERR_INVALID_ARG, call(**bad), rec, cnt)
    for bad in (dict(planes=P(pl, 4)), dict(r=P(rec, 4)), dict(c=P(cnt, 4)), dict(w=P(ws, 12))):
        expect(F.FT_ERR_MISALIGNED, call(**bad), rec, cnt)
    expect(F.FT_ERR_WORKSPACE_TOO_SMALL, call(n=need - 1), rec, cnt)
    # the workspace size grows with K: the size for K = 8 is short for K = 256
    if F.funnel_peaks_workspace_size(h, 256) > need:
        expect(F.FT_ERR_WORKSPACE_TOO_SMALL, call(K=256), rec, cnt)
    # infinite thresholds are valid (nothing, or everything, passes)
    assert call(thr=math.inf) == F.FT_OK


def test_verify_errors(env):
    lib, plan, e = env["lib"], env["plan"], env
    h, K = plan.handle, env["K"]
    img, rec, cnt, chk = e["images"], e["rec"], e["cnt"], e["chk"]

    def call(K=K, D=3, tau=0.1, lmin=16, i=P(img), r=P(rec), c=P(cnt), o=P(chk)):
        return lib.funnel_verify(h, i, r, c, K, D, tau, lmin, o, None)

    for bad in (dict(K=0), dict(K=257), dict(D=0), dict(D=4), dict(tau=NAN), dict(lmin=-1), dict(i=None),
                dict(r=None), dict(c=None), dict(o=None)):
        expect(F.FT_ERR_INVALID_ARG, call(**bad), chk)
    for bad in (dict(i=P(img, 4)), dict(r=P(rec, 4)), dict(c=P(cnt, 8)), dict(o=P(chk, 4))):
        expect(F.FT_ERR_MISALIGNED, call(**bad), chk)


def test_refine_errors(env):
    lib, plan, e = env["lib"], env["plan"], env
    h, K = plan.handle, env["K"]
    need = F.funnel_refine_workspace_size(h, K)
    img, rec, cnt, out, ws = e["images"], e["rec"], e["cnt"], e["ref"], e["rf_ws"]

    def call(K=K, iters=4, i=P(img), r=P(rec), c=P(cnt), o=P(out), w=P(ws), n=need, plan_h=h):
        return lib.funnel_refine(plan_h, i, r, c, K, iters, o, w, n, None)

    for bad in (dict(K=0), dict(K=257), dict(iters=-1), dict(iters=17), dict(i=None), dict(o=None),
                dict(w=None)):
        expect(F.FT_ERR_INVALID_ARG, call(**bad), out)
    for bad in (dict(i=P(img, 4)), dict(r=P(rec, 4)), dict(o=P(out, 4)), dict(w=P(ws, 4))):
        expect(F.FT_ERR_MISALIGNED, call(**bad), out)
    expect(F.FT_ERR_WORKSPACE_TOO_SMALL, call(n=need - 1), out)
    # refinement needs a uniform plan
    rp = F.RaggedPlan([(64, 64), (32, 96)])
    expect(F.FT_ERR_INVALID_ARG, call(plan_h=rp.handle), out)
    # and power-of-two row lengths
    odd = F.FunnelPlan(1, 96, 64)
    n_odd = F.funnel_refine_workspace_size(odd.handle, K)
    big = e["ws"].new_zeros(n_odd + 64)
    expect(F.FT_ERR_UNSUPPORTED_SIZE, call(plan_h=odd.handle, w=P(big), n=n_odd), out)


def test_volume_errors(env):
    import torch
    lib = env["lib"]
    vp = F.VolumePlan(1, 32, 32, 32)
    h, K = vp.handle, 4
    vol = torch.rand((1, 32, 32, 32), device="cuda")
    par = torch.full((1, vp.param_elems), float(SENT), device="cuda")
    need = F.funnel_volume_workspace_size(h)
    ws = torch.zeros(vp.ws.numel() + 64, dtype=torch.uint8, device="cuda")
    expect(F.FT_ERR_MISALIGNED, lib.funnel_volume_forward(h, P(vol, 4), P(par), P(ws), need, None), par)
    expect(F.FT_ERR_MISALIGNED, lib.funnel_volume_forward(h, P(vol), P(par, 8), P(ws), need, None), par)
    expect(F.FT_ERR_WORKSPACE_TOO_SMALL, lib.funnel_volume_forward(h, P(vol), P(par), P(ws), need - 1, None), par)
    expect(F.FT_ERR_INVALID_ARG, lib.funnel_volume_forward(h, None, P(par), P(ws), need, None), par)

    pneed = F.funnel_volume_peaks_workspace_size(h, K)
    pws = torch.zeros(pneed + 64, dtype=torch.uint8, device="cuda")
    rec = torch.full((1, 1, K, F.PLANE_PEAK_WORDS), SENT, dtype=torch.int32, device="cuda")
    cnt = torch.full((1, 1), SENT, dtype=torch.int32, device="cuda")

    def call(K=K, thr=0.0, radius=1, flags=0, p=P(par), r=P(rec), c=P(cnt), w=P(pws), n=pneed):
        return lib.funnel_volume_peaks(h, p, K, thr, radius, flags, r, c, w, n, None)

    for bad in (dict(K=0), dict(K=257), dict(radius=0), dict(radius=3), dict(thr=NAN), dict(flags=8),
                dict(p=None), dict(w=None)):
        expect(F.FT_ERR_INVALID_ARG, call(**bad), rec, cnt)
    for bad in (dict(p=P(par, 4)), dict(r=P(rec, 4)), dict(c=P(cnt, 4)), dict(w=P(pws, 4))):
        expect(F.FT_ERR_MISALIGNED, call(**bad), rec, cnt)
    expect(F.FT_ERR_WORKSPACE_TOO_SMALL, call(n=pneed - 1), rec, cnt)


def test_binding_rejects_short_buffers(env):
    """The binding checks extents, types and devices before calling: a short
    or mistyped buffer raises instead of being written past its end."""
    import torch
    plan = env["plan"]
    short = torch.empty((1, plan.plane_elems), device="cuda")
    with pytest.raises(ValueError):
        plan.forward(env["images"], short)
    with pytest.raises(ValueError):
        plan.forward(env["images"].double())
    with pytest.raises(ValueError):
        plan.forward(env["images"].cpu())
    with pytest.raises(ValueError):
        plan.adjoint(env["planes"], torch.empty((1, 64, 64), device="cuda"))
    with pytest.raises(ValueError):
        plan.peaks(short)
    rec_bad = torch.zeros((2, 2, 8, F.PEAK_WORDS), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        plan.verify(env["images"], rec_bad, env["cnt"])
    with pytest.raises(ValueError):
        plan.refine(env["images"], env["rec"], env["cnt"][:1])
    rp = F.RaggedPlan([(64, 64), (32, 96)])
    with pytest.raises(ValueError):
        rp.forward(torch.zeros(rp.image_floats - 4, device="cuda"))
    with pytest.raises(ValueError):
        rp.adjoint(torch.zeros(rp.plane_floats - 4, device="cuda"))
