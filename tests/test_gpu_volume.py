"""The funnel transform of volumes (App. A) on the GPU against the FP64 oracle.

Tolerance: rel L2 <= 1e-5 over each parameter volume, as for images: four
FP32 passes (z DFT, x' pass, y' pass, inverse omega_3 DFT), each a few
roundings of relative size 6e-8 per butterfly stage along every path, add in
quadrature to about 1e-6.  Peaks: bitwise identical lists on the same
parameter volume (the procedure is exact), and on the oracle's own volume
identical wherever the FP32 error cannot reorder the cells."""
import numpy as np
import pytest

from helpers import rel_l2
from oracle import funnel_oracle as O
from paper_1904_09409_amd import funnel as F
from paper_1904_09409_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5
ROW_ROLE, YCOL_ROLE = 1, 2


def say(*a):
    print(*a, flush=True)


def volumes(B, Nz, Ny, Nx, seed):
    return [synth.sheet_volume(Nz, Ny, Nx, (2, 4), 0.1, np.random.default_rng([91, seed, Nz, Ny, Nx, i]))
            for i in range(B)]


@pytest.mark.parametrize("B,Nz,Ny,Nx,pad", [
    (2, 32, 32, 32, 0),      # padded depth 96: LDS-resident column passes
    (3, 64, 32, 64, 0),      # 160; rows and columns differ
    (2, 64, 64, 64, 0),      # 192
    (2, 48, 96, 96, 0),      # 240; mixed-radix rows and columns
    (3, 72, 48, 40, 0),      # 160; a width that is not a multiple of the y' tile
    (2, 64, 128, 64, 320),   # enlarged padding
    (1, 128, 64, 128, 0),    # 320
])
def test_every_volume_variant_matches_oracle(B, Nz, Ny, Nx, pad):
    import torch
    say(f"volume {B} x {Nz}x{Ny}x{Nx} pad={pad}")
    vols = volumes(B, Nz, Ny, Nx, 1)
    x = torch.from_numpy(np.stack([v.volume for v in vols])).cuda()
    plan = F.VolumePlan(B, Nz, Ny, Nx, pad)
    refs = [O.forward_volume(v.volume.astype(np.float64), pad) for v in vols[:2]]
    defaults = F.funnel_volume_variants(plan.handle)
    assert defaults[4:] == [-1] * 8          # z space only
    tried = 0
    for role in (0, ROW_ROLE, YCOL_ROLE, 3):   # depth DFT, x' pass, y' pass, inverse w3 DFT
        for v in range(F.MAX_VARIANTS):
            try:
                F.funnel_volume_set_variant(plan.handle, role, v)
            except F.FunnelError:
                continue
            tried += 1
            P = plan.views(plan.forward(x))["z"]
            torch.cuda.synchronize()
            got = P.cpu().numpy()
            worst = max(rel_l2(got[b], refs[b]) for b in range(len(refs)))
            say(f"  role {role} variant {v}: worst rel L2 {worst:.2e}")
            assert worst <= TOL, (role, v, worst)
        F.funnel_volume_set_variant(plan.handle, role, defaults[role])
    assert tried >= 3


def test_volume_workload_256():
    """The benchmark shape, 4 x 256^3 (padded depth 768), autotuned: sampled
    (m2, m1) lines of two volumes against the oracle's per-line evaluation,
    every line through the whole padded depth."""
    import torch
    B, N = 4, 256
    say("volume workload 4 x 256^3")
    vols = synth.volume_batch(B, N, seed=0)
    x = torch.from_numpy(np.stack([v.volume for v in vols])).cuda()
    plan = F.VolumePlan(B, N, N, N)
    for r in plan.autotune():
        say(f"  tuned {r['name']}: variant {r['variant']} of {r['n_tried']} ({r['ms']:.3f} ms chain)")
    params = plan.forward(x)
    P = plan.views(params)["z"]
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    lines = [(int(r), int(c)) for r, c in zip(rng.integers(0, N, 6), rng.integers(0, N, 6))] + [(N // 2, N // 2)]
    for b in (1, 3):
        want = O.forward_volume_lines(vols[b].volume.astype(np.float64), lines)
        got = np.stack([P[b, :, r, c].cpu().numpy() for r, c in lines], axis=1)
        e = rel_l2(got, want)
        say(f"  volume {b}: {len(lines)} sampled lines rel L2 {e:.2e}")
        assert e <= TOL
    # every sheet of every volume is detected within one cell of its Eq. A.9 cell
    from pins import expected_cell_volume, torus_dist
    rec, cnt = plan.peaks(params, K=16)
    got = F.plane_peaks_to_numpy(rec, cnt)
    for b, v in enumerate(vols):
        for sh in v.sheets:
            z, r, c = expected_cell_volume(sh, N, N, N, plan.Nzp)
            assert any(torus_dist(int(g["z"]), z, plan.Nzp) <= 1 and torus_dist(int(g["row"]), r, N) <= 1
                       and torus_dist(int(g["col"]), c, N) <= 1 for g in got[b][0]), (b, sh, (z, r, c))
        say(f"  volume {b}: all {len(v.sheets)} sheets among the first 16 peaks")


@pytest.mark.parametrize("shape,radius,flags", [
    ((3, 64, 32, 64), 1, 0), ((3, 64, 32, 64), 2, 0), ((3, 64, 32, 64), 1, F.FT_PEAK_CLAMP_BORDER),
    ((3, 64, 32, 64), 1, F.FT_PEAK_KEEP_PAD_BOUNDARY),
    ((2, 72, 48, 40), 1, 0), ((2, 72, 48, 40), 2, F.FT_PEAK_CLAMP_BORDER),   # width below one tile
    ((2, 48, 96, 96), 1, 0), ((2, 48, 96, 96), 2, 0),                         # a full and a partial tile per row
])
def test_volume_peaks_exact_on_shared_volume(shape, radius, flags):
    """The GPU's 3D peak lists equal the oracle's list procedure run on the
    very same (GPU) parameter volumes, record by record; plane parameters
    within float rounding of Eq. A.9 read backwards.  Widths that fill the
    64-column tiles take the 16-byte staging path, the others the scalar one."""
    import torch
    (B, Nz, Ny, Nx), K = shape, 24
    say(f"volume peaks {shape} radius {radius} flags {flags}")
    vols = volumes(B, Nz, Ny, Nx, 2)
    x = torch.from_numpy(np.stack([v.volume for v in vols])).cuda()
    plan = F.VolumePlan(B, Nz, Ny, Nx)
    params = plan.forward(x)
    rec, cnt = plan.peaks(params, K=K, threshold=0.0, radius=radius, flags=flags)
    got = [g[0] for g in F.plane_peaks_to_numpy(rec, cnt)]
    Ph = plan.views(params)["z"].abs().cpu().numpy().astype(np.float64)
    mask = None if flags & F.FT_PEAK_KEEP_PAD_BOUNDARY else O.volume_boundary_mask(Nz, Ny, Nx, plan.Nzp)
    for b in range(B):
        want = O.peaks_list_volume(Ph[b], K, 0.0, radius, mask, wrap=not (flags & F.FT_PEAK_CLAMP_BORDER))
        idx = [(int(g["z"]) * Ny + int(g["row"])) * Nx + int(g["col"]) for g in got[b]]
        assert idx == want, (b, idx[:5], want[:5])
        for g in got[b]:
            a, bb, c = O.plane_params(int(g["z"]), int(g["row"]), int(g["col"]), Nz, Ny, Nx, plan.Nzp)
            assert g["value"] == np.float32(Ph[b].flat[(int(g["z"]) * Ny + int(g["row"])) * Nx + int(g["col"])])
            assert abs(g["a"] - a) <= 1e-6 and abs(g["b"] - bb) <= 1e-6 and abs(g["c"] - c) <= 1e-4 * max(1, abs(c))
    say(f"  counts {cnt.cpu().numpy().tolist()}")


def vpeak_volumes(kind, shape, rng):
    """|P|-like parameter volumes that drive each path of the 3D tile kernel."""
    nz, ny, nx = shape
    if kind == "noise":     # ~1/27 of the cells are maxima: about 76 keys per 8 x 4 x 64 tile
        return np.abs(rng.standard_normal(shape))
    if kind == "checker":   # a maximum at every (even, even, even) cell: 256 keys per tile
        P = 0.1 * rng.random(shape)
        P[::2, ::2, ::2] += 1.0 + rng.random((nz // 2, ny // 2, nx // 2))
        return P
    if kind == "levels":    # five levels: exact ties everywhere
        return np.floor(rng.random(shape) * 5.0) / 5.0
    raise ValueError(kind)


@pytest.mark.parametrize("radius,K", [(1, 16), (2, 40)])
def test_volume_peaks_exact_many_tiles(radius, K):
    """Parameter volumes of 3,072 tiles each, more than the GPU runs at once,
    so most tiles see a cutoff published by earlier ones: lists identical to
    the literal procedure on the same FP32 volumes, for the register sort,
    the block sort of more than 128 keys and exact ties."""
    import torch
    B, Nz, Ny, Nx = 3, 128, 128, 128
    say(f"volume peaks many tiles radius {radius} K {K}")
    plan = F.VolumePlan(B, Nz, Ny, Nx)
    params = plan.forward(torch.zeros((B, Nz, Ny, Nx), dtype=torch.float32, device="cuda"))
    Pz = plan.views(params)["z"]
    rng = np.random.default_rng([73, radius, K])
    kinds = ["noise", "checker", "levels"]
    host = [vpeak_volumes(k, tuple(Pz.shape[1:]), rng).astype(np.float32) for k in kinds]
    Pz.copy_(torch.from_numpy(np.stack(host)))
    rec, cnt = plan.peaks(params, K=K, threshold=0.0, radius=radius)
    got = [g[0] for g in F.plane_peaks_to_numpy(rec, cnt)]
    for rep in range(2):   # which keys the partial lists hold depends on timing; the result does not
        rec2, cnt2 = plan.peaks(params, K=K, threshold=0.0, radius=radius)
        assert [[g.tolist() for g in v] for v in F.plane_peaks_to_numpy(rec2, cnt2)] == \
            [[g.tolist() for g in v] for v in F.plane_peaks_to_numpy(rec, cnt)], rep
    mask = O.volume_boundary_mask(Nz, Ny, Nx, plan.Nzp)
    for b in range(B):
        want = O.peaks_list_volume(host[b].astype(np.float64), K, 0.0, radius, mask, True)
        idx = [(int(g["z"]) * Ny + int(g["row"])) * Nx + int(g["col"]) for g in got[b]]
        assert idx == want, (kinds[b], idx[:5], want[:5])
    say(f"  counts {cnt.cpu().numpy().tolist()}")


def _close_call(Po, i, delta):
    """Whether FP32 error (delta) could change cell i's place in the order or
    its local-maximum status: a neighbour within 2 delta of its |P|."""
    nz, ny, nx = Po.shape
    z, rem = divmod(i, ny * nx)
    r, c = divmod(rem, nx)
    v = Po[z, r, c]
    win = Po[np.ix_([(z + d) % nz for d in (-1, 0, 1)], [(r + d) % ny for d in (-1, 0, 1)],
                    [(c + d) % nx for d in (-1, 0, 1)])].copy()
    win[1, 1, 1] = np.inf
    return np.abs(win - v).min() <= 2 * delta


def test_volume_peaks_find_the_planes():
    """Plane -> point on the GPU: each volume holds 2-4 sheets (widths 1-2
    voxels, noise 0.1).  The GPU's peak list equals the oracle's list on its
    own FP64 volume up to the first place where FP32 error can decide (two
    candidates within twice the largest |P| error of each other, or a cell
    with a neighbour that close), and every sheet's Eq. A.9 cell is within
    one cell of a detected peak."""
    import torch
    from pins import expected_cell_volume, torus_dist
    B, Nz, Ny, Nx, K = 3, 64, 64, 64, 8
    say("volume peaks find the planes")
    vols = volumes(B, Nz, Ny, Nx, 3)
    x = torch.from_numpy(np.stack([v.volume for v in vols])).cuda()
    plan = F.VolumePlan(B, Nz, Ny, Nx)
    params = plan.forward(x)
    P = plan.views(params)["z"]
    rec, cnt = plan.peaks(params, K=K)
    got = [g[0] for g in F.plane_peaks_to_numpy(rec, cnt)]
    mask = O.volume_boundary_mask(Nz, Ny, Nx, plan.Nzp)
    for b, v in enumerate(vols):
        Po = np.abs(O.forward_volume(v.volume.astype(np.float64)))
        delta = float(np.abs(np.abs(P[b].cpu().numpy()) - Po).max())
        want = O.peaks_list_volume(Po, K, 0.0, 1, mask, True)
        idx = [(int(g["z"]) * Ny + int(g["row"])) * Nx + int(g["col"]) for g in got[b]]
        agree = 0
        for k in range(min(len(idx), len(want))):
            if idx[k] != want[k]:
                flat = Po.ravel()
                assert abs(flat[idx[k]] - flat[want[k]]) <= 2 * delta or _close_call(Po, idx[k], delta) \
                    or _close_call(Po, want[k], delta), (b, k, idx[k], want[k])
                break
            agree += 1
        assert agree >= min(len(v.sheets), K), (b, agree)
        for sh in v.sheets:
            z, r, c = expected_cell_volume(sh, Nz, Ny, Nx, plan.Nzp)
            near = [g for g in got[b] if torus_dist(int(g["z"]), z, plan.Nzp) <= 1
                    and torus_dist(int(g["row"]), r, Ny) <= 1 and torus_dist(int(g["col"]), c, Nx) <= 1]
            assert near, (b, sh, (z, r, c))
        say(f"  volume {b}: {len(v.sheets)} sheets found; lists agree on the first {agree} peaks "
            f"(FP32 error {delta:.1e})")


def test_volume_profile_and_errors():
    """Kernel timing records the four launches with their algorithmic bytes;
    bad calls are rejected before any launch."""
    import torch
    plan = F.VolumePlan(2, 32, 32, 32)
    x = torch.rand((2, 32, 32, 32), device="cuda")
    F.funnel_volume_profile_enable(plan.handle, 16)
    plan.forward(x)
    recs = {r["name"]: r for r in F.funnel_volume_profile_read(plan.handle)}
    F.funnel_volume_profile_disable(plan.handle)
    assert set(recs) == {"volume.A", "volume.Bx", "volume.By", "volume.C"}
    h, lines = 96 // 2 - 1, 32 * 32
    assert recs["volume.By"]["bytes_per_launch"] == 2 * 16.0 * h * lines
    with pytest.raises(F.FunnelError):
        plan.peaks(plan.forward(x), K=0)
    with pytest.raises(F.FunnelError):
        plan.peaks(plan.forward(x), K=4, radius=3)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(F.FunnelError):
        F.funnel_volume_forward(plan.handle, x, plan.new_params(), small)
    with pytest.raises(F.FunnelError):
        F.funnel_volume_set_variant(plan.handle, 5, 0)   # x space: not computed by this plan
    plan3 = F.VolumePlan(2, 32, 32, 32, spaces=F.FT_VOL_SPACE_ALL)
    F.funnel_volume_profile_enable(plan3.handle, 32)
    plan3.forward(x)
    names = {r["name"] for r in F.funnel_volume_profile_read(plan3.handle)}
    F.funnel_volume_profile_disable(plan3.handle)
    assert names == {f"volume.{s}{r}" for s in ("", "x.", "y.") for r in ("A", "Bx", "By", "C")} | {"volume.y.T"}


# ---------------------------------------------------------------- x and y spaces

def world_sheet(space, sh, Nz, Ny, Nx, rng):
    """A sheet of the given space (depth = a col + b row + c in that space's
    axes) rendered in the world volume [Nz, Ny, Nx], background 0."""
    frame = {"z": ((Nz, Ny, Nx), (0, 1, 2)), "x": ((Nx, Nz, Ny), (1, 2, 0)), "y": ((Ny, Nz, Nx), (1, 0, 2))}
    (D, R, C), back = frame[space]
    return np.transpose(synth.render_volume(D, R, C, [sh], 0.0, rng, bg=0.0), back)


@pytest.mark.parametrize("B,Nz,Ny,Nx", [(2, 64, 32, 64), (2, 48, 96, 96)])
def test_volume_spaces_match_oracle(B, Nz, Ny, Nx):
    """All three spaces against the oracle's transform of the volume in each
    space's axis order, for every x' and y' tile variant of the x and y
    spaces (whose rows and columns are the volume's other axes)."""
    import torch
    say(f"volume spaces {B} x {Nz}x{Ny}x{Nx}")
    vols = volumes(B, Nz, Ny, Nx, 4)
    x = torch.from_numpy(np.stack([v.volume for v in vols])).cuda()
    plan = F.VolumePlan(B, Nz, Ny, Nx, spaces=F.FT_VOL_SPACE_ALL)
    assert [n for n, _, _ in plan.space_list] == ["z", "x", "y"]
    refs = {n: [O.forward_volume_space(v.volume.astype(np.float64), n) for v in vols] for n in ("z", "x", "y")}
    defaults = F.funnel_volume_variants(plan.handle)
    assert min(defaults) >= 0
    tried = 0
    for role in (5, 6, 9, 10):   # x space Bx, By; y space Bx, By
        for v in range(12):
            try:
                F.funnel_volume_set_variant(plan.handle, role, v)
            except F.FunnelError:
                continue
            tried += 1
            views = plan.views(plan.forward(x))
            torch.cuda.synchronize()
            worst = max(rel_l2(views[n][b].cpu().numpy(), refs[n][b]) for n in ("z", "x", "y") for b in range(B))
            say(f"  role {role} variant {v}: worst rel L2 over the spaces {worst:.2e}")
            assert worst <= TOL, (role, v, worst)
        F.funnel_volume_set_variant(plan.handle, role, defaults[role])
    assert tried >= 6


def test_volume_steep_planes_found():
    """One sheet of each orientation in one volume: the z sheet focuses in
    the z space, the steep ones (x = a y + b z + c, y = a x + b z + c) in the x
    and y spaces, each within one cell of its Eq. A.9 cell and among the
    first four peaks of its space; plane parameters read back within a cell."""
    import torch
    from pins import expected_cell_volume, torus_dist
    Nz, Ny, Nx = 64, 32, 64
    rng = np.random.default_rng(93)
    geo = {"z": (Nz, Ny, Nx), "x": (Nx, Nz, Ny), "y": (Ny, Nz, Nx)}
    sheets = {}
    vol = np.zeros((Nz, Ny, Nx))
    for n, (D, R, C) in geo.items():
        a, b = float(rng.uniform(-0.7, 0.7)), float(rng.uniform(-0.7, 0.7))
        dc = float(rng.uniform(0.4 * D, 0.6 * D))
        sheets[n] = synth.Sheet(a, b, dc - a * C / 2 - b * R / 2, 1.0)
        vol += world_sheet(n, sheets[n], Nz, Ny, Nx, rng)
    vol = (vol + rng.normal(0.0, 0.02, vol.shape)).astype(np.float32)
    plan = F.VolumePlan(1, Nz, Ny, Nx, spaces=F.FT_VOL_SPACE_ALL)
    params = plan.forward(torch.from_numpy(vol[None].copy()).cuda())
    rec, cnt = plan.peaks(params, K=4)
    got = F.plane_peaks_to_numpy(rec, cnt)[0]
    for si, n in enumerate(("z", "x", "y")):
        D, R, C = geo[n]
        z, r, c = expected_cell_volume(sheets[n], D, R, C, plan.Lp)
        hit = [g for g in got[si] if torus_dist(int(g["z"]), z, plan.Lp) <= 1 and torus_dist(int(g["row"]), r, R) <= 1
               and torus_dist(int(g["col"]), c, C) <= 1]
        assert hit and int(hit[0]["space"]) == si, (n, (z, r, c), got[si])
        sh = sheets[n]
        say(f"  {n} space: sheet a={sh.a:.3f} b={sh.b:.3f} c={sh.c:.2f} -> peak a={hit[0]['a']:.3f} "
            f"b={hit[0]['b']:.3f} c={hit[0]['c']:.2f}")
        # within one cell of the rounded cell: half a bin of rounding plus one bin
        assert abs(hit[0]["a"] - sh.a) <= 3.0 / C + 1e-6 and abs(hit[0]["b"] - sh.b) <= 3.0 / R + 1e-6


def test_volume_peaks_exact_all_spaces():
    """Each space's 3D peak list equals the oracle's list procedure on that
    space's (GPU) parameter volumes, with that space's face cells."""
    import torch
    B, Nz, Ny, Nx, K = 2, 48, 96, 96, 12
    vols = volumes(B, Nz, Ny, Nx, 5)
    x = torch.from_numpy(np.stack([v.volume for v in vols])).cuda()
    plan = F.VolumePlan(B, Nz, Ny, Nx, spaces=F.FT_VOL_SPACE_ALL)
    params = plan.forward(x)
    views = plan.views(params)
    rec, cnt = plan.peaks(params, K=K)
    got = F.plane_peaks_to_numpy(rec, cnt)
    depth = {"z": Nz, "x": Nx, "y": Ny}
    for si, (n, R, C) in enumerate(plan.space_list):
        Ph = views[n].abs().cpu().numpy().astype(np.float64)
        mask = O.volume_boundary_mask(depth[n], R, C, plan.Lp)
        for b in range(B):
            want = O.peaks_list_volume(Ph[b], K, 0.0, 1, mask, True)
            idx = [(int(g["z"]) * R + int(g["row"])) * C + int(g["col"]) for g in got[b][si]]
            assert idx == want, (n, b, idx[:4], want[:4])
            assert all(int(g["space"]) == si and int(g["volume"]) == b for g in got[b][si])
            for g in got[b][si]:
                a, bb, c = O.plane_params(int(g["z"]), int(g["row"]), int(g["col"]), depth[n], R, C, plan.Lp)
                assert abs(g["a"] - a) <= 1e-6 and abs(g["b"] - bb) <= 1e-6 and abs(g["c"] - c) <= 1e-4 * max(1, abs(c))
