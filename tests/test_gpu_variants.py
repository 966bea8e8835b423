"""Every tile variant of every launch against the FP64 oracle.  The plan
starts from default variants and the autotuner may pick any other, so each
one must compute the same transform: for every variant v (register tiles,
LDS-resident tiles, register tiles on a persistent grid), every launch that has a
variant v is switched to it and the forward planes and the adjoint are
compared with the oracle.  The shapes include the benchmark's lengths
(Np = 2048, rows of 1024) and those of the 8 x 2048^2 workload, so every
kernel instantiation a tuned plan can time there is compared too."""
import numpy as np
import pytest

from helpers import rel_l2
from oracle import funnel_oracle as O
from paper_1904_09409_amd import funnel as F
from paper_1904_09409_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("N,M", [
    (128, 128),     # power-of-two lengths: register-resident variants
    (96, 160),      # Np 256 (register-resident), rows 160 and 96 (LDS-resident)
    (240, 320),     # Np 560 = 16*5*7: LDS-resident column variants
    (720, 1280),    # Np 2000 = 16*5^3
    (1080, 1920),   # Np 3000 = 8*3*5^3
    (1024, 1024),   # Np 2048, rows 1024: the benchmark's lengths
    (2048, 2048),   # Np 4096, rows 2048: the 8 x 2048^2 workload's lengths
])
def test_every_variant_matches_oracle(N, M):
    import torch
    B = 2
    imgs = [synth.mixed_lines(N, M, (2, 6), 0.1, np.random.default_rng([31, N, M, i])) for i in range(B)]
    x = torch.from_numpy(np.stack([im.image for im in imgs])).cuda()
    plan = F.FunnelPlan(B, N, M)
    Np = plan.Np
    g = torch.Generator(device="cpu").manual_seed(N + M)
    dP = torch.randn((B, plan.plane_elems), generator=g, dtype=torch.float32)
    refP, refD = [], []
    for b in range(B):
        pr, pi = O.forward(imgs[b].image.astype(np.float64), Np)
        refP.append(np.concatenate([pr.ravel(), pi.ravel()]))
        d = dP[b].numpy().astype(np.float64)
        refD.append(O.adjoint(d[:Np * M].reshape(Np, M), d[Np * M:].reshape(Np, N), N, M, Np))
    dPc = dP.cuda()
    defaults = F.funnel_plan_variants(plan.handle)
    covered = 0
    for v in range(F.MAX_VARIANTS):
        roles = []
        for r in range(12):
            try:
                F.funnel_plan_set_variant(plan.handle, r, v)
                roles.append(r)
            except F.FunnelError:
                F.funnel_plan_set_variant(plan.handle, r, defaults[r])
        if not roles:
            continue
        planes = plan.forward(x)
        dI = plan.adjoint(dPc)
        torch.cuda.synchronize()
        P, G = planes.cpu().numpy(), dI.cpu().numpy()
        worst = max(max(rel_l2(P[b], refP[b]), rel_l2(G[b], refD[b])) for b in range(B))
        say(f"  {N}x{M} variant {v}: roles {roles} worst rel L2 {worst:.2e}")
        assert worst <= TOL, (v, roles, worst)
        covered += len(roles)
    assert covered >= 12
