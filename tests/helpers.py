import numpy as np


def rel_l2(got, want) -> float:
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    den = np.linalg.norm(want.ravel())
    return float(np.linalg.norm((got - want).ravel()) / (den if den > 0 else 1.0))


def nb_max(B, radius, wrap):
    """Largest value among each cell's (2r+1)^2 neighbours (itself excluded),
    toroidal or clamped at the plane's edges."""
    rows, cols = B.shape
    out = np.full(B.shape, -np.inf)
    for dr in range(-radius, radius + 1):
        for dc in range(-radius, radius + 1):
            if dr == 0 and dc == 0:
                continue
            if wrap:
                sh = np.roll(np.roll(B, -dr, axis=0), -dc, axis=1)
            else:
                sh = np.full(B.shape, -np.inf)
                r0, r1 = max(0, -dr), min(rows, rows - dr)
                c0, c1 = max(0, -dc), min(cols, cols - dc)
                sh[r0:r1, c0:c1] = B[r0 + dr:r1 + dr, c0 + dc:c1 + dc]
            out = np.maximum(out, sh)
    return out


def decidable_prefix(Bp, lst, nm, mask, eps):
    """Largest K such that the first K peaks of any plane within eps/2 of Bp
    (element-wise) are the oracle's first K: the first K+1 listed values are
    more than eps apart, and every cell at or above the (K+1)-th value (less
    eps) differs from its largest neighbour by more than eps, so no local
    maximum near the cut can appear, vanish or swap.  The threshold is 0 here,
    which |P| always meets."""
    vals = [Bp.flat[i] for i in lst]
    for K in range(len(lst) - 1, 0, -1):
        if any(abs(a - b) <= eps for a, b in zip(vals[:K], vals[1:K + 1])):
            continue
        region = (Bp >= vals[K] - eps) & ~mask
        if np.any(np.abs(Bp - nm)[region] <= eps):
            continue
        return K
    return 0


def peaks_match_on_decidable_prefix(O, got_ids, P_gpu, P_ref, tol, mask, K, min_prefix):
    """GPU peak list (cell ids) against the literal list on the oracle plane.
    Every cell of the GPU plane must be within tol * max|P| of the oracle's
    (the stated relative bound applied cell by cell; the largest errors sit at
    the peaks, where |P| is large).  Any plane within the measured deviation
    delta of the oracle's has the same first k peaks wherever every
    comparison deciding them is separated by more than 2 delta
    (decidable_prefix at 2.5 delta), so there the lists must agree, and at
    least min_prefix of the K peaks must be decided that way: a path whose
    error grew would decide fewer and fail.  Returns k."""
    Bp = np.abs(P_ref)
    delta = float(np.abs(np.abs(P_gpu) - Bp).max())
    assert delta <= tol * Bp.max(), (delta, tol * Bp.max())
    lst = O.peaks_list(Bp, K + 1, 0.0, 1, mask, True)
    k = decidable_prefix(Bp, lst, nb_max(Bp, 1, True), mask, 2.5 * delta)
    assert list(got_ids[:k]) == lst[:k], (k, list(got_ids[:k]), lst[:k])
    assert k >= min_prefix, (k, min_prefix, delta)
    return k
