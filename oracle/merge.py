"""Voxel-space merge of redundant Gaussians (Sec. II-D), numpy float64.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the benchmark's
CPU-baseline leg, never by the product path.

Steps, in the paper's order:
  1. the caller's eligibility mask M(G) of Eq. (3) selects candidates;
  2. candidates are grouped by voxel (integer cell of mean / voxel size);
  3. within a voxel, Gaussians are taken in insertion order (index order); for
     each newly inserted G_j the squared Mahalanobis distance of Eq. (4) to every
     Gaussian G_i already present is computed with the older one's covariance;
  4. the pair is similar when that squared distance is below the chi-square
     critical value 7.815 (3 degrees of freedom, 95 %);
  5. the merged mean is the closed form of Eq. (6) (the maximiser of Eq. (5));
  6. the merged covariance minimises the sum of squared 2-Wasserstein distances
     of Eq. (9); for two Gaussians that minimiser is the equal-weight W2
     barycenter, the midpoint of the displacement interpolation,
     Sigma_k = 1/4 (I + T) Sigma_i (I + T) with T the optimal map
     Sigma_i^{-1/2} (Sigma_i^{1/2} Sigma_j Sigma_i^{1/2})^{1/2} Sigma_i^{-1/2};
  7. rotation and scale of G_k come from the eigen-decomposition of Sigma_k,
     canonicalised towards the Eq. (10) initial rotation slerp(q_i, q_j, 0.5);
  8. colour and opacity of G_k are those of the older G_i; G_j is removed and the
     map is compacted, survivors keeping their relative order.

`merge_mask` forms M(G) of Eq. (3) from the gradient statistics of the
renderer's backward: the average 3D gradient below tau (0.001 in the paper)
and the insertion keyframe inside [K_min, K_max].

Readings where the paper is silent (listed in the design notes): more than two
Gaussians in a voxel are handled by sequential insertion (policy 0: each new
Gaussian merges into its nearest resident when similar, otherwise becomes a
resident) or by a single best pair per voxel (policy 1); the test uses the
squared distance; argmin ties go to the lowest index; merged means may leave
their voxel (no re-bucketing within one call).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np
from scipy.spatial.transform import Rotation

CHI2_3DOF_95 = 7.815
KEY_BIAS = 1 << 20


def voxel_cells(means: np.ndarray, voxel: float, eligible: np.ndarray):
    """Integer voxel cell of each Gaussian, decided in fp32 (correctly rounded
    division then floor).  Returns (cells [N,3] int64, eligible [N] bool):
    non-finite means and cells outside [-2^20, 2^20) are not eligible."""
    m32 = np.asarray(means, np.float32)
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        q = np.floor(m32 / np.float32(voxel))
    ok = np.all(np.isfinite(q), axis=1)
    ok &= np.all((q >= -KEY_BIAS) & (q < KEY_BIAS), axis=1)
    cells = np.where(ok[:, None], q, 0).astype(np.int64)
    return cells, np.asarray(eligible, bool) & ok


def packed_key(cells: np.ndarray) -> np.ndarray:
    """63-bit key: 21 bits per axis, biased by 2^20, x most significant."""
    c = cells + KEY_BIAS
    return (c[:, 0] << 42) | (c[:, 1] << 21) | c[:, 2]


def group_voxels(means, voxel, eligible) -> Dict[Tuple[int, int, int], List[int]]:
    cells, ok = voxel_cells(means, voxel, eligible)
    groups: Dict[Tuple[int, int, int], List[int]] = {}
    for g in np.nonzero(ok)[0]:
        groups.setdefault(tuple(int(v) for v in cells[g]), []).append(int(g))
    return groups


def rot(q) -> np.ndarray:
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q)
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


def quat_of(R) -> np.ndarray:
    x, y, z, w = Rotation.from_matrix(R).as_quat()
    return np.array([w, x, y, z])


def cov_of(q, s) -> np.ndarray:
    R = rot(q)
    return R @ np.diag(np.asarray(s, np.float64) ** 2) @ R.T


def sym_sqrt(S) -> np.ndarray:
    lam, V = np.linalg.eigh(S)
    return (V * np.sqrt(np.maximum(lam, 0.0))) @ V.T


def mahalanobis2(mu_j, mu_i, Sigma_i) -> float:
    """Eq. (4): (mu_j - mu_i)^T Sigma_i^{-1} (mu_j - mu_i)."""
    d = np.asarray(mu_j, np.float64) - np.asarray(mu_i, np.float64)
    return float(d @ np.linalg.solve(Sigma_i, d))


def merged_mean(mu_i, S_i, mu_j, S_j) -> np.ndarray:
    """Eq. (6)."""
    Pi, Pj = np.linalg.inv(S_i), np.linalg.inv(S_j)
    return np.linalg.solve(Pi + Pj, Pi @ mu_i + Pj @ mu_j)


def w2_sq(S_k, S_i) -> float:
    """Eq. (8): squared W2 distance between zero-mean Gaussians."""
    r = sym_sqrt(S_k)
    return float(np.trace(S_k + S_i - 2.0 * sym_sqrt(r @ S_i @ r)))


def merged_cov(S_i, S_j) -> np.ndarray:
    """Minimiser of Eq. (9): the equal-weight W2 barycenter of S_i and S_j."""
    A = sym_sqrt(S_i)
    Ainv = np.linalg.inv(A)
    T = Ainv @ sym_sqrt(A @ S_j @ A) @ Ainv
    IT = np.eye(3) + T
    Sk = 0.25 * IT @ S_i @ IT
    return 0.5 * (Sk + Sk.T)


def slerp_half(q_i, q_j) -> np.ndarray:
    """Eq. (10) initial rotation with t = 0.5 (shortest path)."""
    a = np.asarray(q_i, np.float64) / np.linalg.norm(q_i)
    b = np.asarray(q_j, np.float64) / np.linalg.norm(q_j)
    if a @ b < 0:
        b = -b
    m = a + b
    return m / np.linalg.norm(m)


def _proper_signed_perms():
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1.0, -1.0), repeat=3):
            P = np.zeros((3, 3))
            for col, row in enumerate(perm):
                P[row, col] = signs[col]
            if np.linalg.det(P) > 0:
                out.append((P, perm))
    return out


_PERMS = _proper_signed_perms()


def canonical_qs(S_k, q_ref):
    """(q, s) with R diag(s^2) R^T = S_k; among the 24 equivalent axis choices
    the one whose quaternion is closest to q_ref, with w >= 0."""
    q, s, _ = canonical_qs_margin(S_k, q_ref)
    return q, s


def canonical_qs_margin(S_k, q_ref):
    """canonical_qs plus how well decided its choice is: the smaller of the
    relative eigen-gap min |lam_a - lam_b| / max lam (the axes themselves) and
    the relative margin between the best and the second-best |<q, q_ref>|
    (the choice among the 24 frames).  A fp32 implementation can only be held
    to the same frame where this is well above its rounding."""
    lam, V = np.linalg.eigh(S_k)
    if np.linalg.det(V) < 0:
        V[:, 0] = -V[:, 0]
    best, best_dot, second = None, -1.0, -1.0
    for P, perm in _PERMS:
        R = V @ P
        q = quat_of(R)
        d = abs(float(q @ q_ref))
        if d > best_dot + 1e-12:
            s = np.sqrt(np.maximum(lam[list(perm)], 0.0))
            best, second, best_dot = (q, s), best_dot, d
        elif d > second:
            second = d
    q, s = best
    if q[0] < 0:
        q = -q
    lmax = max(float(lam.max()), 1e-300)
    gap = min(abs(lam[0] - lam[1]), abs(lam[1] - lam[2]), abs(lam[0] - lam[2])) / lmax
    margin = (best_dot - second) / max(best_dot, 1e-300)
    return q, s, min(gap, margin)


@dataclass
class MergeResult:
    alive: np.ndarray          # [N] bool
    means: np.ndarray          # [N,3] float64 (merged values at the resident's slot)
    quats: np.ndarray          # [N,4]
    scales: np.ndarray         # [N,3]
    covs: np.ndarray           # [N,3,3]
    merged: np.ndarray         # [N] bool: slot holds a merged Gaussian
    absorbed_into: np.ndarray  # [N] int64, -1 unless absorbed
    old_to_new: np.ndarray     # [N] int64, -1 if removed
    n_out: int
    flagged: set               # voxel cells whose decisions lie within the ambiguity band
    frame_margin: np.ndarray = None  # [N] smallest canonical_qs_margin of a merged slot's chain (inf otherwise)


def merge_voxel(members: List[int], means, quats, scales, chi2=CHI2_3DOF_95, policy=0,
                rel_band=1e-4):
    """Merge inside one voxel.  Returns (residents dict slot -> (mu, S, q, s, merged),
    absorbed list of (j, slot), flagged bool)."""
    residents: Dict[int, list] = {}
    order: List[int] = []
    absorbed = []
    flagged = False

    # resident state: mean, covariance, q, s, merged, and the smallest decision
    # margin of canonical_qs_margin over the merges that produced it (inf for
    # an original Gaussian); a chain's later frames depend on its earlier ones
    def state(g):
        mu = np.asarray(means[g], np.float64)
        q = np.asarray(quats[g], np.float64)
        q = q / np.linalg.norm(q)
        s = np.asarray(scales[g], np.float64)
        return [mu, cov_of(q, s), q, s, False, np.inf]

    if policy == 0:
        for j in members:
            sj = state(j)
            if order:
                d2 = np.array([mahalanobis2(sj[0], residents[r][0], residents[r][1]) for r in order])
                k = int(np.argmin(d2))
                if abs(d2[k] / chi2 - 1.0) < rel_band:
                    flagged = True
                srt = np.sort(d2)
                if len(srt) > 1 and srt[1] < chi2 and (srt[1] - srt[0]) <= rel_band * max(srt[1], 1e-30):
                    flagged = True
                if d2[k] < chi2:
                    r = order[k]
                    ri = residents[r]
                    mu = merged_mean(ri[0], ri[1], sj[0], sj[1])
                    S = merged_cov(ri[1], sj[1])
                    q, s, fm = canonical_qs_margin(S, slerp_half(ri[2], sj[2]))
                    residents[r] = [mu, S, q, s, True, min(ri[5], fm)]
                    absorbed.append((j, r))
                    continue
            residents[j] = sj
            order.append(j)
    else:
        for g in members:
            residents[g] = state(g)
        best = None
        d2s = []
        for a_idx, i in enumerate(members):
            for j in members[a_idx + 1:]:
                d2 = mahalanobis2(residents[j][0], residents[i][0], residents[i][1])
                d2s.append(d2)
                if best is None or d2 < best[0]:
                    best = (d2, i, j)
        if best is not None:
            if abs(best[0] / chi2 - 1.0) < rel_band:
                flagged = True
            srt = np.sort(np.array(d2s))
            if len(srt) > 1 and srt[0] < chi2 and (srt[1] - srt[0]) <= rel_band * max(srt[1], 1e-30):
                flagged = True
            if best[0] < chi2:
                _, i, j = best
                ri, rj = residents[i], residents[j]
                mu = merged_mean(ri[0], ri[1], rj[0], rj[1])
                S = merged_cov(ri[1], rj[1])
                q, s, fm = canonical_qs_margin(S, slerp_half(ri[2], rj[2]))
                residents[i] = [mu, S, q, s, True, fm]
                del residents[j]
                absorbed.append((j, i))
    return residents, absorbed, flagged


def voxel_merge(means, quats, scales, voxel, eligible=None, chi2=CHI2_3DOF_95, policy=0,
                voxels=None) -> MergeResult:
    """Whole-map merge.  `voxels` (optional) restricts the work to those cells
    (for sampled checks at full size); other Gaussians are left untouched."""
    m32 = np.asarray(means, np.float32)
    means = m32.astype(np.float64)
    N = means.shape[0]
    if eligible is None:
        eligible = np.ones(N, bool)
    groups = group_voxels(m32, voxel, eligible)
    alive = np.ones(N, bool)
    out_m = means.copy()
    out_q = np.asarray(quats, np.float64).copy()
    out_s = np.asarray(scales, np.float64).copy()
    covs = np.zeros((N, 3, 3))
    merged = np.zeros(N, bool)
    absorbed_into = np.full(N, -1, np.int64)
    frame_margin = np.full(N, np.inf)
    flagged = set()
    cells = groups.keys() if voxels is None else [tuple(v) for v in voxels]
    for cell in cells:
        members = groups.get(cell, [])
        if len(members) < 2:
            continue
        residents, absorbed, flag = merge_voxel(members, means, quats, scales, chi2, policy)
        if flag:
            flagged.add(cell)
        for j, r in absorbed:
            alive[j] = False
            absorbed_into[j] = r
        for r, st in residents.items():
            if st[4]:
                out_m[r], covs[r], out_q[r], out_s[r] = st[0], st[1], st[2], st[3]
                merged[r] = True
                frame_margin[r] = st[5]
    old_to_new = np.full(N, -1, np.int64)
    old_to_new[alive] = np.arange(int(alive.sum()))
    return MergeResult(alive, out_m, out_q, out_s, covs, merged, absorbed_into, old_to_new,
                       int(alive.sum()), flagged, frame_margin)


GRAD_TAU = 1e-3  # the paper's gradient threshold tau of Eq. (3)


def merge_mask(grad_sum, count, tau=GRAD_TAU, kf_index=None, kf_min=0, kf_max=2**31 - 1):
    """M(G) = [grad G < tau and K_min <= K <= K_max] (Eq. (3)) as uint8 [N].

    grad G is the average gradient of each Gaussian, sum / count, taken in fp32
    (the decision is an integer, so it is made in the precision the statistics
    are kept in).  A Gaussian that no view saw (count 0) has no average and is
    not eligible.  kf_index[i] is the keyframe at which Gaussian i entered the
    map (None: every Gaussian is inside the keyframe window)."""
    s32 = np.asarray(grad_sum, np.float32)
    c = np.asarray(count, np.int64)
    with np.errstate(divide="ignore", invalid="ignore"):
        avg = s32 / c.astype(np.float32)
    ok = (c > 0) & (avg < np.float32(tau))
    if kf_index is not None:
        k = np.asarray(kf_index, np.int64)
        ok &= (k >= kf_min) & (k <= kf_max)
    return ok.astype(np.uint8)
