"""Pins of the merge oracle (CPU only).

* the chi-square critical value against scipy;
* voxel cells against exact rational floors and brute-force dictionary grouping,
  with points placed exactly on voxel boundaries;
* Eq. (4) on axis-aligned covariances (closed form);
* Eq. (6) on equal and on isotropic covariances (closed forms);
* the Eq. (9) minimiser: commuting covariances (closed form), equal covariances,
  and an independent numerical minimisation of the Eq. (9) objective written
  with scipy's matrix square root, started from the Eq. (10) initial values;
* hand-built voxels for the sequential-insertion and best-pair readings.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize
import scipy.stats
from scipy.spatial.transform import Rotation

from oracle import merge as M


def test_chi2_critical_value():
    assert round(scipy.stats.chi2.ppf(0.95, 3), 3) == M.CHI2_3DOF_95


def test_voxel_cells_exact_floor_and_boundaries():
    rng = np.random.default_rng(0)
    v = 0.05
    pts = rng.uniform(-3, 3, size=(2000, 3)).astype(np.float32)
    cells, ok = M.voxel_cells(pts, v, np.ones(len(pts), bool))
    assert ok.all()
    v32 = Fraction(float(np.float32(v)))
    for p, c in zip(pts[:300], cells[:300]):
        for x, k in zip(p, c):
            q = Fraction(float(x)) / v32
            f = math.floor(q)
            # fp32 division rounds; away from boundaries it must equal the exact floor
            if abs(q - round(q)) > Fraction(1, 10**5):
                assert k == f
    # power-of-two voxel: boundaries representable exactly; x = k v lies in cell k
    v2 = 0.0625
    ks = np.arange(-40, 40)
    bpts = np.stack([ks * v2, -ks * v2, np.zeros_like(ks, dtype=np.float64)], axis=1).astype(np.float32)
    cells2, _ = M.voxel_cells(bpts, v2, np.ones(len(ks), bool))
    assert np.array_equal(cells2[:, 0], ks) and np.array_equal(cells2[:, 1], -ks)
    # grouping equals a brute-force dictionary
    groups = M.group_voxels(pts, v, np.ones(len(pts), bool))
    brute = {}
    for g, c in enumerate(cells):
        brute.setdefault(tuple(int(a) for a in c), []).append(g)
    assert groups == brute
    # non-finite and out-of-range means are not eligible
    bad = np.array([[np.nan, 0, 0], [1e30, 0, 0], [0.1, 0.1, 0.1]], np.float32)
    _, okb = M.voxel_cells(bad, v, np.ones(3, bool))
    assert okb.tolist() == [False, False, True]


def test_packed_key_order_is_lexicographic():
    rng = np.random.default_rng(1)
    cells = rng.integers(-50, 50, size=(500, 3))
    keys = M.packed_key(cells)
    order_k = np.argsort(keys, kind="stable")
    order_l = np.lexsort((cells[:, 2], cells[:, 1], cells[:, 0]))
    assert np.array_equal(cells[order_k], cells[order_l])


def test_mahalanobis_axis_aligned():
    s = np.array([0.02, 0.05, 0.1])
    S = np.diag(s ** 2)
    d = np.array([0.01, -0.03, 0.2])
    assert abs(M.mahalanobis2(d, np.zeros(3), S) - np.sum((d / s) ** 2)) < 1e-12


def test_merged_mean_closed_forms():
    rng = np.random.default_rng(2)
    A = rng.normal(size=(3, 3))
    S = A @ A.T + 0.1 * np.eye(3)
    mi, mj = rng.normal(size=3), rng.normal(size=3)
    np.testing.assert_allclose(M.merged_mean(mi, S, mj, S), 0.5 * (mi + mj), atol=1e-12)
    a, b = 0.3, 1.7
    np.testing.assert_allclose(M.merged_mean(mi, a * np.eye(3), mj, b * np.eye(3)), (b * mi + a * mj) / (a + b),
                               atol=1e-12)


def _w2sq_scipy(Sk, Si):
    r = scipy.linalg.sqrtm(Sk).real
    return float(np.trace(Sk + Si - 2 * scipy.linalg.sqrtm(r @ Si @ r).real))


def test_merged_cov_commuting_and_equal():
    rng = np.random.default_rng(3)
    R = Rotation.random(random_state=rng).as_matrix()
    si, sj = np.array([0.02, 0.05, 0.03]), np.array([0.04, 0.01, 0.03])
    Si, Sj = R @ np.diag(si ** 2) @ R.T, R @ np.diag(sj ** 2) @ R.T
    np.testing.assert_allclose(M.merged_cov(Si, Sj), R @ np.diag(((si + sj) / 2) ** 2) @ R.T, atol=1e-15)
    np.testing.assert_allclose(M.merged_cov(Si, Si), Si, atol=1e-15)


@pytest.mark.parametrize("seed", [4, 5, 6])
def test_merged_cov_minimises_w2_objective(seed):
    rng = np.random.default_rng(seed)

    def spd():
        R = Rotation.random(random_state=rng).as_matrix()
        s = np.exp(rng.normal(-3.5, 0.5, 3))
        return R, s, R @ np.diag(s ** 2) @ R.T

    Ri, si, Si = spd()
    Rj, sj, Sj = spd()
    scale = np.trace(Si + Sj)

    def obj(x):
        L = np.zeros((3, 3))
        L[np.tril_indices(3)] = x
        Sk = L @ L.T
        return (_w2sq_scipy(Sk, Si) + _w2sq_scipy(Sk, Sj)) / scale

    # Eq. (10) start: slerp(q_i, q_j, 0.5), mean of scales plus the small offsets
    qi, qj = Rotation.from_matrix(Ri).as_quat(), Rotation.from_matrix(Rj).as_quat()
    q0 = M.slerp_half(np.r_[qi[3], qi[:3]], np.r_[qj[3], qj[:3]])
    s0 = (si + sj) / 2 + np.array([0.001, 0.002, 0.003])
    S0 = M.cov_of(q0, s0)
    x0 = np.linalg.cholesky(S0)[np.tril_indices(3)]
    res = scipy.optimize.minimize(obj, x0, method="L-BFGS-B", options=dict(ftol=1e-15, gtol=1e-12, maxiter=5000))
    L = np.zeros((3, 3))
    L[np.tril_indices(3)] = res.x
    S_opt = L @ L.T
    S_cf = M.merged_cov(Si, Sj)
    assert obj(np.linalg.cholesky(S_cf)[np.tril_indices(3)]) <= res.fun * (1 + 1e-9) + 1e-15
    assert np.linalg.norm(S_opt - S_cf) / np.linalg.norm(S_cf) < 1e-3


def test_canonical_qs_reproduces_cov():
    rng = np.random.default_rng(7)
    for _ in range(20):
        A = rng.normal(size=(3, 3)) * 0.05
        S = A @ A.T + 1e-5 * np.eye(3)
        qref = rng.normal(size=4)
        qref /= np.linalg.norm(qref)
        q, s = M.canonical_qs(S, qref)
        assert q[0] >= 0 and abs(np.linalg.norm(q) - 1) < 1e-12
        np.testing.assert_allclose(M.cov_of(q, s), S, atol=1e-14)


def _gauss(mu, s, q=(1, 0, 0, 0)):
    return np.asarray(mu, np.float64), np.asarray(q, np.float64), np.asarray(s, np.float64)


def test_sequential_insertion_voxel():
    s = [0.01, 0.01, 0.01]
    # G0 and G1 are dissimilar (d^2 = 25 > 7.815); G2 sits 1 sigma from G1 and 4 sigma from G0.
    g = [_gauss([0.0, 0.0, 0.0], s), _gauss([0.05, 0.0, 0.0], s), _gauss([0.04, 0.0, 0.0], s)]
    means = np.array([x[0] for x in g])
    quats = np.array([x[1] for x in g])
    scales = np.array([x[2] for x in g])
    res, absorbed, flag = M.merge_voxel([0, 1, 2], means, quats, scales, policy=0)
    assert absorbed == [(2, 1)] and not flag
    assert set(res) == {0, 1}
    np.testing.assert_allclose(res[1][0], [0.045, 0, 0], atol=1e-15)   # equal covariances: midpoint
    # best-pair reading merges the same single pair
    res1, absorbed1, _ = M.merge_voxel([0, 1, 2], means, quats, scales, policy=1)
    assert absorbed1 == [(2, 1)]
    # a fourth Gaussian next to the merged resident merges into it (nearest resident)
    g4 = np.vstack([means, [[0.046, 0.0, 0.0]]])
    res4, absorbed4, _ = M.merge_voxel([0, 1, 2, 3], g4, np.vstack([quats, [1, 0, 0, 0]]),
                                       np.vstack([scales, s]), policy=0)
    assert absorbed4 == [(2, 1), (3, 1)]


def test_voxel_merge_compaction_and_mask():
    rng = np.random.default_rng(8)
    n = 400
    means = rng.uniform(0, 0.4, size=(n, 3)).astype(np.float32)
    means[n // 2:] = means[: n // 2] + rng.uniform(-0.002, 0.002, size=(n // 2, 3)).astype(np.float32)
    scales = np.full((n, 3), 0.01, np.float32)
    quats = np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1))
    elig = np.ones(n, bool)
    elig[::7] = False
    r = M.voxel_merge(means, quats, scales, 0.05, elig)
    assert r.n_out == r.alive.sum() < n
    assert np.all(r.alive[~elig])                       # ineligible Gaussians are never removed
    assert np.all(np.diff(r.old_to_new[r.alive]) == 1)  # stable compaction
    for j in np.nonzero(~r.alive)[0]:
        i = r.absorbed_into[j]
        assert i < j and r.alive[i] and r.merged[i]


# ---- Eq. (10) rotation of the merged Gaussian: the slerp reference and the
# choice among the 24 equivalent eigen-frames

def _wxyz(r):
    x, y, z, w = r.as_quat()
    return np.array([w, x, y, z])


def test_slerp_half_matches_scipy_slerp_on_shortest_path():
    from scipy.spatial.transform import Slerp
    rng = np.random.default_rng(21)
    for k in range(50):
        ra, rb = Rotation.random(random_state=rng), Rotation.random(random_state=rng)
        qa, qb = _wxyz(ra), _wxyz(rb)
        if k % 2:
            qb = -qb  # the same rotation, the other sign: the shortest path must still be taken
        mid = Slerp([0.0, 1.0], Rotation.concatenate([ra, rb]))([0.5])[0]
        got = M.slerp_half(qa, qb)
        assert abs(np.linalg.norm(got) - 1.0) < 1e-12
        np.testing.assert_allclose(M.rot(got), mid.as_matrix(), atol=1e-12)
        # either sign of either input gives the same rotation
        np.testing.assert_allclose(M.rot(M.slerp_half(-qa, qb)), mid.as_matrix(), atol=1e-12)


def test_slerp_half_closed_form_about_one_axis():
    # identity and a rotation by theta about n: halfway is the rotation by theta / 2
    n = np.array([1.0, -2.0, 0.5])
    n /= np.linalg.norm(n)
    for theta in (0.3, 1.7, 3.0):
        qj = np.r_[np.cos(theta / 2), np.sin(theta / 2) * n]
        got = M.slerp_half([1, 0, 0, 0], qj)
        np.testing.assert_allclose(got, np.r_[np.cos(theta / 4), np.sin(theta / 4) * n], atol=1e-14)
        # a negative dot product (theta > pi written as -q): still the short way
        got2 = M.slerp_half([1, 0, 0, 0], -qj)
        np.testing.assert_allclose(got2 * np.sign(got2[0]), got, atol=1e-14)


def _frames():
    """The 24 proper signed axis permutations P, with the permutation p such
    that column c of R P is +-column p[c] of R."""
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1.0, -1.0), repeat=3):
            P = np.zeros((3, 3))
            for c, r in enumerate(perm):
                P[r, c] = signs[c]
            if np.linalg.det(P) > 0:
                out.append((P, perm))
    return out


def test_canonical_qs_returns_the_reference_frame_and_its_scales():
    """Sigma = R diag(s^2) R^T with distinct s.  With q_ref the quaternion of
    R P for any of the 24 frames P, the canonical pair is (+-quat(R P)) and the
    scales follow the axes of R P.  Picking any fixed frame (the first
    eigenvector order, say) fails all but one case."""
    rng = np.random.default_rng(22)
    for trial in range(6):
        R = Rotation.random(random_state=rng).as_matrix()
        s = np.sort(rng.uniform(0.01, 0.05, 3))[rng.permutation(3)]
        S = R @ np.diag(s ** 2) @ R.T
        for P, perm in _frames():
            RP = R @ P
            q_ref = _wxyz(Rotation.from_matrix(RP))
            # a small perturbation of the reference keeps the same nearest frame
            q_ref = q_ref + rng.normal(scale=1e-3, size=4)
            q_ref /= np.linalg.norm(q_ref)
            q, sc = M.canonical_qs(S, q_ref)
            want = _wxyz(Rotation.from_matrix(RP))
            want = want * np.sign(want[0]) if want[0] != 0 else want
            assert q[0] >= 0
            np.testing.assert_allclose(q, want, atol=1e-9)
            np.testing.assert_allclose(sc, s[list(perm)], rtol=1e-12)


def test_canonical_qs_axis_swap_by_ninety_degrees():
    # R = identity, s = (1, 2, 3) cm.  A reference rotated 90 degrees about z
    # takes new x = old y and new y = -old x: scales (2, 1, 3) cm.
    s = np.array([0.01, 0.02, 0.03])
    S = np.diag(s ** 2)
    q, sc = M.canonical_qs(S, np.array([1.0, 0.0, 0.0, 0.0]))
    np.testing.assert_allclose(q, [1, 0, 0, 0], atol=1e-14)
    np.testing.assert_allclose(sc, s, rtol=1e-14)
    qz = np.array([np.cos(np.pi / 4), 0.0, 0.0, np.sin(np.pi / 4)])
    q, sc = M.canonical_qs(S, qz)
    np.testing.assert_allclose(q, qz, atol=1e-14)
    np.testing.assert_allclose(sc, [0.02, 0.01, 0.03], rtol=1e-14)
    # the sign of the reference does not matter
    q2, sc2 = M.canonical_qs(S, -qz)
    np.testing.assert_allclose(q2, qz, atol=1e-14)
    np.testing.assert_allclose(sc2, sc, rtol=1e-14)


def test_merge_of_two_gaussians_with_one_rotation_keeps_it():
    """Same rotation q, scales s_i and s_j: the merged Gaussian has rotation q
    (the slerp of q with itself) and scales (s_i + s_j) / 2 in q's own axis
    order (the commuting closed form of Eq. (9)), whatever the eigenvalue order."""
    rng = np.random.default_rng(23)
    for _ in range(10):
        q = _wxyz(Rotation.random(random_state=rng))
        q = q * np.sign(q[0])
        si = rng.uniform(0.01, 0.04, 3)
        sj = si * rng.uniform(0.9, 1.1, 3)
        mu = rng.uniform(0, 0.04, 3)
        means = np.array([mu, mu + 0.1 * si])
        quats = np.array([q, -q if rng.uniform() < 0.5 else q])
        res, absorbed, _ = M.merge_voxel([0, 1], means, quats, np.array([si, sj]), policy=0)
        assert absorbed == [(1, 0)]
        mu_k, S_k, q_k, s_k, merged, margin = res[0]
        assert margin > 1e-3
        assert merged
        np.testing.assert_allclose(q_k, q, atol=1e-9)
        np.testing.assert_allclose(s_k, (si + sj) / 2, rtol=1e-9)


def test_canonical_margin_flags_undecided_frames():
    """The margin is 0 where the frame is not determined: two equal scales
    (any rotation about that axis fits), or a reference halfway between two of
    the 24 frames (45 degrees about z from the identity's frame)."""
    s = np.array([0.01, 0.02, 0.03])
    _, _, m = M.canonical_qs_margin(np.diag(s ** 2), np.array([1.0, 0, 0, 0]))
    assert m > 0.1
    _, _, m = M.canonical_qs_margin(np.diag([1e-4, 1e-4, 9e-4]), np.array([1.0, 0, 0, 0]))
    assert m == 0.0
    q45 = np.array([np.cos(np.pi / 8), 0, 0, np.sin(np.pi / 8)])
    _, _, m = M.canonical_qs_margin(np.diag(s ** 2), q45)
    assert m < 1e-12
