"""Pins of the oracle's level-of-detail parts against the mathematics and
the paper, independent of the oracle's own formulas.

* Parents (Sec. 3 "Level of Detail", read as opacity-weighted moment
  matching of 8 children): the parent Gaussian must be the mixture's first
  and second moments.  Expected moments come from the law of total
  covariance with rotations built by scipy (not by the oracle's quaternion
  code), and from Monte Carlo samples of the mixture; the parent's
  covariance is rebuilt from its stored scales and quaternion, again with
  scipy's rotation.
* Level rule (Sec. 4.1 "Level of Detail"): exact boundary cases, and pages
  placed by hand at distances that put their projected radius on either side
  of tau and tau / 2.
* Controller (Sec. 5.1.1): a trace worked by hand from the paper's
  sentence (tests/golden/lod_controller_trace.json).
"""
import dataclasses
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from paper_2506_19415_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _rec(mean, scale, quat_wxyz, opacity, sh):
    r = np.zeros(59, np.float32)
    r[0:3] = mean
    r[3:6] = scale
    q = np.asarray(quat_wxyz, np.float64)
    r[6:10] = q / np.linalg.norm(q)
    r[10] = opacity
    r[11:] = np.asarray(sh, np.float32).reshape(-1)
    return r


def _rot(q_wxyz):
    q = np.asarray(q_wxyz, np.float64)
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


def _cov_of(rec):
    """Covariance of a stored record, rotation from scipy."""
    R = _rot(rec[6:10])
    s = np.asarray(rec[3:6], np.float64)
    return R @ np.diag(s * s) @ R.T


def _mixture_moments(children):
    """Opacity-weighted mixture mean and covariance (law of total covariance)."""
    w = children[:, 10].astype(np.float64)
    mu_i = children[:, 0:3].astype(np.float64)
    W = w.sum()
    mu = (w[:, None] * mu_i).sum(0) / W
    cov = np.zeros((3, 3))
    for k in range(children.shape[0]):
        d = mu_i[k] - mu
        cov += w[k] * (_cov_of(children[k]) + np.outer(d, d))
    return mu, cov / W


# Unit quaternions whose float32 components are exactly of norm 1 (the 24
# rotations of the cube): children stored with them have a rotation that is
# exact, so the moments can be pinned at 1e-9.  A general quaternion stored in
# float32 is unit only to about 1e-7, which bounds any pin to that level.
def _exact_quats():
    qs = []
    for i in range(4):
        for sgn in (1.0, -1.0):
            q = np.zeros(4)
            q[i] = sgn
            qs.append(q)
    for bits in range(16):
        qs.append(np.array([0.5 if (bits >> j) & 1 else -0.5 for j in range(4)]))
    return [q for q in qs if q[0] >= 0]


EXACT_Q = _exact_quats()


def _random_children(rng, k=8, spread=0.5, exact_rot=True):
    out = []
    for _ in range(k):
        q = EXACT_Q[rng.integers(len(EXACT_Q))] if exact_rot else rng.normal(size=4)
        out.append(_rec(rng.uniform(-spread, spread, 3), np.exp(rng.normal(-2.5, 0.6, 3)),
                        q, rng.uniform(0.05, 1.0), rng.normal(0, 0.3, 48)))
    return np.stack(out)


def _check_parent(children, parent_d, tol=1e-9):
    mu, cov = _mixture_moments(children)
    assert np.allclose(parent_d[0:3], mu, rtol=0, atol=1e-12 * (1 + np.abs(mu).max()))
    q = parent_d[6:10]
    assert abs(np.linalg.norm(q) - 1.0) < 1e-12
    assert q[0] >= 0.0
    R = _rot(q)
    assert abs(np.linalg.det(R) - 1.0) < 1e-12
    s = parent_d[3:6]
    # descending, up to the rounding of the eigenvalues of a repeated root
    assert s[0] >= s[1] * (1 - 1e-12) and s[1] >= s[2] * (1 - 1e-12) and s[2] >= 0.0, s
    rebuilt = R @ np.diag(s * s) @ R.T
    scale = np.abs(cov).max()
    assert np.abs(rebuilt - cov).max() <= tol * scale, (rebuilt, cov)


def test_parent_of_identical_children_is_the_child():
    rng = np.random.default_rng(11)
    for o, q in zip((0.05, 0.1, 0.2, 0.9), EXACT_Q[3:]):
        child = _rec([1.0, -2.0, 0.5], [0.3, 0.02, 0.1], q, o, rng.normal(0, 0.3, 48))
        kids = np.stack([child] * 8)
        p = oracle.merge_children_d(kids)
        assert np.allclose(p[0:3], child[0:3], rtol=0, atol=1e-12)
        assert np.abs(_cov_of(p) - _cov_of(child)).max() <= 1e-9 * 0.09
        assert sorted(p[3:6].tolist(), reverse=True) == pytest.approx(sorted(child[3:6].astype(float).tolist(),
                                                                             reverse=True), rel=1e-9)
        assert p[10] == pytest.approx(min(1.0, 8 * float(child[10])), rel=1e-12)
        assert np.allclose(p[11:], child[11:], rtol=1e-12, atol=1e-15)


def test_parent_matches_mixture_moments():
    rng = np.random.default_rng(12)
    for _ in range(50):
        kids = _random_children(rng)
        _check_parent(kids, oracle.merge_children_d(kids))
    # general float32 quaternions: unit only to float precision
    for _ in range(50):
        kids = _random_children(rng, exact_rot=False)
        _check_parent(kids, oracle.merge_children_d(kids), tol=1e-6)


def test_parent_sh_and_opacity():
    rng = np.random.default_rng(13)
    kids = _random_children(rng)
    p = oracle.merge_children_d(kids)
    w = kids[:, 10].astype(np.float64)
    sh = (w[:, None] * kids[:, 11:].astype(np.float64)).sum(0) / w.sum()
    assert np.allclose(p[11:], sh, rtol=1e-12, atol=1e-15)
    assert p[10] == pytest.approx(min(1.0, w.sum()), rel=1e-12)
    kids[:, 10] = 0.02
    assert oracle.merge_children_d(kids)[10] == pytest.approx(8 * float(np.float32(0.02)), rel=1e-12)


def test_parent_scale_up():
    """The fixed scale-up of the merged Gaussian (Sec. 3 Level of Detail):
    the parent's covariance is the mixture's times the factor squared; mean,
    rotation, opacity and colour are those of plain moment matching."""
    rng = np.random.default_rng(16)
    for k in (1.25, 1.6, 2.0):
        for _ in range(20):
            kids = _random_children(rng)
            p1 = oracle.merge_children_d(kids)
            pk = oracle.merge_children_d(kids, scale_up=k)
            mu, cov = _mixture_moments(kids)
            assert np.abs(_cov_of(pk) - k * k * cov).max() <= 1e-9 * k * k * np.abs(cov).max()
            assert np.array_equal(pk[0:3], p1[0:3]) and np.array_equal(pk[6:], p1[6:])
            assert np.allclose(pk[3:6], k * p1[3:6], rtol=1e-15, atol=0)


def test_parent_covariance_by_sampling():
    """Sample covariance of the opacity-weighted mixture (no formula of the
    moments involved) against the parent's covariance."""
    rng = np.random.default_rng(14)
    kids = _random_children(rng, spread=0.3)
    p = oracle.merge_children_d(kids)
    w = kids[:, 10].astype(np.float64)
    n = 400_000
    comp = rng.choice(8, size=n, p=w / w.sum())
    z = rng.standard_normal((n, 3))
    pts = np.empty((n, 3))
    for k in range(8):
        m = comp == k
        R = _rot(kids[k, 6:10])
        pts[m] = kids[k, 0:3] + (z[m] * kids[k, 3:6].astype(np.float64)) @ R.T
    emp = np.cov(pts.T)
    cov = _cov_of(p)
    assert np.abs(emp - cov).max() < 0.02 * np.abs(cov).max()
    assert np.abs(pts.mean(0) - p[0:3]).max() < 0.01 * math.sqrt(np.abs(cov).max())


def test_parent_repeated_eigenvalues():
    """Triple and double eigenvalues, axis-aligned and rotated: the parent's
    scales and rotation must still rebuild the mixture covariance."""
    rng = np.random.default_rng(15)
    sig, h = 0.1, 0.3
    # eight isotropic children at one mean: sigma^2 I
    kids = np.stack([_rec([2.0, 1.0, 0.0], [sig] * 3, EXACT_Q[k], 0.5, np.zeros(48)) for k in range(8)])
    p = oracle.merge_children_d(kids)
    assert np.allclose(p[3:6], sig, rtol=1e-7)
    _check_parent(kids, p)
    # isotropic children at +-h along one axis: diag(s^2, s^2, s^2 + h^2), a double eigenvalue
    for rot in (np.eye(3), Rotation.from_rotvec([0.3, -1.1, 0.7]).as_matrix()):
        kids = []
        for k in range(8):
            off = rot @ np.array([0.0, 0.0, h if k < 4 else -h])
            kids.append(_rec(off, [sig] * 3, EXACT_Q[k], 0.25 + 0.05 * (k % 4), np.zeros(48)))
        kids = np.stack(kids)
        p = oracle.merge_children_d(kids)
        _check_parent(kids, p)
        assert p[3] == pytest.approx(math.sqrt(sig * sig + h * h), rel=1e-7)
        assert p[4] == pytest.approx(sig, rel=1e-6) and p[5] == pytest.approx(sig, rel=1e-6)
    # flat coplanar splats (surface Gaussians): a tiny third eigenvalue
    kids = []
    n_rot = Rotation.from_rotvec([0.9, 0.2, -0.4])
    for k in range(8):
        local = np.array([rng.uniform(-0.4, 0.4), rng.uniform(-0.4, 0.4), 0.0])
        q = n_rot * Rotation.from_rotvec([0.0, 0.0, rng.uniform(0, 3)])
        x, y, z, w = q.as_quat()
        kids.append(_rec(n_rot.apply(local), [0.2, 0.15, 0.002], [w, x, y, z], rng.uniform(0.3, 1.0), np.zeros(48)))
    kids = np.stack(kids)
    _check_parent(kids, oracle.merge_children_d(kids), tol=1e-6)
    # the same with the plane along a cube axis (exact rotations)
    kids = []
    for k in range(8):
        local = np.array([rng.uniform(-0.4, 0.4), rng.uniform(-0.4, 0.4), 0.0])
        kids.append(_rec(local, [0.2, 0.15, 0.002], EXACT_Q[k % 2], rng.uniform(0.3, 1.0), np.zeros(48)))
    kids = np.stack(kids)
    p = oracle.merge_children_d(kids)
    _check_parent(kids, p)
    assert p[5] == pytest.approx(0.002, rel=1e-6)


def test_padding_parent_and_stored_record():
    kids = np.zeros((8, 59), np.float32)
    assert not oracle.merge_children_d(kids).any()
    rng = np.random.default_rng(16)
    kids = _random_children(rng)
    kids[:3, 10] = 0.0          # zero-opacity children carry no weight
    p = oracle.merge_children_d(kids)
    _check_parent(kids[3:], oracle.merge_children_d(kids[3:]))
    assert np.allclose(p, oracle.merge_children_d(kids[3:]), rtol=1e-12, atol=1e-15)
    # the stored record is the double record rounded to float
    assert np.array_equal(oracle.merge_children(kids), p.astype(np.float32))


def test_lod_level_boundaries():
    """Level l is the first with fy * R / depth > tau / 2^l: a projected
    radius equal to a threshold belongs to the coarser side."""
    fy, R, tau = 1000.0, 1.0, 32.0
    # 1000 / 31.25 = 32 and 1000 / 62.5 = 16 exactly
    assert oracle.lod_level(fy, R, 31.25, tau, 3) == 1
    assert oracle.lod_level(fy, R, float(np.nextafter(np.float32(31.25), np.float32(0))), tau, 3) == 0
    assert oracle.lod_level(fy, R, 62.5, tau, 3) == 2
    assert oracle.lod_level(fy, R, float(np.nextafter(np.float32(62.5), np.float32(0))), tau, 3) == 1
    assert oracle.lod_level(fy, R, 1e6, tau, 3) == 2
    assert oracle.lod_level(fy, R, 1e6, tau, 2) == 1
    assert oracle.lod_level(fy, R, 1e6, tau, 1) == 0
    assert oracle.lod_level(fy, R, 1.0, tau, 3) == 0
    # four levels: the thresholds keep halving (32, 16, 8)
    assert oracle.lod_level(fy, R, 124.0, tau, 4) == 2
    assert oracle.lod_level(fy, R, 125.0, tau, 4) == 3


def _wall_scene(x0, side=2.0, n_side=16):
    """One page: a flat square of Gaussians in the plane x = x0, facing -x."""
    g = (np.arange(n_side) + 0.5) / n_side * side - side / 2
    yy, zz = np.meshgrid(g, g, indexing="ij")
    n = n_side * n_side
    means = np.stack([np.full(n, x0), yy.ravel(), zz.ravel() + 5.0], 1).astype(np.float32)
    scales = np.tile(np.array([[0.001, 0.01, 0.01]], np.float32), (n, 1))
    quats = np.tile(np.array([[1.0, 0, 0, 0]], np.float32), (n, 1))
    opacity = np.full(n, 0.9, np.float32)
    sh = np.zeros((n, 16, 3), np.float32)
    sh[:, 0, :] = 1.0
    return synth.Scene(means, scales, quats, opacity, sh, (means.min(0), means.max(0)), None)


def test_lod_level_of_hand_placed_pages():
    """A page seen straight on at a chosen distance gets the level its
    projected radius (fy times the page sphere radius over the depth of
    its nearest pixel) gives; fy, not fx, sets the radius."""
    W, H = 320, 240
    sc = _wall_scene(10.0)
    osc = oracle.OracleScene(sc, 256, 3, 0.5, 2.0)
    R = float(osc.get("spheres")[3])
    # the sphere is the half-diagonal of the box of mean +- 3 sigma (rounded
    # outward): half extents 3 * 0.001 across the wall, 15/16 + 3 * 0.01 along it
    h = 15.0 / 16.0 + 0.03
    r_box = math.sqrt(0.003 ** 2 + 2 * h * h)
    assert r_box <= R <= r_box * (1 + 1e-6), (R, r_box)
    tau = 32.0
    for fx_scale, rpx_target, want in [(1.0, 1.25 * tau, 0), (1.0, 0.75 * tau, 1), (1.0, 0.375 * tau, 2),
                                       (1.0, 0.2 * tau, 2), (3.0, 0.75 * tau, 1)]:
        fy = 300.0
        depth = fy * R / rpx_target
        # aimed at a cell centre: the proxy boxes (of the means in each 0.5 m
        # cell) leave gaps between cells, which the far views' few ID pixels
        # could fall into
        cam = synth.look_at([10.0 - depth, 0.25, 5.25], [1.0, 0.0, 0.0], W, H, 60.0)
        cam = dataclasses.replace(cam, fx=fy * fx_scale, fy=fy)
        vm = oracle.OracleVM(osc, 4, (W, H), (80, 60), lod_radius_px=tau)
        vm.frame([cam])
        lvl = vm.get("page_level")
        assert int(lvl[0]) == want, (fx_scale, rpx_target, int(lvl[0]))
        d = float(vm.get("req_direct")[0:1].view(np.float32)[0])
        assert d == pytest.approx(depth, rel=1e-5)


def test_lod_controller_trace():
    g = json.load(open(os.path.join(HERE, "golden", "lod_controller_trace.json")))
    fr = g["frames"]
    tau, step = oracle.lod_control_trace(g["S"], g["tau0"], [f["req_slots"] for f in fr],
                                         [f["missing"] for f in fr], [f["coarse"] for f in fr])
    for i, f in enumerate(fr):
        assert float(tau[i]) == pytest.approx(f["tau"], rel=1e-6), (i, f["why"])
        assert float(step[i]) == pytest.approx(f["step"], rel=1e-6), (i, f["why"])


def test_lod_controller_limits():
    """tau stays within [2^-7, 2^16] px; under the band with nothing coarse,
    or inside the band, it does not move."""
    n = 300
    tau, _ = oracle.lod_control_trace(10, 32.0, [10] * n, [5] * n, [1] * n)
    assert float(tau[-1]) == 65536.0 and np.all(np.diff(tau) >= 0)
    tau, _ = oracle.lod_control_trace(10, 32.0, [1] * n, [0] * n, [1] * n)
    assert float(tau[-1]) == 0.0078125 and np.all(np.diff(tau) <= 0)
    tau, step = oracle.lod_control_trace(10, 32.0, [1] * n, [0] * n, [0] * n)
    assert np.all(tau == 32.0) and np.all(step == 0.125)
    tau, step = oracle.lod_control_trace(10, 32.0, [6] * n, [0] * n, [3] * n)
    assert np.all(tau == 32.0) and np.all(step == 0.125)


def test_lod_controller_ignores_budget_deferrals():
    """Pages the copy budget defers are no sign of memory use: with a pool
    that holds the whole scene and a budget of two pages per frame, the cold
    frames leave requests missing, yet the thresholds only move finer (usage
    under 50 % with coarse requests), as they do without the budget.
    Counting those deferrals as over the band would push tau up every frame."""
    sc = synth.scene_clusters(0)
    osc = oracle.OracleScene(sc, 256, 3, 0.5, 2.0)
    cams = synth.orbit()
    taus = {}
    for budget in (0, 2):
        vm = oracle.OracleVM(osc, 256, (320, 240), (80, 60), copy_budget=budget, lod_radius_px=32.0)
        vm.set_adaptive_lod(True)
        seq, missing = [], 0
        for k in range(4):
            vm.frame([cams[k % len(cams)]])
            seq.append(float(vm.get("lod")[0]))
            missing += vm.counts()["missing"]
        taus[budget] = seq
        if budget:
            assert missing > 0
    for budget in (0, 2):
        assert taus[budget][0] <= 32.0 and np.all(np.diff(taus[budget]) <= 0), (budget, taus[budget])


# ---- the k-means builder (Sec. 3 "Level of Detail") ------------------------
def _records(rng, n, spread=1.0):
    r = np.zeros((n, 59), np.float32)
    r[:, 0:3] = rng.normal(0.0, spread, (n, 3))
    r[:, 3:6] = rng.uniform(0.01, 0.1, (n, 3))
    q = rng.normal(size=(n, 4))
    r[:, 6:10] = q / np.linalg.norm(q, axis=1, keepdims=True)
    r[:, 10] = rng.uniform(0.05, 1.0, n)
    r[:, 11:] = rng.normal(0.0, 0.3, (n, 48))
    return r


def _cluster_mean(r, members, scale_up):
    """Arithmetic means of a cluster, written from the section's merge rule."""
    g = r[members].astype(np.float64)
    q0 = g[0, 6:10]
    sg = np.where(g[:, 6:10] @ q0 < 0.0, -1.0, 1.0)
    q = (g[:, 6:10] * sg[:, None]).mean(0)
    q /= np.linalg.norm(q)
    q *= -1.0 if q[0] < 0 else 1.0
    out = np.zeros(59)
    out[0:3] = g[:, 0:3].mean(0)
    out[3:6] = scale_up * g[:, 3:6].mean(0)
    out[6:10] = q
    out[10:] = g[:, 10:].mean(0)
    return out


def test_kmeans_identical_children():
    """Sixty-four identical records: one cluster holds them all (every
    distance ties, and ties go to the lower cluster), its parent is the
    record with its scales times the factor; the other parents are padding."""
    rng = np.random.default_rng(1)
    r = np.repeat(_records(rng, 1), 64, axis=0)
    p, a, _ = oracle.kmeans_page(r, 8, 1.5)
    assert np.all(a == 0)
    want = r[0].astype(np.float64).copy()
    want[3:6] *= 1.5
    want[6:10] *= -1.0 if want[6] < 0 else 1.0   # parents in w >= 0 form
    np.testing.assert_allclose(p[0], want, rtol=1e-6, atol=1e-7)
    assert np.all(p[1:] == 0.0)


def test_kmeans_separated_groups():
    """Eight tight groups of eight, far apart and listed group by group (as a
    Morton order lists them): the seeds fall one per group, the clusters are
    the groups, and each parent is its group's arithmetic mean (position,
    opacity, SH; sign-aligned normalised quaternion; scale times the factor)."""
    rng = np.random.default_rng(2)
    r = _records(rng, 64, spread=0.05)
    for gi in range(8):
        r[8 * gi:8 * gi + 8, 0] += 10.0 * gi
    p, a, it = oracle.kmeans_page(r, 8, 2.0)
    assert np.array_equal(a, np.repeat(np.arange(8), 8)) and it <= 2
    for gi in range(8):
        np.testing.assert_allclose(p[gi], _cluster_mean(r, np.arange(8 * gi, 8 * gi + 8), 2.0), rtol=2e-6, atol=2e-7)


def test_kmeans_lloyd_fixed_point():
    """A random page of 512 records (12 of them padding) into 64 clusters:
    after convergence every member sits in the cluster whose centroid (the
    mean of its members' features, computed here from the feature definition)
    is nearest, ties to the lower index, and every parent is its cluster's
    arithmetic mean; padding records belong to no cluster."""
    rng = np.random.default_rng(3)
    r = _records(rng, 512, spread=3.0)
    r[500:] = 0.0
    p, a, it = oracle.kmeans_page(r, 64, 1.0)
    assert it < 16
    assert np.all(a[500:] == -1) and np.all(a[:500] >= 0)
    g = r[:500].astype(np.float64)
    c0 = g[:, 0:3].mean(0)
    rms = np.sqrt(((g[:, 0:3] - c0) ** 2).sum() / 500)
    sg = np.where(g[:, 6] < 0, -1.0, 1.0)
    F = np.concatenate([(g[:, 0:3] - c0) / rms, 0.25 * sg[:, None] * g[:, 6:10],
                        0.25 * 0.28209479177387814 * g[:, 11:14], 0.25 * g[:, 10:11]], axis=1)
    used = np.unique(a[:500])
    C = np.stack([F[a[:500] == i].mean(0) for i in used])
    d = ((F[:, None, :] - C[None, :, :]) ** 2).sum(-1)
    nearest = used[np.argmin(d, axis=1)]
    assert np.array_equal(nearest, a[:500])
    for i in range(64):
        m = np.nonzero(a == i)[0]
        if m.size:
            np.testing.assert_allclose(p[i], _cluster_mean(r, m, 1.0), rtol=2e-6, atol=2e-7)
        else:
            assert np.all(p[i] == 0.0)


def test_kmeans_few_members():
    """No more members than clusters: every member is a parent of its own
    (scales times the factor), the rest padding."""
    rng = np.random.default_rng(4)
    r = _records(rng, 16)
    r[5:] = 0.0
    p, a, _ = oracle.kmeans_page(r, 8, 1.25)
    assert np.array_equal(a[:5], np.arange(5)) and np.all(a[5:] == -1)
    for i in range(5):
        np.testing.assert_allclose(p[i], _cluster_mean(r, [i], 1.25), rtol=2e-6, atol=2e-7)
    assert np.all(p[5:] == 0.0)


def test_kmeans_scene_levels():
    """The scene builder's k-means levels: level l of page p is the k-means
    of page p's level l-1 into P/8^l parents."""
    sc = synth.scene_clusters(0, n_clusters=2, per_cluster=1024)
    osc = oracle.OracleScene(sc, 256, 3, 0.5, 2.0, lod_scale_up=1.5, lod_builder=1)
    a0, a1, a2 = (osc.get(f"attr{l}").reshape(-1, 59) for l in range(3))
    for pg in (0, 3, 7):
        p1, _, _ = oracle.kmeans_page(a0[pg * 256:(pg + 1) * 256], 32, 1.5)
        assert np.array_equal(p1.view(np.uint32), a1[pg * 32:(pg + 1) * 32].view(np.uint32))
        p2, _, _ = oracle.kmeans_page(a1[pg * 32:(pg + 1) * 32], 4, 1.5)
        assert np.array_equal(p2.view(np.uint32), a2[pg * 4:(pg + 1) * 4].view(np.uint32))


def test_kmeans_levels_independent_of_threads():
    """The k-means levels are built page by page on several threads; the
    records do not depend on their number."""
    sc = synth.scene_clusters(1, n_clusters=3, per_cluster=1024)
    old = oracle.set_threads(0)
    try:
        got = []
        for nt in (1, 4):
            oracle.set_threads(nt)
            osc = oracle.OracleScene(sc, 256, 3, 0.5, 2.0, lod_scale_up=2.5, lod_builder=1)
            got.append([osc.get(f"attr{l}").view(np.uint32).copy() for l in (1, 2)])
        assert all(np.array_equal(a, b) for a, b in zip(*got))
    finally:
        oracle.set_threads(old)
