"""Pins of the oracle's prefetch stage (features, proposals, the third page-
table stage) on the CPU.

- the pose quaternion is scipy's rotation of the camera-to-world matrix, the
  position is relative to the centre over the extent, the oldest pose
  repeats until four were seen;
- the residency fractions are brute-force counts over v2p;
- proposals are exactly the pages of clusters over the threshold that the
  visibility pass did not request and that are not resident at their
  distance level, nearest first;
- the third stage fills only physical pages used in neither this frame nor
  the previous one, least recently used first, within its budget, never
  touches a page the frame renders, and leaves the image unchanged;
- a prefetched page requested in the next frame is a hit.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from paper_2506_19415_amd import synth

K, H = 32, 16


@pytest.fixture(scope="module")
def setup():
    sc = synth.scene_clusters(0)
    osc = oracle.OracleScene(sc, 256, 1, 0.5, 2.0)
    cams = synth.orbit(24, 25.0, 320, 240)
    means = np.asarray(sc.means, np.float64)
    lo, hi = means.min(0), means.max(0)
    return sc, osc, cams, ((lo + hi) / 2).astype(np.float32), float((hi - lo).max() / 2)


def _vm(osc, center, extent, budget=8, S=64):
    vm = oracle.OracleVM(osc, S, (320, 240), (80, 60))
    vm.set_prefetch(K, H, 0.0, budget, center, extent)
    return vm


def test_pose_features_and_history(setup):
    sc, osc, cams, center, extent = setup
    vm = _vm(osc, center, extent)
    seen = []
    for k in range(6):
        vm.frame([cams[k]])
        seen.append(k)
        x = vm.features(0)
        for slot in range(4):
            c = cams[seen[max(0, len(seen) - 4 + slot)]]
            pos = (np.asarray(c.cam_pos, np.float64) - center) / extent
            R = np.asarray(c.view, np.float64)[:3, :3].T            # camera to world
            q = Rotation.from_matrix(R).as_quat()                    # x y z w
            q = np.array([q[3], q[0], q[1], q[2]])
            q = q if q[0] >= 0 else -q
            assert np.allclose(x[7 * slot: 7 * slot + 3], pos, atol=1e-6), (k, slot)
            assert np.allclose(x[7 * slot + 3: 7 * slot + 7], q, atol=1e-6), (k, slot)


def test_residency_fractions(setup):
    sc, osc, cams, center, extent = setup
    vm = _vm(osc, center, extent)
    for k in range(3):
        vm.frame([cams[k]])
    x = vm.features(0)
    n_pg = osc.get("n_pages")[0] if np.ndim(osc.get("n_pages")) else int(osc.get("n_pages"))
    res = vm.get("v2p") >= 0
    for b in range(H):
        lo, hi = -(-b * n_pg // H), -(-(b + 1) * n_pg // H)
        assert x[28 + b] == pytest.approx(res[lo:hi].mean(), abs=1e-7), b
    assert 0.0 < x[28:].mean() < 1.0


@pytest.fixture(scope="module")
def city():
    sc = synth.scene_city(0, n=100_000, size=300.0, block=60.0, street=12.0)
    cams = synth.path_city(sc, n_frames=40, width=160, height=90)
    osc = oracle.OracleScene(sc, 256, 1, 2.0, 2.0)
    means = np.asarray(sc.means, np.float64)
    lo, hi = means.min(0), means.max(0)
    return osc, cams, ((lo + hi) / 2).astype(np.float32), float((hi - lo).max() / 2)


def test_proposals_and_third_stage(city):
    osc, cams, center, extent = city
    n_pg = int(np.asarray(osc.get("n_pages")).ravel()[0])
    spheres = osc.get("spheres").reshape(-1, 4)
    Kc, S, budget = 64, 250, 6
    vm = oracle.OracleVM(osc, S, (160, 90), (80, 45))
    vm.set_prefetch(Kc, 32, 0.0, budget, center, extent)
    ref = oracle.OracleVM(osc, S, (160, 90), (80, 45))       # the same frames without prefetch
    for k in range(0, 30, 2):       # street level, then climbing: fewer pages per frame, idle pages
        vm.frame([cams[k]])
        ref.frame([cams[k]])
    frame = 15
    rng = np.random.default_rng(0)
    sel = rng.random(Kc) < 0.5
    logits = np.where(sel, 3.0, -3.0).astype(np.float32)[None]
    cam = cams[30]
    vm.frame_prefetch([cam], logits)
    ref.frame([cam])
    # the state after the demand stages is that of the run without prefetch
    v2p_dem, lu_dem = ref.get("v2p"), ref.get("last_used")
    # proposals, brute force
    req = set(vm.get("req_page").tolist())
    want = []
    for p in range(n_pg):
        if not sel[p * Kc // n_pg] or p in req or v2p_dem[p] >= 0:
            continue
        c = spheres[p]
        dx, dy, dz = (np.float32(c[a] - np.float32(cam.cam_pos[a])) for a in range(3))
        d = np.float32(np.sqrt(np.float32(np.float32(dx * dx + dy * dy) + dz * dz)) - c[3])
        d = max(d, np.float32(cam.znear))
        want.append((int(np.float32(d).view(np.uint32)), p))
    want.sort()
    assert len(want) > budget
    keys = vm.get("pf_keys")
    assert [int(k & 0x0fffffff) for k in keys] == [p for _, p in want]
    assert [int((k >> 30) & 0x7fffffff) for k in keys] == [d for d, _ in want]
    n_req, n_pf, n_dem = (int(v) for v in vm.get("pf_counts"))
    assert n_req == len(want) and 0 < n_pf <= budget
    # the demand part of the frame is that of the run without prefetch
    for name in ("req_page", "render_list", "missing"):
        assert np.array_equal(vm.get(name), ref.get(name)), name
    assert np.array_equal(vm.image(), ref.image())
    assert np.array_equal(vm.get("copies")[: 3 * n_dem], ref.get("copies"))
    # prefetch copies went to pages idle for two frames, least recently used first
    cid = vm.get("copy_id").reshape(-1, 4)[n_dem:]
    assert len(cid) == n_pf
    slots = cid[:, 2]
    idle = sorted((lu_dem[s], s) for s in range(S) if lu_dem[s] < frame - 1)
    assert [s for _, s in idle[:n_pf]] == slots.tolist()
    assert not set(slots.tolist()) & set(vm.get("render_list").reshape(-1, 6)[:, 2].tolist())
    assert [int(p) for p in cid[:, 0]] == [p for _, p in want[:n_pf]]
    assert np.all(vm.get("v2p")[cid[:, 0]] >= 0)


def test_prefetched_pages_hit_later():
    """Proposing every cluster along a street-to-aerial city path with idle
    physical pages: later frames find pages the third stage loaded, so
    demand misses fall below those of the plain method on the same frames."""
    sc = synth.scene_city(0, n=100_000, size=300.0, block=60.0, street=12.0)
    cams = synth.path_city(sc, n_frames=40, width=160, height=90)
    osc = oracle.OracleScene(sc, 256, 1, 2.0, 2.0)
    means = np.asarray(sc.means, np.float64)
    lo, hi = means.min(0), means.max(0)
    center, extent = ((lo + hi) / 2).astype(np.float32), float((hi - lo).max() / 2)
    vm = oracle.OracleVM(osc, 250, (160, 90), (80, 45))
    vm.set_prefetch(64, 32, 0.0, 24, center, extent)
    ref = oracle.OracleVM(osc, 250, (160, 90), (80, 45))
    m_pf = m_ref = n_pf = 0
    for k in range(0, 40, 2):
        vm.frame_prefetch([cams[k]], np.full((1, 64), 5.0, np.float32))
        ref.frame([cams[k]])
        n_pf += int(vm.get("pf_counts")[1])
        assert np.array_equal(vm.get("req_page"), ref.get("req_page"))
        if k >= 4:
            m_pf += vm.counts()["misses"]
            m_ref += ref.counts()["misses"]
    assert n_pf > 0 and m_pf < m_ref, (n_pf, m_pf, m_ref)
