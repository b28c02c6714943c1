"""HIP path against the CPU oracle, through the C ABI, on the same seeded inputs.

Bit-exact: frustum candidates, the page-ID buffer, per-page request depths,
request order, page-table state, copy and missing lists, render list, tile
rectangles and depth keys, the sorted (tile, Gaussian) pairs and tile
ranges.  Floating point: conic and colour within 1e-5 relative, images
within 1e-3 absolute per channel (the target of the method's parity claim).
"""
import numpy as np
import pytest

import oracle
from paper_2506_19415_amd import synth

pytestmark = pytest.mark.gpu

NONE32 = np.uint32(0xffffffff)


def _ovm(*a, **kw):
    """The oracle VM with the support-box cut of the tile rectangles, which
    the library makes (its pair list is then the library's; the image is
    that of the plain 3-sigma rectangles either way)."""
    return oracle.OracleVM(*a, support_box=True, **kw)


def _renderer(sc, P, S, img, idbuf, cell, **kw):
    import paper_2506_19415_amd as pkg
    return pkg.Renderer(sc, P, S, img=img, idbuf=idbuf, cell=cell, **kw)


def compare_frame(r, ovm, out, n_views, check_image=True, tag=""):
    """Every intermediate of the last frame of the library against the oracle."""
    g = r.get
    P = int(g("info", np.int64)[1])
    # visibility
    assert np.array_equal(g("cand", np.uint8)[: ovm.get("cand").size], ovm.get("cand")), tag
    assert np.array_equal(g("idbuf", np.uint64)[: ovm.get("idbuf").size], ovm.get("idbuf")), tag
    assert np.array_equal(g("req_direct", np.uint32), ovm.get("req_direct")), tag
    assert np.array_equal(g("req_link", np.uint32), ovm.get("req_link")), tag
    assert np.array_equal(g("page_level", np.int8), ovm.get("page_level")), tag
    req = np.ctypeslib.as_array(out.requests, (out.n_requests,)) if out.n_requests else np.zeros(0, np.int32)
    assert np.array_equal(req, ovm.get("req_page")), tag
    lvl = np.ctypeslib.as_array(out.request_level, (out.n_requests,)) if out.n_requests else np.zeros(0, np.int8)
    assert np.array_equal(lvl, ovm.get("req_level")), tag
    # page table
    for name, dt in [("slot_level", np.int8), ("last_used", np.int32), ("sub_vpage", np.int32),
                     ("sub_last_used", np.int32), ("v2p", np.int32)]:
        assert np.array_equal(g(name, dt), ovm.get(name)), (tag, name)
    assert np.array_equal(g("copies", np.int64), ovm.get("copies")), tag
    assert np.array_equal(g("copy_id", np.int32), ovm.get("copy_id")), tag
    miss = np.ctypeslib.as_array(out.missing, (2 * out.n_missing,)) if out.n_missing else np.zeros(0, np.int32)
    assert np.array_equal(miss, ovm.get("missing")), tag
    c = ovm.counts()
    st = out.stats
    assert (st.requested, st.hits, st.misses, st.evictions, st.copies + st.prefetched, st.missing, st.render_pages) == \
           (c["requests"], c["hits"], c["misses"], c["evictions"], c["copies"], c["missing"], c["render_pages"]), tag
    rl = g("render_list", np.uint32).reshape(-1, 4)
    orl = ovm.get("render_list").reshape(-1, 6)
    assert rl.shape[0] == orl.shape[0]
    assert np.array_equal(rl[:, 0], orl[:, 2] * P + orl[:, 3] * orl[:, 4]), tag
    assert np.array_equal(rl[:, 1], orl[:, 4]) and np.array_equal(rl[:, 2], orl[:, 5]), tag
    compare_splat(r, ovm, n_views, check_image, tag)


def compare_splat(r, ovm, n_views, check_image=True, tag=""):
    g = r.get
    pf, pi = g("pp_float", np.float32).reshape(-1, 12), g("pp_int", np.int32).reshape(-1, 6)
    of, oi = ovm.get("pp_float").reshape(-1, 10), ovm.get("pp_int").reshape(-1, 6)
    assert pf.shape[0] == of.shape[0], tag
    assert np.array_equal(pi[:, 0], oi[:, 0]), tag           # culled
    vis = oi[:, 0] == 0
    assert np.array_equal(pi[vis], oi[vis]), tag              # rect and tile counts
    assert np.array_equal(pf[vis, 2].view(np.uint32), of[vis, 2].view(np.uint32)), tag   # depth keys
    assert np.array_equal(pf[vis, :2], of[vis, :2]), tag      # pixel centre
    np.testing.assert_allclose(pf[vis, 3:10], of[vis, 3:10], rtol=1e-5, atol=1e-7, err_msg=tag)
    # the library's support-box half height and width (its blend skips the
    # pixels beyond them): every row and column where the conic's quadratic
    # form can reach 11.1 is within them
    c64 = pf[vis, 3:6].astype(np.float64)
    det = c64[:, 0] * c64[:, 2] - c64[:, 1] ** 2
    syy, sxx = c64[:, 0] / det, c64[:, 2] / det
    assert np.all(pf[vis, 10].astype(np.float64) >= np.sqrt(11.1 * syy)), tag
    assert np.all(pf[vis, 11].astype(np.float64) >= np.sqrt(11.1 * sxx)), tag
    n_render = pf.shape[0] // n_views
    keys, vals = g("keys", np.uint32), g("vals", np.uint32)
    okeys, ovals = ovm.get("keys"), ovm.get("vals")
    assert keys.shape == okeys.shape, tag
    assert np.array_equal(keys.astype(np.uint64), okeys >> np.uint64(32)), tag
    assert np.array_equal(vals % n_render, ovals), tag
    assert np.array_equal(pf[vals, 2].view(np.uint32).astype(np.uint64), okeys & np.uint64(0xffffffff)), tag
    # an empty tile's range is any (s, s): compare non-empty ranges, and emptiness
    rg = g("ranges", np.uint32)[: ovm.get("ranges").size].reshape(-1, 2)
    org = ovm.get("ranges").reshape(-1, 2)
    ne = org[:, 1] > org[:, 0]
    assert np.array_equal(rg[ne], org[ne]), tag
    assert np.all(rg[~ne, 0] == rg[~ne, 1]), tag
    if check_image:
        img = r.image[:n_views].cpu().numpy()
        ref = ovm.image(n_views)
        err = np.abs(img - ref).max()
        assert err <= 1e-3, (tag, err)


@pytest.fixture(scope="module")
def clusters():
    sc = synth.scene_clusters(0)
    return sc, oracle.OracleScene(sc, 256, 1, 0.5, 2.0)


def test_clusters_all_frames(clusters):
    sc, osc = clusters
    cams = synth.orbit()
    r = _renderer(sc, 256, 64, (320, 240), (80, 60), 0.5, full_scene=True)
    ovm = _ovm(osc, 64, (320, 240), (80, 60))
    for k, cam in enumerate(cams):
        print(f"clusters frame {k}", flush=True)
        _, out = r.frame([cam])
        ovm.frame([cam])
        compare_frame(r, ovm, out, 1, tag=f"frame {k}")
    # the full-scene baseline with the same kernels
    r.render_full([cams[3]])
    ovm.render_full([cams[3]])
    compare_splat(r, ovm, 1, tag="full")
    r.close()


def test_depth_ties():
    """Four Gaussians at every mean: exact depth ties in every tile, broken by
    Gaussian index on both sides (pairs bit-exact), on VM frames and on the
    full-scene render."""
    sc = synth.scene_ties(0)
    osc = oracle.OracleScene(sc, 256, 1, 0.5, 2.0)
    cams = synth.orbit()
    r = _renderer(sc, 256, 64, (320, 240), (80, 60), 0.5, full_scene=True)
    ovm = _ovm(osc, 64, (320, 240), (80, 60))
    for k in range(4):
        print(f"depth ties frame {k}", flush=True)
        _, out = r.frame([cams[k]])
        ovm.frame([cams[k]])
        compare_frame(r, ovm, out, 1, tag=f"ties {k}")
    r.render_full([cams[5]])
    ovm.render_full([cams[5]])
    compare_splat(r, ovm, 1, tag="ties full")
    keys = ovm.get("keys")
    assert np.count_nonzero(keys[1:] == keys[:-1]) > 1000   # tied (tile, depth) pairs
    r.close()


def test_gaussians_covering_every_tile(clusters):
    """Three Gaussians of 12 m scale at the centre of the orbit: each covers
    all 1,200 tiles of a 640x480 image, so its run of pairs crosses several
    emission blocks of 1,024 pairs, and each meets every pixel."""
    sc0, _ = clusters
    rng = np.random.default_rng(7)
    extra = np.array([[0, 0, 0], [1, -1, 0.5], [-1, 1, -0.5]], np.float32)
    k = len(extra)
    sc = synth.Scene(np.concatenate([sc0.means, extra]),
                     np.concatenate([sc0.scales, np.full((k, 3), 12.0, np.float32)]),
                     np.concatenate([sc0.quats, np.tile(np.array([[1, 0, 0, 0]], np.float32), (k, 1))]),
                     np.concatenate([sc0.opacity, np.full(k, 0.3, np.float32)]),
                     np.concatenate([sc0.sh, rng.normal(0, 0.3, (k, 16, 3)).astype(np.float32)]))
    osc = oracle.OracleScene(sc, 256, 1, 0.5, 2.0)
    cams = synth.orbit(8, 25.0, 640, 480)
    r = _renderer(sc, 256, 64, (640, 480), (160, 120), 0.5, full_scene=True)
    ovm = _ovm(osc, 64, (640, 480), (160, 120))
    for f in range(3):
        print(f"covering Gaussians frame {f}", flush=True)
        _, out = r.frame([cams[f]])
        ovm.frame([cams[f]])
        compare_frame(r, ovm, out, 1, tag=f"covering {f}")
        pi = ovm.get("pp_int").reshape(-1, 6)
        tiles = (pi[:, 3] - pi[:, 1]) * (pi[:, 4] - pi[:, 2])
        assert np.count_nonzero(tiles[pi[:, 0] == 0] == 1200) == k
    r.render_full([cams[4]])
    ovm.render_full([cams[4]])
    compare_splat(r, ovm, 1, tag="covering full")
    r.close()


def test_two_views_ragged_image(clusters):
    """Two views per call, an image that is not a multiple of the tile size
    and an ID buffer that does not divide it."""
    sc, osc = clusters
    W, H, Wv, Hv = 330, 250, 70, 50
    cams = [synth.orbit(8, 25.0, W, H)[i] for i in (1, 6)]
    r = _renderer(sc, 256, 96, (W, H), (Wv, Hv), 0.5, max_views=2)
    ovm = _ovm(osc, 96, (W, H), (Wv, Hv))
    for k in range(2):
        _, out = r.frame(cams)
        ovm.frame(cams)
        compare_frame(r, ovm, out, 2, tag=f"two views {k}")
    r.close()


def test_copy_budget_and_no_links(clusters):
    sc, osc = clusters
    cams = synth.orbit()
    r = _renderer(sc, 256, 64, (320, 240), (80, 60), 0.5, copy_budget=5, links=False)
    ovm = _ovm(osc, 64, (320, 240), (80, 60), copy_budget=5, use_links=False)
    for k in range(3):
        _, out = r.frame([cams[k]])
        ovm.frame([cams[k]])
        assert out.stats.copies <= 5
        compare_frame(r, ovm, out, 1, tag=f"budget {k}")
    r.close()


def test_empty_and_inside_views(clusters):
    """A camera looking away from the scene (nothing requested, black image)
    and a camera inside a cluster (proxy boxes straddle the near plane)."""
    sc, osc = clusters
    centre = sc.means[:4096].mean(0)
    away = synth.look_at(centre + np.array([0.0, 0.0, 60.0]), [0.0, 0.0, 1.0], 320, 240, 60.0)
    inside = synth.look_at(centre, [1.0, 0.2, 0.1], 320, 240, 60.0)
    r = _renderer(sc, 256, 64, (320, 240), (80, 60), 0.5)
    ovm = _ovm(osc, 64, (320, 240), (80, 60))
    _, out = r.frame([away])
    ovm.frame([away])
    assert out.n_requests == 0 and out.stats.pairs == 0
    assert float(r.image[0].abs().max()) == 0.0
    compare_frame(r, ovm, out, 1, tag="away")
    _, out = r.frame([inside])
    ovm.frame([inside])
    assert out.n_requests > 0
    compare_frame(r, ovm, out, 1, tag="inside")
    r.close()


def test_padding_page_and_tiny_pool():
    """A scene whose last page is mostly padding, one physical page: every
    frame replaces the resident page."""
    sc = synth.scene_clusters(7, n_clusters=2, per_cluster=700)   # 1400 = 5 pages of 256 + 120
    osc = oracle.OracleScene(sc, 256, 1, 0.5, 2.0)
    cams = synth.orbit(4, 20.0, 160, 128)
    r = _renderer(sc, 256, 1, (160, 128), (40, 32), 0.5)
    ovm = _ovm(osc, 1, (160, 128), (40, 32))
    for k, cam in enumerate(cams):
        _, out = r.frame([cam])
        ovm.frame([cam])
        compare_frame(r, ovm, out, 1, tag=f"tiny pool {k}")
    r.close()


def test_half_form_clusters():
    """Pages stored with SH in bf16 and scale / rotation / opacity in fp16:
    the kernels decode them exactly, so the frame matches the oracle run on
    the same rounded attributes."""
    sc = synth.scene_clusters(0)
    osc = oracle.OracleScene(sc, 256, 1, 0.5, 2.0, attr_format=1)
    cams = synth.orbit()
    r = _renderer(sc, 256, 64, (320, 240), (80, 60), 0.5, attr_format=1)
    ovm = _ovm(osc, 64, (320, 240), (80, 60))
    for k in (0, 3, 5):
        _, out = r.frame([cams[k]])
        ovm.frame([cams[k]])
        assert out.stats.bytes_copied % 124 == 0
        compare_frame(r, ovm, out, 1, tag=f"half {k}")
    r.close()


def test_eight_views_shared_pool(clusters):
    """Eight cameras per call share one pool: requests are the union, per
    page the nearest depth over the views; tiles carry the view index."""
    sc, osc = clusters
    cams = synth.orbit(8, 25.0, 160, 120)
    r = _renderer(sc, 256, 128, (160, 120), (40, 30), 0.5, max_views=8)
    ovm = _ovm(osc, 128, (160, 120), (40, 30))
    _, out = r.frame(cams)
    ovm.frame(cams)
    compare_frame(r, ovm, out, 8, tag="eight views")
    r.close()


def _dense_scene(seed=0, n=40000):
    """A ball of Gaussians (normal, 1 m deviation) seen from 25 m: tiles of
    up to 15,000 pairs.  80 % sub-pixel to a few pixels, 17 % up to ~10 px,
    3 % large and faint; most pixels of the dense tiles stop on the
    transmittance threshold, the outer ones never do."""
    rng = np.random.default_rng(seed)
    means = rng.normal(0.0, 1.0, (n, 3)).clip(-3, 3)
    kind = rng.uniform(size=n)
    s = np.where(kind < 0.8, np.exp(rng.uniform(np.log(0.004), np.log(0.04), n)),
                 np.where(kind < 0.97, np.exp(rng.uniform(np.log(0.04), np.log(0.3), n)),
                          np.exp(rng.uniform(np.log(0.3), np.log(1.5), n))))
    scales = s[:, None] * np.exp(rng.uniform(-0.7, 0.7, (n, 3)))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    op = np.where(kind < 0.97, rng.uniform(0.05, 1.0, n), rng.uniform(0.02, 0.3, n))
    return synth.Scene(means.astype(np.float32), scales.astype(np.float32), q.astype(np.float32),
                       op.astype(np.float32), rng.normal(0.0, 0.4, (n, 16, 3)).astype(np.float32))


def _tile_sums(a, W, H, TX, TY):
    """Per-tile sums of a per-pixel [H][W] array (16x16 tiles, ragged edges)."""
    pad = np.zeros((TY * 16, TX * 16), np.int64)
    pad[:H, :W] = a
    return pad.reshape(TY, 16, TX, 16).sum(axis=(1, 3)).reshape(-1)


def test_dense_tiles():
    """Tiles of 4,096 pairs or more take the band walk (four workgroups per
    tile), the others the strip walk: two views (the ball at the centre, and at the
    ragged bottom-right corner of a 312x232 image), every intermediate and
    the image against the oracle, and the blend's per-tile work counter
    (list entries visited per pixel, up to the stop) equal to the oracle's
    per-pixel visits summed over each tile."""
    import paper_2506_19415_amd as pkg
    sc = _dense_scene()
    osc = oracle.OracleScene(sc, 256, 1, 0.5, 2.0)
    W, H = 312, 232
    c0 = synth.orbit(8, 25.0, W, H)[0]
    eye = np.array([25.0, 0.0, 0.0])
    c1 = synth.look_at(eye, np.array([-1.0, -0.53, 0.41]), W, H, 60.0)
    cams = [c0, c1]
    r = _renderer(sc, 256, 256, (W, H), (78, 58), 0.5, max_views=2, full_scene=True)
    ovm = _ovm(osc, 256, (W, H), (78, 58))
    r.set_flags(pkg.VM3DGS_FLAG_LINKS | pkg.VM3DGS_FLAG_BLEND_STATS)
    for k in range(2):
        print(f"dense tiles frame {k}", flush=True)
        _, out = r.frame(cams)
        ovm.frame(cams)
        compare_frame(r, ovm, out, 2, tag=f"dense {k}")
    TX, TY = (W + 15) // 16, (H + 15) // 16
    rg = ovm.get("ranges").reshape(-1, 2).astype(np.int64)
    n_pairs = rg[:, 1] - rg[:, 0]
    assert np.count_nonzero(n_pairs >= 4096) >= 10 and n_pairs.max() > 8192
    # the long tiles at the corner view are cut by the image edge
    corner = n_pairs[TX * TY:].reshape(TY, TX)
    assert corner[-1, :].max() >= 4096 and corner[:, -1].max() >= 4096
    visits = ovm.get("visits").reshape(2, H, W)
    want = np.concatenate([_tile_sums(visits[v], W, H, TX, TY) for v in range(2)])
    got = r.get("blend_stats", np.uint32).reshape(-1, 2)[: 2 * TX * TY, 0].astype(np.int64)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, [(int(t), int(n_pairs[t]), int(got[t]), int(want[t])) for t in bad[:10]]
    r.close()


@pytest.mark.slow
def test_terrain6m_full_size_sampled():
    """The bench workload at full size in the bench's launch configuration:
    visibility, page table and preprocess compared in full for three frames,
    and the pair lists, ranges and pixels of 48 sampled tiles (ragged last
    tile row included).  The pair buffers start at their minimum (2^20
    pairs), so the first frame outgrows them and is splatted again."""
    import paper_2506_19415_amd as pkg
    sc = synth.scene_terrain(0)
    cams = synth.path_terrain(sc)
    print("terrain6m generated", flush=True)
    r = pkg.Renderer(sc, 1024, 1465, img=(1920, 1080), idbuf=(240, 135), cell=0.5, full_scene=True, pair_capacity=1)
    osc = oracle.OracleScene(sc, 1024, 1, 0.5, 2.0)
    ovm = _ovm(osc, 1465, (1920, 1080), (240, 135))
    TX, TY = 120, 68
    rng = np.random.default_rng(0)
    tiles = np.concatenate([rng.choice(TX * (TY - 1), 40, replace=False), TX * (TY - 1) + rng.choice(TX, 8, replace=False)])
    mask = np.zeros(TX * TY, np.uint8)
    mask[tiles] = 1
    for k in range(3):
        _, out = r.frame([cams[k]])
        ovm.frame([cams[k]], tile_mask=mask)
        print(f"terrain6m frame {k}: {out.n_requests} requests, {out.stats.pairs} pairs", flush=True)
        if k == 0:
            assert out.stats.pairs > (1 << 20)   # the first frame outgrew the pair buffers
        g = r.get
        for name, dt in [("cand", np.uint8), ("idbuf", np.uint64), ("req_direct", np.uint32), ("req_link", np.uint32),
                         ("slot_level", np.int8), ("last_used", np.int32), ("sub_vpage", np.int32), ("v2p", np.int32),
                         ("copies", np.int64)]:
            assert np.array_equal(g(name, dt), ovm.get(name)), (k, name)
        req = np.ctypeslib.as_array(out.requests, (out.n_requests,))
        assert np.array_equal(req, ovm.get("req_page")), k
        pf, pi = g("pp_float", np.float32).reshape(-1, 12), g("pp_int", np.int32).reshape(-1, 6)
        of, oi = ovm.get("pp_float").reshape(-1, 10), ovm.get("pp_int").reshape(-1, 6)
        assert np.array_equal(pi[:, 0], oi[:, 0]), k
        vis = oi[:, 0] == 0
        assert np.array_equal(pi[vis], oi[vis]), k
        assert np.array_equal(pf[vis, :3].view(np.uint32), of[vis, :3].view(np.uint32)), k
        keys, vals = g("keys", np.uint32), g("vals", np.uint32)
        ranges = g("ranges", np.uint32).reshape(-1, 2)
        okeys, ovals = ovm.get("keys"), ovm.get("vals")
        orng = ovm.get("ranges").reshape(-1, 2)
        img = r.image[0].cpu().numpy()
        ref = ovm.image(1)[0]
        for t in tiles:
            s, e = ranges[t]
            os_, oe = orng[t]
            assert np.array_equal(vals[s:e], ovals[os_:oe]), (k, t)
            assert np.all(keys[s:e] == t)
            ty, tx = divmod(int(t), TX)
            blk = (slice(ty * 16, min(ty * 16 + 16, 1080)), slice(tx * 16, tx * 16 + 16))
            assert np.abs(img[blk] - ref[blk]).max() <= 1e-3, (k, t)
    r.close()


@pytest.mark.slow
def test_city50m_full_size_sampled():
    """The default bench workload at full size, in its launch configuration:
    the 50M-Gaussian city with three levels of k-means parents (scales x2.5),
    a pool of 3,907 pages, adaptive thresholds, a 480x270 ID buffer at 1080p.
    Frames 0 and 1 of the street, then 450 and 451 of the aerial phase (a jump
    that evicts, converts pages between levels and copies hundreds of pages):
    visibility, request order and levels, the whole page table, the copy list
    and the preprocess compared in full; the pair lists, pixels and blend
    visit counts of 40 random tiles and of the frame's four longest tiles
    (the band walk)."""
    import paper_2506_19415_amd as pkg
    sc = synth.scene_city(0, n=50_000_000, color="smooth")
    cams = synth.path_city(sc, n_frames=600, width=1920, height=1080)
    print("city50m generated", flush=True)
    r = _renderer(sc, 1024, 3907, (1920, 1080), (480, 270), 2.0, lod_levels=3, lod_radius_px=32.0, lod_scale_up=2.5,
                  lod_builder=1)
    r.set_flags(pkg.VM3DGS_FLAG_LINKS | pkg.VM3DGS_FLAG_ADAPTIVE_LOD | pkg.VM3DGS_FLAG_BLEND_STATS)
    print("city50m library context", flush=True)
    osc = oracle.OracleScene(sc, 1024, 3, 2.0, 2.0, lod_scale_up=2.5, lod_builder=1)
    ovm = _ovm(osc, 3907, (1920, 1080), (480, 270), lod_radius_px=32.0)
    ovm.set_adaptive_lod(True)
    print("city50m oracle context", flush=True)
    TX, TY = 120, 68
    rng = np.random.default_rng(1)
    for k in (0, 1, 450, 451):
        _, out = r.frame([cams[k]])
        g = r.get
        ranges = g("ranges", np.uint32).reshape(-1, 2)[: TX * TY].astype(np.int64)
        n_pairs = np.where(ranges[:, 1] > ranges[:, 0], ranges[:, 1] - ranges[:, 0], 0)
        tiles = np.unique(np.concatenate([rng.choice(TX * TY, 40, replace=False), np.argsort(-n_pairs)[:4]]))
        mask = np.zeros(TX * TY, np.uint8)
        mask[tiles] = 1
        ovm.frame([cams[k]], tile_mask=mask)
        print(f"city50m frame {k}: {out.n_requests} requests, {out.stats.copies} copies, "
              f"{out.stats.pairs} pairs, longest tile {n_pairs.max()}", flush=True)
        for name, dt in [("cand", np.uint8), ("idbuf", np.uint64), ("req_direct", np.uint32), ("req_link", np.uint32),
                         ("page_level", np.int8), ("slot_level", np.int8), ("last_used", np.int32),
                         ("sub_vpage", np.int32), ("sub_last_used", np.int32), ("v2p", np.int32),
                         ("copies", np.int64), ("copy_id", np.int32)]:
            assert np.array_equal(g(name, dt), ovm.get(name)), (k, name)
        req = np.ctypeslib.as_array(out.requests, (out.n_requests,))
        assert np.array_equal(req, ovm.get("req_page")), k
        lvl = np.ctypeslib.as_array(out.request_level, (out.n_requests,))
        assert np.array_equal(lvl, ovm.get("req_level")), k
        rl = g("render_list", np.uint32).reshape(-1, 4)
        orl = ovm.get("render_list").reshape(-1, 6)
        assert rl.shape[0] == orl.shape[0], k
        assert np.array_equal(rl[:, 0], orl[:, 2] * 1024 + orl[:, 3] * orl[:, 4]), k
        assert np.array_equal(rl[:, 1], orl[:, 4]) and np.array_equal(rl[:, 2], orl[:, 5]), k
        pf, pi = g("pp_float", np.float32).reshape(-1, 12), g("pp_int", np.int32).reshape(-1, 6)
        of, oi = ovm.get("pp_float").reshape(-1, 10), ovm.get("pp_int").reshape(-1, 6)
        assert np.array_equal(pi[:, 0], oi[:, 0]), k
        vis = oi[:, 0] == 0
        assert np.array_equal(pi[vis], oi[vis]), k
        assert np.array_equal(pf[vis, :3].view(np.uint32), of[vis, :3].view(np.uint32)), k
        keys, vals = g("keys", np.uint32), g("vals", np.uint32)
        okeys, ovals = ovm.get("keys"), ovm.get("vals")
        orng = ovm.get("ranges").reshape(-1, 2)
        img = r.image[0].cpu().numpy()
        ref = ovm.image(1)[0]
        visits = _tile_sums(ovm.get("visits").reshape(1080, 1920), 1920, 1080, TX, TY)
        bst = g("blend_stats", np.uint32).reshape(-1, 2)[: TX * TY, 0].astype(np.int64)
        for t in tiles:
            s, e = ranges[t]
            os_, oe = orng[t]
            assert np.array_equal(vals[s:e], ovals[os_:oe]), (k, t)
            assert np.all(keys[s:e] == t)
            ty, tx = divmod(int(t), TX)
            blk = (slice(ty * 16, min(ty * 16 + 16, 1080)), slice(tx * 16, tx * 16 + 16))
            assert np.abs(img[blk] - ref[blk]).max() <= 1e-3, (k, t)
            assert bst[t] == visits[t], (k, t, int(n_pairs[t]))
    r.close()


# ---------------------------------------------------------------- LOD levels
@pytest.fixture(scope="module")
def city():
    sc = synth.scene_city(0, n=200_000, size=300.0, block=60.0, street=12.0)
    return sc, synth.path_city(sc, n_frames=30, width=480, height=270)


@pytest.mark.parametrize("L,tau,S,budget,fmt,builder", [(3, 128.0, 64, 0, 0, 0), (3, 256.0, 48, 20, 1, 0),
                                                         (2, 128.0, 80, 0, 0, 0), (3, 128.0, 64, 0, 0, 1)])
def test_lod_city(city, L, tau, S, budget, fmt, builder):
    """Three (or two) LOD levels on a street-to-aerial city path: sub-slot
    reuse, pages converted between levels, evictions of whole physical pages,
    missing pages under pool pressure and a copy budget; moment-matched and
    k-means parents; every intermediate and the image against the oracle."""
    sc, cams = city
    osc = oracle.OracleScene(sc, 512, L, 2.0, 2.0, attr_format=fmt, lod_scale_up=2.5 if builder else 1.0,
                             lod_builder=builder)
    r = _renderer(sc, 512, S, (480, 270), (120, 68), 2.0, lod_levels=L, lod_radius_px=tau,
                  copy_budget=budget, attr_format=fmt, lod_scale_up=2.5 if builder else 1.0, lod_builder=builder)
    ovm = _ovm(osc, S, (480, 270), (120, 68), copy_budget=budget, lod_radius_px=tau)
    seen = np.zeros(L, np.int64)
    evictions = 0
    for k in range(0, 30, 2):
        print(f"lod L={L} tau={tau} S={S} frame {k}", flush=True)
        _, out = r.frame([cams[k]])
        ovm.frame([cams[k]])
        compare_frame(r, ovm, out, 1, tag=f"lod frame {k}")
        seen += np.bincount(ovm.get("req_level"), minlength=L)[:L]
        evictions += out.stats.evictions
    assert np.all(seen > 0), seen          # every level was requested
    assert evictions > 0
    r.close()


@pytest.mark.parametrize("S", [6000, 12000])
def test_large_one_level_table(clusters, S):
    """One level with more pages than the single-workgroup page table holds
    (16,384 pages of 2): the multi-kernel page table, bit-exact as well.  Its
    sorts of the requests and of the pool's slots run in one workgroup from
    the second frame (requests) or throughout (slots); 12,000 slots make that
    sort take two tiles."""
    sc, _ = clusters
    osc = oracle.OracleScene(sc, 2, 1, 0.5, 2.0)
    cams = synth.orbit()
    r = _renderer(sc, 2, S, (320, 240), (80, 60), 0.5)
    ovm = _ovm(osc, S, (320, 240), (80, 60))
    for k in range(4):
        print(f"large table S={S} frame {k}", flush=True)
        _, out = r.frame([cams[k]])
        ovm.frame([cams[k]])
        compare_frame(r, ovm, out, 1, tag=f"large table S={S} {k}")
        print(f"  requests {out.n_requests}", flush=True)
    r.close()


@pytest.mark.parametrize("S", [8192, 3000])
def test_one_level_table_at_its_limit(clusters, S):
    """The single-workgroup page table at its size limit: 8,192 pages of 4,
    8,192 physical pages (or 3,000, with evictions and missing pages), and
    more than 4,096 requests, so that the requests and the candidates each
    fill the 8,192-key sort in LDS.  Bit-exact like the smaller tables."""
    sc, _ = clusters
    osc = oracle.OracleScene(sc, 4, 1, 0.5, 2.0)
    cams = synth.orbit()
    r = _renderer(sc, 4, S, (320, 240), (160, 120), 0.5)
    assert int(r.get("info", np.int64)[0]) == 8192
    ovm = _ovm(osc, S, (320, 240), (160, 120))
    most = 0
    for k in range(4):
        print(f"table at its limit S={S} frame {k}", flush=True)
        _, out = r.frame([cams[k]])
        ovm.frame([cams[k]])
        compare_frame(r, ovm, out, 1, tag=f"limit S={S} {k}")
        most = max(most, out.n_requests)
    assert most > 4096, most
    r.close()


def test_adaptive_lod_thresholds(city):
    """Thresholds that follow memory use: the radius each frame used, and
    every intermediate, equal the oracle's along a path that first overloads
    the pool and then relieves it."""
    import paper_2506_19415_amd as pkg
    sc = synth.scene_city(0, n=400_000, size=300.0, block=60.0, street=12.0)
    cams = synth.path_city(sc, n_frames=60, width=320, height=180)
    osc = oracle.OracleScene(sc, 512, 3, 2.0, 2.0)
    r = _renderer(sc, 512, 60, (320, 180), (80, 45), 2.0, lod_levels=3, lod_radius_px=64.0)
    r.set_flags(pkg.VM3DGS_FLAG_LINKS | pkg.VM3DGS_FLAG_ADAPTIVE_LOD)
    ovm = _ovm(osc, 60, (320, 180), (80, 45), lod_radius_px=64.0)
    ovm.set_adaptive_lod(True)
    taus = []
    for k in range(0, 60, 2):
        print(f"adaptive lod frame {k}", flush=True)
        _, out = r.frame([cams[k]])
        ovm.frame([cams[k]])
        assert out.stats.lod_radius_px == float(ovm.get("lod")[0]), k
        taus.append(out.stats.lod_radius_px)
        compare_frame(r, ovm, out, 1, tag=f"adaptive lod {k}")
    assert max(taus) > 128.0
    r.close()


# ---------------------------------------------------------------- streaming
def test_streaming_one_level(clusters):
    """Streaming (VM3DGS_FLAG_ASYNC_MISSES): frames render what was resident
    when they started and their copies land for the next frame, with a
    staging budget of 10 pages, a pool of 40 and no links (evictions); every
    intermediate, the render set and the image against the oracle's model of
    the same rule."""
    import paper_2506_19415_amd as pkg
    sc, osc = clusters
    cams = synth.orbit()
    r = _renderer(sc, 256, 40, (320, 240), (80, 60), 0.5, copy_budget=10, links=False)
    r.set_flags(pkg.VM3DGS_FLAG_ASYNC_MISSES)
    ovm = _ovm(osc, 40, (320, 240), (80, 60), copy_budget=10, use_links=False)
    ovm.set_async(True)
    rendered = evicted = 0
    for k in list(range(8)) + [0, 1]:
        print(f"streaming one level frame {k}", flush=True)
        _, out = r.frame([cams[k]])
        ovm.frame([cams[k]])
        compare_frame(r, ovm, out, 1, tag=f"streaming {k}")
        assert out.stats.render_pages <= out.stats.hits
        rendered += out.stats.render_pages
        evicted += out.stats.evictions
    assert rendered > 0 and evicted > 0
    r.close()


@pytest.mark.parametrize("S,budget", [(64, 0), (48, 20)])
def test_streaming_lod_city(city, S, budget):
    """Streaming with three LOD levels on the street-to-aerial city path:
    pages resident only at another level are drawn there (fallbacks) and
    their transitions are served after the other misses; page-table state,
    render set and image against the oracle, and the fallback count."""
    import paper_2506_19415_amd as pkg
    sc, cams = city
    osc = oracle.OracleScene(sc, 512, 3, 2.0, 2.0)
    r = _renderer(sc, 512, S, (480, 270), (120, 68), 2.0, lod_levels=3, lod_radius_px=128.0, copy_budget=budget)
    r.set_flags(pkg.VM3DGS_FLAG_LINKS | pkg.VM3DGS_FLAG_ASYNC_MISSES)
    ovm = _ovm(osc, S, (480, 270), (120, 68), copy_budget=budget, lod_radius_px=128.0)
    ovm.set_async(True)
    fallbacks = 0
    for k in range(0, 30, 2):
        print(f"streaming lod S={S} frame {k}", flush=True)
        _, out = r.frame([cams[k]])
        ovm.frame([cams[k]])
        compare_frame(r, ovm, out, 1, tag=f"streaming lod {k}")
        assert out.stats.fallbacks == ovm.counts()["fallbacks"], k
        fallbacks += out.stats.fallbacks
    assert fallbacks > 0
    r.close()
