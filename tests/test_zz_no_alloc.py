"""vm3dgs_frame_noalloc (the frame entry point that allocates nothing; its
pair buffers are the library's fixed device scratch) against vm3dgs_frame,
through the C ABI: two contexts of the same scene take the same cameras, one
through each entry point, and every output of each call is compared.  Two
calls in a row, the second with fewer views (a smaller input); a LOD city
with the multi-kernel page table; a frame with more pairs than the scratch
holds is refused with CAPACITY and the context goes on."""
import numpy as np
import pytest

from paper_2506_19415_amd import synth

pytestmark = pytest.mark.gpu


def _outputs(r, out, n_views):
    g = r.get
    req = np.ctypeslib.as_array(out.requests, (out.n_requests,)).copy() if out.n_requests else np.zeros(0, np.int32)
    lvl = (np.ctypeslib.as_array(out.request_level, (out.n_requests,)).copy() if out.n_requests
           else np.zeros(0, np.int8))
    miss = (np.ctypeslib.as_array(out.missing, (2 * out.n_missing,)).copy() if out.n_missing
            else np.zeros(0, np.int32))
    st = out.stats
    return {
        "image": r.image[:n_views].cpu().numpy().copy(),
        "requests": req, "levels": lvl, "missing": miss,
        "counts": (st.candidates, st.requested, st.direct, st.linked, st.hits, st.misses, st.evictions,
                   st.missing, st.copies, st.render_pages, st.pool_pages_used, st.render_gaussians, st.pairs,
                   st.bytes_copied),
        "keys": g("keys", np.uint32), "vals": g("vals", np.uint32), "ranges": g("ranges", np.uint32),
        "v2p": g("v2p", np.int32), "last_used": g("last_used", np.int32), "sub_vpage": g("sub_vpage", np.int32),
        "copies": g("copies", np.int64),
    }


def _same(a, b, tag):
    for k in a:
        if k == "counts":
            assert a[k] == b[k], (tag, k, a[k], b[k])
        elif k == "image":
            # the same kernels on the same inputs: equal images (well inside
            # the 1e-3 bar of the frame path)
            err = float(np.abs(a[k] - b[k]).max()) if a[k].size else 0.0
            assert err <= 1e-3, (tag, k, err)
            assert np.array_equal(a[k], b[k]), (tag, k, err)
        else:
            assert a[k].shape == b[k].shape and np.array_equal(a[k], b[k]), (tag, k)


def test_noalloc_matches_frame_two_calls():
    import paper_2506_19415_amd as pkg
    sc = synth.scene_clusters(0)
    cams = synth.orbit()
    kw = dict(img=(320, 240), idbuf=(80, 60), cell=0.5, max_views=2)
    ra = pkg.Renderer(sc, 256, 64, **kw)
    rb = pkg.Renderer(sc, 256, 64, **kw)
    for call, views in enumerate([[cams[0], cams[3]], [cams[5]]]):
        print(f"noalloc clusters call {call}: {len(views)} view(s)", flush=True)
        _, oa = ra.frame(views)
        a = _outputs(ra, oa, len(views))
        _, ob = rb.frame_noalloc(views)
        b = _outputs(rb, ob, len(views))
        assert a["counts"][12] > 0
        _same(a, b, f"call {call}")
    ra.close()
    rb.close()


def test_noalloc_matches_frame_lod_city():
    import paper_2506_19415_amd as pkg
    sc = synth.scene_city(0, n=200_000, size=300.0, block=60.0, street=12.0)
    cams = synth.path_city(sc, n_frames=30, width=480, height=270)
    kw = dict(img=(480, 270), idbuf=(120, 68), cell=2.0, lod_levels=3, lod_radius_px=128.0)
    ra = pkg.Renderer(sc, 512, 64, **kw)
    rb = pkg.Renderer(sc, 512, 64, **kw)
    for f in range(0, 30, 3):
        print(f"noalloc city frame {f}", flush=True)
        _, oa = ra.frame([cams[f]])
        a = _outputs(ra, oa, 1)
        _, ob = rb.frame_noalloc([cams[f]])
        b = _outputs(rb, ob, 1)
        _same(a, b, f"city {f}")
    ra.close()
    rb.close()


def test_noalloc_refuses_frames_beyond_its_pairs():
    """1,100 Gaussians of 12 m scale at the centre of the orbit each cover
    all 8,160 tiles of a 1920x1080 image: about 9M pairs, more than the
    7,864,320 the scratch holds.  The no-allocation call returns CAPACITY;
    the next, smaller frame matches vm3dgs_frame again."""
    import paper_2506_19415_amd as pkg
    sc0 = synth.scene_clusters(0)
    rng = np.random.default_rng(11)
    k = 1100
    extra = rng.uniform(-0.5, 0.5, (k, 3)).astype(np.float32)
    sc = synth.Scene(np.concatenate([sc0.means, extra]),
                     np.concatenate([sc0.scales, np.full((k, 3), 12.0, np.float32)]),
                     np.concatenate([sc0.quats, np.tile(np.array([[1, 0, 0, 0]], np.float32), (k, 1))]),
                     np.concatenate([sc0.opacity, np.full(k, 0.05, np.float32)]),
                     np.concatenate([sc0.sh, rng.normal(0, 0.3, (k, 16, 3)).astype(np.float32)]))
    cams = synth.orbit(8, 25.0, 1920, 1080)
    far = synth.orbit(8, 200.0, 1920, 1080)
    kw = dict(img=(1920, 1080), idbuf=(240, 135), cell=0.5)
    ra = pkg.Renderer(sc, 256, 200, **kw)
    rb = pkg.Renderer(sc, 256, 200, **kw)
    print("noalloc capacity: big frame", flush=True)
    _, oa = ra.frame([cams[0]])
    assert oa.stats.pairs > pkg.VM3DGS_NOALLOC_MAX_PAIRS, oa.stats.pairs
    with pytest.raises(pkg.Vm3dgsError) as ei:
        rb.frame_noalloc([cams[0]])
    assert ei.value.code == -6 and "holds 7864320" in str(ei.value)
    # the refused frame went through the page table: the states agree
    for name, dt in [("v2p", np.int32), ("last_used", np.int32), ("slot_level", np.int8)]:
        assert np.array_equal(ra.get(name, dt), rb.get(name, dt)), name
    print("noalloc capacity: next frame", flush=True)
    _, oa = ra.frame([far[2]])
    a = _outputs(ra, oa, 1)
    _, ob = rb.frame_noalloc([far[2]])
    b = _outputs(rb, ob, 1)
    assert a["counts"][12] <= pkg.VM3DGS_NOALLOC_MAX_PAIRS
    _same(a, b, "after refusal")
    ra.close()
    rb.close()
