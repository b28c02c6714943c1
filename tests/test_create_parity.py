"""Create-time paging (Sec. 3) of the library against the oracle, bit for bit,
on the host (no GPU): Morton permutation, records, proxy boxes and tags, links,
page spheres, LOD parents and the encoded page-major store."""
import numpy as np
import pytest

import oracle
import paper_2506_19415_amd as pkg
from paper_2506_19415_amd import synth


def _opts(cell, link_sigma=2.0, fmt=0, scale_up=1.0, builder=0):
    o = pkg.vm3dgs_options_default()
    o.proxy_cell_m = cell
    o.link_sigma = link_sigma
    o.attr_format = fmt
    o.lod_scale_up = scale_up
    o.lod_builder = builder
    return o


def _both(sc, P, L, cell, fmt=0, link_sigma=2.0, scale_up=1.0, builder=0):
    h = pkg.vm3dgs_pages_build(sc, P, L, _opts(cell, link_sigma, fmt, scale_up, builder))
    osc = oracle.OracleScene(sc, P, L, cell, link_sigma, fmt, lod_scale_up=scale_up, lod_builder=builder)
    return h, osc


def _check_same(h, osc, L):
    g = lambda name, dt: pkg.vm3dgs_pages_get(h, name, dt)
    assert np.array_equal(g("perm", np.int64), osc.get("perm"))
    assert np.array_equal(g("rec0", np.float32).view(np.uint32), osc.get("attr0").view(np.uint32))
    for l in range(1, L):
        assert np.array_equal(g(f"rec{l}", np.float32).view(np.uint32), osc.get(f"attr{l}").view(np.uint32)), l
    assert np.array_equal(g("spheres", np.float32).view(np.uint32), osc.get("spheres").view(np.uint32))
    assert np.array_equal(g("cell_box", np.float32).view(np.uint32), osc.get("cell_box").view(np.uint32))
    assert np.array_equal(g("cell_page", np.int32), osc.get("cell_page"))
    assert np.array_equal(g("cell_start", np.int32), osc.get("cell_start"))
    assert np.array_equal(g("link_start", np.int32), osc.get("link_start"))
    assert np.array_equal(g("link_dst", np.int32), osc.get("link_dst"))


def test_clusters_paging_parity():
    sc = synth.scene_clusters(0)
    h, osc = _both(sc, 256, 1, 0.5)
    try:
        _check_same(h, osc, 1)
    finally:
        pkg.vm3dgs_pages_destroy(h)


def test_ragged_last_page_parity():
    sc = synth.scene_clusters(5, n_clusters=3, per_cluster=1111)   # 3333 = 13 pages of 256 + 5
    h, osc = _both(sc, 256, 1, 0.75, link_sigma=1.5)
    try:
        _check_same(h, osc, 1)
        assert osc.n_pages == 14
    finally:
        pkg.vm3dgs_pages_destroy(h)


def test_terrain_paging_parity():
    sc = synth.scene_terrain(0, n_terrain=60000, n_building=40000, n_buildings=6, extent=40.0, path_frames=100)
    h, osc = _both(sc, 1024, 1, 1.0)
    try:
        _check_same(h, osc, 1)
    finally:
        pkg.vm3dgs_pages_destroy(h)


@pytest.mark.parametrize("fmt,scale_up,builder", [(0, 1.0, 0), (1, 1.0, 0), (0, 1.6, 0), (0, 1.0, 1), (1, 2.0, 1)])
def test_lod_and_half_form_parity(fmt, scale_up, builder):
    """Both LOD builders (moment matching; the k-means of Sec. 3), both
    storage forms."""
    sc = synth.scene_city(0, n=40000, size=120.0, block=40.0, street=8.0)
    h, osc = _both(sc, 512, 3, 2.0, fmt=fmt, scale_up=scale_up, builder=builder)
    try:
        _check_same(h, osc, 3)
    finally:
        pkg.vm3dgs_pages_destroy(h)


def _decode_store(store, n_pg, P, L, fmt):
    """Decode the page-major SoA store back to [n][59] per level (reading of the
    layout documented in the kernels)."""
    out = []
    off = 0
    bg = 124 if fmt == 1 else 236
    for l in range(L):
        C = P >> (3 * l)
        blk = np.frombuffer(store, dtype=np.uint8, count=n_pg * C * bg, offset=off).reshape(n_pg, C * bg)
        rec = np.zeros((n_pg, C, 59), np.float32)
        if fmt == 0:
            rec[:] = blk.view(np.float32).reshape(n_pg, 59, C).transpose(0, 2, 1)
        else:
            f = blk.view(np.float32).reshape(n_pg, 31, C)
            u = blk.view(np.uint32).reshape(n_pg, 31, C)
            rec[:, :, 0:3] = f[:, 0:3].transpose(0, 2, 1)
            half = np.stack([(u[:, 3 + k] & 0xffff).astype(np.uint16) for k in range(4)] +
                            [(u[:, 3 + k] >> 16).astype(np.uint16) for k in range(4)], 1).view(np.float16)
            order = [0, 4, 1, 5, 2, 6, 3, 7]   # lo/hi of (sx,sy) (sz,qw) (qx,qy) (qz,o)
            rec[:, :, 3:11] = half[:, order].astype(np.float32).transpose(0, 2, 1)
            lo = (u[:, 7:31] << 16).view(np.float32)
            hi = (u[:, 7:31] & 0xffff0000).view(np.float32)
            sh = np.empty((n_pg, 48, C), np.float32)
            sh[:, 0::2] = lo
            sh[:, 1::2] = hi
            rec[:, :, 11:] = sh.transpose(0, 2, 1)
        out.append(rec.reshape(-1, 59))
        off += n_pg * C * bg
    return out


@pytest.mark.parametrize("fmt", [0, 1])
def test_store_layout_decodes_to_records(fmt):
    sc = synth.scene_clusters(1, n_clusters=2, per_cluster=700)
    h = pkg.vm3dgs_pages_build(sc, 64, 2, _opts(0.5, 2.0, fmt))
    try:
        info = pkg.vm3dgs_pages_get(h, "info", np.int64)
        n_pg, P, L, bg = info[:4]
        assert bg == (124 if fmt else 236)
        store = pkg.vm3dgs_pages_get(h, "store", np.uint8).tobytes()
        assert len(store) == n_pg * (P + P // 8) * bg
        dec = _decode_store(store, n_pg, P, L, fmt)
        for l in range(L):
            rec = pkg.vm3dgs_pages_get(h, f"rec{l}", np.float32).reshape(-1, 59)
            assert np.array_equal(dec[l], rec)
        if fmt == 1:
            # half form: decoded values are the fp16 / bf16 roundings of the fp32 records
            h0 = pkg.vm3dgs_pages_build(sc, 64, 2, _opts(0.5, 2.0, 0))
            full = pkg.vm3dgs_pages_get(h0, "rec0", np.float32).reshape(-1, 59)
            pkg.vm3dgs_pages_destroy(h0)
            assert np.array_equal(dec[0][:, :3], full[:, :3])
            assert np.array_equal(dec[0][:, 3:11], full[:, 3:11].astype(np.float16).astype(np.float32))
            assert np.array_equal(dec[0][:, 11:], oracle.round_bf16_n(full[:, 11:]))
    finally:
        pkg.vm3dgs_pages_destroy(h)


def test_unknown_lod_builder_rejected():
    sc = synth.scene_clusters(0, n_clusters=1, per_cluster=512)
    with pytest.raises(Exception):
        pkg.vm3dgs_pages_build(sc, 256, 2, _opts(0.5, builder=2))
