"""Recall of the requested page set against brute-force truth sets (reported,
not gated), on a small terrain with buildings.

Sec. 4.1 determines the pages to render from a low-resolution page-ID buffer
of a proxy, plus links; it can miss pages whose Gaussians reach the image.
Two truth sets are computed here by brute force over every pixel of the
full-resolution image, in float64, from the projected Gaussians of the
full-scene render:
  touched  pages with a Gaussian whose alpha reaches 1/255 at some pixel;
  blended  pages with a Gaussian that a front-to-back blend of every
           Gaussian at that pixel (depth order, ties by index, stop when
           transmittance would fall below 1e-4) actually takes.
Recall = |requested and truth| / |truth|, per frame, and the share of the
blend weight (alpha times transmittance, summed over pixels) that the
requested pages carry, at three ID-buffer
sizes and with links off and on, on a small terrain with buildings.
"""
import math

import numpy as np

import oracle
from paper_2506_19415_amd import synth

W, H, P = 160, 120, 64


def truth_sets(ovm):
    """Touched and blended page sets of the last full-scene render, by brute
    force in float64.  A Gaussian's alpha can reach 1/255 only where its
    quadratic form is at most 2 ln 255 (opacity <= 1), i.e. within 3.33
    standard deviations along its major axis; each Gaussian is evaluated on
    that window, widened by one pixel, clipped to the image."""
    pf = ovm.get("pp_float").reshape(-1, 10).astype(np.float64)
    pi = ovm.get("pp_int").reshape(-1, 6)
    vis = np.nonzero(pi[:, 0] == 0)[0]
    depth_bits = ovm.get("pp_float").reshape(-1, 10)[:, 2].view(np.uint32)
    order = vis[np.lexsort((vis, depth_bits[vis]))]
    T = np.ones((H, W))
    done = np.zeros((H, W), bool)
    touched, blended = set(), set()
    weight = {}
    for g in order:
        u, v, _, a, b, c, op = pf[g, :7]
        det = a * c - b * b
        if not det > 0.0:
            continue
        lam = 0.5 * (a + c) - math.sqrt(max(0.25 * (a - c) ** 2 + b * b, 0.0))  # smaller eigenvalue of the conic
        r = math.sqrt(2.0 * math.log(255.0) / lam) + 1.0 if lam > 0.0 else float("inf")
        x0, x1 = max(int(math.floor(u - r)), 0), min(int(math.ceil(u + r)), W - 1)
        y0, y1 = max(int(math.floor(v - r)), 0), min(int(math.ceil(v + r)), H - 1)
        if x0 > x1 or y0 > y1:
            continue
        px, py = np.meshgrid(np.arange(x0, x1 + 1, dtype=np.float64), np.arange(y0, y1 + 1, dtype=np.float64))
        dx, dy = u - px, v - py
        power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
        alpha = np.minimum(0.99, op * np.exp(np.minimum(power, 0.0)))
        hit = (power <= 0.0) & (alpha >= 1.0 / 255.0)
        if not hit.any():
            continue
        touched.add(int(g) // P)
        Tw, dw = T[y0:y1 + 1, x0:x1 + 1], done[y0:y1 + 1, x0:x1 + 1]
        take = hit & ~dw
        Tn = Tw * (1.0 - alpha)
        stop = take & (Tn < 1e-4)
        dw |= stop
        take &= ~stop
        if take.any():
            blended.add(int(g) // P)
            weight[int(g) // P] = weight.get(int(g) // P, 0.0) + float((alpha * Tw)[take].sum())
            Tw[take] = Tn[take]
    return touched, blended, weight


def test_page_set_recall_report():
    sc = synth.scene_terrain(0, n_terrain=80_000, n_building=60_000, n_buildings=10, extent=60.0, path_frames=60)
    osc = oracle.OracleScene(sc, P, 1, 0.5, 2.0)
    cams = [synth.path_terrain(sc, 60, W, H)[k] for k in (0, 20, 40)]
    truths = []
    for cam in cams:
        full = oracle.OracleVM(osc, osc.n_pages, (W, H), (W // 4, H // 4))
        full.render_full([cam])
        touched, blended, weight = truth_sets(full)
        assert touched and blended and blended <= touched and set(weight) == blended
        truths.append((touched, blended, weight))
    rows = []
    for idbuf in [(W // 8, H // 8), (W // 4, H // 4), (W, H)]:
        for links in (False, True):
            rec_t, rec_b, rec_w, n_req = [], [], [], []
            for cam, (touched, blended, weight) in zip(cams, truths):
                vm = oracle.OracleVM(osc, osc.n_pages, (W, H), idbuf, use_links=links)
                vm.visibility([cam])
                req = set(int(p) for p in vm.get("req_page"))
                rec_t.append(len(req & touched) / len(touched))
                rec_b.append(len(req & blended) / len(blended))
                rec_w.append(sum(weight[p] for p in req & blended) / sum(weight.values()))
                n_req.append(len(req))
            rows.append((idbuf, links, float(np.mean(rec_t)), float(np.mean(rec_b)), float(np.mean(rec_w)),
                         float(np.mean(n_req))))
    print(f"pages {osc.n_pages}, touched {np.mean([len(t) for t, _, _ in truths]):.0f}, "
          f"blended {np.mean([len(b) for _, b, _ in truths]):.0f} per frame")
    for idbuf, links, rt, rb, rw, nr in rows:
        print(f"ID buffer {idbuf[0]}x{idbuf[1]} links {int(links)}: {nr:.0f} requested, "
              f"recall touched {rt:.3f} blended {rb:.3f} blend weight {rw:.3f}")
        assert 0.0 <= rt <= 1.0 and 0.0 <= rb <= 1.0 and 0.0 <= rw <= 1.0 + 1e-12
    # links only add requests
    for k in range(0, len(rows), 2):
        assert all(rows[k + 1][j] >= rows[k][j] for j in (2, 3, 4))
