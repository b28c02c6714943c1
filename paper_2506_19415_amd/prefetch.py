"""Evaluation of the learned page prefetch (host driver).

The paper names prefetching as future work (Sec. 6).  Here a network proposes
lowest-priority page requests from the last four camera poses and the
current residency; the visibility pass keeps deciding what is rendered.
Training rows, labels and the training itself are the library's
(vm3dgs_prefetch_collect, vm3dgs_prefetch_train); this module orders calls
and measures:

- ``collect``: the library's feature and label rows of plain frames.
- ``evaluate``: the same paths with and without the network: demand misses
  per frame, the stall (the copy stage's milliseconds), and the proposals'
  recall and precision against the next frame's requests.
"""
import numpy as np


def scene_frame(scene):
    """Centre and extent (half the largest side) of the box of the means."""
    m = np.asarray(scene.means, np.float64)
    lo, hi = m.min(0), m.max(0)
    return ((lo + hi) / 2).astype(np.float32), float((hi - lo).max() / 2)


def _resident(r, n_pg, L):
    v2p = r.get("v2p", np.int32).reshape(n_pg, L)
    return (v2p >= 0).any(1)


def collect(r, paths, n_clusters, hist_bins, center, extent):
    """Feature and label rows of every frame but the last of each path, from
    the library (the stage is attached without a network first).
    r: a Renderer of one view; it is reset before each path."""
    r.set_prefetch(None, n_clusters, hist_bins, 0.0, 0, center, extent)
    return r.prefetch_collect(paths)


def evaluate(r, net, paths, n_clusters, hist_bins, threshold, budget, center, extent, skip=2):
    """Demand misses, stall and proposal quality along the paths, with the
    network (net) or without it (net=None).  Frames before `skip` on each
    path (the cold start) are not counted."""
    n_pg, L = int(r.get("info", np.int64)[0]), int(r.get("info", np.int64)[2])
    r.set_prefetch(net, n_clusters, hist_bins, threshold, budget, center, extent)
    misses = stall = frames = 0
    hit_new = n_new = hit_req = n_prop = 0
    for cams in paths:
        r.reset()
        prev_prop = prev_res = None
        for k, cam in enumerate(cams):
            _, out = r.frame([cam])
            req = np.ctypeslib.as_array(out.requests, (out.n_requests,)).copy() if out.n_requests else \
                np.zeros(0, np.int32)
            if k >= skip:
                misses += out.stats.misses
                stall += out.stats.ms_copy
                frames += 1
                if prev_prop is not None:
                    new = set(req[~prev_res[req]].tolist())
                    reqs = set(req.tolist())
                    hit_new += len(prev_prop & new)
                    n_new += len(new)
                    hit_req += len(prev_prop & reqs)
                    n_prop += len(prev_prop)
            # what this frame prefetched (after its demand copies) and the residency before the prefetch
            n_pf = out.stats.prefetched
            if net is not None and n_pf:
                cid = r.get("copy_id", np.int32).reshape(-1, 4)
                prev_prop = set(cid[len(cid) - n_pf:, 0].tolist())
            else:
                prev_prop = set()
            res = _resident(r, n_pg, L)
            if prev_prop:
                res[list(prev_prop)] = False
            prev_res = res
    return {"frames": frames, "misses_per_frame": misses / max(frames, 1), "stall_ms_per_frame": stall / max(frames, 1),
            "recall": hit_new / n_new if n_new else None, "precision": hit_req / n_prop if n_prop else None,
            "proposed": n_prop}
