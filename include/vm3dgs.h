/*
 * vm3dgs.h -- C ABI of the MI355X (gfx950) virtual-memory 3D Gaussian
 * Splatting frame path.
 *
 * Method: Haberl et al., "Virtual Memory for 3D Gaussian Splatting"
 * (arXiv 2506.19415).  Gaussians are grouped into fixed-size pages (Sec. 3,
 * "Page Assignment"); every frame a visibility pass finds the pages the
 * camera needs (Sec. 4.1, "Page Determination": frustum test, a
 * low-resolution page-ID buffer of a proxy, page links and a level of detail
 * from the nearest depth), a page table maps them onto a pool of physical
 * pages with least-recently-used replacement (Sec. 4.1.1), misses are copied
 * from pinned host memory, and only resident Gaussians are splatted with the
 * 3DGS math of Kerbl et al. (Sec. 4.2).
 *
 * Conventions for every entry point:
 *  - plain C types, no exceptions cross the boundary;
 *  - a return value < 0 is an error; vm3dgs_last_error() gives its text;
 *  - after a HIP runtime error the context is poisoned: every later call
 *    returns VM3DGS_E_STATE and only vm3dgs_destroy() is valid;
 *  - one context per host thread at a time (no internal locking);
 *  - "device" pointers are HIP device allocations on the current device,
 *    "host" pointers ordinary host memory.
 */
#ifndef VM3DGS_H
#define VM3DGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vm3dgs vm3dgs;
typedef int32_t vm3dgs_status;

#define VM3DGS_OK 0
#define VM3DGS_E_INVALID_ARG (-1) /* a size, pointer or option is out of range */
#define VM3DGS_E_HOST_OOM (-2)    /* host or pinned host allocation failed */
#define VM3DGS_E_DEVICE_OOM (-3)  /* device allocation failed */
#define VM3DGS_E_HIP (-4)         /* a HIP runtime call failed; context poisoned */
#define VM3DGS_E_STATE (-5)       /* context poisoned by an earlier error */
#define VM3DGS_E_CAPACITY (-6)    /* more views than max_views */

/* Scene in the storage form of Sec. 3 ("Scene Storage"): activated scale and
 * opacity, quaternion w,x,y,z (normalised by create), degree-3 SH with the
 * 16 coefficients of each channel interleaved as sh[k][channel].  All arrays
 * are host memory, borrowed only for the duration of vm3dgs_create. */
typedef struct {
    uint64_t n;
    const float* means;   /* [n][3] metres */
    const float* scales;  /* [n][3] standard deviations, > 0 */
    const float* quats;   /* [n][4] w x y z */
    const float* opacity; /* [n] in [0, 1] */
    const float* sh;      /* [n][16][3] */
} vm3dgs_scene;

#define VM3DGS_FLAG_LINKS 1u           /* expand page links (Sec. 3 "Page Linking") */
#define VM3DGS_FLAG_FULL_SCENE_COPY 2u /* keep all level-0 pages in HBM for vm3dgs_render_full */
#define VM3DGS_FLAG_BLEND_STATS 4u     /* count blend work (stats.blend_evals / blend_alphas); slower */
/* Tile rectangles from the 3-sigma radius alone.  By default each rectangle
 * is cut to the support box of the Gaussian: the pixels where the blend's
 * power can reach -5.55 (with float rounding bounded), outside which every
 * term fails the 1/255 alpha test; the image is the same either way, with
 * fewer (tile, Gaussian) pairs. */
#define VM3DGS_FLAG_SIGMA3_TILES 8u
/* With several LOD levels, move the level-0 radius with memory use
 * (Sec. 5.1.1): aim at 50-80 % of the pool required by the frame.  Above
 * 80 %, or with requests left missing, the radius grows by 1 + step
 * (coarser); under 50 % with coarse levels in use it shrinks by 1 + step
 * (finer).  The step starts at 1/8 and changes by 1 % of itself after a
 * move that repeats (x 1.01) or reverses (x 0.99) a move made at most 4
 * frames earlier.  The radius a frame used is in stats.lod_radius_px; the
 * next frame uses the new one. */
#define VM3DGS_FLAG_ADAPTIVE_LOD 16u
/* Streaming (Sec. 4.3, Sec. 5.1.2): a frame does not wait for its own page
 * copies.  It renders the requested pages that were resident when it
 * started: at the requested level, or, for a page resident only at other
 * levels, at the nearest of them (the finer at equal distance; the level
 * switch is deferred until the copy has landed, and that entry is required
 * for the frame).  Its misses are served in request order (directly seen
 * before linked, then depth), those with such a resident level after all
 * the others; the copies run on the copy stream beside the frame's splat,
 * and the next frame waits for them before it reads or writes the pool.
 * copy_budget_pages is the per-frame staging budget (Sec. 5.1.2: 40 pages).
 * stats.bytes_copied counts the bytes the frame issues. */
#define VM3DGS_FLAG_ASYNC_MISSES 32u

typedef struct {
    uint32_t img_w, img_h;        /* output image, pixels */
    uint32_t idbuf_w, idbuf_h;    /* page-ID buffer, pixels (Sec. 5.1.1: much smaller than the image) */
    uint32_t max_views;           /* views per call, >= 1 */
    uint32_t attr_format;         /* 0: fp32 (236 B/Gaussian); 1: means fp32, scale/quat/opacity fp16, SH bf16 (124 B) */
    uint32_t copy_budget_pages;   /* page copies per frame, 0 = unlimited (Sec. 4.3: staging budget) */
    float idbuf_guard_px;         /* the ID buffer and frustum extend this many image pixels past each edge */
    float proxy_cell_m;           /* proxy grid cell edge, metres */
    float link_sigma;             /* link ellipsoid radius in standard deviations */
    float lod_radius_px;          /* level l is chosen while the projected page radius <= tau / 2^(l-1) */
    uint32_t flags;               /* VM3DGS_FLAG_* */
    void* stream_render;          /* hipStream_t for the frame's kernels, NULL = library-owned stream */
    void* stream_copy;            /* hipStream_t for page copies, NULL = library-owned stream */
    uint64_t pair_capacity;       /* initial (tile, Gaussian) pair capacity; grows on demand; 0 = automatic */
    float lod_scale_up;           /* LOD parents: merged scales times this factor (Sec. 3 Level of Detail:
                                     merged Gaussians are scaled up by a fixed factor to fill gaps); in (0, 16] */
    uint32_t lod_builder;         /* LOD parents (Sec. 3 Level of Detail): 0 = opacity-weighted moment matching
                                     of 8 consecutive Morton children (default); 1 = the section's k-means
                                     clustering of each page on scaled attributes (position first), parents
                                     the clusters' arithmetic means, scales the mean times lod_scale_up.
                                     Other values: VM3DGS_E_INVALID_ARG */
} vm3dgs_options;

/* Fill *o with defaults: 1920x1080 image, 240x135 ID buffer with a 32 px
 * guard band, one view, fp32, unlimited copies, 1 m cells, 2-sigma links,
 * 32 px LOD radius, links on. */
void vm3dgs_options_default(vm3dgs_options* o);

/* Pinhole camera, OpenCV axes (x right, y down, z forward).  view is the
 * row-major 4x4 world-to-camera matrix, cam_pos the camera centre in world
 * space.  Pixel centres are at integer + 0.5 in [0, img_w) x [0, img_h). */
typedef struct {
    float view[16];
    float cam_pos[3];
    float fx, fy, cx, cy, znear;
} vm3dgs_camera;

typedef struct {
    uint32_t candidates;        /* pages passing the frustum test (summed over views) */
    uint32_t requested;         /* unique pages requested */
    uint32_t direct;            /* requested because seen in the ID buffer */
    uint32_t linked;            /* requested only through a link */
    uint32_t hits, misses, evictions, missing, copies;
    uint32_t render_pages;      /* resident requested pages splatted this frame */
    uint32_t pool_pages_used;   /* physical pages holding at least one virtual page */
    uint32_t prefetched;        /* pages copied by the prefetch stage (not awaited by this frame) */
    uint32_t fallbacks;         /* streaming: requested pages drawn at another resident level */
    uint64_t render_gaussians;  /* Gaussians in the render set (incl. padding) x views */
    uint64_t visible_gaussians; /* of those, not culled by the projection */
    uint64_t pairs;             /* (tile, Gaussian) pairs sorted and blended */
    uint64_t bytes_copied;      /* host -> device page bytes */
    uint64_t blend_evals;       /* pixel-Gaussian evaluations (VM3DGS_FLAG_BLEND_STATS only) */
    uint64_t blend_alphas;      /* of those, evaluations that computed alpha (same flag) */
    float ms_visibility, ms_pagetable, ms_copy, ms_preprocess, ms_sort, ms_blend, ms_total;
    float lod_radius_px;        /* level-0 radius this frame used (moves with VM3DGS_FLAG_ADAPTIVE_LOD) */
} vm3dgs_stats;

typedef struct {
    const int32_t* requests;      /* host, context-owned: page ids in service order (class, depth, page) */
    const int8_t* request_level;  /* host, context-owned: LOD level per request */
    uint32_t n_requests;
    const int32_t* missing;       /* host, context-owned: [n_missing][2] page, level not made resident */
    uint32_t n_missing;
    vm3dgs_stats stats;
} vm3dgs_frame_out;

/* Build the paged scene (Sec. 3): Morton-ordered pages of page_size Gaussians
 * (last page padded with zero Gaussians), lod_levels levels (1..3; level l
 * holds page_size / 8^l Gaussians per page, each the opacity-weighted moment
 * match of 8 children), proxy boxes and links, the page-major pinned host
 * store, and a device pool of pool_pages physical pages.
 * Errors: INVALID_ARG if scene or out is NULL, n == 0, page_size == 0,
 * lod_levels not in 1..3, page_size not divisible by 8^(lod_levels-1),
 * pool_pages == 0, image or ID-buffer size 0, max_views == 0 or > 64;
 * HOST_OOM / DEVICE_OOM on allocation failure.  On error *out is NULL. */
vm3dgs_status vm3dgs_create(const vm3dgs_scene* scene, uint32_t page_size, uint32_t pool_pages,
                            uint32_t lod_levels, const vm3dgs_options* opt, vm3dgs** out);

/* One frame for n_views cameras (Sec. 4): visibility, page table, copies of
 * the misses (read by the GPU from the pinned store, on the render stream
 * before the preprocess; prefetch copies on the copy stream), splatting of
 * the resident pages.  image_dev: device, caller-owned,
 * [n_views][img_h][img_w][3] float32, written on the render stream (and on
 * a stream of the library's own that the blend forks from the render stream
 * and joins back to it) and complete when the render stream reaches the end
 * of this call's work (the call returns after that); work of other streams
 * that reads or writes it must be complete before the call.  The frame
 * counter advances on every call.  out may be NULL.  The (tile, Gaussian)
 * pairs of one call are counted in 32 bits (at most 2^32 - 1); the pair
 * buffers grow as needed (a call that outgrows them splats again).
 * Errors: INVALID_ARG (NULL cams/image, n_views == 0), CAPACITY
 * (n_views > max_views, or the pair buffers cannot grow), HIP, STATE. */
vm3dgs_status vm3dgs_frame(vm3dgs* ctx, const vm3dgs_camera* cams, uint32_t n_views, float* image_dev,
                           vm3dgs_frame_out* out);

/* vm3dgs_frame for callers that cannot allocate memory while they run
 * frames (code under stream capture, serving loops, hosts that forbid
 * allocation after set-up): the same frame, with the same kernels and the
 * same results, that allocates nothing.  Every buffer it uses was made by
 * vm3dgs_create, except the (tile, Gaussian) pair buffers, which are one
 * fixed array of device memory per GPU (128 MiB, part of the library's code
 * object, held by each GPU the library runs on until the process ends).  It
 * holds 7,864,320 pairs (VM3DGS_NOALLOC_MAX_PAIRS).  A frame with more pairs
 * returns CAPACITY: the page table, copies and counters of that frame are
 * done (the frame counter advances), its image is not written, and
 * vm3dgs_frame renders the same view with buffers that grow.  Every context
 * on one GPU shares the array, which keeps the last call's pairs; calls that
 * overlap on one GPU (two threads, or contexts on different streams whose
 * frames run at once) race on it and must be serialised by the caller.
 * Arguments, outputs and other errors as vm3dgs_frame. */
#define VM3DGS_NOALLOC_MAX_PAIRS 7864320u
vm3dgs_status vm3dgs_frame_noalloc(vm3dgs* ctx, const vm3dgs_camera* cams, uint32_t n_views, float* image_dev,
                                   vm3dgs_frame_out* out);

/* Splat every level-0 Gaussian of the scene with the same kernels and no
 * paging (the no-virtual-memory baseline of Sec. 5.3).  Needs
 * VM3DGS_FLAG_FULL_SCENE_COPY at create.  image_dev as in vm3dgs_frame;
 * stats may be NULL.  Does not touch the page table. */
vm3dgs_status vm3dgs_render_full(vm3dgs* ctx, const vm3dgs_camera* cams, uint32_t n_views, float* image_dev,
                                 vm3dgs_stats* stats);

/* Copy a named piece of state or of the last frame's intermediates to host
 * memory (parity checks).  Returns the byte size of the item (and copies it
 * when host_dst != NULL and cap >= size), or -1 for an unknown name.
 * Waits for the render stream.  Names: "info", "perm", "spheres", "cell_box",
 * "cell_page", "link_start", "link_dst", "cand", "idbuf", "req_direct",
 * "req_link", "page_level", "slot_level", "last_used", "sub_vpage",
 * "sub_last_used", "v2p", "copies", "copy_id", "render_list", "pp_float",
 * "pp_int", "keys", "vals", "ranges", "host_page" (level-0 attributes of all
 * pages decoded to 59 floats), "blend_stats" (per tile: pixel-Gaussian
 * evaluations and alpha evaluations, two uint32, of the last frame run with
 * VM3DGS_FLAG_BLEND_STATS). */
int64_t vm3dgs_debug_get(vm3dgs* ctx, const char* name, void* host_dst, int64_t cap);

/* Empty the pool and the page table and restart the frame counter (and the
 * prefetch pose history), as after create; the scene stays.  Waits for both
 * streams. */
vm3dgs_status vm3dgs_reset(vm3dgs* ctx);

/* Replace the VM3DGS_FLAG_LINKS / BLEND_STATS / SIGMA3_TILES bits of the options
 * for later frames (VM3DGS_FLAG_FULL_SCENE_COPY is fixed at create).
 * Errors: INVALID_ARG for a NULL context. */
vm3dgs_status vm3dgs_set_flags(vm3dgs* ctx, uint32_t flags);

/* Set the LOD threshold tau (Sec. 4.1 Level of Detail: a page is drawn at
 * level l when l is the first level with projected page radius
 * fy * R / depth > tau / 2^l, capped at L - 1) for later frames, as
 * lod_radius_px at create would; the adaptive controller (Sec. 5.1.1), when
 * on, starts again from this tau with its initial step.
 * Errors: INVALID_ARG for a NULL context or a tau that is not a positive
 * finite number. */
vm3dgs_status vm3dgs_set_lod_radius(vm3dgs* ctx, float tau_px);

/* Block until the render and copy streams are idle. */
vm3dgs_status vm3dgs_sync(vm3dgs* ctx);

/* Create-time paging only (Sec. 3), on the host, with no device work: the
 * same Morton pages, proxy boxes, links, spheres and LOD levels that
 * vm3dgs_create builds.  For inspection and host-side checks.  Items are read
 * with vm3dgs_pages_get ("info", "perm", "spheres", "cell_box", "cell_page",
 * "cell_start", "link_start", "link_dst", "rec0", "rec1", "rec2" (decoded
 * 59-float records per level), "store" (the encoded page-major store)).
 * Errors as for vm3dgs_create (INVALID_ARG, HOST_OOM). */
typedef struct vm3dgs_pages vm3dgs_pages;
vm3dgs_status vm3dgs_pages_build(const vm3dgs_scene* scene, uint32_t page_size, uint32_t lod_levels,
                                 const vm3dgs_options* opt, vm3dgs_pages** out);
int64_t vm3dgs_pages_get(const vm3dgs_pages* pages, const char* name, void* host_dst, int64_t cap);
void vm3dgs_pages_destroy(vm3dgs_pages* pages);

/* Text of the last error of this context (never NULL; "" when none). */
const char* vm3dgs_last_error(const vm3dgs* ctx);

/* Text of the last vm3dgs_create failure in this thread. */
const char* vm3dgs_create_error(void);

/* Release every host and device resource.  NULL is allowed. */
void vm3dgs_destroy(vm3dgs* ctx);

/* ---- Learned page prefetch: the network ----------------------------------
 * The paper leaves prefetching to future work (Sec. 6).  This network
 * proposes lowest-priority page requests; the visibility pass stays the
 * judge of what is rendered.  A multilayer perceptron: dims[0] inputs,
 * ReLU hidden layers, dims[n_layers] logits (one per page cluster), trained
 * with the mean binary cross-entropy of sigmoid(logit) and Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8) on fp32 master weights.  Every matrix product runs
 * on the matrix cores with bf16 operands (weights, inputs, hidden
 * activations, output gradients; round to nearest even) and fp32
 * accumulation.
 *
 * Parameter layout (floats, host or device as stated): per layer l,
 * W_l [dims[l]][dims[l+1]] row-major (input index major), then b_l
 * [dims[l+1]]; vm3dgs_mlp_n_params gives the total.
 * The network owns its device memory; calls are ordered on its stream
 * (stream = NULL: its own); pointers named _dev are device memory the caller
 * owns, and results written there are ready on that stream.  Inputs written
 * on another stream must be complete before a call, and must stay valid
 * until the network's stream has passed it (vm3dgs_mlp_sync). */
typedef struct vm3dgs_mlp vm3dgs_mlp;

/* dims[n_layers + 1], 1 <= n_layers <= 8, widths 1..65536; max_batch rows
 * per call (1..65536).  INVALID_ARG for bad sizes, DEVICE_OOM, HIP. */
vm3dgs_status vm3dgs_mlp_create(const uint32_t* dims, uint32_t n_layers, uint32_t max_batch, void* stream,
                                vm3dgs_mlp** out);
const char* vm3dgs_mlp_create_error(void);
const char* vm3dgs_mlp_last_error(const vm3dgs_mlp* net);
uint64_t vm3dgs_mlp_n_params(const vm3dgs_mlp* net);
/* Weights from host memory (n = vm3dgs_mlp_n_params); resets Adam. */
vm3dgs_status vm3dgs_mlp_set_params(vm3dgs_mlp* net, const float* params_host, uint64_t n);
/* Master weights and Adam moments to host memory (any pointer may be NULL);
 * step = Adam steps taken since the last set_params. */
vm3dgs_status vm3dgs_mlp_get_state(vm3dgs_mlp* net, float* params_host, float* adam_m_host, float* adam_v_host,
                                   uint64_t n, uint32_t* step);
/* x_dev [batch][dims[0]] fp32 -> logits_dev [batch][dims[n_layers]] fp32.
 * CAPACITY when batch > max_batch. */
vm3dgs_status vm3dgs_mlp_forward(vm3dgs_mlp* net, const float* x_dev, uint32_t batch, float* logits_dev);
/* Gradient of the loss for labels y_dev [batch][dims[n_layers]] (0/1 fp32)
 * into grad_dev (parameter layout, fp32); loss_host may be NULL. */
vm3dgs_status vm3dgs_mlp_gradient(vm3dgs_mlp* net, const float* x_dev, const float* y_dev, uint32_t batch,
                                  float* grad_dev, float* loss_host);
/* Forward, backward and one Adam step with learning rate lr; loss_host (the
 * loss before the step) may be NULL (then nothing waits for the device). */
vm3dgs_status vm3dgs_mlp_train_step(vm3dgs_mlp* net, const float* x_dev, const float* y_dev, uint32_t batch,
                                    float lr, float* loss_host);
vm3dgs_status vm3dgs_mlp_sync(vm3dgs_mlp* net);
void vm3dgs_mlp_destroy(vm3dgs_mlp* net);

/* ---- Learned page prefetch: the stage in the frame -----------------------
 * Features of view v (28 + hist_bins floats): its last four camera poses,
 * oldest first (position minus center, over extent; the camera-to-world
 * rotation as a unit quaternion w x y z with w >= 0; the oldest pose repeats
 * until four frames were seen), then the resident fraction (any level) of
 * each of hist_bins equal page-id ranges, after the frame's demand stages.
 * Clusters are n_clusters equal page-id ranges.  A page is proposed when the
 * logit of its cluster exceeds logit_threshold for some view, the frame did
 * not request it and it is not resident at the level its nearest distance
 * (sphere centre distance minus radius, at least znear) gives.  Proposals are
 * served nearest first after the demand misses, only into physical pages used
 * in neither this frame nor the previous one (least recently used first), at
 * most budget_pages per frame; their copies follow the demand copies on the
 * copy stream, this frame does not wait for them or render them, and the
 * next frame waits for them before it reads the pool. */
typedef struct {
    uint32_t n_clusters;        /* network outputs */
    uint32_t hist_bins;         /* network inputs = 28 + hist_bins */
    uint32_t budget_pages;      /* prefetch copies per frame */
    float logit_threshold;
    float center[3];
    float extent;               /* > 0 */
} vm3dgs_prefetch_opts;

/* Attach the stage.  net may be NULL: then only the pose history is kept
 * and vm3dgs_prefetch_features works (gathering training data).  The network
 * must have dims[0] = 28 + hist_bins, n_clusters outputs and max_batch >=
 * max_views, and must not be trained while frames use it.  Poses are
 * recorded from the next frame on.  INVALID_ARG on a mismatch. */
vm3dgs_status vm3dgs_set_prefetch(vm3dgs* ctx, vm3dgs_mlp* net, const vm3dgs_prefetch_opts* opts);
/* Feature rows [n_views][28 + hist_bins] of the current state (the poses of
 * the frames so far and the residency now) into host memory. */
vm3dgs_status vm3dgs_prefetch_features(vm3dgs* ctx, uint32_t n_views, float* x_host);

/* ---- Learned page prefetch: training data and training -------------------
 * Training data are the method's own page sets: camera paths rendered by
 * the plain method (the network's stage off), one view per frame, each path
 * from an empty pool (the context is reset before each path and after the
 * call).  For frame t of a path with a frame t+1, the row is the feature
 * row after frame t (as vm3dgs_prefetch_features gives it), and the label
 * row marks (1.0) every cluster holding a page that frame t+1 requested and
 * that was not resident, at any level, after frame t (0.0 elsewhere). */
typedef struct {
    const vm3dgs_camera* cams;      /* the cameras of all paths, path after path */
    const uint32_t* path_frames;    /* frames of each path */
    uint32_t n_paths;
} vm3dgs_dataset;

/* Rows of the dataset into host memory: x_host [cap_rows][28 + hist_bins],
 * y_host [cap_rows][n_clusters] (either may be NULL to count only); *rows =
 * frames minus paths.  Needs the stage (vm3dgs_set_prefetch, net may be
 * NULL).  CAPACITY when the rows exceed cap_rows (nothing written past it);
 * INVALID_ARG for a missing stage or empty data. */
vm3dgs_status vm3dgs_prefetch_collect(vm3dgs* ctx, const vm3dgs_dataset* data, float* x_host, float* y_host,
                                      uint64_t cap_rows, uint64_t* rows);

typedef struct {
    uint32_t steps;            /* Adam steps */
    uint32_t batch;            /* rows per step, 1..the network's max_batch */
    float lr;                  /* learning rate */
    uint64_t seed;             /* the rows of each step: uniform draws with replacement (splitmix64) */
    float proposal_factor;     /* > 0: set the stage's logit threshold so that the network, on the
                                  training rows, proposes this many times as many clusters as the labels
                                  hold (its (1 - factor * positive rate) quantile); 0: keep it */
    uint32_t log_every;        /* record the loss every log_every steps (0: the first and last only) */
} vm3dgs_train_opts;

typedef struct {
    uint64_t rows;             /* training rows */
    float positive_rate;       /* share of label entries that are 1 */
    float loss_first;          /* mean binary cross-entropy before the first step */
    float loss_last;           /* before the last step */
    float logit_threshold;     /* the stage's threshold after the call */
    float ms_collect, ms_train;
    uint32_t n_losses;         /* recorded losses in losses[] (at most 64, evenly thinned) */
    float losses[64];
} vm3dgs_train_log;

/* Train the network attached to the stage (vm3dgs_set_prefetch with a net)
 * on the dataset's rows with the library's kernels (bf16 matrix products,
 * fp32 Adam), then set its logit threshold (proposal_factor).  The stage
 * options stay; the context is reset.  log may be NULL.  INVALID_ARG for no
 * network, empty data or a batch outside 1..max_batch; HIP, HOST_OOM,
 * DEVICE_OOM. */
vm3dgs_status vm3dgs_prefetch_train(vm3dgs* ctx, const vm3dgs_dataset* data, const vm3dgs_train_opts* opts,
                                    vm3dgs_train_log* log);

/* The network's widths and fp32 master weights to a file, and back: a
 * little-endian binary file, "VM3DGSNN" then uint32 n_layers, uint32
 * dims[n_layers + 1], float params[n_params] (the parameter layout above).
 * Loading needs a network of the same widths and resets its Adam state.
 * INVALID_ARG for a missing file, a bad header or other widths. */
vm3dgs_status vm3dgs_mlp_save(vm3dgs_mlp* net, const char* path);
vm3dgs_status vm3dgs_mlp_load(vm3dgs_mlp* net, const char* path);
/* vm3dgs_mlp_load into the network attached to the stage. */
vm3dgs_status vm3dgs_prefetch_load(vm3dgs* ctx, const char* path);

#ifdef __cplusplus
}
#endif
#endif
