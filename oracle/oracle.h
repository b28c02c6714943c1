/*
 * oracle.h -- plain, slow CPU oracle for the per-frame path of virtual-memory
 * 3D Gaussian Splatting (Haberl et al., "Virtual Memory for 3D Gaussian
 * Splatting", arXiv 2506.19415).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product links, loads or calls
 * this code; only the test-suite, the smoke check and the benchmark's CPU
 * baseline do.  It shares no source with the HIP path.
 *
 * Every step is written as the plain definition (loops, qsort), in the order
 * the paper gives: create-time paging (Sec. 3), page determination with a
 * page-ID buffer, links and LOD (Sec. 4.1), the two-stage page table with
 * LRU replacement (Sec. 4.1.1), and splatting of the resident Gaussians with
 * the 3DGS math of Kerbl et al. (Sec. 4.2).  Decisions that turn floating
 * point into integers (tile rectangles, depth keys, visibility, alpha
 * thresholds) are taken in float32, the precision of the paper's renderer.
 *
 * Gaussian record (59 floats): mean[3] scale[3] quat(w,x,y,z)[4] opacity
 * sh[16][3].
 */
#ifndef VM3DGS_ORACLE_H
#define VM3DGS_ORACLE_H
#include <stdint.h>

#define OR_REC 59

typedef struct {
    int64_t n;
    const float* means;   /* [n][3] */
    const float* scales;  /* [n][3] */
    const float* quats;   /* [n][4] */
    const float* opacity; /* [n]    */
    const float* sh;      /* [n][16][3] */
} or_scene_in;

typedef struct {
    float view[16];   /* world -> camera, row-major, OpenCV axes */
    float cam_pos[3];
    float fx, fy, cx, cy, znear;
} or_camera;

typedef struct or_scene or_scene;
typedef struct or_vm or_vm;

/* ---- math definitions shared (by definition, not by code) with the GPU ---- */
float or_vm_exp(float x);
double or_sh_basis(int k, double x, double y, double z);

/* ---- create time (Sec. 3) ---- */
/* lod_builder: 0 = parents of 8 consecutive children by moment matching,
 * 1 = the section's k-means clustering within the page (or_kmeans_page) */
or_scene* or_scene_build(const or_scene_in* in, int page_size, int lod_levels,
                         double cell_m, double link_sigma, int attr_format, float lod_scale_up, int lod_builder);
void or_scene_free(or_scene* s);
int64_t or_scene_get(const or_scene* s, const char* name, void* dst, int64_t cap);

/* Parent of k children by opacity-weighted moment matching (Sec. 3 "Level
 * of Detail", read as moment matching), its scales then multiplied by
 * scale_up (the section's fixed factor that fills gaps; 1 = moment matching
 * alone): out[59] in double, and the stored float record. */
void or_merge_children_d(const float* children, int k, double scale_up, double* out);
void or_merge_children(const float* children, int k, double scale_up, float* out);

/* The k parents of one page's level from its n records c (Sec. 3 "Level of
 * Detail": k-means on scaled attributes, arithmetic means, a fixed scale-up).
 * out: k records; assign (nullable): the cluster of each record, -1 for
 * padding.  Returns the Lloyd iterations run (KM_ITERS = 16 at most). */
int or_kmeans_page(const float* c, int n, int k, double scale_up, float* out, int32_t* assign);

/* ---- per frame (Sec. 4) ---- */
/* guard_px: the page-ID buffer and the frustum extend this many pixels past
 * each edge of the image */
or_vm* or_vm_create(const or_scene* s, int pool_pages, int copy_budget, int use_links,
                    int img_w, int img_h, int idbuf_w, int idbuf_h, float lod_radius_px, float guard_px);
void or_vm_free(or_vm* vm);
/* tile_mask: NULL = render every tile, else [n_views * TX * TY] bytes, 1 = render */
int or_vm_frame(or_vm* vm, const or_camera* cams, int n_views, const uint8_t* tile_mask);
int64_t or_vm_get(const or_vm* vm, const char* name, void* dst, int64_t cap);

/* Full-scene splat of every level-0 Gaussian (no paging): the reference the
 * VM image is compared with.  Results are read with or_vm_get on a VM made
 * for the same image size. */
int or_render_full(or_vm* vm, const or_camera* cams, int n_views, const uint8_t* tile_mask);

/* Visibility, requests and page table only; brute_force rasterises every
 * proxy box over every ID-buffer pixel. */
int or_vm_visibility(or_vm* vm, const or_camera* cams, int n_views, int brute_force);
/* The page table driven by an explicit request list in service order. */
int or_vm_pagetable(or_vm* vm, int n, const int32_t* pages, const int8_t* levels);
/* Test switches: every page directly requested; tile rectangles from the
 * 3-sigma radius alone (the support box off). */
void or_vm_set_force_all(or_vm* vm, int on);
void or_vm_set_support_box(or_vm* vm, int on);
/* streaming (Sec. 4.3, Sec. 5.1.2): a frame renders what was resident when
 * it started (a page resident only at another level at the nearest such
 * level, the finer at equal distance; that entry is required too), its
 * copies land for the next frame, and level transitions are served after
 * the other misses */
void or_vm_set_async(or_vm* vm, int on);
/* OpenMP threads of the splat loops (n > 0 sets; returns the count in use) */
int or_set_threads(int n);
/* LOD thresholds that follow memory use (several levels only). */
void or_vm_set_adaptive_lod(or_vm* vm, int on);
/* Level of a page (Sec. 4.1 "Level of Detail"): the first l with projected
 * radius fy * radius / depth > tau / 2^l, else L - 1. */
int or_lod_level(float fy, float radius, float depth, float tau, int L);
/* The memory-use controller (Sec. 5.1.1) run over n frames from a fresh
 * state with radius tau0: per frame the pool size S, the physical pages the
 * frame required, the requests left missing and the requested pages at a
 * coarse level; out: the radius and the step after each frame. */
void or_lod_control_trace(int n, int S, float tau0, const int* req_slots, const int* n_missing,
                          const int* n_coarse, float* tau_out, float* step_out);

/* Learned prefetch: n_clusters equal page-id ranges, hist_bins equal ranges
 * for the residency features, proposals where a logit exceeds
 * logit_threshold, at most budget_pages prefetch copies per frame; poses are
 * taken relative to center over extent.  Poses are recorded from the next
 * frame on.  or_vm_features: the feature row of a view from the current
 * state (28 pose floats, then hist_bins fractions).  or_vm_frame_prefetch:
 * a frame whose prefetch stage uses the given logits [n_views][n_clusters]. */
int or_vm_set_prefetch(or_vm* vm, int n_clusters, int hist_bins, float logit_threshold, int budget_pages,
                       const float* center, float extent);
void or_vm_features(const or_vm* vm, int view, float* x);
int or_vm_frame_prefetch(or_vm* vm, const or_camera* cams, int n_views, const float* logits,
                         const uint8_t* tile_mask);

/* ---- learned page prefetch (network oracle, or_mlp.c) ---- */
/* dims[n_layers + 1]; params: per layer W [d_l][d_{l+1}] then b [d_{l+1}];
 * bf16 != 0 rounds the operands of every product to bf16 as the GPU holds
 * them.  z: logits [B][d_L]; grad: parameter layout. */
int64_t or_mlp_n_params(int n_layers, const int* dims);
int or_mlp_forward(int B, int n_layers, const int* dims, const float* params, const float* x, int bf16, double* z);
double or_mlp_backward(int B, int n_layers, const int* dims, const float* params, const float* x, const float* y,
                       int bf16, double* grad, double* z);
void or_adam(int64_t n, float* w, float* m, float* v, const double* g, double lr, double b1, double b2, double eps,
             int t);

/* FP64 reference splat of the last frame's render set with the attributes
 * of src (a scene of the same pages, e.g. the fp32 form of a half scene);
 * image: [n_views][H][W][3] doubles. */
int or_vm_render_fp64(const or_vm* vm, const or_scene* src, const or_camera* cams, int n_views, double* image);

/* fp16 / bf16 round trips (round to nearest even) */
float or_round_f16(float x);
float or_round_bf16(float x);

#endif
