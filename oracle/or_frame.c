/*
 * or_frame.c -- oracle of one VM-3DGS frame (paper Sec. 4).
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Steps, in the paper's order:
 *  1. page determination (Sec. 4.1): page bounding spheres against the view
 *     frustum, then the proxy rendered at low resolution into a page-ID
 *     buffer (nearest depth wins; 0 / all-ones = background, Sec. 5.1.1);
 *  2. reduction (Sec. 5.1.1): per page the nearest depth over its pixels,
 *     then the same depth pushed to every linked page (Sec. 4.1 "Page Links");
 *  3. LOD choice from that depth (Sec. 4.1 "Level of Detail"): level l when
 *     the page's projected radius falls at or below tau / 2^(l-1) pixels;
 *  4. page table (Sec. 4.1.1): stage one marks required entries and drops
 *     hits; stage two places misses into free physical pages in LRU order
 *     and lists the copies;
 *  5. render list (Sec. 4.1.1, last paragraph): resident required pages;
 *  6. splatting (Sec. 4.2, math of Kerbl et al.): EWA projection, SH
 *     colour, per-tile lists ordered by depth then Gaussian index, front-to-
 *     back alpha blending.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

/* memory-use controller of the LOD thresholds (lod_controller below) */
#define LOD_STEP0 0.125f
#define LOD_QUICK 4
#define LOD_TAU_MIN 0.0078125f
#define LOD_TAU_MAX 65536.0f

/* from or_create.c / or_math.c */
int or_scene_P(const or_scene* s);
int or_scene_L(const or_scene* s);
int or_scene_npg(const or_scene* s);
int or_scene_format(const or_scene* s);
const float* or_scene_attr(const or_scene* s, int l);
const float* or_scene_spheres(const or_scene* s);
int64_t or_scene_ncells(const or_scene* s);
const float* or_scene_cellbox(const or_scene* s);
const int32_t* or_scene_cellpage(const or_scene* s);
const int32_t* or_scene_cellstart(const or_scene* s);
const int32_t* or_scene_linkstart(const or_scene* s);
const int32_t* or_scene_linkdst(const or_scene* s);
const int64_t* or_scene_perm(const or_scene* s);
void or_sh_color_f32(const float* sh, float x, float y, float z, float out[3]);

#define NONE32 0xffffffffu
#define NONE64 0xffffffffffffffffull
#define SUBS 64
#define OR_MAX_VIEWS 16

typedef struct {
    int culled;
    float u, v, depth;
    float conic[3];
    float opacity;
    float rgb[3];
    int rect[4];   /* x0 y0 x1 y1, tiles, exclusive upper */
    int tiles;
} pp_t;

typedef struct { int32_t page, level, slot, sub, count; int64_t base; } rl_t;

struct or_vm {
    const or_scene* s;
    int S, budget, use_links, W, H, Wv, Hv, TX, TY;
    float tau;
    float guard;           /* ID buffer and frustum extend this many pixels past each image edge */
    int P, L, n_pg, bytes_g;
    int frame;
    int force_all;         /* test switch: every page is directly requested */
    int support_box;       /* 1: 3-sigma tile rectangles cut to the support box (default 0: plain 3-sigma) */
    int last_full;         /* the last splat was or_render_full (every level-0 Gaussian) */
    /* streaming (Sec. 4.3, Sec. 5.1.2): a frame's copies land for the next
     * frame; it renders what was resident when it started, a page resident
     * only at another level at that level (the switch is deferred) */
    int async;
    int8_t* rlevel;        /* [n_pg] level a requested page is rendered at, -1 none (streaming) */
    int n_fallback;        /* requests rendered at another level (streaming) */
    /* LOD thresholds that follow memory use (Sec. 4.1, Sec. 5.1.1) */
    int adaptive;
    float tau_used, lod_step;
    int lod_dir, lod_last_move, req_slots, n_coarse;
    /* learned prefetch (Sec. 6 future work): configuration, pose history,
     * the logits a frame is given and what the last frame did with them */
    int pf_on, pf_K, pf_H, pf_budget;
    float pf_thr, pf_center[3], pf_extent;
    int pf_n_hist;                 /* poses pushed so far (saturates at 4) */
    float pf_pose[OR_MAX_VIEWS][4][7];
    const float* pf_logits;        /* [n_views][K] for the frame being run, or NULL */
    const or_camera* pf_cams;      /* cameras of the frame being run */
    int n_copy_demand, n_prefetch, n_pf_req;
    uint64_t* pf_keys;             /* [n_pg] sorted prefetch request keys of the last frame */
    float* pf_x;                   /* [n_views][28 + H] features the last frame computed */
    /* page table */
    int8_t* slot_level;
    int32_t* last_used;
    int32_t* sub_vpage;
    int32_t* sub_last_used;
    int32_t* v2p;
    /* last frame */
    int n_views;
    uint8_t* cand;         /* [views][n_pg] */
    uint64_t* idbuf;       /* [views][Hv][Wv] */
    uint32_t* req_direct, * req_link;
    int n_req;
    int32_t* req_page; int8_t* req_level; uint8_t* req_class; uint32_t* req_depth;
    int8_t* page_level;    /* [n_pg] requested level, -1 none */
    int n_copy; int64_t* copy; int32_t* copy_id;   /* [n][3] bytes triples, [n][4] page level slot sub */
    int n_missing; int32_t* missing;               /* [n][2] page level */
    int n_missing_cap;                             /* of them, those left for want of a free pool entry */
    int hits, misses, evictions;
    int n_rl; rl_t* rl; int64_t n_render;
    pp_t* pp;              /* [views][n_render] */
    int64_t n_pairs; uint64_t* keys; uint32_t* vals;
    uint32_t* ranges;      /* [views*TX*TY][2] */
    float* image;          /* [views][H][W][3] */
    float* final_T;        /* [views][H][W] */
    int64_t* contrib;      /* [views][H][W] Gaussians blended per pixel */
    int64_t* visits;       /* [views][H][W] list entries the pixel's loop visits (up to and including the stop) */
};

/* ------------------------------------------------------------------------ */
static inline uint32_t fbits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static inline float bitsf(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

static inline void view_xform(const float* V, float x, float y, float z, float* o)
{
    o[0] = ((V[0] * x + V[1] * y) + V[2] * z) + V[3];
    o[1] = ((V[4] * x + V[5] * y) + V[6] * z) + V[7];
    o[2] = ((V[8] * x + V[9] * y) + V[10] * z) + V[11];
}

/* ---- 1a. frustum: sphere against near plane and the four side planes, which
 * pass through the edges of the image widened by the guard band G ---- */
static int sphere_in_frustum(const or_camera* c, int W, int H, float G, const float* sp)
{
    float p[3];
    view_xform(c->view, sp[0], sp[1], sp[2], p);
    float r = sp[3];
    if (!(p[2] + r > c->znear)) return 0;
    float tl = (c->cx + G) / c->fx, tr = (((float)W + G) - c->cx) / c->fx;
    float tt = (c->cy + G) / c->fy, tb = (((float)H + G) - c->cy) / c->fy;
    float kl = sqrtf(1.0f + tl * tl), kr = sqrtf(1.0f + tr * tr);
    float kt = sqrtf(1.0f + tt * tt), kb = sqrtf(1.0f + tb * tb);
    if (!(p[0] + tl * p[2] >= -(r * kl))) return 0;
    if (!(-p[0] + tr * p[2] >= -(r * kr))) return 0;
    if (!(p[1] + tt * p[2] >= -(r * kt))) return 0;
    if (!(-p[1] + tb * p[2] >= -(r * kb))) return 0;
    return 1;
}

/* ---- 1b. page-ID buffer: it spans image coordinates [-G, W+G) x [-G, H+G);
 * the ray through each buffer pixel centre against each proxy box (slab
 * test); the nearest entry depth wins ---- */
static void pixel_ray(const or_camera* c, int W, int H, float G, int Wv, int Hv, int px, int py, float inv[3])
{
    float sx = ((float)W + 2.0f * G) / (float)Wv, sy = ((float)H + 2.0f * G) / (float)Hv;
    float xc = ((float)px + 0.5f) * sx - G, yc = ((float)py + 0.5f) * sy - G;
    float dcx = (xc - c->cx) / c->fx;
    float dcy = (yc - c->cy) / c->fy;
    const float* V = c->view;
    for (int a = 0; a < 3; a++) {
        float d = (V[a] * dcx + V[4 + a] * dcy) + V[8 + a];
        if (d == 0.0f) d = 1e-30f;
        inv[a] = 1.0f / d;
    }
}

static int ray_box(const float* o, const float* inv, const float* box, float znear, float* depth)
{
    float t0 = -INFINITY, t1 = INFINITY;
    for (int a = 0; a < 3; a++) {
        float ta = (box[a] - o[a]) * inv[a];
        float tb = (box[3 + a] - o[a]) * inv[a];
        float tn = fminf(ta, tb), tf = fmaxf(ta, tb);
        t0 = a == 0 ? tn : fmaxf(t0, tn);
        t1 = a == 0 ? tf : fminf(t1, tf);
    }
    if (t0 <= t1 && t1 > znear) {
        *depth = fmaxf(t0, znear);
        return 1;
    }
    return 0;
}

/* conservative pixel rectangle of a box (inclusive, may be empty) */
static int box_rect(const or_camera* c, int W, int H, float G, int Wv, int Hv, const float* box, int* r)
{
    float vmin[3] = {INFINITY, INFINITY, INFINITY}, vmax[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = 0; k < 8; k++) {
        float p[3];
        view_xform(c->view, box[(k & 1) ? 3 : 0], box[(k & 2) ? 4 : 1], box[(k & 4) ? 5 : 2], p);
        for (int a = 0; a < 3; a++) { vmin[a] = fminf(vmin[a], p[a]); vmax[a] = fmaxf(vmax[a], p[a]); }
    }
    if (!(vmax[2] > c->znear * 0.5f)) return 0;
    float z0 = fmaxf(vmin[2], c->znear * 0.5f), z1 = vmax[2];
    float xs[4] = {vmin[0] / z0, vmin[0] / z1, vmax[0] / z0, vmax[0] / z1};
    float ys[4] = {vmin[1] / z0, vmin[1] / z1, vmax[1] / z0, vmax[1] / z1};
    float xl = fminf(fminf(xs[0], xs[1]), fminf(xs[2], xs[3])), xh = fmaxf(fmaxf(xs[0], xs[1]), fmaxf(xs[2], xs[3]));
    float yl = fminf(fminf(ys[0], ys[1]), fminf(ys[2], ys[3])), yh = fmaxf(fmaxf(ys[0], ys[1]), fmaxf(ys[2], ys[3]));
    float sx = ((float)W + 2.0f * G) / (float)Wv, sy = ((float)H + 2.0f * G) / (float)Hv;
    float fx0 = floorf(((c->fx * xl + c->cx) + G) / sx) - 1.0f, fx1 = floorf(((c->fx * xh + c->cx) + G) / sx) + 1.0f;
    float fy0 = floorf(((c->fy * yl + c->cy) + G) / sy) - 1.0f, fy1 = floorf(((c->fy * yh + c->cy) + G) / sy) + 1.0f;
    fx0 = fmaxf(fx0, 0.0f); fy0 = fmaxf(fy0, 0.0f);
    fx1 = fminf(fx1, (float)(Wv - 1)); fy1 = fminf(fy1, (float)(Hv - 1));
    if (!(fx0 <= fx1) || !(fy0 <= fy1)) return 0;
    r[0] = (int)fx0; r[1] = (int)fy0; r[2] = (int)fx1; r[3] = (int)fy1;
    return 1;
}

/* brute_force != 0 tests every pixel for every box (reference for the rect) */
static void idbuf_render(const or_vm* vm, const or_camera* c, const uint8_t* cand, uint64_t* ib, int brute_force)
{
    int Wv = vm->Wv, Hv = vm->Hv;
    for (int i = 0; i < Wv * Hv; i++) ib[i] = NONE64;
    float* inv = malloc(sizeof(float) * 3 * (size_t)Wv * Hv);
    for (int py = 0; py < Hv; py++)
        for (int px = 0; px < Wv; px++) pixel_ray(c, vm->W, vm->H, vm->guard, Wv, Hv, px, py, inv + 3 * (py * Wv + px));
    const float* boxes = or_scene_cellbox(vm->s);
    const int32_t* cstart = or_scene_cellstart(vm->s);
    for (int p = 0; p < vm->n_pg; p++) {
        if (!cand[p]) continue;
        for (int32_t ci = cstart[p]; ci < cstart[p + 1]; ci++) {
            const float* box = boxes + 6 * ci;
            int r[4] = {0, 0, Wv - 1, Hv - 1};
            if (!brute_force && !box_rect(c, vm->W, vm->H, vm->guard, Wv, Hv, box, r)) continue;
            for (int py = r[1]; py <= r[3]; py++)
                for (int px = r[0]; px <= r[2]; px++) {
                    float d;
                    if (!ray_box(c->cam_pos, inv + 3 * (py * Wv + px), box, c->znear, &d)) continue;
                    uint64_t key = ((uint64_t)fbits(d) << 32) | (uint64_t)(p + 1);
                    if (key < ib[py * Wv + px]) ib[py * Wv + px] = key;
                }
        }
    }
    free(inv);
}

/* ---- 4. page table ------------------------------------------------------- */
typedef struct { int64_t k1, k2, k3; int32_t a, b; } ck;

static int cmp_ck(const void* x, const void* y)
{
    const ck* p = x; const ck* q = y;
    if (p->k1 != q->k1) return p->k1 < q->k1 ? -1 : 1;
    if (p->k2 != q->k2) return p->k2 < q->k2 ? -1 : 1;
    return (p->k3 > q->k3) - (p->k3 < q->k3);
}

static int cap_of(int level) { return 1 << (3 * level); }

static void assign(or_vm* vm, int32_t p, int lvl, int s, int j, uint8_t* req_sub, uint8_t* slot_req)
{
    int32_t old = vm->sub_vpage[s * SUBS + j];
    if (old >= 0) {
        vm->v2p[old * vm->L + lvl] = -1;
        vm->evictions++;
    }
    vm->sub_vpage[s * SUBS + j] = p;
    vm->sub_last_used[s * SUBS + j] = vm->frame;
    vm->last_used[s] = vm->frame;
    vm->v2p[p * vm->L + lvl] = s * SUBS + j;
    req_sub[s * SUBS + j] = 1;
    slot_req[s] = 1;
    int64_t Pl = vm->P >> (3 * lvl);
    int64_t base = 0;
    for (int l = 0; l < lvl; l++) base += (int64_t)vm->n_pg * (vm->P >> (3 * l)) * vm->bytes_g;
    int64_t* cp = vm->copy + 3 * vm->n_copy;
    cp[0] = base + (int64_t)p * Pl * vm->bytes_g;
    cp[1] = ((int64_t)s * vm->P + (int64_t)j * Pl) * vm->bytes_g;
    cp[2] = Pl * vm->bytes_g;
    int32_t* id = vm->copy_id + 4 * vm->n_copy;
    id[0] = p; id[1] = lvl; id[2] = s; id[3] = j;
    vm->n_copy++;
}

static void prefetch_stage(or_vm* vm, uint8_t* req_sub, uint8_t* slot_req);

static void page_table(or_vm* vm)
{
    int S = vm->S, L = vm->L;
    uint8_t* req_sub = calloc((size_t)S * SUBS, 1);
    uint8_t* slot_req = calloc((size_t)S, 1);
    int32_t* miss = malloc(sizeof(int32_t) * 2 * (size_t)(vm->n_req > 0 ? vm->n_req : 1));
    int nm = 0;
    vm->hits = vm->misses = vm->evictions = 0;
    vm->n_fallback = 0;
    /* stage 1: required entries, hits refresh last use, misses keep request
     * order.  Streaming: a miss whose page is resident at another level is
     * drawn at that level this frame (the resident level nearest to the
     * requested one, the finer at equal distance): that entry is required
     * too, and these misses (level transitions) are served after the others */
    int32_t* later = malloc(sizeof(int32_t) * 2 * (size_t)(vm->n_req > 0 ? vm->n_req : 1));
    int nl = 0;
    for (int i = 0; i < vm->n_req; i++) {
        int32_t p = vm->req_page[i];
        int l = vm->req_level[i];
        int32_t e = vm->v2p[p * L + l];
        if (vm->async) vm->rlevel[p] = -1;
        if (e >= 0) {
            int s = e / SUBS, j = e % SUBS;
            req_sub[s * SUBS + j] = 1;
            slot_req[s] = 1;
            vm->sub_last_used[s * SUBS + j] = vm->frame;
            vm->last_used[s] = vm->frame;
            vm->hits++;
            if (vm->async) vm->rlevel[p] = (int8_t)l;
            continue;
        }
        int fl = -1;
        if (vm->async)
            for (int d = 1; d < L && fl < 0; d++) {
                if (l - d >= 0 && vm->v2p[p * L + l - d] >= 0) fl = l - d;
                else if (l + d < L && vm->v2p[p * L + l + d] >= 0) fl = l + d;
            }
        if (fl >= 0) {
            int32_t f = vm->v2p[p * L + fl];
            int s = f / SUBS, j = f % SUBS;
            req_sub[s * SUBS + j] = 1;
            slot_req[s] = 1;
            vm->sub_last_used[s * SUBS + j] = vm->frame;
            vm->last_used[s] = vm->frame;
            vm->rlevel[p] = (int8_t)fl;
            vm->n_fallback++;
            later[2 * nl] = p; later[2 * nl + 1] = l; nl++;
        } else {
            miss[2 * nm] = p; miss[2 * nm + 1] = l; nm++;
        }
    }
    for (int i = 0; i < nl; i++) { miss[2 * nm] = later[2 * i]; miss[2 * nm + 1] = later[2 * i + 1]; nm++; }
    free(later);
    vm->misses = nm;
    /* stage 2 candidate lists, fixed at the start of the stage */
    ck* wl = malloc(sizeof(ck) * (size_t)S);
    int nw = 0;
    for (int s = 0; s < S; s++)
        if (!slot_req[s]) { wl[nw].k1 = vm->last_used[s]; wl[nw].k2 = s; wl[nw].k3 = 0; wl[nw].a = s; wl[nw].b = 0; nw++; }
    qsort(wl, (size_t)nw, sizeof(ck), cmp_ck);
    ck* cl[3] = {NULL, NULL, NULL};
    int ncl[3] = {0, 0, 0};
    for (int l = 1; l < L; l++) {
        cl[l] = malloc(sizeof(ck) * (size_t)S * SUBS);
        for (int s = 0; s < S; s++) {
            if (vm->slot_level[s] != l) continue;
            for (int j = 0; j < cap_of(l); j++) {
                if (req_sub[s * SUBS + j]) continue;
                ck* c = cl[l] + ncl[l]++;
                c->k1 = vm->sub_vpage[s * SUBS + j] < 0 ? -1 : vm->sub_last_used[s * SUBS + j];
                c->k2 = s; c->k3 = j; c->a = s; c->b = j;
            }
        }
        qsort(cl[l], (size_t)ncl[l], sizeof(ck), cmp_ck);
    }
    int pw = 0, pc[3] = {0, 0, 0};
    int fresh[3][2];             /* slot converted this frame per level and its next free sub */
    int32_t* fresh_list[3] = {NULL, NULL, NULL};
    int fresh_n[3] = {0, 0, 0}, fresh_h[3] = {0, 0, 0};
    for (int l = 0; l < 3; l++) { fresh[l][0] = -1; fresh[l][1] = 0; fresh_list[l] = malloc(sizeof(int32_t) * (size_t)(S + 1)); }
    vm->n_copy = 0; vm->n_missing = 0; vm->n_missing_cap = 0;
    for (int i = 0; i < nm; i++) {
        int32_t p = miss[2 * i];
        int l = miss[2 * i + 1];
        if (vm->budget > 0 && vm->n_copy >= vm->budget) {
            vm->missing[2 * vm->n_missing] = p; vm->missing[2 * vm->n_missing + 1] = l; vm->n_missing++;
            continue;
        }
        int ts = -1, tj = -1;
        if (l > 0) {
            /* (1) a free or oldest non-required sub-slot of an existing level-l page */
            while (pc[l] < ncl[l]) {
                ck* c = cl[l] + pc[l]++;
                if (vm->slot_level[c->a] == l && !req_sub[c->a * SUBS + c->b]) { ts = c->a; tj = c->b; break; }
            }
            /* (2) remaining sub-slots of pages converted to level l in this frame */
            while (ts < 0 && fresh_h[l] < fresh_n[l]) {
                int s = fresh_list[l][fresh_h[l]];
                int j = -1;
                for (int t = 0; t < cap_of(l); t++)
                    if (!req_sub[s * SUBS + t] && vm->sub_vpage[s * SUBS + t] < 0 && vm->slot_level[s] == l) { j = t; break; }
                if (j >= 0) { ts = s; tj = j; } else fresh_h[l]++;
            }
        }
        if (ts < 0) {
            /* (3) the least recently used wholly free physical page, converted to level l */
            while (pw < nw) {
                int s = wl[pw++].a;
                if (slot_req[s]) continue;
                int oldl = vm->slot_level[s];
                if (oldl >= 0)
                    for (int j = 0; j < cap_of(oldl); j++) {
                        int32_t op = vm->sub_vpage[s * SUBS + j];
                        if (op >= 0) { vm->v2p[op * L + oldl] = -1; vm->evictions++; }
                    }
                for (int j = 0; j < SUBS; j++) { vm->sub_vpage[s * SUBS + j] = -1; vm->sub_last_used[s * SUBS + j] = -1; }
                vm->slot_level[s] = (int8_t)l;
                ts = s; tj = 0;
                if (l > 0) fresh_list[l][fresh_n[l]++] = s;
                break;
            }
        }
        if (ts < 0) {
            vm->missing[2 * vm->n_missing] = p; vm->missing[2 * vm->n_missing + 1] = l; vm->n_missing++;
            vm->n_missing_cap++;
            continue;
        }
        assign(vm, p, l, ts, tj, req_sub, slot_req);
    }
    (void)fresh;
    vm->n_copy_demand = vm->n_copy;
    vm->req_slots = 0;
    for (int s = 0; s < S; s++) vm->req_slots += slot_req[s];
    vm->n_prefetch = 0;
    vm->n_pf_req = 0;
    if (vm->pf_on && vm->pf_logits) prefetch_stage(vm, req_sub, slot_req);
    for (int l = 0; l < 3; l++) { free(cl[l]); free(fresh_list[l]); }
    free(wl); free(miss); free(req_sub); free(slot_req);
}

/* ---- 5. learned prefetch -------------------------------------------------
 * Features of a view: its last four camera poses (position relative to the
 * scene centre over the extent, and the camera-to-world rotation as a unit
 * quaternion with w >= 0; the oldest pose repeats until four were seen) and
 * the resident fraction of each of H equal ranges of page ids.  Clusters are
 * K equal ranges of page ids (Morton order, so spatially compact).  A page is
 * proposed when some view's logit of its cluster exceeds the threshold, it is
 * not requested by the visibility pass, and it is not resident at the level
 * its distance gives.  Proposals are served after the demand misses, nearest
 * first, into physical pages used in neither this frame nor the previous one
 * (least recently used first), up to the prefetch budget; nothing proposed
 * is rendered in this frame. */
static void pose_of(const or_camera* c, const or_vm* vm, float* o)
{
    const float* V = c->view;
    double M[3][3];                       /* camera to world: transpose of the view rotation */
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) M[i][j] = V[4 * j + i];
    double w, x, y, z, tr = M[0][0] + M[1][1] + M[2][2];
    if (tr > 0.0) {
        double S = sqrt(tr + 1.0) * 2.0;
        w = 0.25 * S; x = (M[2][1] - M[1][2]) / S; y = (M[0][2] - M[2][0]) / S; z = (M[1][0] - M[0][1]) / S;
    } else if (M[0][0] > M[1][1] && M[0][0] > M[2][2]) {
        double S = sqrt(1.0 + M[0][0] - M[1][1] - M[2][2]) * 2.0;
        w = (M[2][1] - M[1][2]) / S; x = 0.25 * S; y = (M[0][1] + M[1][0]) / S; z = (M[0][2] + M[2][0]) / S;
    } else if (M[1][1] > M[2][2]) {
        double S = sqrt(1.0 + M[1][1] - M[0][0] - M[2][2]) * 2.0;
        w = (M[0][2] - M[2][0]) / S; x = (M[0][1] + M[1][0]) / S; y = 0.25 * S; z = (M[1][2] + M[2][1]) / S;
    } else {
        double S = sqrt(1.0 + M[2][2] - M[0][0] - M[1][1]) * 2.0;
        w = (M[1][0] - M[0][1]) / S; x = (M[0][2] + M[2][0]) / S; y = (M[1][2] + M[2][1]) / S; z = 0.25 * S;
    }
    double n = sqrt(w * w + x * x + y * y + z * z);
    if (w < 0.0) n = -n;
    for (int a = 0; a < 3; a++) o[a] = (float)(((double)c->cam_pos[a] - vm->pf_center[a]) / vm->pf_extent);
    o[3] = (float)(w / n); o[4] = (float)(x / n); o[5] = (float)(y / n); o[6] = (float)(z / n);
}

static void push_poses(or_vm* vm, const or_camera* cams, int n_views)
{
    for (int v = 0; v < n_views && v < OR_MAX_VIEWS; v++) {
        float cur[7];
        pose_of(&cams[v], vm, cur);
        if (vm->pf_n_hist == 0)
            for (int k = 0; k < 4; k++) memcpy(vm->pf_pose[v][k], cur, sizeof cur);
        else {
            for (int k = 0; k < 3; k++) memcpy(vm->pf_pose[v][k], vm->pf_pose[v][k + 1], sizeof cur);
            memcpy(vm->pf_pose[v][3], cur, sizeof cur);
        }
    }
    if (vm->pf_n_hist < 4) vm->pf_n_hist++;
}

/* feature row of view v from the current state: 28 pose floats, H fractions */
static void features(const or_vm* vm, int v, float* x)
{
    for (int k = 0; k < 4; k++) memcpy(x + 7 * k, vm->pf_pose[v][k], 7 * sizeof(float));
    int H = vm->pf_H, n_pg = vm->n_pg;
    for (int b = 0; b < H; b++) {
        int64_t lo = ((int64_t)b * n_pg + H - 1) / H, hi = ((int64_t)(b + 1) * n_pg + H - 1) / H;
        int cnt = 0;
        for (int64_t p = lo; p < hi; p++) {
            int res = 0;
            for (int l = 0; l < vm->L; l++) res |= vm->v2p[p * vm->L + l] >= 0;
            cnt += res;
        }
        x[28 + b] = hi > lo ? (float)cnt / (float)(hi - lo) : 0.0f;
    }
}

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

static void prefetch_stage(or_vm* vm, uint8_t* req_sub, uint8_t* slot_req)
{
    int n_pg = vm->n_pg, L = vm->L, K = vm->pf_K, nv = vm->n_views, S = vm->S;
    const or_camera* cams = vm->pf_cams;
    const float* sp = or_scene_spheres(vm->s);
    for (int v = 0; v < nv; v++) features(vm, v, vm->pf_x + (size_t)v * (28 + vm->pf_H));
    float fy = cams[0].fy;
    for (int v = 1; v < nv; v++) fy = fmaxf(fy, cams[v].fy);
    int n = 0;
    for (int p = 0; p < n_pg; p++) {
        int c = (int)((int64_t)p * K / n_pg);
        int sel = 0;
        for (int v = 0; v < nv; v++) sel |= vm->pf_logits[(size_t)v * K + c] > vm->pf_thr;
        if (!sel || vm->page_level[p] >= 0) continue;
        const float* q = sp + 4 * p;
        float dmin = INFINITY;
        for (int v = 0; v < nv; v++) {
            float dx = q[0] - cams[v].cam_pos[0], dy = q[1] - cams[v].cam_pos[1], dz = q[2] - cams[v].cam_pos[2];
            float d = fmaxf(sqrtf((dx * dx + dy * dy) + dz * dz) - q[3], cams[v].znear);
            dmin = fminf(dmin, d);
        }
        int lvl = 0;
        if (L > 1) {
            float rpx = (fy * q[3]) / dmin;
            float thr = vm->tau;
            while (lvl < L - 1 && !(rpx > thr)) { lvl++; thr = thr * 0.5f; }
        }
        if (vm->v2p[p * L + lvl] >= 0) continue;
        vm->pf_keys[n++] = (2ull << 61) | ((uint64_t)fbits(dmin) << 30) | ((uint64_t)lvl << 28) | (uint64_t)p;
    }
    qsort(vm->pf_keys, (size_t)n, sizeof(uint64_t), cmp_u64);
    vm->n_pf_req = n;
    /* physical pages used in neither this frame nor the previous one */
    ck* el = malloc(sizeof(ck) * (size_t)(S > 0 ? S : 1));
    int ne = 0;
    for (int s = 0; s < S; s++)
        if (!slot_req[s] && vm->last_used[s] < vm->frame - 1) {
            el[ne].k1 = vm->last_used[s]; el[ne].k2 = s; el[ne].k3 = 0; el[ne].a = s; el[ne].b = 0; ne++;
        }
    qsort(el, (size_t)ne, sizeof(ck), cmp_ck);
    int32_t* fresh = malloc(sizeof(int32_t) * 3 * (size_t)(S + 1));
    int fn[3] = {0, 0, 0}, fh[3] = {0, 0, 0}, pe = 0;
    for (int i = 0; i < n && vm->n_prefetch < vm->pf_budget; i++) {
        int32_t p = (int32_t)(vm->pf_keys[i] & 0x0fffffffu);
        int l = (int)((vm->pf_keys[i] >> 28) & 3u);
        int ts = -1, tj = -1;
        while (l > 0 && ts < 0 && fh[l] < fn[l]) {
            int s = fresh[l * (S + 1) + fh[l]];
            for (int t = 0; t < cap_of(l) && ts < 0; t++)
                if (vm->slot_level[s] == l && !req_sub[s * SUBS + t] && vm->sub_vpage[s * SUBS + t] < 0) { ts = s; tj = t; }
            if (ts < 0) fh[l]++;
        }
        if (ts < 0) {
            while (pe < ne) {
                int s = el[pe++].a;
                if (slot_req[s]) continue;
                int oldl = vm->slot_level[s];
                if (oldl >= 0)
                    for (int j = 0; j < cap_of(oldl); j++) {
                        int32_t op = vm->sub_vpage[s * SUBS + j];
                        if (op >= 0) { vm->v2p[op * L + oldl] = -1; vm->evictions++; }
                    }
                for (int j = 0; j < SUBS; j++) { vm->sub_vpage[s * SUBS + j] = -1; vm->sub_last_used[s * SUBS + j] = -1; }
                vm->slot_level[s] = (int8_t)l;
                ts = s; tj = 0;
                if (l > 0) fresh[l * (S + 1) + fn[l]++] = s;
                break;
            }
        }
        if (ts < 0) break;                 /* no physical page left for prefetching */
        assign(vm, p, l, ts, tj, req_sub, slot_req);
        vm->n_prefetch++;
    }
    free(fresh);
    free(el);
}

/* ---- 6. splatting -------------------------------------------------------- */
/* Support box of a projected Gaussian (an optional cut of its tile
 * rectangle, off by default).  Blending accepts a term only where
 * power >= -5.55, that is where the quadratic form Q = d^T Sigma'^-1 d is at
 * most 11.1; over a column at horizontal offset dx the smallest Q is
 * dx^2 / Sigma'_xx, so the accepted region lies within
 * |dx| <= sqrt(11.1 Sigma'_xx) (and the same for rows).  The float
 * evaluation of the power errs by less than 5e-7 kap Q with
 * kap = (a + c)^2 / det >= cond(Sigma') + 2, so the threshold is divided by
 * (1 - 5e-7 kap).  The box edges u -+ h and the pixel and tile offsets taken
 * from them are float values, each rounding off by at most 2^-24 (|u| + h):
 * 1/64 pixel plus 1e-6 (|u| + h) is added to cover them.  A footprint with
 * 5e-7 kap >= 1/2 keeps its rectangle.  Tiles outside the box hold no accepted pixel of the
 * Gaussian, so cutting the rectangle to it leaves the image unchanged (pinned
 * by image identity and a float64 brute force of the accepted region); it
 * only predicts which pairs a renderer that makes this cut emits. */
static void support_box_cut(float a, float cc, float det, float u, float v, int TX, int TY,
                            float* x0, float* x1, float* y0, float* y1)
{
    float kap = ((a + cc) * (a + cc)) / det;
    float e = 5e-7f * kap;
    if (!(e < 0.5f)) return;
    float f = 1.0f / (1.0f - e);
    float rx = sqrtf((11.11f * f) * a), ry = sqrtf((11.11f * f) * cc);
    float hx = rx + (0.015625f + 1e-6f * (fabsf(u) + rx));
    float hy = ry + (0.015625f + 1e-6f * (fabsf(v) + ry));
    float bx0 = fminf(fmaxf(floorf((u - hx) / 16.0f), 0.0f), (float)TX);
    float bx1 = fminf(fmaxf(floorf((u + hx) / 16.0f) + 1.0f, 0.0f), (float)TX);
    float by0 = fminf(fmaxf(floorf((v - hy) / 16.0f), 0.0f), (float)TY);
    float by1 = fminf(fmaxf(floorf((v + hy) / 16.0f) + 1.0f, 0.0f), (float)TY);
    *x0 = fmaxf(*x0, bx0); *x1 = fminf(*x1, bx1);
    *y0 = fmaxf(*y0, by0); *y1 = fminf(*y1, by1);
}

static void preprocess_one(const float* g, const or_camera* c, int W, int H, int TX, int TY, int support_box,
                           pp_t* o)
{
    memset(o, 0, sizeof *o);
    o->culled = 1;
    float op = g[10];
    if (op == 0.0f) return;                       /* padding */
    float t[3];
    view_xform(c->view, g[0], g[1], g[2], t);
    float tx = t[0], ty = t[1], tz = t[2];
    if (!(tz > c->znear)) return;
    /* covariance Sigma = R S S^T R^T */
    float w = g[6], x = g[7], y = g[8], z = g[9];
    float R[3][3];
    R[0][0] = 1.0f - 2.0f * (y * y + z * z);
    R[0][1] = 2.0f * (x * y - w * z);
    R[0][2] = 2.0f * (x * z + w * y);
    R[1][0] = 2.0f * (x * y + w * z);
    R[1][1] = 1.0f - 2.0f * (x * x + z * z);
    R[1][2] = 2.0f * (y * z - w * x);
    R[2][0] = 2.0f * (x * z - w * y);
    R[2][1] = 2.0f * (y * z + w * x);
    R[2][2] = 1.0f - 2.0f * (x * x + y * y);
    float M[3][3];
    for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) M[i][j] = R[i][j] * g[3 + j];
    float Sg[3][3];
    for (int i = 0; i < 3; i++)
        for (int k = 0; k < 3; k++) Sg[i][k] = (M[i][0] * M[k][0] + M[i][1] * M[k][1]) + M[i][2] * M[k][2];
    /* EWA: Jacobian of the perspective map at the (clamped) centre */
    const float* V = c->view;
    float limx = 1.3f * ((0.5f * (float)W) / c->fx);
    float limy = 1.3f * ((0.5f * (float)H) / c->fy);
    float cxz = fminf(limx, fmaxf(-limx, tx / tz)) * tz;
    float cyz = fminf(limy, fmaxf(-limy, ty / tz)) * tz;
    float tz2 = tz * tz;
    float j00 = c->fx / tz, j02 = -((c->fx * cxz) / tz2);
    float j11 = c->fy / tz, j12 = -((c->fy * cyz) / tz2);
    float T0[3], T1[3];
    for (int j = 0; j < 3; j++) {
        T0[j] = j00 * V[j] + j02 * V[8 + j];
        T1[j] = j11 * V[4 + j] + j12 * V[8 + j];
    }
    float U0[3], U1[3];
    for (int j = 0; j < 3; j++) {
        U0[j] = (T0[0] * Sg[0][j] + T0[1] * Sg[1][j]) + T0[2] * Sg[2][j];
        U1[j] = (T1[0] * Sg[0][j] + T1[1] * Sg[1][j]) + T1[2] * Sg[2][j];
    }
    float a = ((U0[0] * T0[0] + U0[1] * T0[1]) + U0[2] * T0[2]) + 0.3f;
    float b = (U0[0] * T1[0] + U0[1] * T1[1]) + U0[2] * T1[2];
    float cc = ((U1[0] * T1[0] + U1[1] * T1[1]) + U1[2] * T1[2]) + 0.3f;
    float det = a * cc - b * b;
    if (!(det > 0.0f)) return;
    float inv = 1.0f / det;
    float mid = 0.5f * (a + cc);
    float lam = mid + sqrtf(fmaxf(0.1f, mid * mid - det));
    float rad = ceilf(3.0f * sqrtf(lam));
    float u = (c->fx * tx) / tz + (c->cx - 0.5f);
    float v = (c->fy * ty) / tz + (c->cy - 0.5f);
    float x0 = fminf(fmaxf(floorf((u - rad) / 16.0f), 0.0f), (float)TX);
    float x1 = fminf(fmaxf(floorf(((u + rad) + 15.0f) / 16.0f), 0.0f), (float)TX);
    float y0 = fminf(fmaxf(floorf((v - rad) / 16.0f), 0.0f), (float)TY);
    float y1 = fminf(fmaxf(floorf(((v + rad) + 15.0f) / 16.0f), 0.0f), (float)TY);
    if (support_box) support_box_cut(a, cc, det, u, v, TX, TY, &x0, &x1, &y0, &y1);
    int ix0 = (int)x0, ix1 = (int)x1, iy0 = (int)y0, iy1 = (int)y1;
    if (ix1 <= ix0 || iy1 <= iy0) return;
    /* colour from SH in the viewing direction */
    float d0 = g[0] - c->cam_pos[0], d1 = g[1] - c->cam_pos[1], d2 = g[2] - c->cam_pos[2];
    float len = sqrtf((d0 * d0 + d1 * d1) + d2 * d2);
    or_sh_color_f32(g + 11, d0 / len, d1 / len, d2 / len, o->rgb);
    o->culled = 0;
    o->u = u; o->v = v; o->depth = tz;
    o->conic[0] = cc * inv; o->conic[1] = -b * inv; o->conic[2] = a * inv;
    o->opacity = op;
    o->rect[0] = ix0; o->rect[1] = iy0; o->rect[2] = ix1; o->rect[3] = iy1;
    o->tiles = (ix1 - ix0) * (iy1 - iy0);
    (void)W; (void)H;
}

typedef struct { uint32_t depth; uint32_t idx; } dk;

static int cmp_dk(const void* a, const void* b)
{
    const dk* x = a; const dk* y = b;
    if (x->depth != y->depth) return x->depth < y->depth ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* per tile: Gaussians whose rectangle covers the tile, in (depth, index)
 * order; per pixel: front-to-back blending until transmittance would drop
 * below 1e-4 */
static void splat(or_vm* vm, const or_camera* cams, int n_views, const uint8_t* tile_mask,
                  const float* const* gauss, int64_t n_render)
{
    int TX = vm->TX, TY = vm->TY, W = vm->W, H = vm->H;
    int64_t nt = (int64_t)n_views * TX * TY;
    free(vm->pp);
    vm->pp = malloc(sizeof(pp_t) * (size_t)(n_views * n_render > 0 ? n_views * n_render : 1));
    /* independent per Gaussian (and below per tile): OpenMP threads when built with them */
    for (int v = 0; v < n_views; v++) {
        #pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < n_render; r++)
            preprocess_one(gauss[r], &cams[v], W, H, TX, TY, vm->support_box, &vm->pp[v * n_render + r]);
    }
    /* bucket per tile */
    int64_t* cnt = calloc((size_t)nt + 1, sizeof(int64_t));
    for (int v = 0; v < n_views; v++)
        for (int64_t r = 0; r < n_render; r++) {
            pp_t* o = &vm->pp[v * n_render + r];
            if (o->culled) continue;
            for (int ty = o->rect[1]; ty < o->rect[3]; ty++)
                for (int tx = o->rect[0]; tx < o->rect[2]; tx++) {
                    int64_t t = (int64_t)v * TX * TY + ty * TX + tx;
                    if (tile_mask && !tile_mask[t]) continue;
                    cnt[t + 1]++;
                }
        }
    for (int64_t t = 0; t < nt; t++) cnt[t + 1] += cnt[t];
    int64_t np = cnt[nt];
    dk* lists = malloc(sizeof(dk) * (size_t)(np > 0 ? np : 1));
    int64_t* fill = malloc(sizeof(int64_t) * (size_t)(nt > 0 ? nt : 1));
    for (int64_t t = 0; t < nt; t++) fill[t] = cnt[t];
    for (int v = 0; v < n_views; v++)
        for (int64_t r = 0; r < n_render; r++) {
            pp_t* o = &vm->pp[v * n_render + r];
            if (o->culled) continue;
            for (int ty = o->rect[1]; ty < o->rect[3]; ty++)
                for (int tx = o->rect[0]; tx < o->rect[2]; tx++) {
                    int64_t t = (int64_t)v * TX * TY + ty * TX + tx;
                    if (tile_mask && !tile_mask[t]) continue;
                    lists[fill[t]].depth = fbits(o->depth);
                    lists[fill[t]].idx = (uint32_t)r;
                    fill[t]++;
                }
        }
    free(fill);
    free(vm->keys); free(vm->vals); free(vm->ranges);
    vm->n_pairs = np;
    vm->keys = malloc(sizeof(uint64_t) * (size_t)(np > 0 ? np : 1));
    vm->vals = malloc(sizeof(uint32_t) * (size_t)(np > 0 ? np : 1));
    vm->ranges = calloc((size_t)nt * 2, sizeof(uint32_t));
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; t++) {
        qsort(lists + cnt[t], (size_t)(cnt[t + 1] - cnt[t]), sizeof(dk), cmp_dk);
        for (int64_t k = cnt[t]; k < cnt[t + 1]; k++) {
            vm->keys[k] = ((uint64_t)t << 32) | lists[k].depth;
            vm->vals[k] = lists[k].idx;
        }
        vm->ranges[2 * t] = (uint32_t)cnt[t];
        vm->ranges[2 * t + 1] = (uint32_t)cnt[t + 1];
    }
    /* blend */
    free(vm->image); free(vm->final_T); free(vm->contrib); free(vm->visits);
    vm->image = calloc((size_t)n_views * W * H * 3, sizeof(float));
    vm->final_T = calloc((size_t)n_views * W * H, sizeof(float));
    vm->contrib = calloc((size_t)n_views * W * H, sizeof(int64_t));
    vm->visits = calloc((size_t)n_views * W * H, sizeof(int64_t));
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nt; t++) {
            int v = (int)(t / ((int64_t)TX * TY));
            int ty = (int)((t % ((int64_t)TX * TY)) / TX);
            int tx = (int)(t % TX);
            if (tile_mask && !tile_mask[t]) continue;
            for (int py = ty * 16; py < ty * 16 + 16 && py < H; py++)
                for (int px = tx * 16; px < tx * 16 + 16 && px < W; px++) {
                    float T = 1.0f, C[3] = {0.0f, 0.0f, 0.0f};
                    int64_t nb = 0, nvis = cnt[t + 1] - cnt[t];
                    for (int64_t k = cnt[t]; k < cnt[t + 1]; k++) {
                        pp_t* o = &vm->pp[v * n_render + vm->vals[k]];
                        float dx = o->u - (float)px, dy = o->v - (float)py;
                        float q = fmaf(o->conic[0] * dx, dx, (o->conic[2] * dy) * dy);
                        float power = fmaf(-0.5f, q, -((o->conic[1] * dx) * dy));
                        if (power > 0.0f) continue;
                        float alpha = fminf(0.99f, o->opacity * or_vm_exp(power));
                        if (alpha < 1.0f / 255.0f) continue;
                        float Tn = T * (1.0f - alpha);
                        if (Tn < 0.0001f) { nvis = k - cnt[t] + 1; break; }
                        float wgt = alpha * T;
                        for (int ch = 0; ch < 3; ch++) C[ch] = fmaf(o->rgb[ch], wgt, C[ch]);
                        T = Tn;
                        nb++;
                    }
                    int64_t pix = ((int64_t)v * H + py) * W + px;
                    for (int ch = 0; ch < 3; ch++) vm->image[pix * 3 + ch] = C[ch];
                    vm->final_T[pix] = T;
                    vm->contrib[pix] = nb;
                    vm->visits[pix] = nvis;
                }
        }
    free(lists); free(cnt);
}

/* ------------------------------------------------------------------------ */
or_vm* or_vm_create(const or_scene* s, int pool_pages, int copy_budget, int use_links,
                    int W, int H, int Wv, int Hv, float tau, float guard)
{
    if (!s || pool_pages <= 0 || W <= 0 || H <= 0 || Wv <= 0 || Hv <= 0) return NULL;
    or_vm* vm = calloc(1, sizeof(or_vm));
    vm->s = s; vm->S = pool_pages; vm->budget = copy_budget; vm->use_links = use_links;
    vm->W = W; vm->H = H; vm->Wv = Wv; vm->Hv = Hv; vm->tau = tau; vm->guard = guard;
    vm->tau_used = tau; vm->lod_step = LOD_STEP0; vm->lod_dir = 0; vm->lod_last_move = 0;
    vm->TX = (W + 15) / 16; vm->TY = (H + 15) / 16;
    vm->P = or_scene_P(s); vm->L = or_scene_L(s); vm->n_pg = or_scene_npg(s);
    vm->bytes_g = or_scene_format(s) == 1 ? 124 : 236;
    vm->slot_level = malloc((size_t)vm->S);
    memset(vm->slot_level, -1, (size_t)vm->S);
    vm->last_used = malloc(sizeof(int32_t) * (size_t)vm->S);
    vm->sub_vpage = malloc(sizeof(int32_t) * (size_t)vm->S * SUBS);
    vm->sub_last_used = malloc(sizeof(int32_t) * (size_t)vm->S * SUBS);
    for (int i = 0; i < vm->S; i++) vm->last_used[i] = -1;
    for (int i = 0; i < vm->S * SUBS; i++) { vm->sub_vpage[i] = -1; vm->sub_last_used[i] = -1; }
    vm->v2p = malloc(sizeof(int32_t) * (size_t)vm->n_pg * vm->L);
    for (int i = 0; i < vm->n_pg * vm->L; i++) vm->v2p[i] = -1;
    vm->req_direct = malloc(sizeof(uint32_t) * (size_t)vm->n_pg);
    vm->req_link = malloc(sizeof(uint32_t) * (size_t)vm->n_pg);
    vm->req_page = malloc(sizeof(int32_t) * (size_t)vm->n_pg);
    vm->req_level = malloc((size_t)vm->n_pg);
    vm->req_class = malloc((size_t)vm->n_pg);
    vm->req_depth = malloc(sizeof(uint32_t) * (size_t)vm->n_pg);
    vm->page_level = malloc((size_t)vm->n_pg);
    vm->rlevel = malloc((size_t)vm->n_pg);
    for (int p = 0; p < vm->n_pg; p++) vm->rlevel[p] = -1;
    vm->copy = malloc(sizeof(int64_t) * 3 * (size_t)vm->n_pg * vm->L);
    vm->copy_id = malloc(sizeof(int32_t) * 4 * (size_t)vm->n_pg * vm->L);
    vm->missing = malloc(sizeof(int32_t) * 2 * (size_t)vm->n_pg * vm->L);
    vm->rl = malloc(sizeof(rl_t) * (size_t)vm->n_pg);
    return vm;
}

void or_vm_set_bytes_per_gaussian(or_vm* vm, int b) { vm->bytes_g = b; }

void or_vm_free(or_vm* vm)
{
    if (!vm) return;
    free(vm->slot_level); free(vm->last_used); free(vm->sub_vpage); free(vm->sub_last_used); free(vm->v2p);
    free(vm->cand); free(vm->idbuf); free(vm->req_direct); free(vm->req_link);
    free(vm->req_page); free(vm->req_level); free(vm->req_class); free(vm->req_depth); free(vm->page_level);
    free(vm->rlevel);
    free(vm->copy); free(vm->copy_id); free(vm->missing); free(vm->rl);
    free(vm->pp); free(vm->keys); free(vm->vals); free(vm->ranges); free(vm->image); free(vm->final_T);
    free(vm->contrib); free(vm->visits);
    free(vm->pf_keys); free(vm->pf_x);
    free(vm);
}

static void build_render_list(or_vm* vm);

typedef struct { uint64_t key; int32_t page; } rq;

static int cmp_rq(const void* a, const void* b)
{
    const rq* x = a; const rq* y = b;
    return (x->key > y->key) - (x->key < y->key);
}

/* Level of detail of a page (Sec. 4.1 "Level of Detail"): the level follows
 * the nearest depth of the page, read as its projected radius in pixels
 * against halving thresholds: level l is the first with
 * fy * radius / depth > tau / 2^l, and pages at or below tau / 2^(L-2) take
 * the coarsest level L - 1. */
int or_lod_level(float fy, float radius, float depth, float tau, int L)
{
    float rpx = (fy * radius) / depth;
    float thr = tau;
    int lvl = 0;
    while (lvl < L - 1 && !(rpx > thr)) { lvl++; thr = thr * 0.5f; }
    return lvl;
}

/* Thresholds that follow memory use (Sec. 5.1.1, with Sec. 4.1 and Sec. 5.3):
 * the controller aims at 50-80 % of the pool.  Usage is the share of
 * physical pages the frame required; requests left missing for want of a
 * free pool entry count as over the band (those the copy budget defers do
 * not: they say nothing about memory use).  Over 80 % (or anything missing
 * for want of space) the transition distances
 * shrink: tau, the level-0 radius in pixels, is multiplied by 1 + step.
 * Under 50 % while some requested page is at a coarse level they grow:
 * tau is divided by 1 + step.  The step changes by 1 % of itself after each
 * move: up when the move repeats the direction of a move made at most
 * LOD_QUICK frames earlier, down when it reverses such a move.  The new tau
 * is used from the next frame on. */

static void lod_controller(float* tau, float* step, int* dir, int* last_move, int frame, int S, int req_slots,
                           int n_missing, int n_coarse)
{
    int d = 0;
    if (n_missing > 0 || (int64_t)req_slots * 5 > (int64_t)S * 4) d = 1;
    else if ((int64_t)req_slots * 2 < (int64_t)S && n_coarse > 0) d = -1;
    if (d == 0) return;
    float t = d > 0 ? *tau * (1.0f + *step) : *tau / (1.0f + *step);
    *tau = fminf(fmaxf(t, LOD_TAU_MIN), LOD_TAU_MAX);
    if (*dir != 0 && frame - *last_move <= LOD_QUICK)
        *step = *dir == d ? *step * 1.01f : *step * 0.99f;
    *dir = d;
    *last_move = frame;
}

static void lod_control(or_vm* vm)
{
    lod_controller(&vm->tau, &vm->lod_step, &vm->lod_dir, &vm->lod_last_move, vm->frame, vm->S, vm->req_slots,
                   vm->n_missing_cap, vm->n_coarse);
}

void or_lod_control_trace(int n, int S, float tau0, const int* req_slots, const int* n_missing,
                          const int* n_coarse, float* tau_out, float* step_out)
{
    float tau = tau0, step = LOD_STEP0;
    int dir = 0, last = 0;
    for (int f = 0; f < n; f++) {
        lod_controller(&tau, &step, &dir, &last, f, S, req_slots[f], n_missing[f], n_coarse[f]);
        tau_out[f] = tau;
        step_out[f] = step;
    }
}

/* visibility, requests and page table; brute_force selects the every-pixel raster */
int or_vm_visibility(or_vm* vm, const or_camera* cams, int n_views, int brute_force)
{
    int n_pg = vm->n_pg, Wv = vm->Wv, Hv = vm->Hv;
    vm->n_views = n_views;
    vm->pf_cams = cams;
    if (vm->pf_on) push_poses(vm, cams, n_views);
    free(vm->cand); free(vm->idbuf);
    vm->cand = calloc((size_t)n_views * n_pg, 1);
    vm->idbuf = malloc(sizeof(uint64_t) * (size_t)n_views * Wv * Hv);
    const float* sp = or_scene_spheres(vm->s);
    for (int v = 0; v < n_views; v++) {
        for (int p = 0; p < n_pg; p++)
            vm->cand[(size_t)v * n_pg + p] = (uint8_t)sphere_in_frustum(&cams[v], vm->W, vm->H, vm->guard, sp + 4 * p);
        idbuf_render(vm, &cams[v], vm->cand + (size_t)v * n_pg, vm->idbuf + (size_t)v * Wv * Hv, brute_force);
    }
    /* reduction: nearest depth per page, then links */
    for (int p = 0; p < n_pg; p++) { vm->req_direct[p] = NONE32; vm->req_link[p] = NONE32; }
    for (int64_t i = 0; i < (int64_t)n_views * Wv * Hv; i++) {
        uint64_t k = vm->idbuf[i];
        if (k == NONE64) continue;
        int32_t p = (int32_t)(k & 0xffffffffu) - 1;
        uint32_t d = (uint32_t)(k >> 32);
        if (d < vm->req_direct[p]) vm->req_direct[p] = d;
    }
    if (vm->use_links) {
        const int32_t* ls = or_scene_linkstart(vm->s);
        const int32_t* ld = or_scene_linkdst(vm->s);
        for (int q = 0; q < n_pg; q++) {
            if (vm->req_direct[q] == NONE32) continue;
            for (int32_t e = ls[q]; e < ls[q + 1]; e++)
                if (vm->req_direct[q] < vm->req_link[ld[e]]) vm->req_link[ld[e]] = vm->req_direct[q];
        }
    }
    /* LOD level per requested page and the request order (class, depth, page) */
    float fy = cams[0].fy;
    for (int v = 1; v < n_views; v++) fy = fmaxf(fy, cams[v].fy);
    rq* r = malloc(sizeof(rq) * (size_t)n_pg);
    int nr = 0;
    for (int p = 0; p < n_pg; p++) {
        uint32_t d = vm->req_direct[p] < vm->req_link[p] ? vm->req_direct[p] : vm->req_link[p];
        if (vm->force_all && d == NONE32) { d = 0x3f800000u; vm->req_direct[p] = d; }
        vm->page_level[p] = -1;
        if (d == NONE32) continue;
        uint32_t cls = vm->req_direct[p] != NONE32 ? 0u : 1u;
        int lvl = vm->L > 1 ? or_lod_level(fy, sp[4 * p + 3], bitsf(d), vm->tau, vm->L) : 0;
        vm->page_level[p] = (int8_t)lvl;
        r[nr].key = ((uint64_t)cls << 61) | ((uint64_t)d << 30) | (uint64_t)p;
        r[nr].page = p;
        nr++;
    }
    qsort(r, (size_t)nr, sizeof(rq), cmp_rq);
    vm->n_req = nr;
    for (int i = 0; i < nr; i++) {
        int32_t p = r[i].page;
        vm->req_page[i] = p;
        vm->req_level[i] = vm->page_level[p];
        vm->req_class[i] = (uint8_t)(r[i].key >> 61);
        vm->req_depth[i] = (uint32_t)((r[i].key >> 30) & 0x7fffffffu);
    }
    free(r);
    vm->n_coarse = 0;
    for (int p = 0; p < n_pg; p++) vm->n_coarse += vm->page_level[p] > 0;
    vm->tau_used = vm->tau;
    page_table(vm);
    build_render_list(vm);
    if (vm->adaptive && vm->L > 1) lod_control(vm);
    vm->frame++;
    return 0;
}

/* render list: resident required pages in page order (streaming: at the
 * level stage 1 found resident when the frame started) */
static void build_render_list(or_vm* vm)
{
    int n_pg = vm->n_pg;
    vm->n_rl = 0;
    vm->n_render = 0;
    for (int p = 0; p < n_pg; p++) {
        int l = vm->page_level[p];
        if (l < 0) continue;
        if (vm->async) l = vm->rlevel[p];
        if (l < 0) continue;
        int32_t e = vm->v2p[p * vm->L + l];
        if (e < 0) continue;
        rl_t* x = &vm->rl[vm->n_rl++];
        x->page = p; x->level = l; x->slot = e / SUBS; x->sub = e % SUBS;
        x->count = vm->P >> (3 * l);
        x->base = vm->n_render;
        vm->n_render += x->count;
    }
}

/* Drive the page table with an explicit request list (already in service
 * order); used to check the replacement rule on hand-worked traces. */
int or_vm_pagetable(or_vm* vm, int n, const int32_t* pages, const int8_t* levels)
{
    for (int p = 0; p < vm->n_pg; p++) vm->page_level[p] = -1;
    vm->n_req = n;
    for (int i = 0; i < n; i++) {
        vm->req_page[i] = pages[i];
        vm->req_level[i] = levels ? levels[i] : 0;
        vm->page_level[pages[i]] = vm->req_level[i];
    }
    page_table(vm);
    build_render_list(vm);
    vm->frame++;
    return 0;
}

void or_vm_set_force_all(or_vm* vm, int on) { vm->force_all = on; }

int or_vm_set_prefetch(or_vm* vm, int n_clusters, int hist_bins, float logit_threshold, int budget_pages,
                       const float* center, float extent)
{
    if (n_clusters < 1 || hist_bins < 1 || !(extent > 0.0f)) return -1;
    vm->pf_on = 1;
    vm->pf_K = n_clusters; vm->pf_H = hist_bins; vm->pf_thr = logit_threshold; vm->pf_budget = budget_pages;
    for (int a = 0; a < 3; a++) vm->pf_center[a] = center[a];
    vm->pf_extent = extent;
    vm->pf_n_hist = 0;
    free(vm->pf_keys); free(vm->pf_x);
    vm->pf_keys = malloc(sizeof(uint64_t) * (size_t)(vm->n_pg > 0 ? vm->n_pg : 1));
    vm->pf_x = calloc((size_t)OR_MAX_VIEWS * (28 + hist_bins), sizeof(float));
    return 0;
}

void or_vm_features(const or_vm* vm, int view, float* x) { features(vm, view, x); }

int or_vm_frame_prefetch(or_vm* vm, const or_camera* cams, int n_views, const float* logits,
                         const uint8_t* tile_mask)
{
    vm->pf_logits = logits;
    int r = or_vm_frame(vm, cams, n_views, tile_mask);
    vm->pf_logits = NULL;
    return r;
}

void or_vm_set_support_box(or_vm* vm, int on) { vm->support_box = on; }

void or_vm_set_async(or_vm* vm, int on) { vm->async = on; }

/* threads of the per-Gaussian and per-tile loops (1 = single-threaded;
 * returns the count in use, 1 when built without OpenMP) */
int or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

void or_vm_set_adaptive_lod(or_vm* vm, int on) { vm->adaptive = on; }

int or_vm_frame(or_vm* vm, const or_camera* cams, int n_views, const uint8_t* tile_mask)
{
    vm->last_full = 0;
    or_vm_visibility(vm, cams, n_views, 0);
    const float** g = malloc(sizeof(float*) * (size_t)(vm->n_render > 0 ? vm->n_render : 1));
    for (int i = 0; i < vm->n_rl; i++) {
        const float* a = or_scene_attr(vm->s, vm->rl[i].level);
        int64_t Pl = vm->rl[i].count;
        for (int64_t k = 0; k < Pl; k++)
            g[vm->rl[i].base + k] = a + ((int64_t)vm->rl[i].page * Pl + k) * OR_REC;
    }
    splat(vm, cams, n_views, tile_mask, g, vm->n_render);
    free(g);
    return 0;
}

int or_render_full(or_vm* vm, const or_camera* cams, int n_views, const uint8_t* tile_mask)
{
    int64_t n = (int64_t)vm->n_pg * vm->P;
    const float** g = malloc(sizeof(float*) * (size_t)n);
    const float* a = or_scene_attr(vm->s, 0);
    for (int64_t k = 0; k < n; k++) g[k] = a + k * OR_REC;
    vm->n_views = n_views;
    vm->n_render = n;
    vm->last_full = 1;
    splat(vm, cams, n_views, tile_mask, g, n);
    free(g);
    return 0;
}

/* ---- FP64 reference render of the current render set ----------------------
 * The last frame's render list, with the attributes of `src` (a scene of the
 * same pages: the half-precision scene gives the decoded half attributes, an
 * fp32 scene the original ones), splatted in double with libm exp: the same
 * steps as the float path (EWA with 0.3 dilation, 3-sigma tile rectangles,
 * SH colour, per-tile (depth, index) order, alpha = min(0.99, o e^power),
 * skip below 1/255, stop before T < 1e-4), no rounding to float anywhere.
 * image: [n_views][H][W][3] doubles. */
typedef struct { double u, v, depth, ca, cb, cc, o, rgb[3]; int x0, y0, x1, y1, ok; } ppd_t;

static void preprocess_d(const float* g, const or_camera* c, int W, int H, int TX, int TY, ppd_t* o)
{
    memset(o, 0, sizeof *o);
    double op = g[10];
    if (op == 0.0) return;
    const float* V = c->view;
    double t[3];
    for (int r = 0; r < 3; r++) t[r] = (double)V[4 * r] * g[0] + (double)V[4 * r + 1] * g[1] + (double)V[4 * r + 2] * g[2] + V[4 * r + 3];
    if (!(t[2] > c->znear)) return;
    double w = g[6], x = g[7], y = g[8], z = g[9];
    double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                      {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                      {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    double M[3][3], Sg[3][3];
    for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) M[i][j] = R[i][j] * g[3 + j];
    for (int i = 0; i < 3; i++) for (int k = 0; k < 3; k++) Sg[i][k] = M[i][0] * M[k][0] + M[i][1] * M[k][1] + M[i][2] * M[k][2];
    double limx = 1.3 * (0.5 * W / c->fx), limy = 1.3 * (0.5 * H / c->fy);
    double cxz = fmin(limx, fmax(-limx, t[0] / t[2])) * t[2], cyz = fmin(limy, fmax(-limy, t[1] / t[2])) * t[2];
    double j00 = c->fx / t[2], j02 = -(c->fx * cxz) / (t[2] * t[2]);
    double j11 = c->fy / t[2], j12 = -(c->fy * cyz) / (t[2] * t[2]);
    double T0[3], T1[3], U0[3], U1[3];
    for (int j = 0; j < 3; j++) { T0[j] = j00 * V[j] + j02 * V[8 + j]; T1[j] = j11 * V[4 + j] + j12 * V[8 + j]; }
    for (int j = 0; j < 3; j++) {
        U0[j] = T0[0] * Sg[0][j] + T0[1] * Sg[1][j] + T0[2] * Sg[2][j];
        U1[j] = T1[0] * Sg[0][j] + T1[1] * Sg[1][j] + T1[2] * Sg[2][j];
    }
    double a = U0[0] * T0[0] + U0[1] * T0[1] + U0[2] * T0[2] + 0.3;
    double b = U0[0] * T1[0] + U0[1] * T1[1] + U0[2] * T1[2];
    double cc = U1[0] * T1[0] + U1[1] * T1[1] + U1[2] * T1[2] + 0.3;
    double det = a * cc - b * b;
    if (!(det > 0.0)) return;
    double mid = 0.5 * (a + cc), lam = mid + sqrt(fmax(0.1, mid * mid - det));
    double rad = ceil(3.0 * sqrt(lam));
    double u = c->fx * t[0] / t[2] + (c->cx - 0.5), v = c->fy * t[1] / t[2] + (c->cy - 0.5);
    int x0 = (int)fmin(fmax(floor((u - rad) / 16.0), 0.0), TX), x1 = (int)fmin(fmax(floor((u + rad + 15.0) / 16.0), 0.0), TX);
    int y0 = (int)fmin(fmax(floor((v - rad) / 16.0), 0.0), TY), y1 = (int)fmin(fmax(floor((v + rad + 15.0) / 16.0), 0.0), TY);
    if (x1 <= x0 || y1 <= y0) return;
    double d0 = g[0] - c->cam_pos[0], d1 = g[1] - c->cam_pos[1], d2 = g[2] - c->cam_pos[2];
    double len = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    for (int ch = 0; ch < 3; ch++) {
        double acc = 0.0;
        for (int k = 0; k < 16; k++) acc += or_sh_basis(k, d0 / len, d1 / len, d2 / len) * g[11 + 3 * k + ch];
        acc += 0.5;
        o->rgb[ch] = acc > 0.0 ? acc : 0.0;
    }
    o->u = u; o->v = v; o->depth = t[2];
    o->ca = cc / det; o->cb = -b / det; o->cc = a / det; o->o = op;
    o->x0 = x0; o->y0 = y0; o->x1 = x1; o->y1 = y1; o->ok = 1;
}

typedef struct { double depth; int64_t idx; } dd_t;

static int cmp_dd(const void* x, const void* y)
{
    const dd_t* a = x; const dd_t* b = y;
    if (a->depth != b->depth) return a->depth < b->depth ? -1 : 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

int or_vm_render_fp64(const or_vm* vm, const or_scene* src, const or_camera* cams, int n_views, double* image)
{
    int W = vm->W, H = vm->H, TX = vm->TX, TY = vm->TY;
    int64_t n = vm->n_render;
    const float** g = malloc(sizeof(float*) * (size_t)(n > 0 ? n : 1));
    if (vm->last_full) {
        const float* a = or_scene_attr(src, 0);
        for (int64_t k = 0; k < n; k++) g[k] = a + k * OR_REC;
    } else {
        for (int i = 0; i < vm->n_rl; i++) {
            const float* a = or_scene_attr(src, vm->rl[i].level);
            int64_t Pl = vm->rl[i].count;
            for (int64_t k = 0; k < Pl; k++) g[vm->rl[i].base + k] = a + ((int64_t)vm->rl[i].page * Pl + k) * OR_REC;
        }
    }
    ppd_t* pp = malloc(sizeof(ppd_t) * (size_t)(n > 0 ? n : 1));
    dd_t* list = malloc(sizeof(dd_t) * (size_t)(n > 0 ? n : 1));
    for (int v = 0; v < n_views; v++) {
        for (int64_t r = 0; r < n; r++) preprocess_d(g[r], &cams[v], W, H, TX, TY, &pp[r]);
        for (int ty = 0; ty < TY; ty++)
            for (int tx = 0; tx < TX; tx++) {
                int64_t m = 0;
                for (int64_t r = 0; r < n; r++)
                    if (pp[r].ok && pp[r].x0 <= tx && tx < pp[r].x1 && pp[r].y0 <= ty && ty < pp[r].y1) {
                        list[m].depth = pp[r].depth; list[m].idx = r; m++;
                    }
                qsort(list, (size_t)m, sizeof(dd_t), cmp_dd);
                for (int py = ty * 16; py < ty * 16 + 16 && py < H; py++)
                    for (int px = tx * 16; px < tx * 16 + 16 && px < W; px++) {
                        double T = 1.0, C[3] = {0.0, 0.0, 0.0};
                        for (int64_t q = 0; q < m; q++) {
                            const ppd_t* o = &pp[list[q].idx];
                            double dx = o->u - px, dy = o->v - py;
                            double power = -0.5 * (o->ca * dx * dx + o->cc * dy * dy) - o->cb * dx * dy;
                            if (power > 0.0) continue;
                            double alpha = fmin(0.99, o->o * exp(power));
                            if (alpha < 1.0 / 255.0) continue;
                            double Tn = T * (1.0 - alpha);
                            if (Tn < 1e-4) break;
                            for (int ch = 0; ch < 3; ch++) C[ch] += o->rgb[ch] * alpha * T;
                            T = Tn;
                        }
                        double* out = image + (((size_t)v * H + py) * W + px) * 3;
                        for (int ch = 0; ch < 3; ch++) out[ch] = C[ch];
                    }
            }
    }
    free(list); free(pp); free(g);
    return 0;
}

static int64_t put(void* dst, int64_t cap, const void* src, int64_t bytes)
{
    if (dst && cap >= bytes && bytes > 0) memcpy(dst, src, (size_t)bytes);
    return bytes;
}

int64_t or_vm_get(const or_vm* vm, const char* name, void* dst, int64_t cap)
{
    int64_t nv = vm->n_views;
    int64_t npp = nv * vm->n_render;
    if (!strcmp(name, "frame")) { int64_t v = vm->frame; return put(dst, cap, &v, 8); }
    if (!strcmp(name, "cand")) return put(dst, cap, vm->cand, nv * vm->n_pg);
    if (!strcmp(name, "idbuf")) return put(dst, cap, vm->idbuf, 8 * nv * vm->Wv * vm->Hv);
    if (!strcmp(name, "req_direct")) return put(dst, cap, vm->req_direct, 4 * (int64_t)vm->n_pg);
    if (!strcmp(name, "req_link")) return put(dst, cap, vm->req_link, 4 * (int64_t)vm->n_pg);
    if (!strcmp(name, "page_level")) return put(dst, cap, vm->page_level, vm->n_pg);
    if (!strcmp(name, "req_page")) return put(dst, cap, vm->req_page, 4 * (int64_t)vm->n_req);
    if (!strcmp(name, "req_level")) return put(dst, cap, vm->req_level, vm->n_req);
    if (!strcmp(name, "req_class")) return put(dst, cap, vm->req_class, vm->n_req);
    if (!strcmp(name, "slot_level")) return put(dst, cap, vm->slot_level, vm->S);
    if (!strcmp(name, "last_used")) return put(dst, cap, vm->last_used, 4 * (int64_t)vm->S);
    if (!strcmp(name, "sub_vpage")) return put(dst, cap, vm->sub_vpage, 4 * (int64_t)vm->S * SUBS);
    if (!strcmp(name, "sub_last_used")) return put(dst, cap, vm->sub_last_used, 4 * (int64_t)vm->S * SUBS);
    if (!strcmp(name, "v2p")) return put(dst, cap, vm->v2p, 4 * (int64_t)vm->n_pg * vm->L);
    if (!strcmp(name, "copies")) return put(dst, cap, vm->copy, 24 * (int64_t)vm->n_copy);
    if (!strcmp(name, "copy_id")) return put(dst, cap, vm->copy_id, 16 * (int64_t)vm->n_copy);
    if (!strcmp(name, "missing")) return put(dst, cap, vm->missing, 8 * (int64_t)vm->n_missing);
    if (!strcmp(name, "lod")) {
        float f[2] = {vm->tau_used, vm->tau};
        return put(dst, cap, f, sizeof f);
    }
    if (!strcmp(name, "pf_keys")) return put(dst, cap, vm->pf_keys, 8 * (int64_t)vm->n_pf_req);
    if (!strcmp(name, "pf_x")) return put(dst, cap, vm->pf_x, 4 * (int64_t)vm->n_views * (28 + vm->pf_H));
    if (!strcmp(name, "pf_counts")) {
        int64_t c[3] = {vm->n_pf_req, vm->n_prefetch, vm->n_copy_demand};
        return put(dst, cap, c, sizeof c);
    }
    if (!strcmp(name, "counts")) {
        int64_t c[9] = {vm->n_req, vm->hits, vm->misses, vm->evictions, vm->n_copy, vm->n_missing, vm->n_rl, vm->n_render,
                        vm->n_fallback};
        return put(dst, cap, c, sizeof c);
    }
    if (!strcmp(name, "render_list")) {
        int64_t bytes = 24 * (int64_t)vm->n_rl;
        if (dst && cap >= bytes)
            for (int i = 0; i < vm->n_rl; i++) {
                int32_t* o = (int32_t*)dst + 6 * i;
                o[0] = vm->rl[i].page; o[1] = vm->rl[i].level; o[2] = vm->rl[i].slot;
                o[3] = vm->rl[i].sub; o[4] = vm->rl[i].count; o[5] = (int32_t)vm->rl[i].base;
            }
        return bytes;
    }
    if (!strcmp(name, "pp_float")) {         /* [n][10] u v depth conic3 opacity rgb3 */
        int64_t bytes = 40 * npp;
        if (dst && cap >= bytes)
            for (int64_t i = 0; i < npp; i++) {
                const pp_t* o = &vm->pp[i];
                float* f = (float*)dst + 10 * i;
                f[0] = o->u; f[1] = o->v; f[2] = o->depth;
                f[3] = o->conic[0]; f[4] = o->conic[1]; f[5] = o->conic[2];
                f[6] = o->opacity; f[7] = o->rgb[0]; f[8] = o->rgb[1]; f[9] = o->rgb[2];
            }
        return bytes;
    }
    if (!strcmp(name, "pp_int")) {           /* [n][6] culled x0 y0 x1 y1 tiles */
        int64_t bytes = 24 * npp;
        if (dst && cap >= bytes)
            for (int64_t i = 0; i < npp; i++) {
                const pp_t* o = &vm->pp[i];
                int32_t* q = (int32_t*)dst + 6 * i;
                q[0] = o->culled; q[1] = o->rect[0]; q[2] = o->rect[1]; q[3] = o->rect[2]; q[4] = o->rect[3]; q[5] = o->tiles;
            }
        return bytes;
    }
    if (!strcmp(name, "n_pairs")) { int64_t v = vm->n_pairs; return put(dst, cap, &v, 8); }
    if (!strcmp(name, "keys")) return put(dst, cap, vm->keys, 8 * vm->n_pairs);
    if (!strcmp(name, "vals")) return put(dst, cap, vm->vals, 4 * vm->n_pairs);
    if (!strcmp(name, "ranges")) return put(dst, cap, vm->ranges, 8 * nv * vm->TX * vm->TY);
    if (!strcmp(name, "image")) return put(dst, cap, vm->image, 12 * nv * vm->W * vm->H);
    if (!strcmp(name, "final_T")) return put(dst, cap, vm->final_T, 4 * nv * vm->W * vm->H);
    if (!strcmp(name, "contrib")) return put(dst, cap, vm->contrib, 8 * nv * vm->W * vm->H);
    if (!strcmp(name, "visits")) return put(dst, cap, vm->visits, 8 * nv * vm->W * vm->H);
    return -1;
}
