// api.cpp -- the C ABI of include/vm3dgs.h: context, frame scheduler, copies.
//
// One frame (Sec. 4 of the paper):
//   render stream: camera upload -> one launch of the frame's clears ->
//                  visibility kernels -> page table kernel(s) -> readback of
//                  the counters
//   host:          waits for the counters (the one place the host waits on
//                  the device before splatting, like the paper's fence
//                  before its page-table update, Sec. 5.1.3); the copy list
//                  stays on the device
//   render stream: the GPU reads the missed pages from the pinned page-major
//                  store into their pool slots (k_copy_pages), then
//                  preprocess -> depth sort -> scan of tile counts -> pair
//                  emission -> tile sort -> ranges -> blend into the
//                  caller's image, with the pair count kept on the device
//                  and grids bounded by the last frame's count
//   copy stream:   prefetch copies, which the next frame waits for
//   end:           one readback launch (pair count, request keys and levels,
//                  missing list, flags); a frame with more pairs than its
//                  bounds is splatted again with larger ones
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "vm3dgs_impl.h"

namespace vm {
bool pagetable_l1_fits(int n_pg, int S);
}

using namespace vm;

// memory-use controller of the LOD thresholds (lod_control below)
constexpr float kLodStep0 = 0.125f, kLodTauMin = 0.0078125f, kLodTauMax = 65536.0f;
constexpr int kLodQuick = 4;

struct vm3dgs {
    vm3dgs_options opt{};
    PagedScene ps;
    int S = 0, L = 1, P = 0, n_pg = 0, TX = 0, TY = 0;
    hipStream_t sr = nullptr, sc = nullptr;
    bool own_sr = false, own_sc = false;
    hipStream_t sb = nullptr;   // the blend's second stream, forked from sr and joined back
    hipEvent_t ev_bfork = nullptr, ev_bjoin = nullptr;
    hipEvent_t ev_copy = nullptr;
    hipEvent_t ev_sync = nullptr;   // host waits inside a frame spin on this event
    hipEvent_t ev[8] = {};
    // scene on the device
    float4* d_sph = nullptr; float4* d_clo = nullptr; float4* d_chi = nullptr;
    int32_t* d_ls = nullptr; int32_t* d_ld = nullptr;
    uint8_t* d_pool = nullptr; uint8_t* d_full = nullptr; uint8_t* h_store = nullptr;
    const uint8_t* h_store_dev = nullptr;   // the pinned store as the GPU addresses it
    uint32_t* d_cp_err = nullptr;           // sticky flag: a copy command out of bounds
    unsigned long long* d_pf_bytes = nullptr;   // bytes of prefetch copies (copy stream)
    int64_t* d_level_base = nullptr;
    CamK* d_cams = nullptr; CamK* h_cams = nullptr;
    // visibility
    uint8_t* d_cand = nullptr; float4* d_rays = nullptr; unsigned long long* d_idbuf = nullptr;
    int4* d_crect = nullptr; uint32_t* d_carea = nullptr; uint32_t* d_coffs = nullptr;
    uint32_t* d_rd = nullptr; uint32_t* d_rl = nullptr; int8_t* d_plevel = nullptr; uint64_t* d_keys = nullptr;
    uint32_t* d_ctr = nullptr; uint32_t* h_ctr = nullptr;
    // page table
    int8_t* d_slot_level = nullptr; int32_t* d_last_used = nullptr; int32_t* d_sub_vpage = nullptr;
    int32_t* d_sub_lu = nullptr; int32_t* d_v2p = nullptr; uint8_t* d_req_sub = nullptr; uint8_t* d_slot_req = nullptr;
    uint32_t* d_miss = nullptr;
    // copy commands, two lists used in turn by consecutive frames: the copies
    // a frame leaves running on the copy stream read theirs while the next
    // frame's page table writes the other
    CopyCmd* d_copies_buf[2] = {nullptr, nullptr}; int cpb = 0;
    CopyCmd* d_copies = nullptr; CopyCmd* h_copies = nullptr; int32_t* d_copy_id = nullptr;
    int32_t* d_missing = nullptr; int32_t* h_missing = nullptr;
    uint64_t* h_keys = nullptr;
    // several LOD levels: candidate lists and request order of the multi-kernel page table
    uint64_t* d_lkeys_alt = nullptr; uint64_t* d_wkeys[2] = {nullptr, nullptr};
    uint64_t* d_ck[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
    uint32_t* d_lflag = nullptr; uint32_t* d_lpos = nullptr; int32_t* d_fresh = nullptr;
    uint32_t* d_lflag2 = nullptr; uint32_t* d_lpos2 = nullptr; int8_t* d_rlevel = nullptr;   // streaming
    // streaming (VM3DGS_FLAG_ASYNC_MISSES): the demand copies of the last frame,
    // on the copy stream, which the next frame waits for before it touches the pool
    hipEvent_t ev_async = nullptr;
    bool async_pending = false;
    int8_t* d_lvl_out = nullptr; int8_t* h_lvl = nullptr;
    RenderEntry* d_rlist = nullptr; RenderEntry* d_rlist_full = nullptr;
    // splat
    uint64_t cap_render = 0;
    float4* d_xy = nullptr; float4* d_conic = nullptr; float4* d_rgb = nullptr;   // xy: centre, support half-widths
    uint32_t* d_depth = nullptr; uint2* d_rect = nullptr; uint32_t* d_tiles = nullptr;
    uint32_t* d_dkey[2] = {nullptr, nullptr}; uint32_t* d_dval[2] = {nullptr, nullptr};
    uint32_t* d_offs = nullptr;
    uint64_t cap_pairs = 0;
    // pairs the launches after the scan cover (their grids), per kind of
    // frame: 1.5 times the last count; a frame with more is splatted again
    uint32_t pair_grid[2] = {1u << 20, 1u << 20};   // VM frames, full-scene renders
    int pair_kind = 0;                              // of the splat in flight
    uint32_t pair_cover = 0;                        // its bound
    uint32_t* d_pkey[2] = {nullptr, nullptr}; uint32_t* d_pval[2] = {nullptr, nullptr};
    uint32_t* d_emit_start = nullptr;
    // vm3dgs_frame_noalloc: this device's fixed scratch, and whether the call
    // in flight splats into it; the sorted pairs of the last splat
    uint8_t* d_noalloc = nullptr;
    bool noalloc = false;
    const uint32_t* last_pk = nullptr; const uint32_t* last_pv = nullptr;
    uint2* d_ranges = nullptr; uint32_t* d_tile_order = nullptr;
    // zero block: counters | look-back error flag | tickets | histograms (cleared per frame)
    uint32_t* d_zero = nullptr;
    uint64_t* d_status = nullptr; size_t status_words = 0;
    SortWork sw;
    uint32_t* d_total = nullptr; uint32_t* h_total = nullptr;
    // device addresses of the pinned host buffers that readbacks write, and
    // the readbacks queued since the last wait
    void* hd_total = nullptr; void* hd_ctr = nullptr; void* hd_keys = nullptr; void* hd_lvl = nullptr;
    void* hd_missing = nullptr;
    ReadSegs rb;
    uint2* d_bstats = nullptr; uint2* h_bstats = nullptr;
    int frame = 0;
    bool multi = false;   // multi-kernel page table (several levels or a large table)
    // LOD threshold control from memory use (VM3DGS_FLAG_ADAPTIVE_LOD)
    float lod_tau = 0.0f, lod_step = kLodStep0;
    int lod_dir = 0, lod_last_move = 0;
    // learned prefetch: configuration, pose history (host), features, proposals
    bool pf_on = false, pf_pending = false;
    vm3dgs_prefetch_opts pf{};
    vm3dgs_mlp* pf_net = nullptr;
    int pf_n_hist = 0;
    std::vector<float> pf_pose;                 // [max_views][4][7]
    float* d_pf_x = nullptr; float* h_pf_x = nullptr;   // [max_views][28 + H]
    uint64_t* d_pf_keys[2] = {nullptr, nullptr}; uint64_t* d_pf_idle[2] = {nullptr, nullptr};
    const uint64_t* pf_sorted = nullptr;
    hipEvent_t ev_pf = nullptr;
    uint32_t last_n_pfreq = 0, last_n_pf = 0;
    // last frame, for vm3dgs_debug_get and the frame output
    uint32_t last_views = 0, last_n_render = 0, last_n_pairs = 0, last_n_copy = 0, last_n_missing = 0;
    uint32_t last_n_xlong = 0xffffffffu;   // longest tiles of the last splat (none yet: room for all)
    uint32_t last_n_req = 0, last_n_rl = 0;
    // the last frame's request and level-1/2 candidate counts (all ones: none yet)
    uint32_t hint_req = ~0u, hint_cand[3] = {~0u, ~0u, ~0u};
    int last_pbuf = 0, last_dbuf = 0;
    std::vector<int32_t> out_req, out_missing;
    std::vector<int8_t> out_req_level;
    std::string err;
    bool poisoned = false;
};

namespace {

thread_local std::string g_create_error;

struct HipError {
    hipError_t e;
    const char* what;
    int line;
};

#define HIPCHK(x)                                        \
    do {                                                 \
        hipError_t e_ = (x);                             \
        if (e_ != hipSuccess) throw HipError{e_, #x, __LINE__}; \
    } while (0)

template <class T>
void dalloc(T** p, size_t count) {
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, sizeof(T) * count);
    if (e != hipSuccess) throw HipError{e, "hipMalloc", __LINE__};
}

template <class T>
void dfree(T*& p) {
    if (p) hipFree((void*)p);
    p = nullptr;
}

template <class T>
void halloc(T** p, size_t count) {
    if (count == 0) count = 1;
    hipError_t e = hipHostMalloc((void**)p, sizeof(T) * count, hipHostMallocDefault);
    if (e != hipSuccess) throw HipError{e, "hipHostMalloc", __LINE__};
}

template <class T>
void hfree(T*& p) {
    if (p) hipHostFree((void*)p);
    p = nullptr;
}

int bits_for(uint64_t n) {
    int b = 0;
    while ((1ull << b) < n) ++b;
    return b;
}

void to_camk(const vm3dgs_camera& c, CamK& k) {
    for (int i = 0; i < 12; ++i) k.V[i] = c.view[i];
    for (int i = 0; i < 3; ++i) k.pos[i] = c.cam_pos[i];
    k.fx = c.fx; k.fy = c.fy; k.cx = c.cx; k.cy = c.cy; k.znear = c.znear;
}

void free_all(vm3dgs* c) {
    if (c->sr) hipStreamSynchronize(c->sr);
    if (c->sc) hipStreamSynchronize(c->sc);
    dfree(c->d_sph); dfree(c->d_clo); dfree(c->d_chi); dfree(c->d_ls); dfree(c->d_ld);
    dfree(c->d_pool); dfree(c->d_full); hfree(c->h_store); dfree(c->d_level_base);
    dfree(c->d_cp_err); dfree(c->d_pf_bytes);
    dfree(c->d_cams); hfree(c->h_cams);
    dfree(c->d_cand); dfree(c->d_rays); dfree(c->d_idbuf);
    dfree(c->d_crect); dfree(c->d_carea); dfree(c->d_coffs); dfree(c->d_rd); dfree(c->d_rl); dfree(c->d_plevel);
    dfree(c->d_keys); c->d_ctr = nullptr; hfree(c->h_ctr);
    dfree(c->d_slot_level); dfree(c->d_last_used); dfree(c->d_sub_vpage); dfree(c->d_sub_lu); dfree(c->d_v2p);
    dfree(c->d_req_sub); dfree(c->d_slot_req); dfree(c->d_miss);
    dfree(c->d_copies_buf[0]); dfree(c->d_copies_buf[1]); c->d_copies = nullptr; hfree(c->h_copies); dfree(c->d_copy_id); dfree(c->d_missing); hfree(c->h_missing);
    hfree(c->h_keys);
    dfree(c->d_lkeys_alt); dfree(c->d_wkeys[0]); dfree(c->d_wkeys[1]);
    for (auto& q : c->d_ck) { dfree(q[0]); dfree(q[1]); }
    dfree(c->d_lflag); dfree(c->d_lpos); dfree(c->d_fresh);
    dfree(c->d_lflag2); dfree(c->d_lpos2); dfree(c->d_rlevel);
    if (c->ev_async) hipEventDestroy(c->ev_async); dfree(c->d_lvl_out); hfree(c->h_lvl);
    dfree(c->d_rlist); dfree(c->d_rlist_full);
    dfree(c->d_xy); dfree(c->d_conic); dfree(c->d_rgb); dfree(c->d_depth); dfree(c->d_rect); dfree(c->d_tiles);
    for (int i = 0; i < 2; ++i) { dfree(c->d_dkey[i]); dfree(c->d_dval[i]); dfree(c->d_pkey[i]); dfree(c->d_pval[i]); }
    dfree(c->d_emit_start);
    dfree(c->d_offs); dfree(c->d_ranges); dfree(c->d_tile_order); dfree(c->d_total); hfree(c->h_total);
    dfree(c->d_zero); dfree(c->d_status); dfree(c->d_bstats); hfree(c->h_bstats);
    if (c->ev_copy) hipEventDestroy(c->ev_copy);
    if (c->ev_sync) hipEventDestroy(c->ev_sync);
    if (c->ev_pf) hipEventDestroy(c->ev_pf);
    dfree(c->d_pf_x); hfree(c->h_pf_x);
    for (int i = 0; i < 2; ++i) { dfree(c->d_pf_keys[i]); dfree(c->d_pf_idle[i]); }
    for (auto& e : c->ev)
        if (e) hipEventDestroy(e);
    if (c->own_sr && c->sr) hipStreamDestroy(c->sr);
    if (c->own_sc && c->sc) hipStreamDestroy(c->sc);
    if (c->sb) hipStreamDestroy(c->sb);
    if (c->ev_bfork) hipEventDestroy(c->ev_bfork);
    if (c->ev_bjoin) hipEventDestroy(c->ev_bjoin);
}

constexpr int ZB_CTR = 0, ZB_ERR = C_NCOUNTERS, ZB_BYTES = ZB_ERR + 2, ZB_TICKETS = ZB_ERR + 16,
              ZB_HIST = ZB_TICKETS + SortWork::kMaxTickets, ZB_WORDS = ZB_HIST + 256 * SortWork::kMaxHist;

void ensure_status(vm3dgs* c) {
    const size_t need = lb_status_words(std::max({c->cap_pairs, c->cap_render, (uint64_t)c->S * SUBS,
                                                  (uint64_t)c->n_pg}));
    if (need > c->status_words) {
        dfree(c->d_status);
        dalloc(&c->d_status, need);
        HIPCHK(hipMemset(c->d_status, 0, sizeof(uint64_t) * need));
        c->status_words = need;
        c->sw.status = c->d_status;
    }
}

// Wait, inside a frame, for the render stream to reach this point: a spin on
// an event (the frame's readbacks are a few bytes and the host has nothing
// else to do; a sleeping wait adds its wake-up time to every frame).
// device address of pinned host memory
void* host_dev(void* h) {
    void* d = nullptr;
    HIPCHK(hipHostGetDevicePointer(&d, h, 0));
    return d;
}

// queue a readback of bytes at src into pinned host memory (dst: its device
// address); queued readbacks run as one launch at the next flush
void rb_add(vm3dgs* c, const void* src, void* dst, uint64_t bytes) {
    if (bytes == 0) return;
    if (c->rb.n >= ReadSegs::kMax || bytes > 0xffffffffull) throw std::length_error("readback segments exhausted");
    c->rb.seg[c->rb.n++] = ReadSeg{src, dst, (uint32_t)bytes};
}

void rb_flush(vm3dgs* c) {
    if (c->rb.n == 0) return;
    launch_readback(c->sr, c->rb);
    c->rb.n = 0;
    HIPCHK(hipGetLastError());
}

// the queued readbacks, then ev_sync on the render stream after them
void mark_wait(vm3dgs* c) {
    rb_flush(c);
    HIPCHK(hipEventRecord(c->ev_sync, c->sr));
}

// the host waits for ev_sync by spinning: a sleeping wait adds its wake-up
// time to every frame
void spin_on_mark(vm3dgs* c) {
    hipError_t e;
    while ((e = hipEventQuery(c->ev_sync)) == hipErrorNotReady) {
    }
    if (e != hipSuccess) throw HipError{e, "hipEventQuery", __LINE__};
}

// waits for the render stream (queued readbacks first)
void spin_wait(vm3dgs* c) {
    mark_wait(c);
    spin_on_mark(c);
}

// start of a frame's device work: clear counters, tickets and histograms
void begin_work(vm3dgs* c) {
    launch_fill_u32(c->sr, c->d_zero, ZB_WORDS, 0u);
    c->sw.reset();
    c->rb.n = 0;
}


void ensure_pairs(vm3dgs* c, uint64_t n) {
    if (n <= c->cap_pairs) return;
    HIPCHK(hipStreamSynchronize(c->sr));
    const uint64_t cap = std::max<uint64_t>(n + n / 4, 1u << 20);
    for (int i = 0; i < 2; ++i) {
        dfree(c->d_pkey[i]); dfree(c->d_pval[i]);
        dalloc(&c->d_pkey[i], cap);
        dalloc(&c->d_pval[i], cap);
    }
    dfree(c->d_emit_start);
    dalloc(&c->d_emit_start, cap / EMIT_SPAN + 2);

    c->cap_pairs = cap;
    ensure_status(c);
}

// pair buffers of one splat: the context's own, or the fixed scratch of
// vm3dgs_frame_noalloc (status words, keys, values, emission block starts,
// each at a 256-byte boundary)
struct PairBufs {
    uint32_t* key[2]; uint32_t* val[2]; uint32_t* emit_start; uint64_t* status;
    uint64_t cap;
};

PairBufs noalloc_bufs(uint8_t* base, uint64_t* end_bytes = nullptr) {
    PairBufs b{};
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        uint8_t* p = base + off;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    b.status = (uint64_t*)take(8 * (uint64_t)lb_status_words(kNoallocPairs));
    for (int i = 0; i < 2; ++i) b.key[i] = (uint32_t*)take(4 * kNoallocPairs);
    for (int i = 0; i < 2; ++i) b.val[i] = (uint32_t*)take(4 * kNoallocPairs);
    b.emit_start = (uint32_t*)take(4 * (kNoallocPairs / EMIT_SPAN + 2));
    b.cap = kNoallocPairs;
    if (end_bytes) *end_bytes = off;
    return b;
}

// a frame of vm3dgs_frame_noalloc with more pairs than the fixed scratch holds
struct NoallocCapacity {
    uint32_t pairs;
};

SplatArgs splat_args(const vm3dgs* c, const RenderEntry* rl, uint32_t n_rl, const uint8_t* pool, uint32_t n_render,
                     uint32_t n_views) {
    SplatArgs a{};
    a.rl = rl; a.n_rl = (int)n_rl; a.pool = pool; a.P = c->P; a.fmt = c->ps.fmt;
    a.cams = c->d_cams; a.n_views = (int)n_views; a.W = (int)c->opt.img_w; a.H = (int)c->opt.img_h;
    a.TX = c->TX; a.TY = c->TY; a.n_render = n_render;
    a.sigma3_tiles = (c->opt.flags & VM3DGS_FLAG_SIGMA3_TILES) ? 1 : 0;
    a.xy = c->d_xy; a.conic = c->d_conic; a.rgb = c->d_rgb; a.depth = c->d_depth; a.rect = c->d_rect;
    a.tiles = c->d_tiles; a.dkey = c->d_dkey[0]; a.dval = c->d_dval[0];
    return a;
}

void splat_sorted(vm3dgs* c, uint32_t n_render, uint32_t n_views, float* image, vm3dgs_stats* st);

// the render half of a frame: preprocess .. blend for n_render Gaussians per view
void splat(vm3dgs* c, const RenderEntry* rl, uint32_t n_rl, const uint8_t* pool, uint32_t n_render, uint32_t n_views,
           float* image, vm3dgs_stats* st) {
    HIPCHK(hipEventRecord(c->ev[3], c->sr));
    launch_preprocess(c->sr, splat_args(c, rl, n_rl, pool, n_render, n_views));
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(c->ev[4], c->sr));
    splat_sorted(c, n_render, n_views, image, st);
}

// splat after the preprocess: depth sort .. blend
void splat_sorted(vm3dgs* c, uint32_t n_render, uint32_t n_views, float* image, vm3dgs_stats* st) {
    const uint64_t n_total = (uint64_t)n_render * n_views;
    hipEvent_t* ev = c->ev;
    // depth order of the render set (culled entries carry all-ones keys and sort last)
    const int db = onesweep_u32(c->sr, c->sw, c->d_dkey, c->d_dval, (uint32_t)n_total, 0, 32);
    scan_lb_gather(c->sr, c->sw, c->d_tiles, c->d_dval[db], n_total, c->d_offs, c->d_total);
    // the pair count stays on the device: emission, tile sort and ranges read
    // it there, with grids sized for a bound on it; the host checks the count
    // against the bound once the frame is done (splat_pairs_ok)
    PairBufs pbuf{{c->d_pkey[0], c->d_pkey[1]}, {c->d_pval[0], c->d_pval[1]}, c->d_emit_start, c->sw.status,
                  c->cap_pairs};
    if (c->noalloc) pbuf = noalloc_bufs(c->d_noalloc);
    const uint32_t cap = (uint32_t)std::min<uint64_t>({pbuf.cap, (uint64_t)c->pair_grid[c->pair_kind],
                                                       0xffffffffull});
    c->pair_cover = cap;
    // the fixed scratch is shared by every context on the GPU: its status
    // words are cleared so that no word of an earlier call matches an epoch
    if (c->noalloc) launch_fill_u32(c->sr, (uint32_t*)pbuf.status, 2 * (uint64_t)lb_status_words(cap), 0u);
    launch_emit(c->sr, c->d_dval[db], c->d_offs, c->d_tiles, c->d_rect, pbuf.emit_start, (uint32_t)n_total,
                c->d_total, n_render, c->TX, c->TY, pbuf.key[0], pbuf.val[0], cap);
    const uint32_t n_tiles = (uint32_t)(c->TX * c->TY) * n_views;
    uint64_t* const own_status = c->sw.status;
    c->sw.status = pbuf.status;
    const int pb = onesweep_u32_dev(c->sr, c->sw, pbuf.key, pbuf.val, cap, c->d_total, 0,
                                    std::max(1, bits_for(n_tiles)));
    c->sw.status = own_status;
    c->last_pk = pbuf.key[pb]; c->last_pv = pbuf.val[pb];
    launch_ranges(c->sr, pbuf.key[pb], cap, c->d_total, c->d_ranges, n_tiles);
    launch_tile_order(c->sr, c->d_ranges, n_tiles, c->d_tile_order);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(ev[5], c->sr));
    const bool bstats = (c->opt.flags & VM3DGS_FLAG_BLEND_STATS) != 0;
    {
        uint2* const bs = bstats ? c->d_bstats : nullptr;
        const int W = (int)c->opt.img_w, H = (int)c->opt.img_h;
        if (bs) launch_fill_u32(c->sr, (uint32_t*)bs, 2 * (uint64_t)n_tiles, 0u);
        // the longest tiles' alpha band walk on the render stream, the other
        // tiles beside it on the blend stream, joined back; room for half
        // as many longest tiles again as the last frame had (their count is
        // known on the device only; any beyond take the other launch), and
        // one launch alone after a frame without them
        const uint32_t h = c->last_n_xlong;
        const uint32_t x_cap = h == 0 ? 0u : blend_x_cap(n_tiles, h > 0x3fffffffu ? h : h + h / 2 + 8);
        if (x_cap) {
            HIPCHK(hipEventRecord(c->ev_bfork, c->sr));
            HIPCHK(hipStreamWaitEvent(c->sb, c->ev_bfork, 0));
            launch_blend_x(c->sr, c->d_ranges, c->d_tile_order, pbuf.val[pb], c->d_xy, c->d_conic, c->d_rgb, W, H,
                           c->TX, c->TY, (int)n_views, x_cap, image, bs);
            launch_blend(c->sb, c->d_ranges, c->d_tile_order, pbuf.val[pb], c->d_xy, c->d_conic, c->d_rgb, W, H,
                         c->TX, c->TY, (int)n_views, x_cap, image, bs);
            HIPCHK(hipGetLastError());
            HIPCHK(hipEventRecord(c->ev_bjoin, c->sb));
            HIPCHK(hipStreamWaitEvent(c->sr, c->ev_bjoin, 0));
        } else {
            launch_blend(c->sr, c->d_ranges, c->d_tile_order, pbuf.val[pb], c->d_xy, c->d_conic, c->d_rgb, W, H,
                         c->TX, c->TY, (int)n_views, 0u, image, bs);
            HIPCHK(hipGetLastError());
        }
    }
    HIPCHK(hipEventRecord(ev[6], c->sr));
    if (bstats && st) {
        HIPCHK(hipMemcpyAsync(c->h_bstats, c->d_bstats, sizeof(uint2) * n_tiles, hipMemcpyDeviceToHost, c->sr));
        HIPCHK(hipStreamSynchronize(c->sr));
        uint64_t e = 0, al = 0;
        for (uint32_t i = 0; i < n_tiles; ++i) { e += c->h_bstats[i].x; al += c->h_bstats[i].y; }
        st->blend_evals = e;
        st->blend_alphas = al;
    }
    rb_add(c, c->d_total, c->hd_total, sizeof(uint32_t));
    rb_add(c, c->d_zero + ZB_ERR, (uint32_t*)c->hd_total + 1, sizeof(uint32_t));
    rb_add(c, c->d_tile_order + n_tiles + 1, (uint32_t*)c->hd_total + 5, sizeof(uint32_t));
    c->last_views = n_views; c->last_n_render = n_render;
    c->last_pbuf = pb; c->last_dbuf = db;
    if (st) st->render_gaussians = n_total;
}

// after the render stream has passed splat: true when every pair fitted the
// pair buffers; otherwise they are grown and the caller runs splat again
bool splat_pairs_ok(vm3dgs* c, vm3dgs_stats* st) {
    if (c->h_total[1]) throw HipError{hipErrorUnknown, "single-pass scan look-back did not complete", __LINE__};
    const uint32_t n_pairs = c->h_total[0];
    c->last_n_xlong = c->h_total[5];
    const uint64_t want = std::min<uint64_t>((uint64_t)n_pairs + n_pairs / 2 + 1024, 0xffffffffull);
    c->pair_grid[c->pair_kind] = (uint32_t)want;
    if (n_pairs > c->pair_cover) {
        if (c->noalloc) {
            if (n_pairs > kNoallocPairs) throw NoallocCapacity{n_pairs};
            return false;   // a larger grid over the same fixed buffers
        }
        ensure_pairs(c, n_pairs);
        return false;
    }
    c->last_n_pairs = n_pairs;
    if (st) st->pairs = n_pairs;
    return true;
}

// camera pose for the prefetch features: position relative to the centre
// over the extent, camera-to-world rotation as a unit quaternion, w >= 0
void pose_of(const vm3dgs_camera& cam, const vm3dgs_prefetch_opts& o, float* out) {
    double M[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i][j] = cam.view[4 * j + i];
    double w, x, y, z;
    const double tr = M[0][0] + M[1][1] + M[2][2];
    if (tr > 0.0) {
        const double S = std::sqrt(tr + 1.0) * 2.0;
        w = 0.25 * S; x = (M[2][1] - M[1][2]) / S; y = (M[0][2] - M[2][0]) / S; z = (M[1][0] - M[0][1]) / S;
    } else if (M[0][0] > M[1][1] && M[0][0] > M[2][2]) {
        const double S = std::sqrt(1.0 + M[0][0] - M[1][1] - M[2][2]) * 2.0;
        w = (M[2][1] - M[1][2]) / S; x = 0.25 * S; y = (M[0][1] + M[1][0]) / S; z = (M[0][2] + M[2][0]) / S;
    } else if (M[1][1] > M[2][2]) {
        const double S = std::sqrt(1.0 + M[1][1] - M[0][0] - M[2][2]) * 2.0;
        w = (M[0][2] - M[2][0]) / S; x = (M[0][1] + M[1][0]) / S; y = 0.25 * S; z = (M[1][2] + M[2][1]) / S;
    } else {
        const double S = std::sqrt(1.0 + M[2][2] - M[0][0] - M[1][1]) * 2.0;
        w = (M[1][0] - M[0][1]) / S; x = (M[0][2] + M[2][0]) / S; y = (M[1][2] + M[2][1]) / S; z = 0.25 * S;
    }
    double n = std::sqrt(w * w + x * x + y * y + z * z);
    if (w < 0.0) n = -n;
    for (int a = 0; a < 3; ++a) out[a] = (float)(((double)cam.cam_pos[a] - o.center[a]) / o.extent);
    out[3] = (float)(w / n); out[4] = (float)(x / n); out[5] = (float)(y / n); out[6] = (float)(z / n);
}

void push_poses(vm3dgs* c, const vm3dgs_camera* cams, uint32_t n_views) {
    for (uint32_t v = 0; v < n_views; ++v) {
        float cur[7];
        pose_of(cams[v], c->pf, cur);
        float* h = &c->pf_pose[(size_t)v * 28];
        if (c->pf_n_hist == 0)
            for (int k = 0; k < 4; ++k) memcpy(h + 7 * k, cur, sizeof cur);
        else {
            memmove(h, h + 7, sizeof(float) * 21);
            memcpy(h + 21, cur, sizeof cur);
        }
    }
    if (c->pf_n_hist < 4) c->pf_n_hist++;
}

// feature rows of n_views views into d_pf_x: pose history from the host, the
// residency fractions by a kernel (on the render stream)
void pf_features(vm3dgs* c, uint32_t n_views) {
    const int ld = 28 + (int)c->pf.hist_bins;
    for (uint32_t v = 0; v < n_views; ++v) memcpy(c->h_pf_x + (size_t)v * ld, &c->pf_pose[(size_t)v * 28], 28 * 4);
    HIPCHK(hipMemcpy2DAsync(c->d_pf_x, sizeof(float) * ld, c->h_pf_x, sizeof(float) * ld, 28 * sizeof(float),
                            n_views, hipMemcpyHostToDevice, c->sr));
    launch_pf_features(c->sr, c->d_v2p, c->n_pg, c->L, (int)c->pf.hist_bins, (int)n_views, c->d_pf_x);
}

}  // namespace

namespace vm {
bool prefetch_stage_of(const vm3dgs* c, vm3dgs_mlp** net, vm3dgs_prefetch_opts* opts) {
    if (!c || !c->pf_on) return false;
    if (net) *net = c->pf_net;
    if (opts) *opts = c->pf;
    return true;
}
}  // namespace vm

namespace {

// The LOD thresholds follow memory use (Sec. 5.1.1, with Sec. 4.1 and
// Sec. 5.3).  The aim is 50-80 % of the pool, usage being the share of
// physical pages the frame required.  Over 80 %, or with requests left
// missing for want of a free pool entry (not those the copy budget defers,
// which say nothing about memory use), the transition distances shrink: the
// level-0 radius tau (pixels)
// grows by the factor 1 + step.  Under 50 % while some requested page is at
// a coarse level, tau shrinks by the same factor.  After a move the step
// changes by 1 % of itself: up when the move repeats the direction of a
// move made at most kLodQuick frames earlier, down when it reverses one.
// tau stays within [2^-7, 2^16] px.  The new tau is used from the next frame.
void lod_control(vm3dgs* c, uint32_t n_missing_cap, uint32_t req_slots, uint32_t n_coarse) {
    const uint64_t S = (uint64_t)c->S;
    int d = 0;
    if (n_missing_cap > 0 || (uint64_t)req_slots * 5 > S * 4) d = 1;
    else if ((uint64_t)req_slots * 2 < S && n_coarse > 0) d = -1;
    if (d == 0) return;
    const float t = d > 0 ? c->lod_tau * (1.0f + c->lod_step) : c->lod_tau / (1.0f + c->lod_step);
    c->lod_tau = std::min(std::max(t, kLodTauMin), kLodTauMax);
    if (c->lod_dir != 0 && c->frame - c->lod_last_move <= kLodQuick)
        c->lod_step = c->lod_dir == d ? c->lod_step * 1.01f : c->lod_step * 0.99f;
    c->lod_dir = d;
    c->lod_last_move = c->frame;
}

vm3dgs_status fail(vm3dgs* c, const HipError& h) {
    c->err = std::string("HIP error ") + hipGetErrorString(h.e) + " in " + h.what + " (api.cpp:" +
             std::to_string(h.line) + ")";
    c->poisoned = true;
    return VM3DGS_E_HIP;
}

vm3dgs_status bad(vm3dgs* c, const char* m) {
    c->err = m;
    return VM3DGS_E_INVALID_ARG;
}

float ms(hipEvent_t a, hipEvent_t b) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, a, b) != hipSuccess) return 0.0f;
    return t;
}

}  // namespace

extern "C" {

void vm3dgs_options_default(vm3dgs_options* o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->img_w = 1920; o->img_h = 1080; o->idbuf_w = 240; o->idbuf_h = 135; o->max_views = 1;
    o->attr_format = 0; o->copy_budget_pages = 0;
    o->proxy_cell_m = 1.0f; o->link_sigma = 2.0f; o->lod_radius_px = 32.0f; o->idbuf_guard_px = 32.0f;
    o->flags = VM3DGS_FLAG_LINKS;
    o->lod_scale_up = 1.0f;
    o->lod_builder = 0;
}

const char* vm3dgs_create_error(void) { return g_create_error.c_str(); }

vm3dgs_status vm3dgs_create(const vm3dgs_scene* scene, uint32_t page_size, uint32_t pool_pages, uint32_t lod_levels,
                            const vm3dgs_options* opt, vm3dgs** out) {
    g_create_error.clear();
    if (!out) { g_create_error = "out is NULL"; return VM3DGS_E_INVALID_ARG; }
    *out = nullptr;
    vm3dgs_options o;
    if (opt) o = *opt; else vm3dgs_options_default(&o);
    auto inval = [](const char* m) { g_create_error = m; return VM3DGS_E_INVALID_ARG; };
    if (!scene || scene->n == 0 || !scene->means || !scene->scales || !scene->quats || !scene->opacity || !scene->sh)
        return inval("scene is NULL or empty");
    if (page_size == 0 || pool_pages == 0) return inval("page_size and pool_pages must be > 0");
    if (lod_levels < 1 || lod_levels > 3) return inval("lod_levels must be 1..3");
    for (uint32_t l = 1; l < lod_levels; ++l)
        if ((page_size >> (3 * l)) == 0 || ((page_size >> (3 * l)) << (3 * l)) != page_size)
            return inval("page_size must be divisible by 8^(lod_levels-1)");
    if (o.img_w == 0 || o.img_h == 0 || o.idbuf_w == 0 || o.idbuf_h == 0) return inval("image sizes must be > 0");
    if (o.img_w > 65535 * 16 || o.img_h > 65535 * 16) return inval("image too large");
    if (o.max_views == 0 || o.max_views > 64) return inval("max_views must be 1..64");
    if (o.attr_format > 1) return inval("attr_format must be 0 or 1");
    if (!(o.proxy_cell_m > 0.0f) || !(o.link_sigma >= 0.0f) || !(o.lod_radius_px > 0.0f) ||
        !(o.idbuf_guard_px >= 0.0f && o.idbuf_guard_px <= 4096.0f))
        return inval("proxy_cell_m, link_sigma, lod_radius_px out of range");
    if (!(o.lod_scale_up > 0.0f && o.lod_scale_up <= 16.0f)) return inval("lod_scale_up must be in (0, 16]");
    if (o.lod_builder > 1) return inval("lod_builder must be 0 or 1");
    if (scene->n > (uint64_t)INT32_MAX * page_size) return inval("scene too large");

    vm3dgs* c = new (std::nothrow) vm3dgs();
    if (!c) { g_create_error = "host allocation failed"; return VM3DGS_E_HOST_OOM; }
    c->opt = o;
    try {
        std::string e = build_paged_scene(*scene, (int)page_size, (int)lod_levels, (int)o.attr_format,
                                          (double)o.proxy_cell_m, (double)o.link_sigma, (double)o.lod_scale_up,
                                          (int)o.lod_builder, c->ps);
        if (!e.empty()) { g_create_error = e; delete c; return VM3DGS_E_INVALID_ARG; }
    } catch (const std::bad_alloc&) {
        g_create_error = "host allocation failed";
        delete c;
        return VM3DGS_E_HOST_OOM;
    }
    const PagedScene& ps = c->ps;
    c->S = (int)pool_pages; c->L = (int)lod_levels; c->P = (int)page_size; c->n_pg = ps.n_pg;
    c->TX = (int)((o.img_w + 15) / 16); c->TY = (int)((o.img_h + 15) / 16);
    // one level and a table that fits one workgroup's LDS: the single-kernel page
    // table; otherwise the multi-kernel one (sorted candidate lists, ordered walk)
    c->multi = c->L > 1 || !pagetable_l1_fits(c->n_pg, c->S);
    c->lod_tau = o.lod_radius_px;
    try {
        if (o.stream_render) c->sr = (hipStream_t)o.stream_render;
        else { HIPCHK(hipStreamCreateWithFlags(&c->sr, hipStreamNonBlocking)); c->own_sr = true; }
        if (o.stream_copy) c->sc = (hipStream_t)o.stream_copy;
        else { HIPCHK(hipStreamCreateWithFlags(&c->sc, hipStreamNonBlocking)); c->own_sc = true; }
        HIPCHK(hipStreamCreateWithFlags(&c->sb, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&c->ev_bfork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->ev_bjoin, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->ev_copy, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->ev_sync, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->ev_async, hipEventDisableTiming));
        for (auto& e : c->ev) HIPCHK(hipEventCreate(&e));
        {
            // this device's fixed scratch for vm3dgs_frame_noalloc (looked up
            // once per device, with the device current)
            void* p = nullptr;
            HIPCHK(noalloc_scratch(&p));
            uint64_t used = 0;
            noalloc_bufs((uint8_t*)p, &used);
            if (used > kNoallocScratchBytes)
                throw HipError{hipErrorInvalidValue, "fixed scratch layout exceeds its size", __LINE__};
            c->d_noalloc = (uint8_t*)p;
        }
        const int n_pg = c->n_pg, S = c->S, L = c->L, V = (int)o.max_views;
        // frame outputs at their largest, so that no frame call allocates host memory
        c->out_req.reserve((size_t)n_pg);
        c->out_req_level.reserve((size_t)n_pg);
        c->out_missing.reserve((size_t)2 * n_pg * L);
        const int64_t nc = ps.nc();
        // scene metadata
        dalloc(&c->d_sph, n_pg);
        HIPCHK(hipMemcpy(c->d_sph, ps.spheres.data(), sizeof(float) * 4 * n_pg, hipMemcpyHostToDevice));
        dalloc(&c->d_clo, nc); dalloc(&c->d_chi, nc);
        if (nc) {
            HIPCHK(hipMemcpy(c->d_clo, ps.cell_lo.data(), sizeof(float) * 4 * nc, hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(c->d_chi, ps.cell_hi.data(), sizeof(float) * 4 * nc, hipMemcpyHostToDevice));
        }
        dalloc(&c->d_ls, n_pg + 1);
        HIPCHK(hipMemcpy(c->d_ls, ps.link_start.data(), sizeof(int32_t) * (n_pg + 1), hipMemcpyHostToDevice));
        dalloc(&c->d_ld, ps.link_dst.size());
        if (!ps.link_dst.empty())
            HIPCHK(hipMemcpy(c->d_ld, ps.link_dst.data(), sizeof(int32_t) * ps.link_dst.size(), hipMemcpyHostToDevice));
        dalloc(&c->d_level_base, 3);
        HIPCHK(hipMemcpy(c->d_level_base, ps.level_base, sizeof(int64_t) * 3, hipMemcpyHostToDevice));
        // pinned page-major store and the pool
        halloc(&c->h_store, (size_t)ps.store_bytes);
        encode_store(ps, c->h_store);
        {
            void* dp = nullptr;
            HIPCHK(hipHostGetDevicePointer(&dp, c->h_store, 0));
            c->h_store_dev = (const uint8_t*)dp;
        }
        dalloc(&c->d_cp_err, 4);
        HIPCHK(hipMemset(c->d_cp_err, 0, 16));
        dalloc(&c->d_pf_bytes, 1);
        HIPCHK(hipMemset(c->d_pf_bytes, 0, 8));
        const size_t slot_bytes = (size_t)c->P * ps.bytes_g;
        dalloc(&c->d_pool, slot_bytes * S);
        HIPCHK(hipMemset(c->d_pool, 0, slot_bytes * S));
        if (o.flags & VM3DGS_FLAG_FULL_SCENE_COPY) {
            dalloc(&c->d_full, slot_bytes * n_pg);
            HIPCHK(hipMemcpy(c->d_full, c->h_store, slot_bytes * n_pg, hipMemcpyHostToDevice));
        }
        dalloc(&c->d_cams, V); halloc(&c->h_cams, V);
        // visibility
        const int64_t npx = (int64_t)o.idbuf_w * o.idbuf_h;
        dalloc(&c->d_cand, (size_t)V * n_pg); dalloc(&c->d_rays, (size_t)V * npx); dalloc(&c->d_idbuf, (size_t)V * npx);
        dalloc(&c->d_crect, (size_t)V * nc); dalloc(&c->d_carea, (size_t)V * nc); dalloc(&c->d_coffs, (size_t)V * nc + 1);
        dalloc(&c->d_rd, n_pg); dalloc(&c->d_rl, n_pg); dalloc(&c->d_plevel, n_pg);
        dalloc(&c->d_keys, (size_t)2 * n_pg); halloc(&c->h_keys, n_pg);
        dalloc(&c->d_zero, ZB_WORDS);
        HIPCHK(hipMemset(c->d_zero, 0, sizeof(uint32_t) * ZB_WORDS));
        c->d_ctr = c->d_zero + ZB_CTR;
        c->sw.err = c->d_zero + ZB_ERR;
        c->sw.tickets = c->d_zero + ZB_TICKETS;
        c->sw.hist = c->d_zero + ZB_HIST;
        halloc(&c->h_ctr, C_NCOUNTERS);
        // page table (empty pool)
        dalloc(&c->d_slot_level, S); dalloc(&c->d_last_used, S); dalloc(&c->d_sub_vpage, (size_t)S * SUBS);
        dalloc(&c->d_sub_lu, (size_t)S * SUBS); dalloc(&c->d_v2p, (size_t)n_pg * L);
        dalloc(&c->d_req_sub, (size_t)S * SUBS); dalloc(&c->d_slot_req, (size_t)(S + 3) / 4 * 4); dalloc(&c->d_miss, (size_t)n_pg * L);
        HIPCHK(hipMemset(c->d_slot_level, 0xff, S));
        HIPCHK(hipMemset(c->d_last_used, 0xff, sizeof(int32_t) * S));
        HIPCHK(hipMemset(c->d_sub_vpage, 0xff, sizeof(int32_t) * S * SUBS));
        HIPCHK(hipMemset(c->d_sub_lu, 0xff, sizeof(int32_t) * S * SUBS));
        HIPCHK(hipMemset(c->d_v2p, 0xff, sizeof(int32_t) * n_pg * L));
        dalloc(&c->d_copies_buf[0], (size_t)n_pg * L); dalloc(&c->d_copies_buf[1], (size_t)n_pg * L);
        c->d_copies = c->d_copies_buf[0];
        halloc(&c->h_copies, (size_t)n_pg * L);
        dalloc(&c->d_copy_id, (size_t)4 * n_pg * L);
        dalloc(&c->d_missing, (size_t)2 * n_pg * L); halloc(&c->h_missing, (size_t)2 * n_pg * L);
        dalloc(&c->d_rlist, n_pg);
        if (c->multi) {
            dalloc(&c->d_lkeys_alt, n_pg); dalloc(&c->d_lflag, n_pg); dalloc(&c->d_lpos, (size_t)n_pg + 1);
            dalloc(&c->d_lflag2, n_pg); dalloc(&c->d_lpos2, (size_t)n_pg + 1); dalloc(&c->d_rlevel, n_pg);
            dalloc(&c->d_wkeys[0], S); dalloc(&c->d_wkeys[1], S);
            for (int l = 1; l < L; ++l) { dalloc(&c->d_ck[l][0], (size_t)S * SUBS); dalloc(&c->d_ck[l][1], (size_t)S * SUBS); }
            dalloc(&c->d_fresh, (size_t)3 * S);
            dalloc(&c->d_lvl_out, n_pg); halloc(&c->h_lvl, n_pg);
        }
        // splat buffers
        const uint64_t per_view = std::max<uint64_t>((uint64_t)S * c->P,
                                                     (o.flags & VM3DGS_FLAG_FULL_SCENE_COPY) ? (uint64_t)n_pg * c->P : 0);
        if (per_view * V > 0xffffffffull) throw HipError{hipErrorInvalidValue, "render set exceeds 2^32", __LINE__};
        c->cap_render = per_view * V;
        const uint64_t R = c->cap_render;
        dalloc(&c->d_xy, R); dalloc(&c->d_conic, R); dalloc(&c->d_rgb, R); dalloc(&c->d_depth, R);
        dalloc(&c->d_rect, R); dalloc(&c->d_tiles, R); dalloc(&c->d_offs, R + 1);
        for (int i = 0; i < 2; ++i) { dalloc(&c->d_dkey[i], R); dalloc(&c->d_dval[i], R); }
        dalloc(&c->d_ranges, (size_t)c->TX * c->TY * V);
        dalloc(&c->d_tile_order, (size_t)c->TX * c->TY * V + 2);   // + the counts of long and longest tiles
        dalloc(&c->d_bstats, (size_t)c->TX * c->TY * V); halloc(&c->h_bstats, (size_t)c->TX * c->TY * V);
        dalloc(&c->d_total, 4); halloc(&c->h_total, 8);  // [0] pairs, [1] look-back error, [2..3] bytes, [4] copy error, [5] longest tiles
        c->hd_total = host_dev(c->h_total); c->hd_ctr = host_dev(c->h_ctr); c->hd_keys = host_dev(c->h_keys);
        c->hd_missing = host_dev(c->h_missing);
        if (c->h_lvl) c->hd_lvl = host_dev(c->h_lvl);
        c->cap_pairs = 0;
        ensure_pairs(c, o.pair_capacity ? o.pair_capacity : std::max<uint64_t>(R * 4, 1u << 22));
            ensure_status(c);
        if (o.flags & VM3DGS_FLAG_FULL_SCENE_COPY) {
            std::vector<RenderEntry> full((size_t)n_pg);
            for (int p = 0; p < n_pg; ++p)
                full[(size_t)p] = RenderEntry{(uint32_t)p * (uint32_t)c->P, (uint32_t)c->P, (uint32_t)p * (uint32_t)c->P, 0u};
            dalloc(&c->d_rlist_full, n_pg);
            HIPCHK(hipMemcpy(c->d_rlist_full, full.data(), sizeof(RenderEntry) * n_pg, hipMemcpyHostToDevice));
        }
        HIPCHK(hipDeviceSynchronize());
    } catch (const HipError& h) {
        g_create_error = std::string("HIP error ") + hipGetErrorString(h.e) + " in " + h.what;
        const bool oom = h.e == hipErrorOutOfMemory || h.e == hipErrorMemoryAllocation;
        free_all(c);
        delete c;
        return oom ? VM3DGS_E_DEVICE_OOM : VM3DGS_E_HIP;
    } catch (const std::bad_alloc&) {
        g_create_error = "host allocation failed";
        free_all(c);
        delete c;
        return VM3DGS_E_HOST_OOM;
    }
    *out = c;
    return VM3DGS_OK;
}

}  // extern "C"

namespace {

// one frame; with noalloc the pair buffers are the device's fixed scratch and
// nothing is allocated
vm3dgs_status frame_impl(vm3dgs* c, const vm3dgs_camera* cams, uint32_t n_views, float* image,
                         vm3dgs_frame_out* out, bool noalloc) {
    if (!c) return VM3DGS_E_INVALID_ARG;
    if (c->poisoned) return VM3DGS_E_STATE;
    if (!cams || !image || n_views == 0) return bad(c, "cams, image and n_views must be given");
    if (n_views > c->opt.max_views) { c->err = "n_views exceeds max_views"; return VM3DGS_E_CAPACITY; }
    vm3dgs_stats st{};
    struct ModeGuard {
        vm3dgs* c;
        ModeGuard(vm3dgs* c_, bool m) : c(c_) { c->noalloc = m; }
        ~ModeGuard() { c->noalloc = false; }
    } mode(c, noalloc);
    try {
        hipEvent_t* ev = c->ev;
        float fy_max = 0.0f;
        for (uint32_t v = 0; v < n_views; ++v) {
            to_camk(cams[v], c->h_cams[v]);
            fy_max = std::max(fy_max, cams[v].fy);
        }
        HIPCHK(hipEventRecord(ev[0], c->sr));
        HIPCHK(hipMemcpyAsync(c->d_cams, c->h_cams, sizeof(CamK) * n_views, hipMemcpyHostToDevice, c->sr));
        if (c->pf_on) push_poses(c, cams, n_views);
        c->cpb ^= 1;
        c->d_copies = c->d_copies_buf[c->cpb];
        c->sw.reset();
        c->rb.n = 0;
        VisArgs va{};
        va.spheres = c->d_sph; va.n_pg = c->n_pg; va.cell_lo = c->d_clo; va.cell_hi = c->d_chi; va.nc = c->ps.nc();
        va.link_start = c->d_ls; va.link_dst = c->d_ld; va.use_links = (c->opt.flags & VM3DGS_FLAG_LINKS) ? 1 : 0;
        va.cams = c->d_cams; va.n_views = (int)n_views; va.W = (int)c->opt.img_w; va.H = (int)c->opt.img_h;
        va.Wv = (int)c->opt.idbuf_w; va.Hv = (int)c->opt.idbuf_h; va.L = c->L; va.tau = c->lod_tau;
        va.fy_max = fy_max;
        va.guard = c->opt.idbuf_guard_px;
        va.cand = c->d_cand; va.rays = c->d_rays; va.idbuf = c->d_idbuf; va.req_direct = c->d_rd; va.req_link = c->d_rl;
        va.page_level = c->d_plevel; va.req_keys = c->d_keys; va.counters = c->d_ctr;
        va.cell_rects = c->d_crect; va.cell_area = c->d_carea; va.cell_offs = c->d_coffs;
        va.sw = &c->sw;
        {
            // counters, tickets, histograms, ID buffer and request arrays: one launch
            FillSegs fs;
            fs.seg[fs.n++] = FillSeg{c->d_zero, (uint64_t)ZB_WORDS, 0u, 0};
            visibility_clears(va, fs);
            launch_fill_multi(c->sr, fs);
        }
        launch_visibility(c->sr, va);
        HIPCHK(hipGetLastError());
        HIPCHK(hipEventRecord(ev[1], c->sr));
        PtArgs pa{};
        pa.req_keys = c->d_keys; pa.n_pg = c->n_pg; pa.L = c->L; pa.P = c->P; pa.S = c->S; pa.frame = c->frame;
        pa.budget = (int)c->opt.copy_budget_pages; pa.bytes_g = c->ps.bytes_g; pa.page_level = c->d_plevel;
        pa.slot_level = c->d_slot_level; pa.last_used = c->d_last_used; pa.sub_vpage = c->d_sub_vpage;
        pa.sub_last_used = c->d_sub_lu; pa.v2p = c->d_v2p; pa.req_sub = c->d_req_sub; pa.slot_req = c->d_slot_req;
        pa.miss = c->d_miss; pa.copies = c->d_copies; pa.copy_id = c->d_copy_id; pa.missing = c->d_missing;
        pa.counters = c->d_ctr; pa.level_base = c->d_level_base; pa.rl = c->d_rlist;
        const bool streaming = (c->opt.flags & VM3DGS_FLAG_ASYNC_MISSES) != 0;
        pa.streaming = streaming ? 1 : 0; pa.rlevel = c->d_rlevel;
        pa.hint_req = c->hint_req;
        for (int l = 0; l < 3; ++l) pa.hint_cand[l] = c->hint_cand[l];
        if (!c->multi) {
            launch_pagetable(c->sr, pa, 0);
        } else {
            LodWork lw{};
            lw.keys_alt = c->d_lkeys_alt; lw.keys_out = c->d_keys + c->n_pg; lw.level_out = c->d_lvl_out;
            lw.flag = c->d_lflag; lw.pos = c->d_lpos; lw.flag2 = c->d_lflag2; lw.pos2 = c->d_lpos2; lw.wkeys[0] = c->d_wkeys[0]; lw.wkeys[1] = c->d_wkeys[1];
            for (int l = 0; l < 3; ++l) { lw.ck[l][0] = c->d_ck[l][0]; lw.ck[l][1] = c->d_ck[l][1]; }
            lw.fresh = c->d_fresh;
            launch_pagetable_lod(c->sr, pa, c->sw, lw);
        }
        if (c->pf_on && c->pf_net) {
            // features of the state after the demand stages, the network, proposals, third stage
            pf_features(c, n_views);
            const MlpDev& nd = *mlp_dev_of(c->pf_net);
            mlp_input_dev(c->sr, nd, c->d_pf_x, (int)n_views);
            mlp_forward_dev(c->sr, nd, (int)n_views);
            PfArgs fa{};
            fa.logits = nd.logits; fa.K = (int)c->pf.n_clusters; fa.thr = c->pf.logit_threshold;
            fa.page_level = c->d_plevel; fa.v2p = c->d_v2p; fa.sph = c->d_sph; fa.n_pg = c->n_pg; fa.L = c->L;
            fa.tau = c->lod_tau; fa.fy = fy_max; fa.cams = c->d_cams; fa.n_views = (int)n_views;
            fa.keys[0] = c->d_pf_keys[0]; fa.keys[1] = c->d_pf_keys[1];
            fa.idle[0] = c->d_pf_idle[0]; fa.idle[1] = c->d_pf_idle[1];
            fa.S = c->S; fa.P = c->P; fa.frame = c->frame; fa.budget = (int)c->pf.budget_pages;
            fa.bytes_g = c->ps.bytes_g; fa.level_base = c->d_level_base;
            fa.slot_level = c->d_slot_level; fa.last_used = c->d_last_used; fa.sub_vpage = c->d_sub_vpage;
            fa.sub_last_used = c->d_sub_lu; fa.fresh = c->d_fresh;
            fa.copies = c->d_copies; fa.copy_id = c->d_copy_id; fa.counters = c->d_ctr;
            fa.sorted_out = &c->pf_sorted;
            launch_prefetch(c->sr, fa, c->sw);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipEventRecord(ev[2], c->sr));
        // the counters: how many copies, render entries and Gaussians this
        // frame has; the host reads them while the GPU runs the copies and the
        // preprocess, which take these counts from the device
        rb_add(c, c->d_ctr, c->hd_ctr, sizeof(uint32_t) * C_NCOUNTERS);
        mark_wait(c);
        const bool pf_stage = c->pf_on && c->pf_net;
        const uint64_t max_cmd = (uint64_t)c->P * c->ps.bytes_g;
        const uint64_t pool_bytes = max_cmd * (uint64_t)c->S;
        const uint32_t max_copies = (uint32_t)c->n_pg * (uint32_t)c->L;
        CopyRangeDev demand{c->d_ctr + C_NCOPY, pf_stage ? c->d_ctr + C_NPF : nullptr, 0};
        // copies of earlier frames on the copy stream (prefetches, streamed
        // misses) finish before this frame writes or reads the pool; a frame
        // records ev_pf after its ev_async, so waiting for ev_pf covers both
        if (c->pf_pending) {
            HIPCHK(hipStreamWaitEvent(c->sr, c->ev_pf, 0));
            c->pf_pending = false;
            c->async_pending = false;
        }
        if (c->async_pending) {
            HIPCHK(hipStreamWaitEvent(c->sr, c->ev_async, 0));
            c->async_pending = false;
        }
        if (!streaming) {
            // demand copies: read by the GPU from the pinned store, in order before the splat
            launch_copy_pages_dev(c->sr, c->d_copies, demand, max_copies, max_cmd, c->h_store_dev,
                                  (uint64_t)c->ps.store_bytes, c->d_pool, pool_bytes,
                                  (unsigned long long*)(c->d_zero + ZB_BYTES), c->d_cp_err);
        } else {
            // streaming (Sec. 4.3, Sec. 5.1.2): the frame renders what was resident
            // when it started; its copies run on the copy stream beside the splat
            // and the next frame waits for them before it touches the pool
            launch_copy_bytes_dev(c->sr, c->d_copies, demand, max_copies, (unsigned long long*)(c->d_zero + ZB_BYTES));
            HIPCHK(hipEventRecord(c->ev_copy, c->sr));
            HIPCHK(hipStreamWaitEvent(c->sc, c->ev_copy, 0));
            launch_copy_pages_dev(c->sc, c->d_copies, demand, max_copies, max_cmd, c->h_store_dev,
                                  (uint64_t)c->ps.store_bytes, c->d_pool, pool_bytes, c->d_pf_bytes, c->d_cp_err);
            HIPCHK(hipEventRecord(c->ev_async, c->sc));
            c->async_pending = true;
        }
        HIPCHK(hipGetLastError());
        // prefetch copies: on the copy stream, after the page table; not awaited by this frame
        if (pf_stage) {
            HIPCHK(hipEventRecord(c->ev_copy, c->sr));
            HIPCHK(hipStreamWaitEvent(c->sc, c->ev_copy, 0));
            launch_copy_pages_dev(c->sc, c->d_copies, CopyRangeDev{demand.n_copy, demand.n_pf, 1}, max_copies,
                                  max_cmd, c->h_store_dev, (uint64_t)c->ps.store_bytes, c->d_pool, pool_bytes,
                                  c->d_pf_bytes, c->d_cp_err);
            HIPCHK(hipGetLastError());
            HIPCHK(hipEventRecord(c->ev_pf, c->sc));
            c->pf_pending = true;
        }
        // the preprocess of the render set, sized on the device
        HIPCHK(hipEventRecord(ev[3], c->sr));
        launch_preprocess_dev(c->sr, splat_args(c, c->d_rlist, 0, c->d_pool, 0, n_views), c->d_ctr + C_NRENDER,
                              c->d_ctr + C_NRL, c->cap_render);
        HIPCHK(hipGetLastError());
        HIPCHK(hipEventRecord(ev[4], c->sr));
        spin_on_mark(c);
        const uint32_t* k = c->h_ctr;
        const uint32_t n_copy = k[C_NCOPY];
        const uint32_t n_pf = pf_stage ? k[C_NPF] : 0u;
        const uint32_t n_dem = n_copy - n_pf;
        st.lod_radius_px = c->lod_tau;
        if ((c->opt.flags & VM3DGS_FLAG_ADAPTIVE_LOD) && c->L > 1)
            lod_control(c, k[C_NMISSCAP], k[C_REQSLOTS], k[C_NCOARSE]);
        c->last_n_pfreq = (c->pf_on && c->pf_net) ? k[C_NPFREQ] : 0u;
        c->last_n_pf = n_pf;
        st.prefetched = n_pf;
        st.fallbacks = k[C_FALLBACK];
        const uint32_t n_render = k[C_NRENDER];
        c->last_n_copy = n_copy; c->last_n_missing = k[C_NMISSING]; c->last_n_req = k[C_NREQ];
        c->hint_req = k[C_NREQ]; c->hint_cand[1] = k[C_NCAND1]; c->hint_cand[2] = k[C_NCAND2];
        c->last_n_rl = k[C_NRL];
        st.candidates = k[C_CAND]; st.requested = k[C_NREQ]; st.direct = k[C_DIRECT]; st.linked = k[C_LINKED];
        st.hits = k[C_HITS]; st.misses = k[C_MISSES]; st.evictions = k[C_EVICT]; st.missing = k[C_NMISSING];
        st.copies = n_dem; st.render_pages = k[C_NRL]; st.pool_pages_used = k[C_POOLUSED];
        c->pair_kind = 0;
        splat_sorted(c, n_render, n_views, image, &st);
        // outputs of the frame: request order and missing list
        rb_add(c, c->d_keys + c->n_pg, c->hd_keys, sizeof(uint64_t) * c->last_n_req);
        if (c->L > 1) rb_add(c, c->d_lvl_out, c->hd_lvl, c->last_n_req);
        rb_add(c, c->d_missing, c->hd_missing, sizeof(int32_t) * 2 * c->last_n_missing);
        rb_add(c, c->d_zero + ZB_BYTES, (uint32_t*)c->hd_total + 2, 8);
        rb_add(c, c->d_cp_err, (uint32_t*)c->hd_total + 4, 4);
        spin_wait(c);
        if (c->h_total[4]) throw HipError{hipErrorInvalidValue, "a page copy command left the store or the pool",
                                          __LINE__};
        if (!splat_pairs_ok(c, &st)) {
            // more pairs than the buffers held: the same render set again (its
            // pages are resident now) with the grown buffers
            splat(c, c->d_rlist, k[C_NRL], c->d_pool, n_render, n_views, image, &st);
            spin_wait(c);
            if (!splat_pairs_ok(c, &st)) throw std::length_error("pair buffers could not hold the frame's pairs");
        }
        {
            uint64_t b;
            memcpy(&b, c->h_total + 2, 8);
            st.bytes_copied = b;
        }
        c->out_req.resize(c->last_n_req);
        c->out_req_level.resize(c->last_n_req);
        for (uint32_t i = 0; i < c->last_n_req; ++i) {
            c->out_req[i] = (int32_t)(c->h_keys[i] & 0x3fffffffull);
            c->out_req_level[i] = c->L > 1 ? c->h_lvl[i] : (int8_t)0;
        }
        c->out_missing.assign(c->h_missing, c->h_missing + 2 * c->last_n_missing);
        st.ms_visibility = ms(ev[0], ev[1]);
        st.ms_pagetable = ms(ev[1], ev[2]);
        st.ms_copy = ms(ev[2], ev[3]);
        st.ms_preprocess = ms(ev[3], ev[4]);
        st.ms_sort = ms(ev[4], ev[5]);
        st.ms_blend = ms(ev[5], ev[6]);
        st.ms_total = ms(ev[0], ev[6]);
        c->frame++;
    } catch (const HipError& h) {
        return fail(c, h);
    } catch (const NoallocCapacity& e) {
        // the page table has taken the frame; its image is not rendered
        c->frame++;
        c->last_n_pairs = 0;
        c->err = "the frame has " + std::to_string(e.pairs) + " (tile, Gaussian) pairs; vm3dgs_frame_noalloc holds " +
                 std::to_string(kNoallocPairs);
        return VM3DGS_E_CAPACITY;
    } catch (const std::length_error& e) {
        c->err = e.what();
        c->poisoned = true;
        return VM3DGS_E_CAPACITY;
    }
    if (out) {
        out->requests = c->out_req.data();
        out->request_level = c->out_req_level.data();
        out->n_requests = (uint32_t)c->out_req.size();
        out->missing = c->out_missing.data();
        out->n_missing = (uint32_t)(c->out_missing.size() / 2);
        out->stats = st;
    }
    return VM3DGS_OK;
}

}  // namespace

extern "C" {

vm3dgs_status vm3dgs_frame(vm3dgs* c, const vm3dgs_camera* cams, uint32_t n_views, float* image,
                           vm3dgs_frame_out* out) {
    return frame_impl(c, cams, n_views, image, out, false);
}

vm3dgs_status vm3dgs_frame_noalloc(vm3dgs* c, const vm3dgs_camera* cams, uint32_t n_views, float* image,
                                   vm3dgs_frame_out* out) {
    return frame_impl(c, cams, n_views, image, out, true);
}

vm3dgs_status vm3dgs_render_full(vm3dgs* c, const vm3dgs_camera* cams, uint32_t n_views, float* image,
                                 vm3dgs_stats* stats) {
    if (!c) return VM3DGS_E_INVALID_ARG;
    if (c->poisoned) return VM3DGS_E_STATE;
    if (!cams || !image || n_views == 0) return bad(c, "cams, image and n_views must be given");
    if (n_views > c->opt.max_views) { c->err = "n_views exceeds max_views"; return VM3DGS_E_CAPACITY; }
    if (!c->d_full) return bad(c, "vm3dgs_render_full needs VM3DGS_FLAG_FULL_SCENE_COPY at create");
    vm3dgs_stats st{};
    try {
        for (uint32_t v = 0; v < n_views; ++v) to_camk(cams[v], c->h_cams[v]);
        HIPCHK(hipEventRecord(c->ev[0], c->sr));
        HIPCHK(hipMemcpyAsync(c->d_cams, c->h_cams, sizeof(CamK) * n_views, hipMemcpyHostToDevice, c->sr));
        begin_work(c);
        c->pair_kind = 1;
        splat(c, c->d_rlist_full, (uint32_t)c->n_pg, c->d_full, (uint32_t)c->n_pg * (uint32_t)c->P, n_views, image, &st);
        rb_flush(c);
        HIPCHK(hipStreamSynchronize(c->sr));
        if (!splat_pairs_ok(c, &st)) {
            splat(c, c->d_rlist_full, (uint32_t)c->n_pg, c->d_full, (uint32_t)c->n_pg * (uint32_t)c->P, n_views,
                  image, &st);
            rb_flush(c);
            HIPCHK(hipStreamSynchronize(c->sr));
            if (!splat_pairs_ok(c, &st)) throw std::length_error("pair buffers could not hold the frame's pairs");
        }
        st.ms_preprocess = ms(c->ev[3], c->ev[4]);
        st.ms_sort = ms(c->ev[4], c->ev[5]);
        st.ms_blend = ms(c->ev[5], c->ev[6]);
        st.ms_total = ms(c->ev[0], c->ev[6]);
        st.render_pages = (uint32_t)c->n_pg;
    } catch (const HipError& h) {
        return fail(c, h);
    } catch (const std::length_error& e) {
        c->err = e.what();
        c->poisoned = true;
        return VM3DGS_E_CAPACITY;
    }
    if (stats) *stats = st;
    return VM3DGS_OK;
}

vm3dgs_status vm3dgs_reset(vm3dgs* c) {
    if (!c) return VM3DGS_E_INVALID_ARG;
    if (c->poisoned) return VM3DGS_E_STATE;
    try {
        HIPCHK(hipStreamSynchronize(c->sr));
        HIPCHK(hipStreamSynchronize(c->sc));
        const size_t S = c->S, n_pg = c->n_pg, L = c->L;
        HIPCHK(hipMemset(c->d_slot_level, 0xff, S));
        HIPCHK(hipMemset(c->d_last_used, 0xff, sizeof(int32_t) * S));
        HIPCHK(hipMemset(c->d_sub_vpage, 0xff, sizeof(int32_t) * S * SUBS));
        HIPCHK(hipMemset(c->d_sub_lu, 0xff, sizeof(int32_t) * S * SUBS));
        HIPCHK(hipMemset(c->d_v2p, 0xff, sizeof(int32_t) * n_pg * L));
    } catch (const HipError& h) {
        return fail(c, h);
    }
    c->frame = 0;
    c->lod_tau = c->opt.lod_radius_px; c->lod_step = kLodStep0; c->lod_dir = 0; c->lod_last_move = 0;
    c->pf_n_hist = 0;
    c->pf_pending = false;
    c->last_n_copy = c->last_n_missing = c->last_n_req = c->last_n_rl = 0;
    c->last_n_pfreq = c->last_n_pf = 0;
    c->hint_req = ~0u;
    for (auto& h : c->hint_cand) h = ~0u;
    c->last_n_xlong = ~0u;
    return VM3DGS_OK;
}

vm3dgs_status vm3dgs_set_prefetch(vm3dgs* c, vm3dgs_mlp* net, const vm3dgs_prefetch_opts* o) {
    if (!c) return VM3DGS_E_INVALID_ARG;
    if (c->poisoned) return VM3DGS_E_STATE;
    if (!o || o->n_clusters == 0 || o->hist_bins == 0 || !(o->extent > 0.0f)) return bad(c, "prefetch options out of range");
    if (c->n_pg >= (1 << 28)) return bad(c, "prefetch keys hold page ids below 2^28");
    if (net) {
        const MlpDev& d = *mlp_dev_of(net);
        if (d.dims[0] != 28 + (int)o->hist_bins || d.dims[d.n_layers] != (int)o->n_clusters ||
            mlp_max_batch_of(net) < (int)c->opt.max_views)
            return bad(c, "network widths or batch do not match the prefetch options");
    }
    try {
        HIPCHK(hipStreamSynchronize(c->sr));
        HIPCHK(hipStreamSynchronize(c->sc));
        const size_t V = c->opt.max_views, ld = 28 + (size_t)o->hist_bins;
        dfree(c->d_pf_x); hfree(c->h_pf_x);
        dalloc(&c->d_pf_x, V * ld); halloc(&c->h_pf_x, V * ld);
        for (int i = 0; i < 2; ++i) {
            if (!c->d_pf_keys[i]) dalloc(&c->d_pf_keys[i], (size_t)c->n_pg);
            if (!c->d_pf_idle[i]) dalloc(&c->d_pf_idle[i], (size_t)c->S);
        }
        if (!c->d_fresh) dalloc(&c->d_fresh, (size_t)3 * c->S);
        if (!c->ev_pf) HIPCHK(hipEventCreateWithFlags(&c->ev_pf, hipEventDisableTiming));
    } catch (const HipError& h) {
        return fail(c, h);
    }
    c->pf = *o;
    c->pf_net = net;
    c->pf_on = true;
    c->pf_n_hist = 0;
    c->pf_pose.assign((size_t)c->opt.max_views * 28, 0.0f);
    c->pf_sorted = nullptr;
    c->last_n_pfreq = c->last_n_pf = 0;
    return VM3DGS_OK;
}

vm3dgs_status vm3dgs_prefetch_features(vm3dgs* c, uint32_t n_views, float* x) {
    if (!c) return VM3DGS_E_INVALID_ARG;
    if (c->poisoned) return VM3DGS_E_STATE;
    if (!c->pf_on || !x || n_views == 0 || n_views > c->opt.max_views) return bad(c, "no prefetch stage or bad views");
    try {
        pf_features(c, n_views);
        HIPCHK(hipMemcpyAsync(x, c->d_pf_x, sizeof(float) * n_views * (28 + c->pf.hist_bins), hipMemcpyDeviceToHost,
                              c->sr));
        HIPCHK(hipStreamSynchronize(c->sr));
    } catch (const HipError& h) {
        return fail(c, h);
    }
    return VM3DGS_OK;
}

vm3dgs_status vm3dgs_set_flags(vm3dgs* c, uint32_t flags) {
    if (!c) return VM3DGS_E_INVALID_ARG;
    const uint32_t fixed = VM3DGS_FLAG_FULL_SCENE_COPY;
    c->opt.flags = (c->opt.flags & fixed) | (flags & ~fixed);
    return VM3DGS_OK;
}

vm3dgs_status vm3dgs_set_lod_radius(vm3dgs* c, float tau_px) {
    if (!c) return VM3DGS_E_INVALID_ARG;
    if (!(tau_px > 0.0f) || !std::isfinite(tau_px)) return bad(c, "tau_px must be a positive finite number");
    c->opt.lod_radius_px = tau_px;
    c->lod_tau = tau_px; c->lod_step = kLodStep0; c->lod_dir = 0; c->lod_last_move = c->frame;
    return VM3DGS_OK;
}

vm3dgs_status vm3dgs_sync(vm3dgs* c) {
    if (!c) return VM3DGS_E_INVALID_ARG;
    if (c->poisoned) return VM3DGS_E_STATE;
    try {
        HIPCHK(hipStreamSynchronize(c->sr));
        HIPCHK(hipStreamSynchronize(c->sc));
    } catch (const HipError& h) {
        return fail(c, h);
    } catch (const std::length_error& e) {
        c->err = e.what();
        c->poisoned = true;
        return VM3DGS_E_CAPACITY;
    }
    return VM3DGS_OK;
}

const char* vm3dgs_last_error(const vm3dgs* c) { return c ? c->err.c_str() : "context is NULL"; }

void vm3dgs_destroy(vm3dgs* c) {
    if (!c) return;
    free_all(c);
    delete c;
}

struct vm3dgs_pages {
    PagedScene ps;
    std::vector<uint8_t> store;
};

vm3dgs_status vm3dgs_pages_build(const vm3dgs_scene* scene, uint32_t page_size, uint32_t lod_levels,
                                 const vm3dgs_options* opt, vm3dgs_pages** out) {
    g_create_error.clear();
    if (!out) { g_create_error = "out is NULL"; return VM3DGS_E_INVALID_ARG; }
    *out = nullptr;
    vm3dgs_options o;
    if (opt) o = *opt; else vm3dgs_options_default(&o);
    if (!scene || scene->n == 0 || !scene->means || !scene->scales || !scene->quats || !scene->opacity || !scene->sh) {
        g_create_error = "scene is NULL or empty";
        return VM3DGS_E_INVALID_ARG;
    }
    if (page_size == 0 || lod_levels < 1 || lod_levels > 3 || o.attr_format > 1 || !(o.proxy_cell_m > 0.0f) ||
        !(o.lod_scale_up > 0.0f && o.lod_scale_up <= 16.0f) || o.lod_builder > 1) {
        g_create_error = "page_size, lod_levels, attr_format, proxy_cell_m, lod_scale_up or lod_builder out of range";
        return VM3DGS_E_INVALID_ARG;
    }
    for (uint32_t l = 1; l < lod_levels; ++l)
        if ((page_size >> (3 * l)) == 0 || ((page_size >> (3 * l)) << (3 * l)) != page_size) {
            g_create_error = "page_size must be divisible by 8^(lod_levels-1)";
            return VM3DGS_E_INVALID_ARG;
        }
    vm3dgs_pages* p = new (std::nothrow) vm3dgs_pages();
    if (!p) return VM3DGS_E_HOST_OOM;
    try {
        std::string e = build_paged_scene(*scene, (int)page_size, (int)lod_levels, (int)o.attr_format,
                                          (double)o.proxy_cell_m, (double)o.link_sigma, (double)o.lod_scale_up,
                                          (int)o.lod_builder, p->ps);
        if (!e.empty()) { g_create_error = e; delete p; return VM3DGS_E_INVALID_ARG; }
        p->store.resize((size_t)p->ps.store_bytes);
        encode_store(p->ps, p->store.data());
    } catch (const std::bad_alloc&) {
        delete p;
        g_create_error = "host allocation failed";
        return VM3DGS_E_HOST_OOM;
    }
    *out = p;
    return VM3DGS_OK;
}

int64_t vm3dgs_pages_get(const vm3dgs_pages* p, const char* name, void* dst, int64_t cap) {
    if (!p || !name) return -1;
    const std::string n(name);
    const PagedScene& ps = p->ps;
    auto host = [&](const void* src, int64_t bytes) -> int64_t {
        if (dst && cap >= bytes && bytes > 0) memcpy(dst, src, (size_t)bytes);
        return bytes;
    };
    if (n == "info") {
        int64_t v[8] = {ps.n_pg, ps.P, ps.L, ps.bytes_g, ps.nc(), (int64_t)ps.link_dst.size(), ps.store_bytes, 0};
        return host(v, sizeof v);
    }
    if (n == "perm") return host(ps.perm.data(), 8 * (int64_t)ps.perm.size());
    if (n == "spheres") return host(ps.spheres.data(), 4 * (int64_t)ps.spheres.size());
    if (n == "cell_box") {
        const int64_t nc = ps.nc();
        if (dst && cap >= 24 * nc)
            for (int64_t i = 0; i < nc; ++i) {
                float* o = (float*)dst + 6 * i;
                for (int a = 0; a < 3; ++a) { o[a] = ps.cell_lo[(size_t)i * 4 + a]; o[3 + a] = ps.cell_hi[(size_t)i * 4 + a]; }
            }
        return 24 * nc;
    }
    if (n == "cell_page") return host(ps.cell_page.data(), 4 * ps.nc());
    if (n == "cell_start") return host(ps.cell_start.data(), 4 * (int64_t)ps.cell_start.size());
    if (n == "link_start") return host(ps.link_start.data(), 4 * (int64_t)ps.link_start.size());
    if (n == "link_dst") return host(ps.link_dst.data(), 4 * (int64_t)ps.link_dst.size());
    if (n == "rec0") return host(ps.rec[0].data(), 4 * (int64_t)ps.rec[0].size());
    if (n == "rec1" && ps.L > 1) return host(ps.rec[1].data(), 4 * (int64_t)ps.rec[1].size());
    if (n == "rec2" && ps.L > 2) return host(ps.rec[2].data(), 4 * (int64_t)ps.rec[2].size());
    if (n == "store") return host(p->store.data(), (int64_t)p->store.size());
    return -1;
}

void vm3dgs_pages_destroy(vm3dgs_pages* p) { delete p; }

int64_t vm3dgs_debug_get(vm3dgs* c, const char* name, void* dst, int64_t cap) {
    if (!c || !name) return -1;
    const std::string n(name);
    auto host = [&](const void* src, int64_t bytes) -> int64_t {
        if (dst && cap >= bytes && bytes > 0) memcpy(dst, src, (size_t)bytes);
        return bytes;
    };
    auto dev = [&](const void* src, int64_t bytes) -> int64_t {
        if (dst && cap >= bytes && bytes > 0) {
            if (hipStreamSynchronize(c->sr) != hipSuccess) return -1;
            if (hipMemcpy(dst, src, (size_t)bytes, hipMemcpyDeviceToHost) != hipSuccess) return -1;
        }
        return bytes;
    };
    const PagedScene& ps = c->ps;
    const int64_t V = c->last_views ? c->last_views : 1;
    if (n == "info") {
        int64_t v[16] = {ps.n_pg, ps.P, ps.L, ps.bytes_g, ps.nc(), (int64_t)ps.link_dst.size(), c->S, c->frame,
                         c->TX, c->TY, (int64_t)c->cap_pairs, ps.store_bytes, c->last_n_render, c->last_n_pairs,
                         c->last_views, c->last_n_rl};
        return host(v, sizeof v);
    }
    if (n == "perm") return host(ps.perm.data(), 8 * (int64_t)ps.perm.size());
    if (n == "spheres") return host(ps.spheres.data(), 4 * (int64_t)ps.spheres.size());
    if (n == "cell_box") {
        const int64_t nc = ps.nc();
        if (dst && cap >= 24 * nc)
            for (int64_t i = 0; i < nc; ++i) {
                float* o = (float*)dst + 6 * i;
                for (int a = 0; a < 3; ++a) { o[a] = ps.cell_lo[(size_t)i * 4 + a]; o[3 + a] = ps.cell_hi[(size_t)i * 4 + a]; }
            }
        return 24 * nc;
    }
    if (n == "cell_page") return host(ps.cell_page.data(), 4 * ps.nc());
    if (n == "cell_start") return host(ps.cell_start.data(), 4 * (int64_t)ps.cell_start.size());
    if (n == "link_start") return host(ps.link_start.data(), 4 * (int64_t)ps.link_start.size());
    if (n == "link_dst") return host(ps.link_dst.data(), 4 * (int64_t)ps.link_dst.size());
    if (n == "host_page") return host(ps.rec[0].data(), 4 * (int64_t)ps.rec[0].size());
    if (n == "cand") return dev(c->d_cand, V * c->n_pg);
    if (n == "idbuf") return dev(c->d_idbuf, 8 * V * c->opt.idbuf_w * c->opt.idbuf_h);
    if (n == "req_direct") return dev(c->d_rd, 4 * (int64_t)c->n_pg);
    if (n == "req_link") return dev(c->d_rl, 4 * (int64_t)c->n_pg);
    if (n == "page_level") return dev(c->d_plevel, c->n_pg);
    if (n == "req_page") return host(c->out_req.data(), 4 * (int64_t)c->out_req.size());
    if (n == "slot_level") return dev(c->d_slot_level, c->S);
    if (n == "last_used") return dev(c->d_last_used, 4 * (int64_t)c->S);
    if (n == "sub_vpage") return dev(c->d_sub_vpage, 4 * (int64_t)c->S * SUBS);
    if (n == "sub_last_used") return dev(c->d_sub_lu, 4 * (int64_t)c->S * SUBS);
    if (n == "v2p") return dev(c->d_v2p, 4 * (int64_t)c->n_pg * c->L);
    if (n == "pf_keys") return c->pf_sorted ? dev(c->pf_sorted, 8 * (int64_t)c->last_n_pfreq) : 0;
    if (n == "pf_x") return c->d_pf_x ? dev(c->d_pf_x, 4 * (int64_t)c->last_views * (28 + c->pf.hist_bins)) : 0;
    if (n == "pf_logits")
        return c->pf_net ? dev(mlp_dev_of(c->pf_net)->logits, 4 * (int64_t)c->last_views * c->pf.n_clusters) : 0;
    if (n == "copies") return dev(c->d_copies, 24 * (int64_t)c->last_n_copy);
    if (n == "copy_id") return dev(c->d_copy_id, 16 * (int64_t)c->last_n_copy);
    if (n == "missing") return host(c->out_missing.data(), 4 * (int64_t)c->out_missing.size());
    if (n == "render_list") return dev(c->d_rlist, 16 * (int64_t)c->last_n_rl);
    const int64_t nt = (int64_t)c->last_n_render * c->last_views;
    if (n == "pp_float") {
        const int64_t bytes = 48 * nt;
        if (dst && cap >= bytes) {
            std::vector<float4> xy((size_t)nt);
            std::vector<float4> co((size_t)nt), rgb((size_t)nt);
            std::vector<uint32_t> dep((size_t)nt);
            hipStreamSynchronize(c->sr);
            hipMemcpy(xy.data(), c->d_xy, 16 * nt, hipMemcpyDeviceToHost);
            hipMemcpy(co.data(), c->d_conic, 16 * nt, hipMemcpyDeviceToHost);
            hipMemcpy(rgb.data(), c->d_rgb, 16 * nt, hipMemcpyDeviceToHost);
            hipMemcpy(dep.data(), c->d_depth, 4 * nt, hipMemcpyDeviceToHost);
            for (int64_t i = 0; i < nt; ++i) {
                float* f = (float*)dst + 12 * i;
                f[10] = xy[(size_t)i].w;   // support half height
                f[11] = xy[(size_t)i].z;   // support half width
                float d;
                memcpy(&d, &dep[(size_t)i], 4);
                f[0] = xy[(size_t)i].x; f[1] = xy[(size_t)i].y; f[2] = d;
                f[3] = co[(size_t)i].x; f[4] = co[(size_t)i].y; f[5] = co[(size_t)i].z; f[6] = co[(size_t)i].w;
                f[7] = rgb[(size_t)i].x; f[8] = rgb[(size_t)i].y; f[9] = rgb[(size_t)i].z;
            }
        }
        return bytes;
    }
    if (n == "pp_int") {
        const int64_t bytes = 24 * nt;
        if (dst && cap >= bytes) {
            std::vector<uint2> rc((size_t)nt);
            std::vector<uint32_t> dep((size_t)nt), til((size_t)nt);
            hipStreamSynchronize(c->sr);
            hipMemcpy(rc.data(), c->d_rect, 8 * nt, hipMemcpyDeviceToHost);
            hipMemcpy(dep.data(), c->d_depth, 4 * nt, hipMemcpyDeviceToHost);
            hipMemcpy(til.data(), c->d_tiles, 4 * nt, hipMemcpyDeviceToHost);
            for (int64_t i = 0; i < nt; ++i) {
                int32_t* q = (int32_t*)dst + 6 * i;
                q[0] = dep[(size_t)i] == 0xffffffffu ? 1 : 0;
                q[1] = (int32_t)(rc[(size_t)i].x & 0xffffu); q[2] = (int32_t)(rc[(size_t)i].x >> 16);
                q[3] = (int32_t)(rc[(size_t)i].y & 0xffffu); q[4] = (int32_t)(rc[(size_t)i].y >> 16);
                q[5] = (int32_t)til[(size_t)i];
            }
        }
        return bytes;
    }
    if (n == "keys") return dev(c->last_pk, 4 * (int64_t)c->last_n_pairs);
    if (n == "vals") return dev(c->last_pv, 4 * (int64_t)c->last_n_pairs);
    if (n == "ranges") return dev(c->d_ranges, 8 * (int64_t)c->TX * c->TY * V);
    if (n == "depth_order") return dev(c->d_dval[c->last_dbuf], 4 * nt);
    if (n == "blend_stats") return host(c->h_bstats, 8 * (int64_t)c->TX * c->TY * V);
    return -1;
}

}  // extern "C"
