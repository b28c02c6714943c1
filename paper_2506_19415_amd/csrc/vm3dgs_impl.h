// vm3dgs_impl.h -- internal declarations of the VM-3DGS library (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/vm3dgs.h"

namespace vm {

constexpr int REC = 59;   // floats per Gaussian record
constexpr int SUBS = 64;  // sub-slots per physical page
constexpr uint32_t EMIT_SPAN = 1024;  // pairs per workgroup of the pair emission

// vm3dgs_frame_noalloc: the (tile, Gaussian) pair buffers of a frame live in
// a fixed device array of kNoallocScratchBytes per GPU (scratch.hip), laid
// out as the look-back status words of the pair sort, then keys and values
// (two of each, ping-pong), then the emission block starts.  It holds
// kNoallocPairs pairs.
constexpr uint64_t kNoallocScratchBytes = 128ull << 20;
constexpr uint64_t kNoallocPairs = VM3DGS_NOALLOC_MAX_PAIRS;   // 7.5 Mi
// the current device's scratch address, looked up once per device
hipError_t noalloc_scratch(void** out);

// ----------------------------------------------------------- create time
struct PagedScene {
    int64_t n_in = 0;
    int P = 0, L = 1, n_pg = 0, fmt = 0, bytes_g = 236;
    double lo[3] = {0, 0, 0};
    std::vector<int64_t> perm;         // [n_pg*P] input index, -1 = padding
    std::vector<float> rec[3];         // decoded records per level [n_pg*P_l][59]
    std::vector<float> spheres;        // [n_pg][4]
    std::vector<float> cell_lo, cell_hi;  // [nc][4]; lo.w = page id as float bits
    std::vector<int32_t> cell_page, cell_start;  // [nc], [n_pg+1]
    std::vector<int32_t> link_start, link_dst;   // [n_pg+1], [n_links]
    int64_t level_base[3] = {0, 0, 0};  // byte offset of each level in the host store
    int64_t store_bytes = 0;
    int P_l(int l) const { return P >> (3 * l); }
    int64_t nc() const { return (int64_t)cell_page.size(); }
};

// Builds everything of Sec. 3 for the library; returns "" or an error text.
std::string build_paged_scene(const vm3dgs_scene& sc, int page_size, int lod_levels, int fmt, double cell_m,
                              double link_sigma, double lod_scale_up, int lod_builder, PagedScene& out);
// Writes the page-major SoA store of every level into dst (store_bytes).
void encode_store(const PagedScene& ps, uint8_t* dst);

// ----------------------------------------------------------- device sort/scan
// Workspace of the single-pass sorts and scans of one frame.  reset() is
// called when the frame's zero-fill of `zero_base` (counters, histograms,
// tickets) has been enqueued; every launch then takes the next histogram
// block, ticket and epoch.
struct SortWork {
    uint64_t* status = nullptr;   // look-back status words (no clearing needed)
    uint32_t* hist = nullptr;     // [kMaxHist][256], zeroed per frame
    uint32_t* tickets = nullptr;  // [kMaxTickets], zeroed per frame
    uint32_t* err = nullptr;      // look-back spin overrun flag
    static constexpr int kMaxHist = 64;
    static constexpr int kMaxTickets = 128;
    int hist_used = 0, tickets_used = 0;
    uint32_t epoch = 0;
    void reset() { hist_used = 0; tickets_used = 0; }
    uint32_t* next_hist(int n) {
        if (hist_used + n > kMaxHist) throw std::length_error("sort histograms of one frame exhausted");
        uint32_t* p = hist + 256 * (size_t)hist_used;
        hist_used += n;
        return p;
    }
    uint32_t* next_ticket() {
        if (tickets_used >= kMaxTickets) throw std::length_error("sort tickets of one frame exhausted");
        return tickets + tickets_used++;
    }
    uint32_t next_epoch() { epoch = (epoch + 1) & 0x3fffffffu; if (epoch == 0) epoch = 1; return epoch; }
};
size_t lb_status_words(uint64_t n_keys);
int onesweep_u32(hipStream_t st, SortWork& w, uint32_t* keys[2], uint32_t* vals[2], uint32_t n, int begin_bit,
                 int end_bit);
// the same with the key count on the device (at most n_bound, which sizes the grid)
int onesweep_u32_dev(hipStream_t st, SortWork& w, uint32_t* keys[2], uint32_t* vals[2], uint32_t n_bound,
                     const uint32_t* n_dev, int begin_bit, int end_bit);
int onesweep_u64(hipStream_t st, SortWork& w, uint64_t* keys[2], uint32_t* vals[2], uint32_t n, int begin_bit,
                 int end_bit);
int onesweep_u64_dev(hipStream_t st, SortWork& w, uint64_t* keys[2], uint32_t* vals[2], uint32_t n_bound,
                     const uint32_t* n_dev, int begin_bit, int end_bit);
// keys only by one workgroup in one launch (the result in keys[returned
// index], as above), for counts up to a few thousand, where the onesweep
// passes are bound by their launches; its result is the stable sort's when
// keys that agree on the sorted bits are equal (up to 8192 keys it sorts
// without keeping their order)
int sort_small_u64(hipStream_t st, uint64_t* keys[2], uint32_t n_bound, const uint32_t* n_dev, int begin_bit,
                   int end_bit);
// counts up to which sort_small_u64 beats the onesweep passes
constexpr uint32_t kSortSmallMax = 8192;
void scan_lb(hipStream_t st, SortWork& w, const uint32_t* in, uint64_t n, uint32_t* out, uint32_t* total);
void scan_lb_gather(hipStream_t st, SortWork& w, const uint32_t* a, const uint32_t* idx, uint64_t n, uint32_t* out,
                    uint32_t* total);

// ----------------------------------------------------------- kernels' camera
struct CamK {
    float V[12];       // rows of the world->camera transform
    float pos[3];
    float fx, fy, cx, cy, znear;
};

// Counters written by the page-table kernels and read back once per frame.
enum Ctr {
    C_NREQ = 0, C_DIRECT, C_LINKED, C_HITS, C_MISSES, C_EVICT, C_NCOPY, C_NMISSING, C_NRL, C_NRENDER,
    C_CAND, C_POOLUSED, C_NCAND1, C_NCAND2, C_NPFREQ, C_NPF,
    C_REQSLOTS,   // physical pages required after the demand stages
    C_NCOARSE,    // requests at a level above 0
    C_PTERR,      // page-table bound check (never set when the host checks hold)
    C_FALLBACK,   // streaming: requests drawn at another resident level
    C_NMISSCAP,   // LOD table: requests left missing for want of a free pool entry
    C_NCOUNTERS = 24
};

struct RenderEntry {   // one resident requested (sub-)page in render order
    uint32_t pool_off;  // first Gaussian of the block in the pool (Gaussian units)
    uint32_t count;     // Gaussians in the block
    uint32_t base;      // first render index
    uint32_t level;
};

struct CopyCmd {
    int64_t host_off, pool_off, bytes;
};

// ----------------------------------------------------------- launchers
struct VisArgs {
    const float4* spheres; int n_pg;
    const float4* cell_lo; const float4* cell_hi; int64_t nc;
    const int32_t* link_start; const int32_t* link_dst; int use_links;
    const CamK* cams; int n_views;
    int W, H, Wv, Hv, L; float tau; float fy_max; float guard;
    uint8_t* cand; float4* rays; unsigned long long* idbuf;
    uint32_t* req_direct; uint32_t* req_link; int8_t* page_level;
    uint64_t* req_keys; uint32_t* counters;
    int4* cell_rects; uint32_t* cell_area; uint32_t* cell_offs;  // [views*nc], [views*nc], [views*nc + 1]
    SortWork* sw;
};
void launch_visibility(hipStream_t st, const VisArgs& a);

struct PtArgs {
    const uint64_t* req_keys; int n_pg, L, P, S, frame, budget, bytes_g;
    const int8_t* page_level;
    int8_t* slot_level; int32_t* last_used; int32_t* sub_vpage; int32_t* sub_last_used; int32_t* v2p;
    uint8_t* req_sub; uint8_t* slot_req; uint32_t* miss;
    CopyCmd* copies; int32_t* copy_id; int32_t* missing; uint32_t* counters;
    const int64_t* level_base;  // device [3]
    RenderEntry* rl;
    // streaming: the frame renders what was resident when it started (a page
    // resident only at another level at the nearest one); rlevel [n_pg] is
    // the level each requested page is drawn at (several levels only)
    int streaming; int8_t* rlevel;
    // the last frame's request and level-1/2 candidate counts (all ones:
    // none yet); the LOD table sorts such lists by one workgroup when the
    // last frame's fitted
    uint32_t hint_req = ~0u, hint_cand[3] = {~0u, ~0u, ~0u};
};
void launch_pagetable(hipStream_t st, const PtArgs& a, int n_req_host_bound);

// scratch of the LOD page table
struct LodWork {
    uint64_t* keys_alt;     // [n_pg] sort ping-pong for the requests
    uint64_t* keys_out;     // [n_pg] requests in service order (read back)
    int8_t* level_out;      // [n_pg] their levels (read back)
    uint32_t* flag;         // [n_pg]
    uint32_t* pos;          // [n_pg + 1]
    uint32_t* flag2;        // [n_pg] streaming: misses with a resident level (served last)
    uint32_t* pos2;         // [n_pg + 1]
    uint64_t* wkeys[2];     // [S] x 2
    uint64_t* ck[3][2];     // per level 1, 2: [S*64] x 2
    int32_t* fresh;         // [3][S]
};
void launch_pagetable_lod(hipStream_t st, const PtArgs& a, SortWork& sw, const LodWork& w);

struct SplatArgs {
    const RenderEntry* rl; int n_rl;
    const uint8_t* pool; int P; int fmt;
    const CamK* cams; int n_views;
    int W, H, TX, TY;
    uint32_t n_render;  // per view
    int sigma3_tiles;   // 1: 3-sigma tile rectangles only (no support box)
    float4* xy; float4* conic; float4* rgb; uint32_t* depth; uint2* rect; uint32_t* tiles;
    uint32_t* dkey; uint32_t* dval;
};
void launch_preprocess(hipStream_t st, const SplatArgs& a);
// the same with the render set's size read on the device (*n_render_dev
// Gaussians per view in *n_rl_dev entries, at most max_total in all): it is
// queued before the host has read the page table's counters
void launch_preprocess_dev(hipStream_t st, const SplatArgs& a, const uint32_t* n_render_dev, const uint32_t* n_rl_dev,
                           uint64_t max_total);
// pairs counted on the device (*n_pairs_dev); the grids cover the capacity cap
void launch_emit(hipStream_t st, const uint32_t* order, const uint32_t* offsets, const uint32_t* tiles,
                 const uint2* rect, uint32_t* starts, uint32_t n_total, const uint32_t* n_pairs_dev, uint32_t n_render,
                 int TX, int TY, uint32_t* pkey, uint32_t* pval, uint32_t cap);
void launch_ranges(hipStream_t st, const uint32_t* pkey, uint32_t cap, const uint32_t* n_pairs_dev, uint2* ranges,
                   uint32_t n_tiles);
// order: n_tiles + 2 words (the blend order, then the number of long tiles
// and of the longest ones)
void launch_tile_order(hipStream_t st, const uint2* ranges, uint32_t n_tiles, uint32_t* order);
// the blend of the tiles in order, in two launches that may run side by
// side and must be given the same x_cap: launch_blend_x takes the first
// tiles, those with 16384 pairs or more (at most x_cap of them; alpha band
// walk, four workgroups each), launch_blend the others (band walk for those
// with 4096 pairs or more, strip walk for the rest).  stats (or null): per
// tile, the visited list entries and the alpha evaluations, added to
// (cleared by the caller)
void launch_blend(hipStream_t st, const uint2* ranges, const uint32_t* order, const uint32_t* pval, const float4* xy,
                  const float4* conic, const float4* rgb, int W, int H, int TX, int TY, int n_views, uint32_t x_cap,
                  float* image, uint2* stats);
void launch_blend_x(hipStream_t st, const uint2* ranges, const uint32_t* order, const uint32_t* pval,
                    const float4* xy, const float4* conic, const float4* rgb, int W, int H, int TX, int TY,
                    int n_views, uint32_t x_cap, float* image, uint2* stats);
// room for want such tiles of n_tiles (a multiple of 8, at most the walk's limit)
uint32_t blend_x_cap(uint32_t n_tiles, uint32_t want);
// fills done together in one launch (at most kMax)
struct FillSeg {
    void* p; uint64_t n; uint64_t v; int wide;   // wide: 8-byte words, else 4-byte
};
struct FillSegs {
    static constexpr int kMax = 8;
    FillSeg seg[kMax];
    int n = 0;
};
void launch_fill_multi(hipStream_t st, const FillSegs& f);
// device-to-host readbacks at one point of a stream, in one launch: the GPU
// writes each segment into mapped pinned host memory (at most kMax)
struct ReadSeg {
    const void* src; void* dst; uint32_t bytes;   // dst: device address of pinned host memory
};
struct ReadSegs {
    static constexpr int kMax = 8;
    ReadSeg seg[kMax];
    int n = 0;
};
void launch_readback(hipStream_t st, const ReadSegs& r);
void visibility_clears(const VisArgs& a, FillSegs& f);
void launch_fill_u32(hipStream_t st, uint32_t* p, uint64_t n, uint32_t v);
void launch_fill_u64(hipStream_t st, unsigned long long* p, uint64_t n, unsigned long long v);


// ---------------------------------------------------------------- prefetch network
// Device state of the network (k_mlp.hip).  Layer l maps dims[l] -> dims[l+1];
// act[l] is its bf16 input [b_pad][kpad[l]] (kpad = dims rounded up to 32,
// the padding columns and the rows past the batch are zero), dz[l] the bf16
// gradient of its output [b_pad][dims[l+1]], wb[l] its bf16 weights
// [kpad[l]][dims[l+1]] (padding rows zero).  master/adam_m/adam_v/grad use
// the parameter layout: per layer W [dims[l]][dims[l+1]] then b.
struct MlpDev {
    int n_layers = 0;
    int dims[9] = {};
    int kpad[9] = {};
    int64_t off[9] = {};
    int b_pad = 0;
    float* master = nullptr; float* adam_m = nullptr; float* adam_v = nullptr; float* grad = nullptr;
    uint16_t* wb[8] = {};
    uint16_t* act[8] = {};
    uint16_t* dz[8] = {};
    float* logits = nullptr;
    float* loss_part = nullptr;
};
void mlp_input_dev(hipStream_t st, const MlpDev& d, const float* x, int B);
void mlp_forward_dev(hipStream_t st, const MlpDev& d, int B);
void mlp_backward_dev(hipStream_t st, const MlpDev& d, const float* y, int B);
void mlp_adam_dev(hipStream_t st, const MlpDev& d, float lr, float b1, float b2, float eps, int t);
void mlp_sync_bf16_dev(hipStream_t st, const MlpDev& d);


// learned prefetch (k_prefetch.hip)
struct PfArgs {
    const float* logits; int K; float thr;
    const int8_t* page_level; int32_t* v2p; const float4* sph; int n_pg, L; float tau, fy;
    const CamK* cams; int n_views;
    uint64_t* keys[2]; uint64_t* idle[2];
    int S, P, frame, budget, bytes_g;
    const int64_t* level_base;
    int8_t* slot_level; int32_t* last_used; int32_t* sub_vpage; int32_t* sub_last_used; int32_t* fresh;
    CopyCmd* copies; int32_t* copy_id; uint32_t* counters;
    const uint64_t** sorted_out;   // receives the buffer holding the sorted proposals
};
void launch_pf_features(hipStream_t st, const int32_t* v2p, int n_pg, int L, int H, int n_views, float* x);
void launch_prefetch(hipStream_t st, const PfArgs& a, SortWork& sw);
const MlpDev* mlp_dev_of(const vm3dgs_mlp* net);
int mlp_max_batch_of(const vm3dgs_mlp* net);
hipStream_t mlp_stream_of(const vm3dgs_mlp* net);
// rows idx[i] of src [.][width] into dst [n][width] (k_mlp.hip)
void launch_gather_rows(hipStream_t st, const float* src, const uint32_t* idx, uint32_t n, uint32_t width,
                        float* dst);
// the prefetch stage of a context: its network (or NULL) and options; false without a stage
bool prefetch_stage_of(const vm3dgs* ctx, vm3dgs_mlp** net, vm3dgs_prefetch_opts* opts);

// a range of copy commands whose bounds the kernel reads on the device: of
// *n_copy commands the last *n_pf (none when n_pf is null) are prefetches;
// prefetch 0 takes the others (the demand copies), 1 the prefetches
struct CopyRangeDev {
    const uint32_t* n_copy = nullptr;
    const uint32_t* n_pf = nullptr;
    int prefetch = 0;
};
// total bytes of the commands of such a range (at most max_count) into *out
void launch_copy_bytes_dev(hipStream_t st, const CopyCmd* cmds, CopyRangeDev r, uint32_t max_count,
                           unsigned long long* out);
// copies of the misses of such a range by the GPU from the pinned host store
// (16 KB chunks, workgroups striding over them); bytes_done accumulates the
// bytes copied, err is set by a command outside the store or the pool
void launch_copy_pages_dev(hipStream_t st, const CopyCmd* cmds, CopyRangeDev r, uint32_t max_count,
                           uint64_t max_cmd_bytes, const uint8_t* host, uint64_t host_bytes, uint8_t* pool,
                           uint64_t pool_bytes, unsigned long long* bytes_done, uint32_t* err);

}  // namespace vm
