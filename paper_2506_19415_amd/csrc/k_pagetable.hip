// k_pagetable.hip -- page table of Sec. 4.1.1 on the device.
//
// Stage one walks the required pages: hits mark their physical page as
// required and refresh its last use; the rest are misses, kept in request
// order (class, depth, page).  Stage two places the misses into physical
// pages that are not required this frame, least recently used first (ties to
// the lower physical page), evicting what they held, and lists the copies;
// misses beyond the free pages or the copy budget become "missing".  The
// render list then holds the resident required pages in page order.
//
// One LOD level: everything in one 1024-thread workgroup (requests sorted by
// a bitonic network in LDS, hits and placements in parallel).  Several LOD
// levels: the placement of a miss depends on the ones before it (sub-slots
// of a physical page fill up), so one wave walks the misses in order over
// candidate lists sorted beforehand.
#include <algorithm>
#include <stdexcept>

#include "kcommon.h"
#include "vm3dgs_impl.h"

namespace vmk {

using vm::CopyCmd;
using vm::RenderEntry;

constexpr int PT_NT = 1024;
constexpr int PT_MAXK = 8192;  // requests / slots sorted in LDS
constexpr int RL_SEG = 65536;  // pages per segment of the LOD render list (one byte each in LDS)

// ascending bitonic sort of n (power of two, <= PT_MAXK) keys in LDS
__device__ void bitonic_lds(uint64_t* s, int n) {
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n; i += PT_NT) {
                const int l = i ^ j;
                if (l > i) {
                    const uint64_t a = s[i], b = s[l];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) { s[i] = b; s[l] = a; }
                }
            }
            __syncthreads();
        }
    }
}

__device__ int pow2_at_least(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

struct PtL1 {
    uint64_t* keys_sorted;  // out: requests in service order
    int n_pg, P, S, frame, budget, bytes_g, streaming;
    const int8_t* page_level;
    int8_t* slot_level; int32_t* last_used; int32_t* sub_vpage; int32_t* sub_last_used; int32_t* v2p;
    uint8_t* slot_req; uint32_t* miss;
    CopyCmd* copies; int32_t* copy_id; int32_t* missing; uint32_t* counters;
    RenderEntry* rl;
};

// requested pages resident now, in page order; returns their number
__device__ uint32_t l1_render_list(const PtL1& a, uint32_t* scan_sh) {
    const int t = threadIdx.x;
    uint32_t n_rl = 0;
    for (int base = 0; base < a.n_pg; base += PT_NT) {
        const int p = base + t;
        bool r = false;
        int32_t e = -1;
        if (p < a.n_pg && a.page_level[p] >= 0) {
            e = a.v2p[p];
            r = e >= 0;
        }
        uint32_t tot;
        const uint32_t ex = block_excl_scan<PT_NT>(r ? 1u : 0u, scan_sh, &tot);
        if (r) {
            RenderEntry q;
            q.pool_off = (uint32_t)((e / vmk::SUBS) * a.P);
            q.count = (uint32_t)a.P;
            q.base = (n_rl + ex) * (uint32_t)a.P;
            q.level = 0;
            a.rl[n_rl + ex] = q;
        }
        n_rl += tot;
        __syncthreads();
    }
    return n_rl;
}

__global__ __launch_bounds__(PT_NT) void k_pagetable_l1(const uint64_t* __restrict__ req_keys, PtL1 a) {
    __shared__ uint64_t s[PT_MAXK];
    __shared__ uint32_t scan_sh[PT_NT / WAVE];
    __shared__ uint32_t s_cnt[4];
    const int t = threadIdx.x;
    const int n = (int)a.counters[vm::C_NREQ];
    if (n > PT_MAXK || a.S > PT_MAXK) {   // host checks these bounds; never reached
        if (t == 0) a.counters[vm::C_PTERR] = 1;
        return;
    }
    if (t < 4) s_cnt[t] = 0;
    // ---- requests in service order
    const int np2 = pow2_at_least(n > 1 ? n : 1);
    for (int i = t; i < np2; i += PT_NT) s[i] = i < n ? req_keys[i] : ~0ull;
    __syncthreads();
    bitonic_lds(s, np2);
    for (int i = t; i < n; i += PT_NT) a.keys_sorted[i] = s[i];
    for (int i = t; i < a.S; i += PT_NT) a.slot_req[i] = 0;
    __syncthreads();
    // ---- stage 1: hits refresh last use; misses keep request order
    uint32_t n_miss = 0;
    for (int base = 0; base < n; base += PT_NT) {
        const int i = base + t;
        bool miss = false;
        int32_t p = 0;
        if (i < n) {
            p = (int32_t)(s[i] & 0x3fffffffull);
            const int32_t e = a.v2p[p];
            if (e >= 0) {
                const int sl = e / vmk::SUBS;
                a.slot_req[sl] = 1;
                a.last_used[sl] = a.frame;
                a.sub_last_used[e] = a.frame;
            } else {
                miss = true;
            }
        }
        uint32_t tot;
        const uint32_t ex = block_excl_scan<PT_NT>(miss ? 1u : 0u, scan_sh, &tot);
        if (miss) a.miss[n_miss + ex] = (uint32_t)p;
        n_miss += tot;
    }
    __syncthreads();
    // streaming: the frame renders the pages resident when it started (the
    // placements below only take pages no request of this frame holds)
    uint32_t n_rl = 0;
    if (a.streaming) n_rl = l1_render_list(a, scan_sh);
    // ---- stage 2 candidates: physical pages not required, (last use, slot) ascending
    uint64_t* cand = s;
    uint32_t n_free = 0;
    for (int base = 0; base < a.S; base += PT_NT) {
        const int sl = base + t;
        const bool fr = sl < a.S && a.slot_req[sl] == 0;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<PT_NT>(fr ? 1u : 0u, scan_sh, &tot);
        if (fr) cand[n_free + ex] = ((uint64_t)(uint32_t)(a.last_used[sl] + 1) << 32) | (uint32_t)sl;
        n_free += tot;
    }
    __syncthreads();
    {
        const int np = pow2_at_least(n_free > 1 ? (int)n_free : 1);
        for (int i = (int)n_free + t; i < np; i += PT_NT) cand[i] = ~0ull;
        __syncthreads();
        bitonic_lds(cand, np);
    }
    __syncthreads();
    uint32_t n_take = n_miss < n_free ? n_miss : n_free;
    if (a.budget > 0 && n_take > (uint32_t)a.budget) n_take = (uint32_t)a.budget;
    // ---- placements (independent with one level)
    for (uint32_t i = t; i < n_miss; i += PT_NT) {
        const int32_t p = (int32_t)a.miss[i];
        if (i < n_take) {
            const int sl = (int)(cand[i] & 0xffffffffull);
            const int32_t old = a.sub_vpage[sl * vmk::SUBS];
            if (old >= 0) {
                a.v2p[old] = -1;
                atomicAdd(&s_cnt[0], 1u);
            }
            a.sub_vpage[sl * vmk::SUBS] = p;
            a.sub_last_used[sl * vmk::SUBS] = a.frame;
            a.last_used[sl] = a.frame;
            a.slot_level[sl] = 0;
            a.v2p[p] = sl * vmk::SUBS;
            CopyCmd c;
            c.host_off = (int64_t)p * a.P * a.bytes_g;
            c.pool_off = (int64_t)sl * a.P * a.bytes_g;
            c.bytes = (int64_t)a.P * a.bytes_g;
            a.copies[i] = c;
            a.copy_id[4 * i] = p; a.copy_id[4 * i + 1] = 0; a.copy_id[4 * i + 2] = sl; a.copy_id[4 * i + 3] = 0;
        } else {
            a.missing[2 * (i - n_take)] = p;
            a.missing[2 * (i - n_take) + 1] = 0;
        }
    }
    __syncthreads();
    __threadfence_block();
    // ---- render list: requested and resident pages in page order (streaming:
    // built above, before the placements)
    if (!a.streaming) n_rl = l1_render_list(a, scan_sh);
    uint32_t used = 0;
    for (int sl = t; sl < a.S; sl += PT_NT) used += a.sub_vpage[sl * vmk::SUBS] >= 0 ? 1u : 0u;
    used = wave_sum(used);
    if (__lane_id() == 0) atomicAdd(&s_cnt[1], used);
    __syncthreads();
    if (t == 0) {
        a.counters[vm::C_HITS] = (uint32_t)n - n_miss;
        a.counters[vm::C_MISSES] = n_miss;
        a.counters[vm::C_EVICT] = s_cnt[0];
        a.counters[vm::C_NCOPY] = n_take;
        a.counters[vm::C_NMISSING] = n_miss - n_take;
        a.counters[vm::C_NRL] = n_rl;
        a.counters[vm::C_REQSLOTS] = n_rl;   // one level: one physical page per render entry
        a.counters[vm::C_NRENDER] = n_rl * (uint32_t)a.P;
        a.counters[vm::C_POOLUSED] = s_cnt[1];
    }
}

// ------------------------------------------------------------------ LOD path
// Several levels: a level-l physical page holds 8^l sub-pages.  Candidate
// lists are built and sorted in parallel; one thread then places the misses
// in request order (each placement can change what the next one finds).

// stage 1 over the sorted requests: hits, miss flags (request order kept)
// unused key slots past the compacted requests sort last
// Streaming: a miss whose page is resident at another level is drawn at the
// resident level nearest to the requested one (the finer at equal distance),
// that entry is required too, and it is flagged in flag2 (served after the
// other misses); rlevel receives the level each request is drawn at.  Two
// requests never name one page, so the marks of different threads are of
// different entries (the byte and int stores of equal values to one physical
// page's flags and last use are the same values).
__global__ void k_ptl_hits(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ counters,
                           const int8_t* __restrict__ page_level, int n_pg, int L, const int32_t* __restrict__ v2p,
                           uint8_t* __restrict__ req_sub, uint8_t* __restrict__ slot_req,
                           int32_t* __restrict__ last_used, int32_t* __restrict__ sub_last_used, int frame,
                           uint32_t* __restrict__ miss_flag, uint64_t* __restrict__ keys_out,
                           int8_t* __restrict__ level_out, int streaming, uint32_t* __restrict__ miss_flag2,
                           int8_t* __restrict__ rlevel) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pg) return;
    const uint32_t n = counters[vm::C_NREQ];
    uint32_t flag = 0, flag2 = 0;
    if ((uint32_t)i < n) {
        const uint64_t key = keys[i];
        const int32_t pg = (int32_t)(key & 0x3fffffffull);
        const int l = page_level[pg];
        keys_out[i] = key;
        level_out[i] = (int8_t)l;
        int32_t e = v2p[pg * L + l];
        int drawn = e >= 0 ? l : -1;
        if (e < 0 && streaming) {
            for (int d = 1; d < L && drawn < 0; ++d) {
                if (l - d >= 0 && v2p[pg * L + l - d] >= 0) drawn = l - d;
                else if (l + d < L && v2p[pg * L + l + d] >= 0) drawn = l + d;
            }
            if (drawn >= 0) e = v2p[pg * L + drawn];
        }
        if (e >= 0) {
            req_sub[e] = 1;
            slot_req[e / vmk::SUBS] = 1;
            last_used[e / vmk::SUBS] = frame;
            sub_last_used[e] = frame;
        }
        if (drawn != l) {
            flag = drawn < 0 ? 1u : 0u;
            flag2 = drawn < 0 ? 0u : 1u;
        }
        if (streaming) rlevel[pg] = (int8_t)drawn;
    }
    miss_flag[i] = flag;
    if (streaming) miss_flag2[i] = flag2;
}

// misses in service order: request order, and with streaming the misses
// drawn at another level (flag2, positions pos2 after the first list's total)
__global__ void k_ptl_miss_list(const uint64_t* __restrict__ keys, const int8_t* __restrict__ page_level, int n_pg,
                                const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                                const uint32_t* __restrict__ flag2, const uint32_t* __restrict__ pos2,
                                uint32_t* __restrict__ miss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pg) return;
    const uint32_t pg = (uint32_t)(keys[i] & 0x3fffffffull);
    if (flag[i]) miss[pos[i]] = pg | ((uint32_t)page_level[pg] << 30);
    else if (flag2 && flag2[i]) miss[pos[n_pg] + pos2[i]] = pg | ((uint32_t)page_level[pg] << 30);
}

// candidate keys: whole free pages (last use + 1, slot; all-ones for required
// pages, which sort last) and, per level l >= 1, the non-required sub-slots
// of level-l pages (0 for empty else last use + 1, slot * 64 + sub), listed
// in counters[C_NCAND1 / C_NCAND2] entries
__global__ void k_ptl_cand_keys(int S, int L, int idx_bits, const int8_t* __restrict__ slot_level,
                                const int32_t* __restrict__ last_used, const int32_t* __restrict__ sub_vpage,
                                const int32_t* __restrict__ sub_last_used, const uint8_t* __restrict__ req_sub,
                                const uint8_t* __restrict__ slot_req, uint64_t* __restrict__ wkeys,
                                uint64_t* __restrict__ ck1, uint64_t* __restrict__ ck2, uint32_t* __restrict__ counters) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)S * vmk::SUBS) return;
    const int s = (int)(i / vmk::SUBS), j = (int)(i % vmk::SUBS);
    if (j == 0)
        wkeys[s] = slot_req[s] ? ~0ull : (((uint64_t)(uint32_t)(last_used[s] + 1) << idx_bits) | (uint64_t)s);
    const int l = slot_level[s];
    bool ok1 = false, ok2 = false;
    uint64_t key = ~0ull;
    if (l >= 1 && j < (1 << (3 * l)) && !req_sub[i]) {
        const uint32_t k1 = sub_vpage[i] < 0 ? 0u : (uint32_t)(sub_last_used[i] + 1);
        key = ((uint64_t)k1 << idx_bits) | (uint64_t)i;
        ok1 = l == 1;
        ok2 = l == 2;
    }
    // appended, wave by wave, to the level's list (its sort restores the order)
    const uint64_t b1 = __ballot(ok1), b2 = __ballot(ok2);
    uint32_t base1 = 0, base2 = 0;
    if (__lane_id() == 0) {
        if (b1) base1 = atomicAdd(&counters[vm::C_NCAND1], (uint32_t)__popcll(b1));
        if (b2) base2 = atomicAdd(&counters[vm::C_NCAND2], (uint32_t)__popcll(b2));
    }
    base1 = (uint32_t)__shfl((int)base1, 0, WAVE);
    base2 = (uint32_t)__shfl((int)base2, 0, WAVE);
    const uint64_t lt = lanemask_lt();
    if (ok1) ck1[base1 + (uint32_t)__popcll(b1 & lt)] = key;
    if (ok2) ck2[base2 + (uint32_t)__popcll(b2 & lt)] = key;
}

struct PtWalk {
    const uint32_t* miss; const uint64_t* wkeys; const uint64_t* ck[3];
    int S, L, P, frame, budget, bytes_g;
    uint64_t idx_mask;
    const int64_t* level_base;
    int8_t* slot_level; int32_t* last_used; int32_t* sub_vpage; int32_t* sub_last_used; int32_t* v2p;
    uint8_t* req_sub; uint8_t* slot_req; int32_t* fresh;   // fresh: [3][S]
    CopyCmd* copies; int32_t* copy_id; int32_t* missing; uint32_t* counters;
};

// One wave: the misses in request order over the sorted candidate lists.  The
// walk's state is uniform (every lane computes it alike and stores the same
// values); the scans of a candidate list read 64 entries at a time and take the
// first usable one by ballot, and the sub-slots of a physical page are read and
// cleared one per lane.
__device__ __forceinline__ int lane_i(int x, int i) { return __builtin_amdgcn_readlane(x, i); }

__global__ __launch_bounds__(WAVE) void k_ptl_walk(PtWalk a) {
    if (blockIdx.x != 0) return;
    const int lane = (int)__lane_id();
    const uint32_t n_miss = a.counters[vm::C_MISSES];
    const uint32_t n_s = (uint32_t)a.S;
    const uint32_t ncl[3] = {0u, a.counters[vm::C_NCAND1], a.counters[vm::C_NCAND2]};
    uint32_t pw = 0, pc[3] = {0, 0, 0}, fn[3] = {0, 0, 0}, fh[3] = {0, 0, 0};
    uint32_t n_copy = 0, n_missing = 0, n_missing_cap = 0, evict = 0;
    for (uint32_t i = 0; i < n_miss; ++i) {
        const uint32_t m = a.miss[i];
        const int32_t p = (int32_t)(m & 0x3fffffffu);
        const int l = (int)(m >> 30);
        if (a.budget > 0 && n_copy >= (uint32_t)a.budget) {
            a.missing[2 * n_missing] = p; a.missing[2 * n_missing + 1] = l; ++n_missing;
            continue;
        }
        int ts = -1, tj = -1;
        const int cap = 1 << (3 * l);
        if (l > 0) {
            // (1) non-required sub-slots of level-l pages, in candidate order
            while (pc[l] < ncl[l]) {
                const uint32_t k = pc[l] + (uint32_t)lane;
                int idx = 0;
                bool ok = false;
                if (k < ncl[l]) {
                    idx = (int)(a.ck[l][k] & a.idx_mask);
                    ok = a.slot_level[idx / vmk::SUBS] == l && !a.req_sub[idx];
                }
                const uint64_t b = __builtin_amdgcn_ballot_w64(ok);
                if (b != 0) {
                    const int f = (int)__builtin_ctzll(b);
                    const int id = lane_i(idx, f);
                    ts = id / vmk::SUBS; tj = id % vmk::SUBS;
                    pc[l] += (uint32_t)f + 1u;
                    break;
                }
                pc[l] = min(pc[l] + (uint32_t)WAVE, ncl[l]);
            }
            // (2) remaining sub-slots of pages converted to level l in this frame
            while (ts < 0 && fh[l] < fn[l]) {
                const int s = a.fresh[l * a.S + fh[l]];
                bool ok = false;
                if (a.slot_level[s] == l && lane < cap)
                    ok = !a.req_sub[s * vmk::SUBS + lane] && a.sub_vpage[s * vmk::SUBS + lane] < 0;
                const uint64_t b = __builtin_amdgcn_ballot_w64(ok);
                if (b != 0) { ts = s; tj = (int)__builtin_ctzll(b); } else ++fh[l];
            }
        }
        if (ts < 0) {
            // (3) the least recently used wholly free physical page
            while (pw < n_s) {
                const uint32_t k = pw + (uint32_t)lane;
                const uint64_t wk = k < n_s ? a.wkeys[k] : ~0ull;
                const bool real = wk != ~0ull;
                const int s = real ? (int)(wk & a.idx_mask) : 0;
                const bool ok = real && !a.slot_req[s];
                const uint64_t b_end = __builtin_amdgcn_ballot_w64(!real);
                const uint64_t b_ok = __builtin_amdgcn_ballot_w64(ok);
                // usable entries before the first all-ones key (the end of the list)
                const uint64_t before_end = b_end != 0 ? ((1ull << __builtin_ctzll(b_end)) - 1ull) : ~0ull;
                const uint64_t b = b_ok & before_end;
                if (b != 0) {
                    const int f = (int)__builtin_ctzll(b);
                    ts = lane_i(s, f); tj = 0;
                    pw += (uint32_t)f + 1u;
                    break;
                }
                if (b_end != 0) { pw = n_s; break; }
                pw += (uint32_t)WAVE;
            }
            if (ts >= 0) {
                const int oldl = a.slot_level[ts];
                bool ev = false;
                if (oldl >= 0 && lane < (1 << (3 * oldl))) {
                    const int32_t op = a.sub_vpage[ts * vmk::SUBS + lane];
                    if (op >= 0) { a.v2p[op * a.L + oldl] = -1; ev = true; }
                }
                evict += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(ev));
                a.sub_vpage[ts * vmk::SUBS + lane] = -1;
                a.sub_last_used[ts * vmk::SUBS + lane] = -1;
                __threadfence_block();   // the cleared sub-slots before any lane reads them again
                a.slot_level[ts] = (int8_t)l;
                if (l > 0) a.fresh[l * a.S + fn[l]] = ts;
                if (l > 0) ++fn[l];
            }
        }
        if (ts < 0) {   // no free pool entry
            a.missing[2 * n_missing] = p; a.missing[2 * n_missing + 1] = l; ++n_missing;
            ++n_missing_cap;
            continue;
        }
        const int e = ts * vmk::SUBS + tj;
        const int32_t old = a.sub_vpage[e];
        if (old >= 0) { a.v2p[old * a.L + l] = -1; ++evict; }
        a.sub_vpage[e] = p;
        a.sub_last_used[e] = a.frame;
        a.last_used[ts] = a.frame;
        a.v2p[p * a.L + l] = e;
        a.req_sub[e] = 1;
        a.slot_req[ts] = 1;
        if (lane == 0) {
            const int64_t Pl = a.P >> (3 * l);
            CopyCmd c;
            c.host_off = a.level_base[l] + (int64_t)p * Pl * a.bytes_g;
            c.pool_off = ((int64_t)ts * a.P + (int64_t)tj * Pl) * a.bytes_g;
            c.bytes = Pl * a.bytes_g;
            a.copies[n_copy] = c;
            a.copy_id[4 * n_copy] = p; a.copy_id[4 * n_copy + 1] = l;
            a.copy_id[4 * n_copy + 2] = ts; a.copy_id[4 * n_copy + 3] = tj;
        }
        ++n_copy;
        __threadfence_block();   // this placement before the next miss's scans
    }
    if (lane == 0) {
        a.counters[vm::C_EVICT] = evict;
        a.counters[vm::C_NCOPY] = n_copy;
        a.counters[vm::C_NMISSING] = n_missing;
        a.counters[vm::C_NMISSCAP] = n_missing_cap;
    }
}

// render list with per-level counts, and the number of occupied physical pages
// streaming: a requested page is drawn at rlevel (the level stage one found
// resident when the frame started), otherwise at its requested level if resident
__global__ __launch_bounds__(PT_NT) void k_ptl_render_list(const int8_t* __restrict__ page_level,
                                                           const int32_t* __restrict__ v2p, int n_pg, int L, int P,
                                                           int S, const int8_t* __restrict__ slot_level,
                                                           const int32_t* __restrict__ sub_vpage,
                                                           const uint8_t* __restrict__ slot_req,
                                                           RenderEntry* __restrict__ rl, uint32_t* __restrict__ counters,
                                                           const int8_t* __restrict__ rlevel) {
    __shared__ uint32_t scan_sh[PT_NT / WAVE];
    __shared__ int8_t s_lvl[RL_SEG];   // per page of the segment: level rendered, or -1
    __shared__ uint32_t s_used, s_reqd;
    const int t = threadIdx.x;
    if (t == 0) { s_used = 0; s_reqd = 0; }
    uint32_t n_rl = 0, n_g = 0;
    // segments of RL_SEG pages: a coalesced pass marks the rendered pages in
    // LDS (the loads of a thread are independent, so they are in flight
    // together); thread t then takes the consecutive pages [t K, (t + 1) K) of
    // the segment, one scan over the threads places its entries in page order
    for (int seg = 0; seg < n_pg; seg += RL_SEG) {
        const int n = min(RL_SEG, n_pg - seg);
        for (int i = t; i < n; i += PT_NT) {
            int l = page_level[seg + i];
            if (l >= 0 && rlevel) l = rlevel[seg + i];
            s_lvl[i] = (int8_t)((l >= 0 && v2p[(int64_t)(seg + i) * L + l] >= 0) ? l : -1);
        }
        __syncthreads();
        const int K = (n + PT_NT - 1) / PT_NT;
        const int i0 = min(n, t * K), i1 = min(n, i0 + K);
        uint32_t n_mine = 0, g_mine = 0;
        for (int i = i0; i < i1; ++i) {
            const int l = s_lvl[i];
            if (l >= 0) { ++n_mine; g_mine += (uint32_t)(P >> (3 * l)); }
        }
        uint32_t tot, totg;
        const uint32_t ex = block_excl_scan<PT_NT>(n_mine, scan_sh, &tot);
        const uint32_t exg = block_excl_scan<PT_NT>(g_mine, scan_sh, &totg);
        uint32_t k = n_rl + ex, base = n_g + exg;
        for (int i = i0; i < i1; ++i) {
            const int l = s_lvl[i];
            if (l < 0) continue;
            const int32_t e = v2p[(int64_t)(seg + i) * L + l];
            const uint32_t cnt = (uint32_t)(P >> (3 * l));
            RenderEntry q;
            q.pool_off = (uint32_t)((e / vmk::SUBS) * P + (e % vmk::SUBS) * (int)cnt);
            q.count = cnt;
            q.base = base;
            q.level = (uint32_t)l;
            rl[k++] = q;
            base += cnt;
        }
        n_rl += tot;
        n_g += totg;
        __syncthreads();   // s_lvl is rewritten by the next segment
    }
    uint32_t used = 0, reqd = 0;
    for (int s = t; s < S; s += PT_NT) {
        reqd += slot_req[s] ? 1u : 0u;
        const int l = slot_level[s];
        if (l < 0) continue;
        bool any = false;
        for (int j = 0; j < (1 << (3 * l)); ++j) any = any || sub_vpage[s * vmk::SUBS + j] >= 0;
        used += any ? 1u : 0u;
    }
    used = wave_sum(used);
    reqd = wave_sum(reqd);
    if (__lane_id() == 0) { atomicAdd(&s_used, used); atomicAdd(&s_reqd, reqd); }
    __syncthreads();
    if (t == 0) {
        counters[vm::C_NRL] = n_rl;
        counters[vm::C_REQSLOTS] = s_reqd;
        counters[vm::C_NRENDER] = n_g;
        counters[vm::C_POOLUSED] = s_used;
        counters[vm::C_HITS] = counters[vm::C_NREQ] - counters[vm::C_MISSES];
    }
}

__global__ void k_ptl_count_misses(const uint32_t* __restrict__ total, const uint32_t* __restrict__ total2,
                                   uint32_t* __restrict__ counters) {
    const uint32_t t2 = total2 ? *total2 : 0u;
    counters[vm::C_MISSES] = *total + t2;
    counters[vm::C_FALLBACK] = t2;
}


// ------------------------------------------------------------------ page copies
// Miss streaming by the GPU itself: workgroups take 16 KB chunks of the copy
// commands in turn, read each from the pinned host store (over PCIe, with many
// loads in flight) and write it into the pool; the commands and their count
// stay on the device, so the copies are queued before the host knows it.
// Offsets and sizes are multiples of 4 bytes (Gaussian records are 236 or 124
// bytes); 16-byte accesses where the command allows.  A command that would
// leave the store or the pool is skipped and flagged.
constexpr int CP_NT = 256;
constexpr uint32_t CP_CHUNK = 16384;

__device__ __forceinline__ void copy_chunk(const vm::CopyCmd* __restrict__ cmds, uint32_t c, uint32_t ch,
                                           const uint8_t* __restrict__ host, uint64_t host_bytes,
                                           uint8_t* __restrict__ pool, uint64_t pool_bytes,
                                           unsigned long long* __restrict__ bytes_done, uint32_t* __restrict__ err) {
    const vm::CopyCmd cmd = cmds[c];
    const uint64_t h0 = (uint64_t)cmd.host_off, p0 = (uint64_t)cmd.pool_off, nb = (uint64_t)cmd.bytes;
    if (cmd.host_off < 0 || cmd.pool_off < 0 || cmd.bytes < 0 || h0 + nb > host_bytes || p0 + nb > pool_bytes) {
        if (threadIdx.x == 0 && ch == 0) atomicOr(err, 1u);
        return;
    }
    const uint64_t lo = (uint64_t)ch * CP_CHUNK;
    if (lo >= nb) return;
    const uint64_t hi = lo + CP_CHUNK < nb ? lo + CP_CHUNK : nb;
    if (threadIdx.x == 0) atomicAdd(bytes_done, (unsigned long long)(hi - lo));
    if (((h0 | p0 | lo | hi) & 15) == 0) {
        const uint4* src = (const uint4*)(host + h0 + lo);
        uint4* dst = (uint4*)(pool + p0 + lo);
        const uint32_t n = (uint32_t)((hi - lo) / 16);
        for (uint32_t i = threadIdx.x; i < n; i += CP_NT * 4) {
            uint4 v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (i + k * CP_NT < n) v[k] = src[i + k * CP_NT];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (i + k * CP_NT < n) dst[i + k * CP_NT] = v[k];
        }
    } else {
        const uint32_t* src = (const uint32_t*)(host + h0 + lo);
        uint32_t* dst = (uint32_t*)(pool + p0 + lo);
        const uint32_t n = (uint32_t)((hi - lo) / 4);
        for (uint32_t i = threadIdx.x; i < n; i += CP_NT) dst[i] = src[i];
    }
}

// the commands of a range read on the device (demand: the first n_copy - n_pf,
// prefetch: the last n_pf), at most max_count of them; workgroups stride over
// the chunks
__device__ __forceinline__ void dev_range(const vm::CopyRangeDev& r, uint32_t max_count, uint32_t& first,
                                          uint32_t& count) {
    const uint32_t nc = *r.n_copy, np = r.n_pf ? *r.n_pf : 0u;
    first = r.prefetch ? nc - np : 0u;
    count = r.prefetch ? np : nc - np;
    if (first > max_count) first = max_count;
    if (count > max_count - first) count = max_count - first;
}

__global__ __launch_bounds__(CP_NT) void k_copy_pages(const vm::CopyCmd* __restrict__ cmds, vm::CopyRangeDev r,
                                                          uint32_t max_count, uint32_t chunks_per_cmd,
                                                          const uint8_t* __restrict__ host, uint64_t host_bytes,
                                                          uint8_t* __restrict__ pool, uint64_t pool_bytes,
                                                          unsigned long long* __restrict__ bytes_done,
                                                          uint32_t* __restrict__ err) {
    uint32_t first, count;
    dev_range(r, max_count, first, count);
    const uint64_t items = (uint64_t)count * chunks_per_cmd;
    for (uint64_t it = blockIdx.x; it < items; it += gridDim.x)
        copy_chunk(cmds, first + (uint32_t)(it / chunks_per_cmd), (uint32_t)(it % chunks_per_cmd), host, host_bytes,
                   pool, pool_bytes, bytes_done, err);
}

// bytes of the copy commands of a range (read on the device, at most
// max_count commands) into *out (one workgroup)
__global__ __launch_bounds__(PT_NT) void k_copy_bytes(const vm::CopyCmd* __restrict__ cmds, vm::CopyRangeDev r,
                                                     uint32_t max_count, unsigned long long* __restrict__ out) {
    __shared__ unsigned long long part[PT_NT / WAVE];
    uint32_t first, n;
    dev_range(r, max_count, first, n);
    unsigned long long b = 0;
    for (uint32_t i = threadIdx.x; i < n; i += PT_NT) b += (unsigned long long)cmds[first + i].bytes;
    for (int o = WAVE / 2; o > 0; o >>= 1) b += __shfl_down(b, o);
    if (__lane_id() == 0) part[threadIdx.x / WAVE] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int w = 0; w < PT_NT / WAVE; ++w) s += part[w];
        *out = s;
    }
}

}  // namespace vmk

namespace vm {
using namespace vmk;

bool pagetable_l1_fits(int n_pg, int S) { return n_pg <= PT_MAXK && S <= PT_MAXK; }

void launch_pagetable(hipStream_t st, const PtArgs& a, int) {
    PtL1 k;
    k.keys_sorted = const_cast<uint64_t*>(a.req_keys) + a.n_pg;  // second half of the key buffer
    k.n_pg = a.n_pg; k.P = a.P; k.S = a.S; k.frame = a.frame; k.budget = a.budget; k.bytes_g = a.bytes_g;
    k.streaming = a.streaming;
    k.page_level = a.page_level;
    k.slot_level = a.slot_level; k.last_used = a.last_used; k.sub_vpage = a.sub_vpage;
    k.sub_last_used = a.sub_last_used; k.v2p = a.v2p; k.slot_req = a.slot_req; k.miss = a.miss;
    k.copies = a.copies; k.copy_id = a.copy_id; k.missing = a.missing; k.counters = a.counters; k.rl = a.rl;
    hipLaunchKernelGGL(k_pagetable_l1, dim3(1), dim3(PT_NT), 0, st, a.req_keys, k);
}

}  // namespace vm

namespace vm {

static int bits_for_u(uint64_t n) {
    int b = 0;
    while ((1ull << b) < n) ++b;
    return b;
}

void launch_pagetable_lod(hipStream_t st, const PtArgs& a, SortWork& sw, const LodWork& w) {
    const int n_pg = a.n_pg, S = a.S, L = a.L;
    const unsigned nb_pg = (unsigned)((n_pg + 255) / 256);
    // requests in service order: the counters[C_NREQ] keys the visibility
    // stage wrote (the sort's grid covers n_pg, its kernels read the count)
    uint64_t* rk[2] = {const_cast<uint64_t*>(a.req_keys), w.keys_alt};
    uint32_t* nov[2] = {nullptr, nullptr};
    const int kb = a.hint_req <= kSortSmallMax
                       ? sort_small_u64(st, rk, (uint32_t)n_pg, a.counters + vm::C_NREQ, 0, 64)
                       : onesweep_u64_dev(st, sw, rk, nov, (uint32_t)n_pg, a.counters + vm::C_NREQ, 0, 64);
    const uint64_t* keys = rk[kb];
    launch_fill_u32(st, (uint32_t*)a.req_sub, ((uint64_t)S * SUBS + 3) / 4, 0u);
    launch_fill_u32(st, (uint32_t*)a.slot_req, ((uint64_t)S + 3) / 4, 0u);
    hipLaunchKernelGGL(k_ptl_hits, dim3(nb_pg), dim3(256), 0, st, keys, (const uint32_t*)a.counters, a.page_level,
                       n_pg, L, (const int32_t*)a.v2p, a.req_sub, a.slot_req, a.last_used, a.sub_last_used, a.frame,
                       w.flag, w.keys_out, w.level_out, a.streaming, w.flag2, a.rlevel);
    scan_lb(st, sw, w.flag, (uint64_t)n_pg, w.pos, w.pos + n_pg);
    if (a.streaming) scan_lb(st, sw, w.flag2, (uint64_t)n_pg, w.pos2, w.pos2 + n_pg);
    hipLaunchKernelGGL(k_ptl_count_misses, dim3(1), dim3(1), 0, st, (const uint32_t*)(w.pos + n_pg),
                       a.streaming ? (const uint32_t*)(w.pos2 + n_pg) : nullptr, a.counters);
    hipLaunchKernelGGL(k_ptl_miss_list, dim3(nb_pg), dim3(256), 0, st, keys, a.page_level, n_pg,
                       (const uint32_t*)w.flag, (const uint32_t*)w.pos,
                       a.streaming ? (const uint32_t*)w.flag2 : nullptr, (const uint32_t*)w.pos2, a.miss);
    const int idx_bits = bits_for_u((uint64_t)S * SUBS);
    // one bit above the largest eligible key, so that the all-ones keys of
    // ineligible entries sort strictly after every eligible one
    const int end_bit = idx_bits + bits_for_u((uint64_t)a.frame + 2) + 1;
    hipLaunchKernelGGL(k_ptl_cand_keys, dim3((unsigned)(((uint64_t)S * SUBS + 255) / 256)), dim3(256), 0, st, S, L,
                       idx_bits, (const int8_t*)a.slot_level, (const int32_t*)a.last_used,
                       (const int32_t*)a.sub_vpage, (const int32_t*)a.sub_last_used, (const uint8_t*)a.req_sub,
                       (const uint8_t*)a.slot_req, w.wkeys[0], w.ck[1][0], w.ck[2][0], a.counters);
    uint64_t* wk[2] = {w.wkeys[0], w.wkeys[1]};
    // the pool's slots (S keys): one workgroup for up to two of its tiles
    const int wb = (uint32_t)S <= 2 * kSortSmallMax
                       ? sort_small_u64(st, wk, (uint32_t)S, nullptr, 0, std::max(8, end_bit))
                       : onesweep_u64(st, sw, wk, nov, (uint32_t)S, 0, std::max(8, end_bit));
    PtWalk pw;
    pw.wkeys = wk[wb];
    pw.ck[0] = nullptr;
    if (end_bit > 64) throw std::length_error("LOD page table: frame counter and pool size exceed the 64-bit keys");
    for (int l = 1; l < 3; ++l) {
        pw.ck[l] = nullptr;
        if (l < L) {
            uint64_t* ck[2] = {w.ck[l][0], w.ck[l][1]};
            const uint32_t* n_cand = a.counters + (l == 1 ? vm::C_NCAND1 : vm::C_NCAND2);
            const int cb = a.hint_cand[l] <= kSortSmallMax
                               ? sort_small_u64(st, ck, (uint32_t)S * SUBS, n_cand, 0, std::max(8, end_bit))
                               : onesweep_u64_dev(st, sw, ck, nov, (uint32_t)S * SUBS, n_cand, 0,
                                                  std::max(8, end_bit));
            pw.ck[l] = ck[cb];
        }
    }
    pw.miss = a.miss;
    pw.S = S; pw.L = L; pw.P = a.P; pw.frame = a.frame; pw.budget = a.budget; pw.bytes_g = a.bytes_g;
    pw.idx_mask = (1ull << idx_bits) - 1;
    pw.level_base = a.level_base;
    pw.slot_level = a.slot_level; pw.last_used = a.last_used; pw.sub_vpage = a.sub_vpage;
    pw.sub_last_used = a.sub_last_used; pw.v2p = a.v2p; pw.req_sub = a.req_sub; pw.slot_req = a.slot_req;
    pw.fresh = w.fresh; pw.copies = a.copies; pw.copy_id = a.copy_id; pw.missing = a.missing;
    pw.counters = a.counters;
    hipLaunchKernelGGL(k_ptl_walk, dim3(1), dim3(WAVE), 0, st, pw);
    hipLaunchKernelGGL(k_ptl_render_list, dim3(1), dim3(PT_NT), 0, st, (const int8_t*)a.page_level,
                       (const int32_t*)a.v2p, n_pg, L, a.P, S, (const int8_t*)a.slot_level,
                       (const int32_t*)a.sub_vpage, (const uint8_t*)a.slot_req, a.rl, a.counters,
                       a.streaming ? (const int8_t*)a.rlevel : nullptr);
}

}  // namespace vm

namespace vm {

void launch_copy_bytes_dev(hipStream_t st, const CopyCmd* cmds, CopyRangeDev r, uint32_t max_count,
                           unsigned long long* out) {
    hipLaunchKernelGGL(vmk::k_copy_bytes, dim3(1), dim3(vmk::PT_NT), 0, st, cmds, r, max_count, out);
}

void launch_copy_pages_dev(hipStream_t st, const CopyCmd* cmds, CopyRangeDev r, uint32_t max_count,
                           uint64_t max_cmd_bytes, const uint8_t* host, uint64_t host_bytes, uint8_t* pool,
                           uint64_t pool_bytes, unsigned long long* bytes_done, uint32_t* err) {
    if (max_count == 0) return;
    const uint32_t per = (uint32_t)((max_cmd_bytes + vmk::CP_CHUNK - 1) / vmk::CP_CHUNK);
    // 8 workgroups per compute unit, striding over the chunks
    const uint32_t nb = (uint32_t)std::min<uint64_t>((uint64_t)max_count * per, 2048);
    hipLaunchKernelGGL(vmk::k_copy_pages, dim3(nb), dim3(vmk::CP_NT), 0, st, cmds, r, max_count, per, host,
                       host_bytes, pool, pool_bytes, bytes_done, err);
}

}  // namespace vm
