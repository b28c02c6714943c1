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
#include "kcommon.h"
#include "vm3dgs_impl.h"

namespace vmk {

using vm::CopyCmd;
using vm::RenderEntry;

constexpr int PT_NT = 1024;
constexpr int PT_MAXK = 8192;  // requests / slots sorted in LDS

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
    int n_pg, P, S, frame, budget, bytes_g;
    const int8_t* page_level;
    int8_t* slot_level; int32_t* last_used; int32_t* sub_vpage; int32_t* sub_last_used; int32_t* v2p;
    uint8_t* slot_req; uint32_t* miss;
    CopyCmd* copies; int32_t* copy_id; int32_t* missing; uint32_t* counters;
    RenderEntry* rl;
};

__global__ __launch_bounds__(PT_NT) void k_pagetable_l1(const uint64_t* __restrict__ req_keys, PtL1 a) {
    __shared__ uint64_t s[PT_MAXK];
    __shared__ uint32_t scan_sh[PT_NT / WAVE];
    __shared__ uint32_t s_cnt[4];
    const int t = threadIdx.x;
    const int n = (int)a.counters[vm::C_NREQ];
    if (n > PT_MAXK || a.S > PT_MAXK) {   // host checks these bounds; never reached
        if (t == 0) a.counters[vm::C_NCOUNTERS - 1] = 1;
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
    // ---- render list: requested and resident pages in page order
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
        a.counters[vm::C_NRENDER] = n_rl * (uint32_t)a.P;
        a.counters[vm::C_POOLUSED] = s_cnt[1];
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
    k.page_level = a.page_level;
    k.slot_level = a.slot_level; k.last_used = a.last_used; k.sub_vpage = a.sub_vpage;
    k.sub_last_used = a.sub_last_used; k.v2p = a.v2p; k.slot_req = a.slot_req; k.miss = a.miss;
    k.copies = a.copies; k.copy_id = a.copy_id; k.missing = a.missing; k.counters = a.counters; k.rl = a.rl;
    hipLaunchKernelGGL(k_pagetable_l1, dim3(1), dim3(PT_NT), 0, st, a.req_keys, k);
}

}  // namespace vm
