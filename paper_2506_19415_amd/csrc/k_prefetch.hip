// Learned prefetch on the device: the residency features, the proposals from
// the network's logits, and the third page-table stage that serves them into
// physical pages idle for two frames.  Prefetching is the paper's future work
// (Sec. 6); the visibility pass alone decides what a frame renders.
//
//  k_pf_hist     resident fraction of each of H equal page-id ranges, into
//                every view's feature row (after the 28 pose floats).
//  k_pf_select   per page: proposed when some view's logit of its cluster is
//                over the threshold, it is not requested by the frame, and it
//                is not resident at the level its nearest distance gives; key
//                (2 << 61 | distance bits << 30 | level << 28 | page), else
//                all-ones.
//  k_pf_idle     per physical page: (last use + 1, slot) when it was used in
//                neither this frame nor the previous one, else all-ones.
//  k_pf_walk     one thread: proposals nearest first, into the remaining sub-
//                slots of pages converted in this stage or the least recently
//                used idle page, up to the budget; copies follow the demand
//                copies in the copy list.
#include "kcommon.h"
#include "vm3dgs_impl.h"

namespace vmk {

using vm::CamK;

__global__ void k_pf_hist(const int32_t* __restrict__ v2p, int n_pg, int L, int H, int n_views, int ldx,
                          float* __restrict__ x) {
    const int b = blockIdx.x;
    const int64_t lo = ((int64_t)b * n_pg + H - 1) / H, hi = ((int64_t)(b + 1) * n_pg + H - 1) / H;
    uint32_t cnt = 0;
    for (int64_t p = lo + threadIdx.x; p < hi; p += blockDim.x) {
        bool res = false;
        for (int l = 0; l < L; ++l) res = res || v2p[p * L + l] >= 0;
        cnt += res ? 1u : 0u;
    }
    cnt = wave_sum(cnt);
    __shared__ uint32_t sh[4];
    if (__lane_id() == 0) sh[threadIdx.x / WAVE] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t c = 0;
        for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) c += sh[w];
        const float f = hi > lo ? (float)c / (float)(hi - lo) : 0.0f;
        for (int v = 0; v < n_views; ++v) x[(size_t)v * ldx + 28 + b] = f;
    }
}

__global__ void k_pf_select(const float* __restrict__ logits, int K, float thr, const int8_t* __restrict__ page_level,
                            const int32_t* __restrict__ v2p, const float4* __restrict__ sph, int n_pg, int L,
                            float tau, float fy, const CamK* __restrict__ cams, int n_views,
                            uint64_t* __restrict__ keys, uint32_t* __restrict__ counters) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_pg) return;
    const int c = (int)((int64_t)p * K / n_pg);
    bool sel = false;
    for (int v = 0; v < n_views; ++v) sel = sel || logits[(size_t)v * K + c] > thr;
    uint64_t key = ~0ull;
    if (sel && page_level[p] < 0) {
        const float4 q = sph[p];
        float dmin = __builtin_inff();
        for (int v = 0; v < n_views; ++v) {
            const CamK& cm = cams[v];
            const float dx = q.x - cm.pos[0], dy = q.y - cm.pos[1], dz = q.z - cm.pos[2];
            const float d = fmaxf(sqrtf((dx * dx + dy * dy) + dz * dz) - q.w, cm.znear);
            dmin = fminf(dmin, d);
        }
        int lvl = 0;
        if (L > 1) {
            const float rpx = (fy * q.w) / dmin;
            float t = tau;
            while (lvl < L - 1 && !(rpx > t)) { ++lvl; t = t * 0.5f; }
        }
        if (v2p[(int64_t)p * L + lvl] < 0)
            key = (2ull << 61) | ((uint64_t)__float_as_uint(dmin) << 30) | ((uint64_t)lvl << 28) | (uint64_t)p;
    }
    keys[p] = key;
    const uint64_t b = __ballot(key != ~0ull);
    if (__lane_id() == 0 && b) atomicAdd(&counters[vm::C_NPFREQ], (uint32_t)__popcll(b));
}

__global__ void k_pf_idle(const int32_t* __restrict__ last_used, int S, int frame, int idx_bits,
                          uint64_t* __restrict__ keys) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const int32_t lu = last_used[s];
    keys[s] = lu < frame - 1 ? (((uint64_t)(uint32_t)(lu + 1) << idx_bits) | (uint64_t)s) : ~0ull;
}

struct PfWalk {
    const uint64_t* req; const uint64_t* idle;
    int S, L, P, frame, budget, bytes_g, n_pg;
    uint64_t idx_mask;
    const int64_t* level_base;
    int8_t* slot_level; int32_t* last_used; int32_t* sub_vpage; int32_t* sub_last_used; int32_t* v2p;
    int32_t* fresh;      // [3][S]
    vm::CopyCmd* copies; int32_t* copy_id; uint32_t* counters;
};

__global__ void k_pf_walk(PfWalk a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t n_copy = a.counters[vm::C_NCOPY];
    uint32_t evict = 0, n_pf = 0, pe = 0;
    uint32_t fn[3] = {0, 0, 0}, fh[3] = {0, 0, 0};
    for (int i = 0; i < a.n_pg && n_pf < (uint32_t)a.budget; ++i) {
        const uint64_t key = a.req[i];
        if (key == ~0ull) break;
        const int32_t p = (int32_t)(key & 0x0fffffffu);
        const int l = (int)((key >> 28) & 3u);
        int ts = -1, tj = -1;
        while (l > 0 && ts < 0 && fh[l] < fn[l]) {
            const int s = a.fresh[l * a.S + fh[l]];
            for (int t = 0; t < (1 << (3 * l)) && ts < 0; ++t)
                if (a.slot_level[s] == l && a.sub_vpage[s * vmk::SUBS + t] < 0) { ts = s; tj = t; }
            if (ts < 0) ++fh[l];
        }
        if (ts < 0 && pe < (uint32_t)a.S) {
            const uint64_t ik = a.idle[pe];
            if (ik != ~0ull) {
                ++pe;
                const int s = (int)(ik & a.idx_mask);
                const int oldl = a.slot_level[s];
                if (oldl >= 0)
                    for (int j = 0; j < (1 << (3 * oldl)); ++j) {
                        const int32_t op = a.sub_vpage[s * vmk::SUBS + j];
                        if (op >= 0) { a.v2p[op * a.L + oldl] = -1; ++evict; }
                    }
                for (int j = 0; j < vmk::SUBS; ++j) {
                    a.sub_vpage[s * vmk::SUBS + j] = -1;
                    a.sub_last_used[s * vmk::SUBS + j] = -1;
                }
                a.slot_level[s] = (int8_t)l;
                ts = s; tj = 0;
                if (l > 0) a.fresh[l * a.S + fn[l]++] = s;
            }
        }
        if (ts < 0) break;                 // no idle physical page left
        const int e = ts * vmk::SUBS + tj;
        const int32_t old = a.sub_vpage[e];
        if (old >= 0) { a.v2p[old * a.L + l] = -1; ++evict; }
        a.sub_vpage[e] = p;
        a.sub_last_used[e] = a.frame;
        a.last_used[ts] = a.frame;
        a.v2p[p * a.L + l] = e;
        const int64_t Pl = a.P >> (3 * l);
        vm::CopyCmd cmd;
        cmd.host_off = a.level_base[l] + (int64_t)p * Pl * a.bytes_g;
        cmd.pool_off = ((int64_t)ts * a.P + (int64_t)tj * Pl) * a.bytes_g;
        cmd.bytes = Pl * a.bytes_g;
        a.copies[n_copy] = cmd;
        a.copy_id[4 * n_copy] = p; a.copy_id[4 * n_copy + 1] = l;
        a.copy_id[4 * n_copy + 2] = ts; a.copy_id[4 * n_copy + 3] = tj;
        ++n_copy;
        ++n_pf;
    }
    a.counters[vm::C_NCOPY] = n_copy;
    a.counters[vm::C_NPF] = n_pf;
    a.counters[vm::C_EVICT] += evict;
}

}  // namespace vmk

namespace vm {
using namespace vmk;

static int bits_u(uint64_t n) {
    int b = 0;
    while ((1ull << b) < n) ++b;
    return b;
}

void launch_pf_features(hipStream_t st, const int32_t* v2p, int n_pg, int L, int H, int n_views, float* x) {
    hipLaunchKernelGGL(k_pf_hist, dim3((unsigned)H), dim3(256), 0, st, v2p, n_pg, L, H, n_views, 28 + H, x);
}

void launch_prefetch(hipStream_t st, const PfArgs& a, SortWork& sw) {
    const unsigned nb = (unsigned)((a.n_pg + 255) / 256);
    hipLaunchKernelGGL(k_pf_select, dim3(nb), dim3(256), 0, st, a.logits, a.K, a.thr, a.page_level,
                       (const int32_t*)a.v2p, a.sph, a.n_pg, a.L, a.tau, a.fy, a.cams, a.n_views, a.keys[0],
                       a.counters);
    uint32_t* nov[2] = {nullptr, nullptr};
    uint64_t* rk[2] = {a.keys[0], a.keys[1]};
    const int kb = onesweep_u64(st, sw, rk, nov, (uint32_t)a.n_pg, 0, 64);
    const int idx_bits = bits_u((uint64_t)a.S);
    const int end_bit = idx_bits + bits_u((uint64_t)a.frame + 2) + 1;
    if (end_bit > 64) throw std::length_error("prefetch: frame counter and pool size exceed the 64-bit keys");
    hipLaunchKernelGGL(k_pf_idle, dim3((unsigned)((a.S + 255) / 256)), dim3(256), 0, st, (const int32_t*)a.last_used,
                       a.S, a.frame, idx_bits, a.idle[0]);
    uint64_t* ik[2] = {a.idle[0], a.idle[1]};
    const int ib = onesweep_u64(st, sw, ik, nov, (uint32_t)a.S, 0, std::max(8, end_bit));
    PfWalk w;
    w.req = rk[kb]; w.idle = ik[ib];
    w.S = a.S; w.L = a.L; w.P = a.P; w.frame = a.frame; w.budget = a.budget; w.bytes_g = a.bytes_g; w.n_pg = a.n_pg;
    w.idx_mask = (1ull << idx_bits) - 1;
    w.level_base = a.level_base;
    w.slot_level = a.slot_level; w.last_used = a.last_used; w.sub_vpage = a.sub_vpage;
    w.sub_last_used = a.sub_last_used; w.v2p = a.v2p; w.fresh = a.fresh;
    w.copies = a.copies; w.copy_id = a.copy_id; w.counters = a.counters;
    hipLaunchKernelGGL(k_pf_walk, dim3(1), dim3(64), 0, st, w);
    *a.sorted_out = rk[kb];
}

}  // namespace vm
