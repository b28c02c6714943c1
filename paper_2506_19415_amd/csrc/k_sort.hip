// k_sort.hip -- device-wide exclusive scan and stable LSD radix sort for
// gfx950 (wave64).  Used for the per-frame depth order of the render set,
// the (tile, Gaussian) pair order, request order and page-table candidates.
//
// Radix pass = histogram (wave-aggregated, per-wave LDS bins) -> exclusive
// scan of the digit-major block histograms -> stable scatter: each wave
// ranks 64 keys per round with ballot-based digit matching, the block
// stages its tile in LDS in digit order and writes runs coalesced.
#include <algorithm>

#include "kcommon.h"
#include "vm3dgs_impl.h"

namespace vmk {

constexpr int RS_NT = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_NT * RS_ITEMS;     // 4096 keys per block
constexpr int RS_WAVES = RS_NT / WAVE;
constexpr int RS_WAVE_SPAN = RS_TILE / RS_WAVES;  // 1024 consecutive keys per wave

constexpr int SC_NT = 256;
constexpr int SC_ITEMS = 16;
constexpr int SC_TILE = SC_NT * SC_ITEMS;

// ------------------------------------------------------------------ scan
struct InPlain {
    const uint32_t* a;
    __device__ uint32_t operator()(uint64_t i) const { return a[i]; }
};
struct InGather {  // a[idx[i]]
    const uint32_t* a;
    const uint32_t* idx;
    __device__ uint32_t operator()(uint64_t i) const { return a[idx[i]]; }
};

template <class In>
__global__ __launch_bounds__(SC_NT) void k_scan_reduce(In in, uint64_t n, uint32_t* bsum) {
    __shared__ uint32_t sh[SC_NT / WAVE];
    const uint64_t base = (uint64_t)blockIdx.x * SC_TILE;
    uint32_t s = 0;
#pragma unroll 4
    for (int i = 0; i < SC_ITEMS; ++i) {
        const uint64_t k = base + (uint64_t)i * SC_NT + threadIdx.x;
        if (k < n) s += in(k);
    }
    s = wave_sum(s);
    if (__lane_id() == 0) sh[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < SC_NT / WAVE; ++w) t += sh[w];
        bsum[blockIdx.x] = t;
    }
}

// single block: exclusive scan of nb block sums in place; total -> *total
__global__ __launch_bounds__(1024) void k_scan_bsums(uint32_t* bsum, uint32_t nb, uint32_t* total) {
    __shared__ uint32_t sh[1024 / WAVE];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += 1024) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < nb ? bsum[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<1024>(v, sh, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

// each thread owns SC_ITEMS consecutive elements
template <class In>
__global__ __launch_bounds__(SC_NT) void k_scan_down(In in, uint64_t n, const uint32_t* bsum, uint32_t* out) {
    __shared__ uint32_t sh[SC_NT / WAVE];
    const uint64_t base = (uint64_t)blockIdx.x * SC_TILE + (uint64_t)threadIdx.x * SC_ITEMS;
    uint32_t v[SC_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        v[i] = (base + i < n) ? in(base + i) : 0u;
        s += v[i];
    }
    uint32_t tot;
    uint32_t run = bsum[blockIdx.x] + block_excl_scan<SC_NT>(s, sh, &tot);
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

// ------------------------------------------------------------------ radix
template <typename K>
__device__ __forceinline__ uint32_t digit_of(K k, int shift) {
    return (uint32_t)((k >> shift) & (K)0xff);
}

template <typename K>
__global__ __launch_bounds__(RS_NT) void k_rs_hist(const K* __restrict__ keys, uint32_t n, int shift,
                                                  uint32_t* __restrict__ hist, uint32_t nb) {
    __shared__ uint32_t h[RS_WAVES][256];
    for (int i = threadIdx.x; i < RS_WAVES * 256; i += RS_NT) (&h[0][0])[i] = 0;
    __syncthreads();
    const int w = threadIdx.x / WAVE;
    const uint64_t lt = lanemask_lt();
    const uint32_t base = blockIdx.x * RS_TILE + w * RS_WAVE_SPAN;
    for (int r = 0; r < RS_WAVE_SPAN / WAVE; ++r) {
        const uint32_t idx = base + r * WAVE + __lane_id();
        const bool valid = idx < n;
        const uint32_t d = valid ? digit_of(keys[idx], shift) : 0u;
        const uint64_t peers = match_digit8(d, valid);
        if (valid && (peers & lt) == 0) h[w][d] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int i = 0; i < RS_WAVES; ++i) t += h[i][threadIdx.x];
    hist[(uint64_t)threadIdx.x * nb + blockIdx.x] = t;
}

template <typename K>
__global__ __launch_bounds__(RS_NT) void k_rs_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                     K* __restrict__ kout, uint32_t* __restrict__ vout, uint32_t n,
                                                     int shift, const uint32_t* __restrict__ offs, uint32_t nb,
                                                     int has_vals) {
    __shared__ uint32_t wc[RS_WAVES][256];
    __shared__ uint32_t dbase[256];
    __shared__ uint32_t scan_sh[RS_NT / WAVE];
    __shared__ K skey[RS_TILE];
    __shared__ uint32_t sval[RS_TILE];
    for (int i = threadIdx.x; i < RS_WAVES * 256; i += RS_NT) (&wc[0][0])[i] = 0;
    __syncthreads();
    const int w = threadIdx.x / WAVE;
    const uint64_t lt = lanemask_lt();
    const uint32_t tile0 = blockIdx.x * RS_TILE;
    const uint32_t base = tile0 + w * RS_WAVE_SPAN;
    K key[RS_ITEMS];
    uint32_t val[RS_ITEMS];
    uint32_t rank[RS_ITEMS];
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const uint32_t idx = base + r * WAVE + __lane_id();
        const bool valid = idx < n;
        key[r] = valid ? kin[idx] : (K)0;
        val[r] = (valid && has_vals) ? vin[idx] : 0u;
        const uint32_t d = digit_of(key[r], shift);
        const uint64_t peers = match_digit8(d, valid);
        uint32_t old = valid ? wc[w][d] : 0u;
        rank[r] = old + (uint32_t)__popcll(peers & lt);
        if (valid && (peers & lt) == 0) wc[w][d] = old + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: block-local start, then the wave offsets inside the digit
    {
        const int d = threadIdx.x;
        uint32_t c[RS_WAVES], tot = 0;
#pragma unroll
        for (int i = 0; i < RS_WAVES; ++i) { c[i] = wc[i][d]; tot += c[i]; }
        uint32_t all;
        const uint32_t start = block_excl_scan<RS_NT>(tot, scan_sh, &all);
        dbase[d] = start;
        uint32_t run = start;
#pragma unroll
        for (int i = 0; i < RS_WAVES; ++i) { wc[i][d] = run; run += c[i]; }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const uint32_t idx = base + r * WAVE + __lane_id();
        if (idx < n) {
            const uint32_t d = digit_of(key[r], shift);
            const uint32_t lp = wc[w][d] + rank[r];
            skey[lp] = key[r];
            sval[lp] = val[r];
        }
    }
    __syncthreads();
    const uint32_t cnt = min((uint32_t)RS_TILE, n - tile0);
#pragma unroll 4
    for (int i = 0; i < RS_ITEMS; ++i) {
        const uint32_t j = i * RS_NT + threadIdx.x;
        if (j < cnt) {
            const K k = skey[j];
            const uint32_t d = digit_of(k, shift);
            const uint32_t g = offs[(uint64_t)d * nb + blockIdx.x] + (j - dbase[d]);
            kout[g] = k;
            if (has_vals) vout[g] = sval[j];
        }
    }
}

// ------------------------------------------------------------------ single pass
// Decoupled look-back (chained scan): a block takes its tile number from an
// atomic ticket, so every earlier tile belongs to a block that is already
// running; it publishes its local total, then adds the published totals of
// earlier tiles until it meets an inclusive prefix.  Status word (64 bit):
// epoch (30 bits) | flag (2 bits: 1 = aggregate, 2 = inclusive) | value (32).
// The epoch is unique per launch, so stale words read as "not ready" and no
// clearing is needed.  Spins are bounded: on overrun a flag is raised (the
// host reports it) and the kernel still finishes.
constexpr uint64_t LB_AGG = 1, LB_INC = 2;
constexpr uint32_t LB_SPIN_LIMIT = 1u << 22;

__device__ __forceinline__ uint64_t lb_pack(uint32_t epoch, uint64_t flag, uint32_t v) {
    return ((uint64_t)epoch << 34) | (flag << 32) | v;
}
__device__ __forceinline__ void lb_store(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t lb_load(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// exclusive prefix of `tile` for one lane's column `col` of the status matrix
// (status[tile * ncol + col]); `mine` is this tile's total.  Publishes too.
__device__ uint32_t lb_lookback(uint64_t* status, uint32_t ncol, uint32_t col, uint32_t tile, uint32_t epoch,
                                uint32_t mine, uint32_t* err) {
    if (tile == 0) {
        lb_store(&status[col], lb_pack(epoch, LB_INC, mine));
        return 0;
    }
    lb_store(&status[(uint64_t)tile * ncol + col], lb_pack(epoch, LB_AGG, mine));
    uint32_t prefix = 0;
    int64_t p = (int64_t)tile - 1;
    uint32_t spins = 0;
    while (p >= 0) {
        const uint64_t w = lb_load(&status[(uint64_t)p * ncol + col]);
        if ((uint32_t)(w >> 34) != epoch || ((w >> 32) & 3u) == 0) {
            if (++spins > LB_SPIN_LIMIT) { atomicOr(err, 1u); break; }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        prefix += (uint32_t)w;
        if (((w >> 32) & 3u) == LB_INC) break;
        --p;
    }
    lb_store(&status[(uint64_t)tile * ncol + col], lb_pack(epoch, LB_INC, prefix + mine));
    return prefix;
}

// one-launch exclusive scan; the last tile writes the total
template <class In>
__global__ __launch_bounds__(SC_NT) void k_scan_lb(In in, uint64_t n, uint32_t* out, uint32_t* total,
                                                   uint64_t* status, uint32_t* ticket, uint32_t epoch,
                                                   uint32_t* err) {
    __shared__ uint32_t sh[SC_NT / WAVE];
    __shared__ uint32_t s_tile, s_prefix;
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint64_t base = (uint64_t)tile * SC_TILE + (uint64_t)threadIdx.x * SC_ITEMS;
    uint32_t v[SC_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        v[i] = (base + i < n) ? in(base + i) : 0u;
        s += v[i];
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan<SC_NT>(s, sh, &tot);
    if (threadIdx.x == 0) s_prefix = lb_lookback(status, 1, 0, tile, epoch, tot, err);
    __syncthreads();
    uint32_t run = s_prefix + ex;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (total && (uint64_t)(tile + 1) * SC_TILE >= n && threadIdx.x == SC_NT - 1) *total = run;
}

// digit histograms of several 8-bit passes in one read of the keys
template <typename K>
__global__ __launch_bounds__(RS_NT) void k_os_hist(const K* __restrict__ keys, uint32_t n, int shift0, int passes,
                                                  uint32_t* __restrict__ ghist) {
    __shared__ uint32_t h[4][256];
    for (int i = threadIdx.x; i < 4 * 256; i += RS_NT) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint64_t lt = lanemask_lt();
    const int w = threadIdx.x / WAVE;
    const uint32_t base = blockIdx.x * RS_TILE + w * RS_WAVE_SPAN;
    for (int r = 0; r < RS_WAVE_SPAN / WAVE; ++r) {
        const uint32_t idx = base + r * WAVE + __lane_id();
        const bool valid = idx < n;
        const K k = valid ? keys[idx] : (K)0;
        for (int p = 0; p < passes; ++p) {
            const uint32_t d = digit_of(k, shift0 + 8 * p);
            const uint64_t peers = match_digit8(d, valid);
            if (valid && (peers & lt) == 0) atomicAdd(&h[p][d], (uint32_t)__popcll(peers));
        }
    }
    __syncthreads();
    for (int p = 0; p < passes; ++p) {
        const uint32_t c = h[p][threadIdx.x];
        if (c) atomicAdd(&ghist[p * 256 + threadIdx.x], c);
    }
}

// one stable 8-bit pass: local ranking (ballot digit matching per wave), look-back
// over earlier tiles per digit, LDS staging in digit order, coalesced writes
// HV: values travel with the keys (without them no value pointer is touched)
template <typename K, bool HV>
__global__ __launch_bounds__(RS_NT) void k_os_pass(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                  K* __restrict__ kout, uint32_t* __restrict__ vout, uint32_t n,
                                                  int shift, const uint32_t* __restrict__ ghist_pass,
                                                  uint64_t* status, uint32_t* ticket, uint32_t epoch, uint32_t* err) {
    constexpr bool has_vals = HV;
    __shared__ uint32_t wc[RS_WAVES][256];
    __shared__ uint32_t dbase[256];
    __shared__ uint32_t gbase[256];
    __shared__ uint32_t scan_sh[RS_NT / WAVE];
    __shared__ K skey[RS_TILE];
    __shared__ uint32_t sval[RS_TILE];
    __shared__ uint32_t s_tile;
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    for (int i = threadIdx.x; i < RS_WAVES * 256; i += RS_NT) (&wc[0][0])[i] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    const int w = threadIdx.x / WAVE;
    const uint64_t lt = lanemask_lt();
    const uint32_t tile0 = tile * RS_TILE;
    const uint32_t base = tile0 + w * RS_WAVE_SPAN;
    K key[RS_ITEMS];
    uint32_t val[RS_ITEMS];
    uint32_t rank[RS_ITEMS];
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const uint32_t idx = base + r * WAVE + __lane_id();
        const bool valid = idx < n;
        key[r] = valid ? kin[idx] : (K)0;
        val[r] = (valid && has_vals) ? vin[idx] : 0u;
        const uint32_t d = digit_of(key[r], shift);
        const uint64_t peers = match_digit8(d, valid);
        const uint32_t old = valid ? wc[w][d] : 0u;
        rank[r] = old + (uint32_t)__popcll(peers & lt);
        if (valid && (peers & lt) == 0) wc[w][d] = old + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        const int d = threadIdx.x;
        uint32_t c[RS_WAVES], tot = 0;
#pragma unroll
        for (int i = 0; i < RS_WAVES; ++i) { c[i] = wc[i][d]; tot += c[i]; }
        uint32_t all;
        const uint32_t start = block_excl_scan<RS_NT>(tot, scan_sh, &all);
        dbase[d] = start;
        uint32_t run = start;
#pragma unroll
        for (int i = 0; i < RS_WAVES; ++i) { wc[i][d] = run; run += c[i]; }
        // global start of digit d: all keys with smaller digits, then earlier tiles
        uint32_t gall;
        const uint32_t dstart = block_excl_scan<RS_NT>(ghist_pass[d], scan_sh, &gall);
        gbase[d] = dstart + lb_lookback(status, 256, (uint32_t)d, tile, epoch, tot, err);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const uint32_t idx = base + r * WAVE + __lane_id();
        if (idx < n) {
            const uint32_t d = digit_of(key[r], shift);
            const uint32_t lp = wc[w][d] + rank[r];
            skey[lp] = key[r];
            sval[lp] = val[r];
        }
    }
    __syncthreads();
    const uint32_t cnt = tile0 < n ? min((uint32_t)RS_TILE, n - tile0) : 0u;
#pragma unroll 4
    for (int i = 0; i < RS_ITEMS; ++i) {
        const uint32_t j = i * RS_NT + threadIdx.x;
        if (j < cnt) {
            const K k = skey[j];
            const uint32_t d = digit_of(k, shift);
            const uint32_t g = gbase[d] + (j - dbase[d]);
            kout[g] = k;
            if (has_vals) vout[g] = sval[j];
        }
    }
}

}  // namespace vmk

// ------------------------------------------------------------------ host
namespace vm {

using namespace vmk;

static uint32_t div_up(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

size_t scan_temp_words(uint64_t n) { return (size_t)div_up(n, SC_TILE) + 16; }

template <class In>
static void scan_impl(hipStream_t st, In in, uint64_t n, uint32_t* out, uint32_t* total, uint32_t* temp) {
    const uint32_t nb = div_up(n, SC_TILE);
    if (nb == 0) {
        hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(1024), 0, st, temp, 0u, total);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce<In>, dim3(nb), dim3(SC_NT), 0, st, in, n, temp);
    hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(1024), 0, st, temp, nb, total);
    hipLaunchKernelGGL(k_scan_down<In>, dim3(nb), dim3(SC_NT), 0, st, in, n, (const uint32_t*)temp, out);
}

void scan_excl(hipStream_t st, const uint32_t* in, uint64_t n, uint32_t* out, uint32_t* total, uint32_t* temp) {
    scan_impl(st, InPlain{in}, n, out, total, temp);
}

void scan_excl_gather(hipStream_t st, const uint32_t* a, const uint32_t* idx, uint64_t n, uint32_t* out,
                      uint32_t* total, uint32_t* temp) {
    scan_impl(st, InGather{a, idx}, n, out, total, temp);
}

size_t radix_temp_words(uint64_t n) {
    const uint32_t nb = div_up(n, RS_TILE);
    return (size_t)256 * nb + scan_temp_words((uint64_t)256 * nb) + 16;
}

template <typename K>
static int radix_impl(hipStream_t st, K* keys[2], uint32_t* vals[2], uint32_t n, int begin_bit, int end_bit,
                      uint32_t* temp) {
    int cur = 0;
    if (n == 0) return 0;
    const uint32_t nb = div_up(n, RS_TILE);
    uint32_t* hist = temp;
    uint32_t* stemp = temp + (size_t)256 * nb;
    const int has_vals = vals[0] != nullptr;
    for (int shift = begin_bit; shift < end_bit; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist<K>, dim3(nb), dim3(RS_NT), 0, st, (const K*)keys[cur], n, shift, hist, nb);
        scan_impl(st, InPlain{hist}, (uint64_t)256 * nb, hist, nullptr, stemp);
        hipLaunchKernelGGL(k_rs_scatter<K>, dim3(nb), dim3(RS_NT), 0, st, (const K*)keys[cur],
                           (const uint32_t*)vals[cur], keys[cur ^ 1], vals[cur ^ 1], n, shift,
                           (const uint32_t*)hist, nb, has_vals);
        cur ^= 1;
    }
    return cur;
}

int radix_sort_u32(hipStream_t st, uint32_t* keys[2], uint32_t* vals[2], uint32_t n, int begin_bit, int end_bit,
                   uint32_t* temp) {
    return radix_impl<uint32_t>(st, keys, vals, n, begin_bit, end_bit, temp);
}

int radix_sort_u64(hipStream_t st, uint64_t* keys[2], uint32_t* vals[2], uint32_t n, int begin_bit, int end_bit,
                   uint32_t* temp) {
    return radix_impl<uint64_t>(st, keys, vals, n, begin_bit, end_bit, temp);
}

// ---------------------------------------------------------------- onesweep
size_t lb_status_words(uint64_t n_keys) { return (size_t)256 * div_up(n_keys, RS_TILE) + 256; }

template <typename K>
static int onesweep_impl(hipStream_t st, SortWork& w, K* keys[2], uint32_t* vals[2], uint32_t n, int begin_bit,
                         int end_bit) {
    if (n == 0) return 0;
    const uint32_t nb = div_up(n, RS_TILE);
    const int passes = (end_bit - begin_bit + 7) / 8;
    const int has_vals = vals[0] != nullptr;
    int cur = 0;
    for (int p0 = 0; p0 < passes; p0 += 4) {
        const int np = std::min(4, passes - p0);
        uint32_t* gh = w.next_hist(np);
        hipLaunchKernelGGL(k_os_hist<K>, dim3(nb), dim3(RS_NT), 0, st, (const K*)keys[cur], n, begin_bit + 8 * p0,
                           np, gh);
        for (int p = 0; p < np; ++p) {
            const int shift = begin_bit + 8 * (p0 + p);
            if (has_vals)
                hipLaunchKernelGGL((k_os_pass<K, true>), dim3(nb), dim3(RS_NT), 0, st, (const K*)keys[cur],
                                   (const uint32_t*)vals[cur], keys[cur ^ 1], vals[cur ^ 1], n, shift,
                                   (const uint32_t*)(gh + 256 * p), w.status, w.next_ticket(), w.next_epoch(), w.err);
            else
                hipLaunchKernelGGL((k_os_pass<K, false>), dim3(nb), dim3(RS_NT), 0, st, (const K*)keys[cur],
                                   (const uint32_t*)nullptr, keys[cur ^ 1], (uint32_t*)nullptr, n, shift,
                                   (const uint32_t*)(gh + 256 * p), w.status, w.next_ticket(), w.next_epoch(), w.err);
            cur ^= 1;
        }
    }
    return cur;
}

int onesweep_u32(hipStream_t st, SortWork& w, uint32_t* keys[2], uint32_t* vals[2], uint32_t n, int begin_bit,
                 int end_bit) {
    return onesweep_impl<uint32_t>(st, w, keys, vals, n, begin_bit, end_bit);
}

int onesweep_u64(hipStream_t st, SortWork& w, uint64_t* keys[2], uint32_t* vals[2], uint32_t n, int begin_bit,
                 int end_bit) {
    return onesweep_impl<uint64_t>(st, w, keys, vals, n, begin_bit, end_bit);
}

void scan_lb(hipStream_t st, SortWork& w, const uint32_t* in, uint64_t n, uint32_t* out, uint32_t* total) {
    const uint32_t nb = std::max(1u, div_up(n, SC_TILE));
    hipLaunchKernelGGL(k_scan_lb<InPlain>, dim3(nb), dim3(SC_NT), 0, st, InPlain{in}, n, out, total, w.status,
                       w.next_ticket(), w.next_epoch(), w.err);
}

void scan_lb_gather(hipStream_t st, SortWork& w, const uint32_t* a, const uint32_t* idx, uint64_t n, uint32_t* out,
                    uint32_t* total) {
    const uint32_t nb = std::max(1u, div_up(n, SC_TILE));
    hipLaunchKernelGGL(k_scan_lb<InGather>, dim3(nb), dim3(SC_NT), 0, st, InGather{a, idx}, n, out, total, w.status,
                       w.next_ticket(), w.next_epoch(), w.err);
}

}  // namespace vm
