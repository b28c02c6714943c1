// k_sort.hip -- single-pass exclusive scan and onesweep stable LSD radix sort
// for gfx950 (wave64).  Used for the per-frame depth order of the render set,
// the (tile, Gaussian) pair order, request order and page-table candidates.
//
// Radix: one histogram kernel reads the keys once for up to four 8-bit
// passes (LDS counters per key); each pass is one kernel: a block takes its
// tile by ticket, ranks its keys per wave with ballot digit matching, finds
// each digit's global start by a decoupled look-back over earlier tiles,
// stages the tile in LDS in digit order and writes runs coalesced.  Threads
// per block and keys per thread are template parameters of the kernels.
#include "kcommon.h"
#include "vm3dgs_impl.h"

namespace vmk {

constexpr int RS_MIN_TILE = 4096;       // keys per block (tile)

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

// ------------------------------------------------------------------ radix
template <typename K>
__device__ __forceinline__ uint32_t digit_of(K k, int shift) {
    return (uint32_t)((k >> shift) & (K)0xff);
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

// digit histograms of several 8-bit passes in one read of the keys: every
// key adds one to its digit's counter in LDS (four copies, wave w using copy
// w mod 4, summed at the end, so that the waves of a block spread over them)
template <typename K, int NT, int ITEMS>
__global__ __launch_bounds__(NT) void k_os_hist(const K* __restrict__ keys, uint32_t n_arg,
                                                const uint32_t* __restrict__ n_dev, int shift0, int passes,
                                                uint32_t* __restrict__ ghist) {
    const uint32_t n = n_dev ? min(*n_dev, n_arg) : n_arg;
    constexpr int NC = 4;
    constexpr int TILE_K = NT * ITEMS;
    __shared__ uint32_t h[NC][4][256];
    for (int i = threadIdx.x; i < NC * 4 * 256; i += NT) (&h[0][0][0])[i] = 0;
    __syncthreads();
    const int w = (threadIdx.x / WAVE) % NC;
    const uint32_t base = blockIdx.x * TILE_K + threadIdx.x;
    K kr[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = base + r * NT;
        kr[r] = idx < n ? keys[idx] : (K)0;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        if (base + r * NT < n)
            for (int p = 0; p < passes; ++p) atomicAdd(&h[w][p][digit_of(kr[r], shift0 + 8 * p)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < passes * 256; i += NT) {
        const int p = i >> 8, d = i & 255;
        uint32_t c = 0;
#pragma unroll
        for (int v = 0; v < NC; ++v) c += h[v][p][d];
        if (c) atomicAdd(&ghist[i], c);
    }
}

// one stable 8-bit pass: local ranking (ballot digit matching per wave), look-back
// over earlier tiles per digit, LDS staging in digit order, coalesced writes.
// NT threads, ITEMS keys each; each wave ranks ITEMS consecutive rows of 64
// keys and the first 256 threads do the per-digit work.
// HV: values travel with the keys (without them no value pointer is touched)
template <typename K, bool HV, int NT, int ITEMS>
__global__ __launch_bounds__(NT) void k_os_pass(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                K* __restrict__ kout, uint32_t* __restrict__ vout, uint32_t n_arg,
                                                const uint32_t* __restrict__ n_dev,
                                                int shift, const uint32_t* __restrict__ ghist_pass,
                                                uint64_t* status, uint32_t* ticket, uint32_t epoch, uint32_t* err) {
    const uint32_t n = n_dev ? min(*n_dev, n_arg) : n_arg;
    constexpr bool has_vals = HV;
    constexpr int NW = NT / WAVE;
    constexpr int TILE_K = NT * ITEMS, SPAN = TILE_K / NW;
    static_assert(NT >= 256, "the digit phase needs 256 threads");
    __shared__ uint32_t wc[NW][256];
    __shared__ uint32_t dbase[256];
    __shared__ uint32_t gbase[256];
    __shared__ uint32_t scan_sh[NW];
    __shared__ K skey[TILE_K];
    __shared__ uint32_t sval[TILE_K];
    __shared__ uint32_t s_tile;
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    for (int i = threadIdx.x; i < NW * 256; i += NT) (&wc[0][0])[i] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t tile0 = tile * TILE_K;
    if (tile0 >= n && tile > 0) return;   // beyond the keys (grid sized for a capacity bound)
    const int w = threadIdx.x / WAVE;
    const uint64_t lt = lanemask_lt();
    const uint32_t base = tile0 + w * SPAN;
    K key[ITEMS];
    uint32_t val[ITEMS];
    uint32_t rank[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = base + r * WAVE + __lane_id();
        const bool valid = idx < n;
        key[r] = valid ? kin[idx] : (K)0;
        val[r] = (valid && has_vals) ? vin[idx] : 0u;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const bool valid = base + r * WAVE + __lane_id() < n;
        const uint32_t d = digit_of(key[r], shift);
        const uint64_t peers = match_digit8(d, valid);
        const uint32_t old = valid ? wc[w][d] : 0u;
        rank[r] = old + (uint32_t)__popcll(peers & lt);
        if (valid && (peers & lt) == 0) wc[w][d] = old + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        const int d = threadIdx.x;
        const bool dig = d < 256;
        uint32_t c[NW], tot = 0;
#pragma unroll
        for (int i = 0; i < NW; ++i) { c[i] = dig ? wc[i][d] : 0u; tot += c[i]; }
        uint32_t all;
        const uint32_t start = block_excl_scan<NT>(tot, scan_sh, &all);
        if (dig) {
            dbase[d] = start;
            uint32_t run = start;
#pragma unroll
            for (int i = 0; i < NW; ++i) { wc[i][d] = run; run += c[i]; }
        }
        // global start of digit d: all keys with smaller digits, then earlier tiles
        uint32_t gall;
        const uint32_t dstart = block_excl_scan<NT>(dig ? ghist_pass[d] : 0u, scan_sh, &gall);
        if (dig) gbase[d] = dstart + lb_lookback(status, 256, (uint32_t)d, tile, epoch, tot, err);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = base + r * WAVE + __lane_id();
        if (idx < n) {
            const uint32_t d = digit_of(key[r], shift);
            const uint32_t lp = wc[w][d] + rank[r];
            skey[lp] = key[r];
            sval[lp] = val[r];
        }
    }
    __syncthreads();
    const uint32_t cnt = tile0 < n ? min((uint32_t)TILE_K, n - tile0) : 0u;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = i * NT + threadIdx.x;
        if (j < cnt) {
            const K k = skey[j];
            const uint32_t d = digit_of(k, shift);
            const uint32_t g = gbase[d] + (j - dbase[d]);
            kout[g] = k;
            if (has_vals) vout[g] = sval[j];
        }
    }
}

// ------------------------------------------------------------------ one workgroup
// Keys only, up to a few thousand, by one workgroup in one launch.  Up to
// SS_TILE keys: a bitonic sort in LDS (the count padded to a power of two
// with all-ones keys), comparing the keys' bits in [begin_bit, end_bit); it
// is not stable, so it gives the stable sort's result when keys that agree
// on those bits are equal (as the page table's are: each holds its page,
// slot or sub-slot index, or is all ones).  More keys: a stable LSD radix
// sort, per pass tiles of SS_TILE keys in order, each ranked like a
// onesweep tile (ballot digit matching per wave, a scan over digits) and
// written to its digit's running position after a digit histogram of all
// keys, ping-ponging between the two buffers in global memory as the
// onesweep passes do.  Either way the result is in buffer passes % 2.
constexpr int SS_NT = 1024, SS_ITEMS = 8, SS_TILE = SS_NT * SS_ITEMS;

template <typename K>
__global__ __launch_bounds__(SS_NT) void k_sort_small(K* __restrict__ k0, K* __restrict__ k1, uint32_t n_arg,
                                                      const uint32_t* __restrict__ n_dev, int begin_bit,
                                                      int passes) {
    constexpr int NW = SS_NT / WAVE, SPAN = SS_TILE / NW;
    __shared__ uint32_t wc[NW][256];
    __shared__ uint32_t gpos[256];
    __shared__ uint32_t scan_sh[NW];
    __shared__ K sk[SS_TILE];
    const uint32_t n = n_dev ? min(*n_dev, n_arg) : n_arg;
    if (n <= (uint32_t)SS_TILE) {
        const int nbits = 8 * passes;
        const K mask = (nbits >= (int)(8 * sizeof(K)) ? ~(K)0 : (((K)1 << nbits) - 1)) << begin_bit;
        uint32_t N = 1;
        while (N < n) N <<= 1;
        for (uint32_t i = threadIdx.x; i < N; i += SS_NT) sk[i] = i < n ? k0[i] : ~(K)0;
        __syncthreads();
        // a stage with j < 64 keeps each wave within its own blocks of 128
        // keys (its lanes' pairs t hold i in [128 (t / 64), 128 (t / 64 + 1))),
        // and a wave's LDS accesses take effect in order: it needs no
        // workgroup barrier, only one that keeps the compiler's order
        for (uint32_t k = 2; k <= N; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t t = threadIdx.x; t < N / 2; t += SS_NT) {
                    const uint32_t i = 2 * t - (t & (j - 1));   // t with a 0 bit inserted at j
                    const K a = sk[i], b = sk[i + j];
                    const bool up = (i & k) == 0;
                    if (((a & mask) > (b & mask)) == up) { sk[i] = b; sk[i + j] = a; }
                }
                if (j >= (uint32_t)WAVE) __syncthreads();
                else __builtin_amdgcn_wave_barrier();
            }
            __syncthreads();
        }
        K* __restrict__ out = (passes & 1) ? k1 : k0;
        for (uint32_t i = threadIdx.x; i < n; i += SS_NT) out[i] = sk[i];
        return;
    }
    const uint32_t n_tiles = (n + SS_TILE - 1) / SS_TILE;
    const int w = threadIdx.x / WAVE;
    const uint64_t lt = lanemask_lt();
    for (int p = 0; p < passes; ++p) {
        const K* __restrict__ src = (p & 1) ? k1 : k0;
        K* __restrict__ dst = (p & 1) ? k0 : k1;
        const int shift = begin_bit + 8 * p;
        // digit starts over all keys
        for (int i = threadIdx.x; i < 256; i += SS_NT) wc[0][i] = 0;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < n; i += SS_NT) atomicAdd(&wc[0][digit_of(src[i], shift)], 1u);
        __syncthreads();
        {
            const int d = threadIdx.x;
            uint32_t all;
            const uint32_t start = block_excl_scan<SS_NT>(d < 256 ? wc[0][d] : 0u, scan_sh, &all);
            if (d < 256) gpos[d] = start;
        }
        __syncthreads();
        for (uint32_t t = 0; t < n_tiles; ++t) {
            for (int i = threadIdx.x; i < NW * 256; i += SS_NT) (&wc[0][0])[i] = 0;
            __syncthreads();
            const uint32_t base = t * SS_TILE + w * SPAN;
            K key[SS_ITEMS];
            uint32_t rank[SS_ITEMS];
#pragma unroll
            for (int r = 0; r < SS_ITEMS; ++r) {
                const uint32_t idx = base + r * WAVE + __lane_id();
                key[r] = idx < n ? src[idx] : (K)0;
            }
#pragma unroll
            for (int r = 0; r < SS_ITEMS; ++r) {
                const bool valid = base + r * WAVE + __lane_id() < n;
                const uint32_t d = digit_of(key[r], shift);
                const uint64_t peers = match_digit8(d, valid);
                const uint32_t old = valid ? wc[w][d] : 0u;
                rank[r] = old + (uint32_t)__popcll(peers & lt);
                if (valid && (peers & lt) == 0) wc[w][d] = old + (uint32_t)__popcll(peers);
            }
            __syncthreads();
            {
                // per digit: the waves' starts from the digit's running position
                const int d = threadIdx.x;
                if (d < 256) {
                    uint32_t run = gpos[d];
#pragma unroll
                    for (int i = 0; i < NW; ++i) { const uint32_t c = wc[i][d]; wc[i][d] = run; run += c; }
                    gpos[d] = run;
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < SS_ITEMS; ++r)
                if (base + r * WAVE + __lane_id() < n) dst[wc[w][digit_of(key[r], shift)] + rank[r]] = key[r];
            __syncthreads();
        }
    }
}

}  // namespace vmk

// ------------------------------------------------------------------ host
namespace vm {

using namespace vmk;

static uint32_t div_up(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// ---------------------------------------------------------------- onesweep
size_t lb_status_words(uint64_t n_keys) { return (size_t)256 * div_up(n_keys, RS_MIN_TILE) + 256; }

// n: the number of keys, or with n_dev a bound on it (the grid covers n keys,
// the kernels sort min(*n_dev, n))
template <typename K, int NT, int ITEMS>
static int onesweep_items(hipStream_t st, SortWork& w, K* keys[2], uint32_t* vals[2], uint32_t n,
                          const uint32_t* n_dev, int begin_bit, int end_bit) {
    const uint32_t nb = div_up(n, NT * ITEMS);
    const int passes = (end_bit - begin_bit + 7) / 8;
    const int has_vals = vals[0] != nullptr;
    int cur = 0;
    for (int p0 = 0; p0 < passes; p0 += 4) {
        const int np = std::min(4, passes - p0);
        uint32_t* gh = w.next_hist(np);
        hipLaunchKernelGGL((k_os_hist<K, NT, ITEMS>), dim3(nb), dim3(NT), 0, st, (const K*)keys[cur], n, n_dev,
                           begin_bit + 8 * p0, np, gh);
        for (int p = 0; p < np; ++p) {
            const int shift = begin_bit + 8 * (p0 + p);
            if (has_vals)
                hipLaunchKernelGGL((k_os_pass<K, true, NT, ITEMS>), dim3(nb), dim3(NT), 0, st, (const K*)keys[cur],
                                   (const uint32_t*)vals[cur], keys[cur ^ 1], vals[cur ^ 1], n, n_dev, shift,
                                   (const uint32_t*)(gh + 256 * p), w.status, w.next_ticket(), w.next_epoch(), w.err);
            else
                hipLaunchKernelGGL((k_os_pass<K, false, NT, ITEMS>), dim3(nb), dim3(NT), 0, st, (const K*)keys[cur],
                                   (const uint32_t*)nullptr, keys[cur ^ 1], (uint32_t*)nullptr, n, n_dev, shift,
                                   (const uint32_t*)(gh + 256 * p), w.status, w.next_ticket(), w.next_epoch(), w.err);
            cur ^= 1;
        }
    }
    return cur;
}

// 4096 keys per block (tile), 512 threads of 8 keys: measured on 1M 32-bit
// depth keys (four passes) and 3M 13-bit tile keys (two passes), 512 threads
// sort the depth keys 7 % faster than 256 and 1 % faster than 1024; smaller
// tiles make every pass slower (more blocks, longer look-back chains)
constexpr int SORT_NT = 512;
template <typename K>
static int onesweep_impl(hipStream_t st, SortWork& w, K* keys[2], uint32_t* vals[2], uint32_t n,
                         const uint32_t* n_dev, int begin_bit, int end_bit) {
    if (n == 0) return 0;
    return onesweep_items<K, SORT_NT, RS_MIN_TILE / SORT_NT>(st, w, keys, vals, n, n_dev, begin_bit, end_bit);
}

int onesweep_u32(hipStream_t st, SortWork& w, uint32_t* keys[2], uint32_t* vals[2], uint32_t n, int begin_bit,
                 int end_bit) {
    return onesweep_impl<uint32_t>(st, w, keys, vals, n, nullptr, begin_bit, end_bit);
}

int onesweep_u32_dev(hipStream_t st, SortWork& w, uint32_t* keys[2], uint32_t* vals[2], uint32_t n_bound,
                     const uint32_t* n_dev, int begin_bit, int end_bit) {
    return onesweep_impl<uint32_t>(st, w, keys, vals, n_bound, n_dev, begin_bit, end_bit);
}

int onesweep_u64(hipStream_t st, SortWork& w, uint64_t* keys[2], uint32_t* vals[2], uint32_t n, int begin_bit,
                 int end_bit) {
    return onesweep_impl<uint64_t>(st, w, keys, vals, n, nullptr, begin_bit, end_bit);
}

int onesweep_u64_dev(hipStream_t st, SortWork& w, uint64_t* keys[2], uint32_t* vals[2], uint32_t n_bound,
                     const uint32_t* n_dev, int begin_bit, int end_bit) {
    return onesweep_impl<uint64_t>(st, w, keys, vals, n_bound, n_dev, begin_bit, end_bit);
}

int sort_small_u64(hipStream_t st, uint64_t* keys[2], uint32_t n_bound, const uint32_t* n_dev, int begin_bit,
                   int end_bit) {
    const int passes = (end_bit - begin_bit + 7) / 8;
    if (n_bound == 0 || passes == 0) return 0;
    hipLaunchKernelGGL(k_sort_small<uint64_t>, dim3(1), dim3(SS_NT), 0, st, keys[0], keys[1], n_bound, n_dev,
                       begin_bit, passes);
    return passes & 1;
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
