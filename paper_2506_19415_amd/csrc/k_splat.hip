// k_splat.hip -- splatting of the resident Gaussians (Sec. 4.2: the 3DGS math
// of Kerbl et al.) on gfx950.
//
//  k_preprocess  one thread per (view, render Gaussian): coalesced SoA loads
//                from the pool block, EWA projection (0.3 px^2 dilation),
//                conic, 3-sigma radius, 16x16 tile rectangle, degree-3 SH
//                colour, view depth.  Padding (opacity 0) and Gaussians in
//                front of the near plane are culled.
//  k_emit        pairs in depth order, balanced over pairs: each workgroup
//                writes 1024 consecutive pairs, finding their Gaussians by
//                binary search over the runs of pairs in LDS.
//  k_ranges      [start, end) of every tile in the tile-sorted pairs.
//  k_tile_order  blend order of the tiles: by decreasing power-of-two class
//                of their pair counts, so that the longest tiles start first
//                and the short ones fill in behind them.
//  k_blend       one 256-thread workgroup per 16x16 tile, one pixel per
//                thread, one 4 x 16 strip per wave (a long tile: four
//                workgroups, one 1 x 16 column per wave); each wave walks
//                the tile's pairs on its own (registers, no LDS, no
//                barriers); per pixel front-to-back blending until
//                transmittance would fall below 1e-4; the wave stops when
//                all its pixels are done.
#include "kcommon.h"
#include "vm3dgs_impl.h"

namespace vmk {

using vm::CamK;
using vm::RenderEntry;

__device__ __forceinline__ void load_gauss(const uint8_t* __restrict__ blk, uint32_t C, uint32_t i, int fmt,
                                           Gauss& g) {
    if (fmt == 0) {
        const float* f = (const float*)blk;
#pragma unroll
        for (int a = 0; a < 3; ++a) g.m[a] = f[(size_t)a * C + i];
#pragma unroll
        for (int a = 0; a < 3; ++a) g.s[a] = f[(size_t)(3 + a) * C + i];
#pragma unroll
        for (int a = 0; a < 4; ++a) g.q[a] = f[(size_t)(6 + a) * C + i];
        g.o = f[(size_t)10 * C + i];
#pragma unroll
        for (int a = 0; a < 48; ++a) g.sh[a] = f[(size_t)(11 + a) * C + i];
    } else {
        const float* f = (const float*)blk;
        const uint32_t* u = (const uint32_t*)blk;
#pragma unroll
        for (int a = 0; a < 3; ++a) g.m[a] = f[(size_t)a * C + i];
        const uint32_t p0 = u[(size_t)3 * C + i], p1 = u[(size_t)4 * C + i];
        const uint32_t p2 = u[(size_t)5 * C + i], p3 = u[(size_t)6 * C + i];
        g.s[0] = f16_lo(p0); g.s[1] = f16_hi(p0); g.s[2] = f16_lo(p1); g.q[0] = f16_hi(p1);
        g.q[1] = f16_lo(p2); g.q[2] = f16_hi(p2); g.q[3] = f16_lo(p3); g.o = f16_hi(p3);
#pragma unroll
        for (int m = 0; m < 24; ++m) {
            const uint32_t w = u[(size_t)(7 + m) * C + i];
            g.sh[2 * m] = bf16_lo(w);
            g.sh[2 * m + 1] = bf16_hi(w);
        }
    }
}

struct PreArgs {
    const RenderEntry* rl; int n_rl;
    const uint8_t* pool; int fmt; int bytes_g;
    const CamK* cams;
    int W, H, TX, TY;
    uint32_t n_render; uint64_t n_total;
    int sigma3_tiles;
    float4* xy; float4* conic; float4* rgb; uint32_t* depth; uint2* rect; uint32_t* tiles;
    uint32_t* dkey; uint32_t* dval;
};

__global__ __launch_bounds__(256) void k_preprocess(PreArgs a) {
    const uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= a.n_total) return;
    const uint32_t v = (uint32_t)(f / a.n_render);
    const uint32_t gi = (uint32_t)(f - (uint64_t)v * a.n_render);
    // render entry holding gi: last entry with base <= gi
    int lo = 0, hi = a.n_rl - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.rl[mid].base <= gi) lo = mid; else hi = mid - 1;
    }
    const RenderEntry e = a.rl[lo];
    const uint32_t i = gi - e.base;
    Gauss g;
    load_gauss(a.pool + (size_t)e.pool_off * a.bytes_g, e.count, i, a.fmt, g);
    const CamK& c = a.cams[v];

    bool ok = g.o != 0.0f;  // padding
    const float3 t = view_xform(c.V, g.m[0], g.m[1], g.m[2]);
    ok = ok && (t.z > c.znear);
    float u = 0.f, vv = 0.f, ca = 0.f, cb = 0.f, cc2 = 0.f;
    int ix0 = 0, iy0 = 0, ix1 = 0, iy1 = 0;
    float hx = __builtin_inff(), hy = __builtin_inff();
    float col[3] = {0.f, 0.f, 0.f};
    if (ok) {
        const float w = g.q[0], x = g.q[1], y = g.q[2], z = g.q[3];
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
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k) M[r][k] = R[r][k] * g.s[k];
        float S[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k) S[r][k] = (M[r][0] * M[k][0] + M[r][1] * M[k][1]) + M[r][2] * M[k][2];
        const float limx = 1.3f * ((0.5f * (float)a.W) / c.fx);
        const float limy = 1.3f * ((0.5f * (float)a.H) / c.fy);
        const float cxz = fminf(limx, fmaxf(-limx, t.x / t.z)) * t.z;
        const float cyz = fminf(limy, fmaxf(-limy, t.y / t.z)) * t.z;
        const float tz2 = t.z * t.z;
        const float j00 = c.fx / t.z, j02 = -((c.fx * cxz) / tz2);
        const float j11 = c.fy / t.z, j12 = -((c.fy * cyz) / tz2);
        float T0[3], T1[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            T0[k] = j00 * c.V[k] + j02 * c.V[8 + k];
            T1[k] = j11 * c.V[4 + k] + j12 * c.V[8 + k];
        }
        float U0[3], U1[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            U0[k] = (T0[0] * S[0][k] + T0[1] * S[1][k]) + T0[2] * S[2][k];
            U1[k] = (T1[0] * S[0][k] + T1[1] * S[1][k]) + T1[2] * S[2][k];
        }
        const float A = ((U0[0] * T0[0] + U0[1] * T0[1]) + U0[2] * T0[2]) + 0.3f;
        const float B = (U0[0] * T1[0] + U0[1] * T1[1]) + U0[2] * T1[2];
        const float Cc = ((U1[0] * T1[0] + U1[1] * T1[1]) + U1[2] * T1[2]) + 0.3f;
        const float det = A * Cc - B * B;
        ok = det > 0.0f;
        if (ok) {
            const float inv = 1.0f / det;
            const float mid = 0.5f * (A + Cc);
            const float lam = mid + sqrtf(fmaxf(0.1f, mid * mid - det));
            const float rad = ceilf(3.0f * sqrtf(lam));
            u = (c.fx * t.x) / t.z + (c.cx - 0.5f);
            vv = (c.fy * t.y) / t.z + (c.cy - 0.5f);
            float x0 = fminf(fmaxf(floorf((u - rad) / 16.0f), 0.0f), (float)a.TX);
            float x1 = fminf(fmaxf(floorf(((u + rad) + 15.0f) / 16.0f), 0.0f), (float)a.TX);
            float y0 = fminf(fmaxf(floorf((vv - rad) / 16.0f), 0.0f), (float)a.TY);
            float y1 = fminf(fmaxf(floorf(((vv + rad) + 15.0f) / 16.0f), 0.0f), (float)a.TY);
            // support box: outside it the blend's power is below -5.55 even
            // with the rounding of its float evaluation (bounded through
            // kap = (A + Cc)^2 / det); ill-conditioned footprints keep the
            // 3-sigma rectangle
            if (!a.sigma3_tiles) {
                const float kap = ((A + Cc) * (A + Cc)) / det;
                const float e = 5e-7f * kap;
                if (e < 0.5f) {
                    const float fm = 1.0f / (1.0f - e);
                    // plus a margin over the float rounding of the box
                    // edges and of the offsets taken from them
                    const float rx = sqrtf((11.11f * fm) * A), ry = sqrtf((11.11f * fm) * Cc);
                    hx = rx + (0.015625f + 1e-6f * (fabsf(u) + rx));
                    hy = ry + (0.015625f + 1e-6f * (fabsf(vv) + ry));
                    const float bx0 = fminf(fmaxf(floorf((u - hx) / 16.0f), 0.0f), (float)a.TX);
                    const float bx1 = fminf(fmaxf(floorf((u + hx) / 16.0f) + 1.0f, 0.0f), (float)a.TX);
                    const float by0 = fminf(fmaxf(floorf((vv - hy) / 16.0f), 0.0f), (float)a.TY);
                    const float by1 = fminf(fmaxf(floorf((vv + hy) / 16.0f) + 1.0f, 0.0f), (float)a.TY);
                    x0 = fmaxf(x0, bx0); x1 = fminf(x1, bx1);
                    y0 = fmaxf(y0, by0); y1 = fminf(y1, by1);
                }
            }
            ix0 = (int)x0; ix1 = (int)x1; iy0 = (int)y0; iy1 = (int)y1;
            ok = ix1 > ix0 && iy1 > iy0;
            ca = Cc * inv; cb = -B * inv; cc2 = A * inv;
        }
        if (ok) {
            const float d0 = g.m[0] - c.pos[0], d1 = g.m[1] - c.pos[1], d2 = g.m[2] - c.pos[2];
            const float len = sqrtf((d0 * d0 + d1 * d1) + d2 * d2);
            const float X = d0 / len, Y = d1 / len, Z = d2 / len;
            const float xx = X * X, yy = Y * Y, zz = Z * Z;
            const float xy_ = X * Y, yz = Y * Z, xz = X * Z;
            float b[16];
            b[0] = ShConst::k0;
            b[1] = ShConst::k1 * Y;
            b[2] = ShConst::k2 * Z;
            b[3] = ShConst::k3 * X;
            b[4] = ShConst::k4 * xy_;
            b[5] = ShConst::k5 * yz;
            b[6] = ShConst::k6 * ((2.0f * zz - xx) - yy);
            b[7] = ShConst::k7 * xz;
            b[8] = ShConst::k8 * (xx - yy);
            b[9] = (ShConst::k9 * Y) * (3.0f * xx - yy);
            b[10] = (ShConst::k10 * xy_) * Z;
            b[11] = (ShConst::k11 * Y) * ((4.0f * zz - xx) - yy);
            b[12] = (ShConst::k12 * Z) * ((2.0f * zz - 3.0f * xx) - 3.0f * yy);
            b[13] = (ShConst::k13 * X) * ((4.0f * zz - xx) - yy);
            b[14] = (ShConst::k14 * Z) * (xx - yy);
            b[15] = (ShConst::k15 * X) * (xx - 3.0f * yy);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float acc = b[0] * g.sh[ch];
#pragma unroll
                for (int k = 1; k < 16; ++k) acc = acc + b[k] * g.sh[k * 3 + ch];
                acc = acc + 0.5f;
                col[ch] = acc > 0.0f ? acc : 0.0f;
            }
        }
    }
    a.xy[f] = make_float4(u, vv, ok ? hx : __builtin_inff(), ok ? hy : __builtin_inff());
    a.conic[f] = make_float4(ca, cb, cc2, ok ? g.o : 0.0f);
    a.rgb[f] = make_float4(col[0], col[1], col[2], 0.0f);
    a.depth[f] = ok ? __float_as_uint(t.z) : NONE32;
    a.rect[f] = ok ? make_uint2((uint32_t)ix0 | ((uint32_t)iy0 << 16), (uint32_t)ix1 | ((uint32_t)iy1 << 16))
                   : make_uint2(0u, 0u);
    a.tiles[f] = ok ? (uint32_t)((ix1 - ix0) * (iy1 - iy0)) : 0u;
    a.dkey[f] = ok ? __float_as_uint(t.z) : NONE32;
    a.dval[f] = (uint32_t)f;
}

// Pair emission balanced over pairs: workgroup b writes pairs
// [b EMIT_SPAN, (b + 1) EMIT_SPAN).  k_emit_starts records, for every block
// boundary, the depth-ordered Gaussian whose run of pairs holds it; k_emit
// loads the runs from there (each Gaussian with a run has at least one pair,
// so at most EMIT_SPAN + 1 runs meet a block) and each thread finds the owner
// of its pairs by binary search in LDS.  A pair's tile comes from the run's
// first tile key and width (a float reciprocal corrected to the exact
// quotient).
using vm::EMIT_SPAN;

__global__ void k_emit_starts(const uint32_t* __restrict__ offs, const uint32_t* __restrict__ order,
                              const uint32_t* __restrict__ tiles, uint32_t n_total, uint32_t n_start,
                              uint32_t* __restrict__ start) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_total) return;
    const uint32_t off = offs[i], cnt = tiles[order[i]];
    if (cnt == 0) return;
    // blocks past the pair capacity are not launched (n_start bounds the table)
    for (uint32_t b = (off + EMIT_SPAN - 1) / EMIT_SPAN; b * EMIT_SPAN < off + cnt && b < n_start; ++b) start[b] = i;
}

__global__ __launch_bounds__(256) void k_emit(const uint32_t* __restrict__ order, const uint32_t* __restrict__ offs,
                                              const uint2* __restrict__ rect, const uint32_t* __restrict__ start,
                                              uint32_t n_total, const uint32_t* __restrict__ n_pairs_dev,
                                              uint32_t n_render, int TX, int TY, uint32_t* __restrict__ pkey,
                                              uint32_t* __restrict__ pval, uint32_t cap) {
    __shared__ uint32_t s_off[EMIT_SPAN + 1];
    __shared__ uint32_t s_f[EMIT_SPAN + 1];
    __shared__ uint32_t s_kb[EMIT_SPAN + 1];
    __shared__ uint32_t s_wd[EMIT_SPAN + 1];
    __shared__ float s_inv[EMIT_SPAN + 1];
    // pairs beyond the capacity are not written (the frame is run again with
    // larger buffers)
    const uint32_t n_pairs = min(*n_pairs_dev, cap);
    const uint32_t p0 = blockIdx.x * EMIT_SPAN;
    if (p0 >= n_pairs) return;
    const uint32_t p1 = min(p0 + EMIT_SPAN, n_pairs);
    const uint32_t g0 = start[blockIdx.x];
    const uint32_t n_runs = min(EMIT_SPAN + 1, n_total - g0);
    for (uint32_t t = threadIdx.x; t < n_runs; t += 256) {
        const uint32_t g = g0 + t;
        const uint32_t f = order[g];
        const uint2 r = rect[f];
        const uint32_t x0 = r.x & 0xffffu, y0 = r.x >> 16, x1 = r.y & 0xffffu;
        const uint32_t wd = x1 > x0 ? x1 - x0 : 1u;
        s_off[t] = offs[g];
        s_f[t] = f;
        s_kb[t] = (f / n_render) * (uint32_t)(TX * TY) + y0 * (uint32_t)TX + x0;
        s_wd[t] = wd;
        s_inv[t] = 1.0f / (float)wd;
    }
    __syncthreads();
    for (uint32_t j = p0 + threadIdx.x; j < p1; j += 256) {
        // owner: the last run starting at or before j (zero-length runs share
        // the next start and come before it)
        int lo = 0, hi = (int)n_runs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= j) lo = mid; else hi = mid - 1;
        }
        const uint32_t q = j - s_off[lo];
        const uint32_t wd = s_wd[lo];
        uint32_t qy = (uint32_t)((float)q * s_inv[lo]);
        if (qy * wd > q) --qy;
        else if ((qy + 1) * wd <= q) ++qy;
        pkey[j] = s_kb[lo] + qy * (uint32_t)TX + (q - qy * wd);
        pval[j] = s_f[lo];
    }
}

constexpr int TO_NT = 1024;

// classes at or above this one hold the long tiles (1024 pairs or more)
constexpr int BL_LONG_CLASS = 11;

// order[n_tiles] receives the number of long tiles (a prefix of the order)
__global__ __launch_bounds__(TO_NT) void k_tile_order(const uint2* __restrict__ ranges, uint32_t n_tiles,
                                                      uint32_t* __restrict__ order) {
    __shared__ uint32_t cnt[33];
    if (threadIdx.x < 33) cnt[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < n_tiles; t += TO_NT) {
        const uint2 r = ranges[t];
        atomicAdd(&cnt[32 - __clz(r.y - r.x)], 1u);   // class 0: empty, c: count in [2^(c-1), 2^c)
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int c = 32; c >= 0; --c) {
            const uint32_t k = cnt[c];
            cnt[c] = acc;
            acc += k;
            if (c == BL_LONG_CLASS) order[n_tiles] = acc;
        }
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < n_tiles; t += TO_NT) {
        const uint2 r = ranges[t];
        order[atomicAdd(&cnt[32 - __clz(r.y - r.x)], 1u)] = t;
    }
}

__global__ void k_ranges(const uint32_t* __restrict__ key, uint32_t cap, const uint32_t* __restrict__ n_dev,
                         uint2* __restrict__ ranges) {
    const uint32_t n = min(*n_dev, cap);
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t t = key[i];
    if (i == 0 || key[i - 1] != t) ranges[t].x = i;
    if (i == n - 1 || key[i + 1] != t) ranges[t].y = i + 1;
}

// One 256-thread workgroup per 16x16 tile, one pixel per thread, one 4 x 16
// strip (4 columns, 16 rows) per wave.  The four waves of a tile work
// independently (no LDS, no barriers), so a wave whose strip holds most of
// the tile's work (a horizon band, say) is not held back at every batch by
// the others.  A long tile (1024 pairs or more, the first ones of the blend
// order) goes to four workgroups of four waves, one pixel column per wave
// (lanes 0..15 the column's rows): sixteen waves on its pairs instead of
// four, the long tiles no longer the tail of the launch.  Each wave walks
// the tile's depth-ordered pairs in chunks of 64, one pair per lane, with the
// gathers of the next chunk in flight while it blends the current one.
// Each lane first tests its Gaussian's support box (outside it no term passes
// the alpha test) against the strip's pixels that still blend: the box's
// columns and rows give a 64-bit mask of the strip's pixels (bit = lane), and
// the lanes whose mask meets the wave's live mask form the chunk's work list.
// A Gaussian that only covers pixels already stopped (an opaque band under a
// sky that never stops, say) is so skipped by one test per 64 Gaussians.  The
// wave takes the listed Gaussians in order, four at a time, and broadcasts
// each from its lane through scalar registers (v_readlane).  The exponents of
// four Gaussians are evaluated together, then the four are blended in order
// (the pixel state after one decides whether the next one is taken); the
// lanes evaluate with the pixel's "live" flag as a predicate, and the wave
// stops when no lane is live.  STATS counts, per tile, the algorithmic work:
// per pixel the list entries the front-to-back loop visits (up to and
// including the one at which it stops), and the alpha evaluations.
constexpr int BL_NT = TILE * TILE;

__device__ __forceinline__ float uniform_f(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}

// lane i's value of x, in a scalar register (i uniform)
__device__ __forceinline__ float lane_f(float x, int i) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), i));
}

// Long tiles given four workgroups each, at most (the others of a larger
// count keep one).  The launch carries BL_LONG_CAP * 4 workgroups for them;
// those without a long tile exit at once.
constexpr uint32_t BL_LONG_CAP = 1024;
static_assert(BL_LONG_CAP % 8 == 0, "long workgroups come in groups of 32, four per XCD slot");

// A wave's strip: SW columns by 16 rows of the tile, lane = row * SW +
// column (SW = 1: lanes 16..63 idle).  Pixels of the strip (bit = lane)
// whose centre lies in the box |px - u| <= hx, |py - v| <= hy; (sx, sy) is
// the strip's first pixel.  The support half-widths carry a pixel of margin,
// more than the rounding of these differences.
template <int SW>
__device__ __forceinline__ uint64_t strip_box_mask(float u, float v, float hx, float hy, float sx, float sy) {
    static_assert(SW == 1 || SW == 4, "strips of 1 or 4 columns");
    const float c0 = fmaxf(ceilf((u - hx) - sx), 0.0f), c1 = fminf(floorf((u + hx) - sx), (float)(SW - 1));
    const float r0 = fmaxf(ceilf((v - hy) - sy), 0.0f), r1 = fminf(floorf((v + hy) - sy), 15.0f);
    if (!(c0 <= c1) || !(r0 <= r1)) return 0ull;
    const int ic0 = (int)c0, ic1 = (int)c1, ir0 = (int)r0, ir1 = (int)r1;
    const uint64_t cols = (uint64_t)(((2u << ic1) - 1u) & ~((1u << ic0) - 1u));
    // one bit per row in [ir0, ir1] at the row's first column
    constexpr uint64_t first_cols = SW == 4 ? 0x1111111111111111ull : 0xffffull;   // bit row * SW, rows 0..15
    const uint64_t rows = (first_cols >> (SW * (15 - ir1))) & (~0ull << (SW * ir0));
    return rows * cols;
}

// Number of workgroups k_blend is launched with for n_tiles tiles.
__host__ __device__ inline uint32_t blend_long_slots(uint32_t n_tiles) {
    return ((n_tiles < BL_LONG_CAP ? n_tiles : BL_LONG_CAP) + 7u) & ~7u;
}

template <bool STATS>
__global__ __launch_bounds__(BL_NT) void k_blend(const uint2* __restrict__ ranges, const uint32_t* __restrict__ order,
                                                 const uint32_t* __restrict__ pval, const float4* __restrict__ xy,
                                                 const float4* __restrict__ conic, const float4* __restrict__ rgb,
                                                 int W, int H, int TX, int TY, int n_views,
                                                 float* __restrict__ image, uint2* __restrict__ stats) {
    __shared__ uint32_t s_st[2][BL_NT / WAVE];
    // Workgroups [0, 4 * slots) serve the long tiles, the rest the others in
    // order.  Workgroup ids go round-robin over the eight XCDs, so a long
    // tile's four workgroups are taken 8 ids apart (one XCD, one L2 for the
    // tile's Gaussians).
    const uint32_t n_tiles = (uint32_t)(TX * TY) * (uint32_t)n_views;
    const uint32_t slots = blend_long_slots(n_tiles);
    const uint32_t n_long = min(order[n_tiles], slots);
    const uint32_t b = blockIdx.x;
    uint32_t idx, group = 0;
    bool long_tile = false;
    if (b < 4 * slots) {
        const uint32_t s = b >> 3;
        idx = (s >> 2) * 8 + (b & 7);
        group = s & 3;
        if (idx >= n_long) return;
        long_tile = true;
    } else {
        idx = b - 4 * slots + n_long;
        if (idx >= n_tiles) return;
    }
    const uint32_t tile = order[idx];
    const uint32_t per_view = (uint32_t)(TX * TY);
    const uint32_t view = tile / per_view;
    const uint32_t t = tile - view * per_view;
    const int tx = (int)(t % (uint32_t)TX), ty = (int)(t / (uint32_t)TX);
    const int wave = (int)(threadIdx.x / WAVE);
    const int lane = (int)__lane_id();
    // short: a 4 x 16 strip per wave; long: column group * 4 + wave
    const int sx = long_tile ? tx * TILE + (int)group * 4 + wave : tx * TILE + wave * 4;
    const int px = long_tile ? sx : sx + lane % 4;
    const int py = long_tile ? ty * TILE + lane : ty * TILE + lane / 4;
    const bool inside = (!long_tile || lane < TILE) && px < W && py < H;
    const uint2 rg = ranges[tile];
    const float fpx = (float)px, fpy = (float)py;
    // first pixel of this wave's strip, in scalar registers
    const float strip_x = uniform_f((float)sx);
    const float strip_y = uniform_f((float)(ty * TILE));
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    uint32_t n_visit = inside ? rg.y - rg.x : 0u, n_alpha = 0;   // list entries the pixel's loop visits
    bool live = inside;   // this pixel still blends
    uint64_t live_m = __builtin_amdgcn_ballot_w64(live);   // the wave's live pixels
    bool wave_live = live_m != 0;
    // chunk registers: this chunk's Gaussian (centre and support half-widths;
    // conic and opacity; colour), the next chunk's, and the pair value of the
    // one after
    float4 n_p = make_float4(0.f, 0.f, 0.f, 0.f);
    float4 n_co = n_p, n_cl = n_p;
    if (rg.x + lane < rg.y) {
        const uint32_t f = pval[rg.x + lane];
        n_p = xy[f];
        n_co = conic[f];
        n_cl = rgb[f];
    }
    uint32_t n_f = rg.x + WAVE + lane < rg.y ? pval[rg.x + WAVE + lane] : 0u;
    for (uint32_t base = rg.x; base < rg.y && wave_live; base += WAVE) {
        const float4 gp = n_p;
        const float4 gb = n_co, gc = n_cl;
        const bool valid = base + lane < rg.y;
        if (base + WAVE + lane < rg.y) {
            n_p = xy[n_f];
            n_co = conic[n_f];
            n_cl = rgb[n_f];
        }
        n_f = base + 2 * WAVE + lane < rg.y ? pval[base + 2 * WAVE + lane] : 0u;
        // the chunk's Gaussians whose support box meets a live pixel of the
        // strip (every pixel rejects the others)
        const uint64_t box = !valid ? 0ull
                             : long_tile ? strip_box_mask<1>(gp.x, gp.y, gp.z, gp.w, strip_x, strip_y)
                                         : strip_box_mask<4>(gp.x, gp.y, gp.z, gp.w, strip_x, strip_y);
        uint64_t mask = __builtin_amdgcn_ballot_w64((box & live_m) != 0ull);
        while (mask != 0 && wave_live) {
            int ii[4];
            bool ok[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ok[u] = mask != 0;
                ii[u] = ok[u] ? (int)__builtin_ctzll(mask) : 0;
                mask = ok[u] ? (mask & (mask - 1)) : mask;
            }
            // exponents and in-range masks of the four (exp(-5.55) < 1/255 and
            // opacity <= 1: outside [-5.55, 0] a term fails the alpha test);
            // one ballot per compare, no lane booleans
            float pw[4];
            uint64_t mk[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float gu = lane_f(gp.x, ii[u]), gv = lane_f(gp.y, ii[u]);
                const float ca = lane_f(gb.x, ii[u]), cb = lane_f(gb.y, ii[u]), cc = lane_f(gb.z, ii[u]);
                const float dx = gu - fpx, dy = gv - fpy;
                const float q = fmaf(ca * dx, dx, (cc * dy) * dy);
                pw[u] = fmaf(-0.5f, q, -((cb * dx) * dy));
                mk[u] = __builtin_amdgcn_ballot_w64(pw[u] <= 0.0f) & __builtin_amdgcn_ballot_w64(pw[u] >= -5.55f) &
                        (ok[u] ? ~0ull : 0ull);
            }
            if (((mk[0] | mk[1] | mk[2] | mk[3]) & live_m) == 0) continue;   // no live pixel in range of any
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float power = pw[u];
                if ((mk[u] & live_m) != 0) {
                    const bool in = live && power <= 0.0f && power >= -5.55f;
                    if (STATS) n_alpha += in ? 1u : 0u;
                    // every lane computes; the pixel's state changes only where "in"
                    const float op = lane_f(gb.w, ii[u]);
                    const float alpha = fminf(0.99f, op * vm_exp_core(__builtin_amdgcn_fmed3f(power, -6.0f, 0.0f)));
                    const bool take = in && alpha >= 1.0f / 255.0f;
                    const float Tn = T * (1.0f - alpha);
                    const bool stop = take && Tn < 0.0001f;
                    const bool add = take && !stop;
                    const float wgt = alpha * T;
                    const float n0 = fmaf(lane_f(gc.x, ii[u]), wgt, C0);
                    const float n1 = fmaf(lane_f(gc.y, ii[u]), wgt, C1);
                    const float n2 = fmaf(lane_f(gc.z, ii[u]), wgt, C2);
                    C0 = add ? n0 : C0;
                    C1 = add ? n1 : C1;
                    C2 = add ? n2 : C2;
                    T = add ? Tn : T;
                    if (STATS && stop) n_visit = base + (uint32_t)ii[u] + 1u - rg.x;
                    live = live && !stop;
                    live_m = __builtin_amdgcn_ballot_w64(live);
                }
            }
            wave_live = live_m != 0;   // the wave stops when every pixel is done
        }
    }
    if (inside) {
        float* o = image + (((size_t)view * H + py) * W + px) * 3;
        o[0] = C0; o[1] = C1; o[2] = C2;
    }
    if (STATS) {
        const uint32_t e = wave_sum(n_visit), al = wave_sum(n_alpha);
        if (lane == 0) { s_st[0][threadIdx.x / WAVE] = e; s_st[1][threadIdx.x / WAVE] = al; }
        __syncthreads();
        if (threadIdx.x == 0) {   // stats cleared before the launch: a long tile's four add up
            uint32_t se = 0, sa = 0;
            for (int i = 0; i < BL_NT / WAVE; ++i) { se += s_st[0][i]; sa += s_st[1][i]; }
            atomicAdd(&stats[tile].x, se);
            atomicAdd(&stats[tile].y, sa);
        }
    }
}

}  // namespace vmk

namespace vm {
using namespace vmk;

static unsigned nblk(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

void launch_preprocess(hipStream_t st, const SplatArgs& s) {
    PreArgs a;
    a.rl = s.rl; a.n_rl = s.n_rl; a.pool = s.pool; a.fmt = s.fmt; a.bytes_g = s.fmt == 1 ? 124 : 236;
    a.cams = s.cams; a.W = s.W; a.H = s.H; a.TX = s.TX; a.TY = s.TY;
    a.n_render = s.n_render; a.n_total = (uint64_t)s.n_render * s.n_views;
    a.sigma3_tiles = s.sigma3_tiles;
    a.xy = s.xy; a.conic = s.conic; a.rgb = s.rgb; a.depth = s.depth; a.rect = s.rect; a.tiles = s.tiles;
    a.dkey = s.dkey; a.dval = s.dval;
    if (a.n_total == 0 || s.n_rl == 0) return;
    hipLaunchKernelGGL(k_preprocess, dim3(nblk(a.n_total, 256)), dim3(256), 0, st, a);
}

void launch_emit(hipStream_t st, const uint32_t* order, const uint32_t* offsets, const uint32_t* tiles,
                 const uint2* rect, uint32_t* starts, uint32_t n_total, const uint32_t* n_pairs_dev, uint32_t n_render,
                 int TX, int TY, uint32_t* pkey, uint32_t* pval, uint32_t cap) {
    if (n_total == 0 || cap == 0) return;
    const uint32_t n_blocks = nblk(cap, EMIT_SPAN);
    hipLaunchKernelGGL(k_emit_starts, dim3(nblk(n_total, 256)), dim3(256), 0, st, offsets, order, tiles, n_total,
                       n_blocks, starts);
    hipLaunchKernelGGL(k_emit, dim3(n_blocks), dim3(256), 0, st, order, offsets, rect, (const uint32_t*)starts,
                       n_total, n_pairs_dev, n_render, TX, TY, pkey, pval, cap);
}

void launch_ranges(hipStream_t st, const uint32_t* pkey, uint32_t cap, const uint32_t* n_pairs_dev, uint2* ranges,
                   uint32_t n_tiles) {
    launch_fill_u64(st, (unsigned long long*)ranges, n_tiles, 0ull);
    if (cap) hipLaunchKernelGGL(k_ranges, dim3(nblk(cap, 256)), dim3(256), 0, st, pkey, cap, n_pairs_dev, ranges);
}

void launch_tile_order(hipStream_t st, const uint2* ranges, uint32_t n_tiles, uint32_t* order) {
    if (n_tiles) hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(TO_NT), 0, st, ranges, n_tiles, order);
}

void launch_blend(hipStream_t st, const uint2* ranges, const uint32_t* order, const uint32_t* pval, const float4* xy,
                  const float4* conic, const float4* rgb, int W, int H, int TX, int TY, int n_views, float* image,
                  uint2* stats) {
    const uint32_t n_tiles = (uint32_t)(TX * TY * n_views);
    if (!n_tiles) return;
    const uint32_t n_blocks = n_tiles + 4 * blend_long_slots(n_tiles);
    if (stats) {
        launch_fill_u32(st, (uint32_t*)stats, 2 * (uint64_t)n_tiles, 0u);
        hipLaunchKernelGGL(k_blend<true>, dim3(n_blocks), dim3(BL_NT), 0, st, ranges, order, pval, xy, conic, rgb, W,
                           H, TX, TY, n_views, image, stats);
    } else {
        hipLaunchKernelGGL(k_blend<false>, dim3(n_blocks), dim3(BL_NT), 0, st, ranges, order, pval, xy, conic, rgb, W,
                           H, TX, TY, n_views, image, stats);
    }
}

}  // namespace vm
