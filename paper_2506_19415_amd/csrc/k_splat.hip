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
//  k_blend       per pixel front-to-back blending until the transmittance
//                would fall below 1e-4.  Short tiles: one 256-thread
//                workgroup, a 4 x 16 strip per wave, each wave walking the
//                pairs on its own (registers, no barriers).  Long tiles:
//                four workgroups (16 x 4 bands), chunks of 256 pairs,
//                Gaussian-parallel selection of the terms that pass the
//                alpha test into per-pixel bit masks (LDS), then
//                pixel-parallel compositing of the selected terms in order.
#include <type_traits>

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
    // counts on the device (launched before the host has read them):
    // n_render and n_rl from these words, n_total bounded by max_total, and
    // the grid strides over the entries
    const uint32_t* n_render_dev; const uint32_t* n_rl_dev; int n_views; uint64_t max_total;
    int sigma3_tiles;
    float4* xy; float4* conic; float4* rgb; uint32_t* depth; uint2* rect; uint32_t* tiles;
    uint32_t* dkey; uint32_t* dval;
};

__device__ __forceinline__ void preprocess_one(const PreArgs& a, uint64_t f);

__global__ __launch_bounds__(256) void k_preprocess(PreArgs a) {
    if (a.n_render_dev) {
        a.n_render = *a.n_render_dev;
        a.n_rl = (int)*a.n_rl_dev;
        a.n_total = (uint64_t)a.n_render * (uint32_t)a.n_views;
        if (a.n_total > a.max_total) a.n_total = a.max_total;
        if (a.n_rl == 0) return;
        for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f < a.n_total;
             f += (uint64_t)gridDim.x * blockDim.x)
            preprocess_one(a, f);
        return;
    }
    const uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f < a.n_total) preprocess_one(a, f);
}

__device__ __forceinline__ void preprocess_one(const PreArgs& a, uint64_t f) {
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

// The blend's long tiles: tile-order classes from this one up (counts of
// 2^12 or more).  order[n_tiles] receives their number (a prefix of the
// order), order[n_tiles + 1] that of the tiles from BL_XLONG_CLASS up
// (counts of 2^14 or more, the alpha band walk's).
constexpr int BL_LONG_CLASS = 13;
constexpr int BL_XLONG_CLASS = 15;
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
            if (c == BL_XLONG_CLASS) order[n_tiles + 1] = acc;
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

// k_blend: 256-thread workgroups, depth-ordered pairs in chunks, per pixel
// front-to-back blending until the transmittance would fall below 1e-4.
// Two ways of walking a tile's pairs, chosen per tile:
//
// Strip walk (tiles of fewer than BL_LONG pairs; one workgroup, one pixel
// per thread).  A 4 x 16 strip (4 columns, 16 rows) per wave, and the four
// waves of the tile work independently (registers only, no barriers), so a
// wave whose strip holds most of the work (a horizon band, say) is not held
// back by the others.  Each wave reads the pairs in chunks of 64, one per
// lane, with the gathers of the next chunk in flight; each lane tests its
// Gaussian's support box (outside it no term passes the alpha test) against
// the strip's pixels that still blend, and the lanes whose box meets one
// form the chunk's work list.  The wave takes the listed Gaussians in
// order, four at a time, broadcasting each from its lane through scalar
// registers (v_readlane): the exponents of the four are evaluated together,
// then the four are blended in order, every lane with its pixel's "live"
// flag as a predicate.  The wave stops when no lane is live.
//
// Band walk (tiles of BL_LONG pairs or more: the far end of a street, a
// horizon, where thousands of Gaussians of a few pixels each meet in one
// tile).  Broadcasting those to a strip of pixels wastes most lanes (each
// covers a handful), so the tile goes to four workgroups, one 16 x 4 band
// each (on one XCD, so the tile's Gaussians are read through one L2), and a
// workgroup takes the pairs in chunks of 256, one per thread, in two phases:
//  1. selection, Gaussian-parallel: each thread evaluates its Gaussian over
//     the live pixels of its support box within the band (boxes of more
//     than BL_SEL_BOX pixels are evaluated by their whole wave, one pixel
//     per lane), and where a term passes the alpha test sets the Gaussian's
//     bit in the pixel's 256-bit mask in LDS;
//  2. compositing, pixel-parallel (wave w: row w of the band, lanes 0..15):
//     each pixel walks its mask bits in depth order, evaluating those terms
//     again (the same float operations on the same values, hence the same
//     decisions) and blending them; the chunk's Gaussians are read from LDS.
// Both walks evaluate a term with the same float operations, so either
// yields the same image.
//
// STATS counts, per tile, the algorithmic work: per pixel the list entries
// the front-to-back loop visits (up to and including the one at which it
// stops), and the alpha evaluations (terms in the power range at pixels
// still blending; the band walk counts those live when the chunk starts).
constexpr int BL_NT = TILE * TILE;
constexpr uint32_t BL_LONG = 4096;   // tiles with this many pairs take the band walk
constexpr int BL_BANDS = 4;          // workgroups (16 x 4 bands) per long tile
constexpr int BL_BAND_PX = TILE * TILE / BL_BANDS;
constexpr int BL_CH = BL_NT;         // pairs per band-walk chunk, one per thread
constexpr int BL_WORDS = BL_CH / 32;
constexpr int BL_SEL_BOX = 16;       // larger boxes are evaluated by the whole wave
constexpr int BL_APAD = BL_BAND_PX + 1;   // alpha row stride: a term's pixels, one word of padding
// Long tiles given a band walk, at most (the others of a larger count take
// the strip walk).
constexpr uint32_t BL_LONG_CAP = 2048;
constexpr uint32_t BL_XLONG = 16384;   // tiles with this many pairs take the alpha band walk
static_assert(BL_LONG == (1u << (BL_LONG_CLASS - 1)), "the long tiles are whole tile-order classes");
static_assert(BL_XLONG == (1u << (BL_XLONG_CLASS - 1)) && BL_XLONG >= BL_LONG, "the longest tiles too");
static_assert(BL_BANDS == 4 && BL_BAND_PX == WAVE && BL_NT / WAVE == BL_BANDS, "band layout: one band row per wave");

__device__ __forceinline__ float uniform_f(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}

// lane i's value of x, in a scalar register (i uniform)
__device__ __forceinline__ float lane_f(float x, int i) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), i));
}
__device__ __forceinline__ int lane_i(int x, int i) { return __builtin_amdgcn_readlane(x, i); }

// The exponent of a Gaussian at a pixel (its centre (u, v), conic
// (ca, cb, cc)), as every walk evaluates it; a term can pass the alpha test
// only for power in [-5.55, 0] (exp(-5.55) < 1/255, opacity <= 1).
__device__ __forceinline__ float blend_power(float u, float v, float ca, float cb, float cc, float fpx, float fpy) {
    const float dx = u - fpx, dy = v - fpy;
    const float q = fmaf(ca * dx, dx, (cc * dy) * dy);
    return fmaf(-0.5f, q, -((cb * dx) * dy));
}
__device__ __forceinline__ bool power_in_range(float power) { return power <= 0.0f && power >= -5.55f; }
__device__ __forceinline__ float blend_alpha(float power, float op) {
    return fminf(0.99f, op * vm_exp_core(__builtin_amdgcn_fmed3f(power, -6.0f, 0.0f)));
}

// Pixels of a 4 x 16 strip (bit = lane = row * 4 + column) whose centre lies
// in the box |px - u| <= hx, |py - v| <= hy; (sx, sy) is the strip's first
// pixel.  The support half-widths carry a margin above the rounding of
// these differences.
__device__ __forceinline__ uint64_t strip_box_mask(float u, float v, float hx, float hy, float sx, float sy) {
    const float c0 = fmaxf(ceilf((u - hx) - sx), 0.0f), c1 = fminf(floorf((u + hx) - sx), 3.0f);
    const float r0 = fmaxf(ceilf((v - hy) - sy), 0.0f), r1 = fminf(floorf((v + hy) - sy), 15.0f);
    if (!(c0 <= c1) || !(r0 <= r1)) return 0ull;
    const int ic0 = (int)c0, ic1 = (int)c1, ir0 = (int)r0, ir1 = (int)r1;
    const uint64_t cols = (uint64_t)(((2u << ic1) - 1u) & ~((1u << ic0) - 1u));
    // one bit per row in [ir0, ir1] at the row's first column
    constexpr uint64_t first_cols = 0x1111111111111111ull;   // bit row * 4, rows 0..15
    const uint64_t rows = (first_cols >> (4 * (15 - ir1))) & (~0ull << (4 * ir0));
    return rows * cols;
}

// LDS of the band walk: the chunk's Gaussians (centre and support
// half-widths; conic and opacity; colour), the per-pixel masks of the
// chunk's selected Gaussians, word-major (consecutive pixels read
// consecutive words: no bank conflicts), and the band's live pixels, 16 bits
// per row.
struct BlendLds {
    float4 g[3][BL_CH];
    uint32_t mask[BL_WORDS][BL_BAND_PX];
    uint32_t live[BL_BANDS];
    uint32_t st[2][BL_NT / WAVE];
};


// LDS of the alpha band walk (the longest tiles): the alphas that the selection finds (term t,
// band pixel q at t * BL_APAD + q: the lanes of a wave, on consecutive
// terms, write distinct banks), the chunk's colours, the per-pixel masks of
// the chunk's selected Gaussians, word-major (consecutive pixels read
// consecutive words: no bank conflicts), and the band's live pixels, 16 bits
// per row.
struct AlphaLds {
    float alpha[BL_CH * BL_APAD];
    float4 col[BL_CH];
    uint32_t mask[BL_WORDS][BL_BAND_PX];
    uint32_t live[BL_BANDS];
    uint32_t st[2][BL_NT / WAVE];
};
// per-pixel blend state
struct PixelBlend {
    float T, C0, C1, C2;
    bool live;
    uint32_t n_visit;
};

// one term of a pixel's front-to-back loop; returns whether the pixel stops
__device__ __forceinline__ bool blend_term(PixelBlend& px, float alpha, bool in, float r, float g, float b) {
    const bool take = in && alpha >= 1.0f / 255.0f;
    const float Tn = px.T * (1.0f - alpha);
    const bool stop = take && Tn < 0.0001f;
    const bool add = take && !stop;
    const float wgt = alpha * px.T;
    const float n0 = fmaf(r, wgt, px.C0), n1 = fmaf(g, wgt, px.C1), n2 = fmaf(b, wgt, px.C2);
    px.C0 = add ? n0 : px.C0;
    px.C1 = add ? n1 : px.C1;
    px.C2 = add ? n2 : px.C2;
    px.T = add ? Tn : px.T;
    return stop;
}

template <bool STATS>
__device__ __forceinline__ void strip_walk(uint2 rg, const uint32_t* __restrict__ pval, const float4* __restrict__ xy,
                                           const float4* __restrict__ conic, const float4* __restrict__ rgb, int tx,
                                           int ty, int W, int H, PixelBlend& pb, uint32_t& n_alpha, int& px_out,
                                           int& py_out) {
    const int wave = (int)(threadIdx.x / WAVE);
    const int lane = (int)__lane_id();
    const int px = tx * TILE + wave * 4 + lane % 4;
    const int py = ty * TILE + lane / 4;
    px_out = px; py_out = py;
    const bool inside = px < W && py < H;
    const float fpx = (float)px, fpy = (float)py;
    // first pixel of this wave's strip, in scalar registers
    const float strip_x = uniform_f((float)(tx * TILE + wave * 4));
    const float strip_y = uniform_f((float)(ty * TILE));
    pb.live = inside;
    pb.n_visit = inside ? rg.y - rg.x : 0u;
    uint64_t live_m = __builtin_amdgcn_ballot_w64(pb.live);   // the wave's live pixels
    bool wave_live = live_m != 0;
    // chunk registers: this chunk's Gaussian, the next chunk's, and the pair
    // value of the one after
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
        const uint64_t box = valid ? strip_box_mask(gp.x, gp.y, gp.z, gp.w, strip_x, strip_y) : 0ull;
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
            // exponents and in-range masks of the four; one ballot per
            // compare, no lane booleans
            float pw[4];
            uint64_t mk[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                pw[u] = blend_power(lane_f(gp.x, ii[u]), lane_f(gp.y, ii[u]), lane_f(gb.x, ii[u]),
                                    lane_f(gb.y, ii[u]), lane_f(gb.z, ii[u]), fpx, fpy);
                mk[u] = __builtin_amdgcn_ballot_w64(pw[u] <= 0.0f) & __builtin_amdgcn_ballot_w64(pw[u] >= -5.55f) &
                        (ok[u] ? ~0ull : 0ull);
            }
            if (((mk[0] | mk[1] | mk[2] | mk[3]) & live_m) == 0) continue;   // no live pixel in range of any
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if ((mk[u] & live_m) != 0) {
                    const bool in = pb.live && power_in_range(pw[u]);
                    if (STATS) n_alpha += in ? 1u : 0u;
                    // every lane computes; the pixel's state changes only where "in"
                    const float alpha = blend_alpha(pw[u], lane_f(gb.w, ii[u]));
                    const bool stop = blend_term(pb, alpha, in, lane_f(gc.x, ii[u]), lane_f(gc.y, ii[u]),
                                                 lane_f(gc.z, ii[u]));
                    if (STATS && stop) pb.n_visit = base + (uint32_t)ii[u] + 1u - rg.x;
                    pb.live = pb.live && !stop;
                    live_m = __builtin_amdgcn_ballot_w64(pb.live);
                }
            }
            wave_live = live_m != 0;   // the wave stops when every pixel is done
        }
    }
}

// value of sub-lane j of this lane's quad (DPP quad_perm [j, j, j, j]; 0
// from an inactive lane)
__device__ __forceinline__ int quad_bcast_i(int x, int j) {
    switch (j) {
    case 0: return __builtin_amdgcn_mov_dpp(x, 0x00, 0xf, 0xf, true);
    case 1: return __builtin_amdgcn_mov_dpp(x, 0x55, 0xf, 0xf, true);
    case 2: return __builtin_amdgcn_mov_dpp(x, 0xaa, 0xf, 0xf, true);
    default: return __builtin_amdgcn_mov_dpp(x, 0xff, 0xf, 0xf, true);
    }
}
__device__ __forceinline__ float quad_bcast(float x, int j) {
    return __builtin_bit_cast(float, quad_bcast_i(__builtin_bit_cast(int, x), j));
}

// 16 bits, one per quad of a wave-wide mask in which the lanes of a quad agree
__device__ __forceinline__ uint32_t quad_live16(uint64_t m) {
    uint64_t x = m & 0x1111111111111111ull;   // lane 4c -> bit 4c
    x = (x | (x >> 3)) & 0x0303030303030303ull;
    x = (x | (x >> 6)) & 0x000f000f000f000full;
    x = (x | (x >> 12)) & 0x000000ff000000ffull;
    x = (x | (x >> 24)) & 0xffffull;
    return (uint32_t)x;
}

// phase 1 for one Gaussian and one band pixel (q = row * 16 + column, at
// image position (fx, fy))
__device__ __forceinline__ void select_term(BlendLds& L, uint32_t bit, int word, int q, float fx, float fy, float u,
                                            float v, float ca, float cb, float cc, float op, uint32_t& n_alpha) {
    const float power = blend_power(u, v, ca, cb, cc, fx, fy);
    if (power_in_range(power)) {
        ++n_alpha;
        if (blend_alpha(power, op) >= 1.0f / 255.0f) atomicOr(&L.mask[word][q], bit);
    }
}

// phase 1 for chunk term jt and band pixel q (= row * 16 + column, at image
// position (fx, fy)): a term that passes the alpha test is selected and
// its alpha kept
__device__ __forceinline__ void select_alpha_term(AlphaLds& L, int jt, int q, float fx, float fy, float u, float v, float ca,
                                            float cb, float cc, float op, uint32_t& n_alpha) {
    const float power = blend_power(u, v, ca, cb, cc, fx, fy);
    if (power_in_range(power)) {
        ++n_alpha;
        const float a = blend_alpha(power, op);
        if (a >= 1.0f / 255.0f) {
            atomicOr(&L.mask[jt >> 5][q], 1u << (jt & 31));
            L.alpha[jt * BL_APAD + q] = a;
        }
    }
}

template <bool STATS>
__device__ __forceinline__ void band_walk(BlendLds& L, uint2 rg, const uint32_t* __restrict__ pval,
                                          const float4* __restrict__ xy, const float4* __restrict__ conic,
                                          const float4* __restrict__ rgb, int tx, int ty, int band, int W, int H,
                                          PixelBlend& pb, uint32_t& n_alpha, int& px_out, int& py_out) {
    const int t = (int)threadIdx.x, wave = t / WAVE, lane = (int)__lane_id();
    // the band: columns tx * 16 + [0, 16), rows by0 + [0, 4).  Compositing:
    // wave w takes row w, a quad of lanes per pixel (column lane / 4); the
    // quad's lanes hold the same pixel state and sub-lane k = lane % 4
    // evaluates every fourth selected term
    const int by0 = ty * TILE + band * (TILE / BL_BANDS);
    const int col = lane >> 2, sub = lane & 3;
    const int q = wave * TILE + col;   // band pixel of the quad
    const int px = tx * TILE + col, py = by0 + wave;
    px_out = sub == 0 ? px : W;   // one lane of the quad writes the pixel
    py_out = py;
    const float fpx = (float)px, fpy = (float)py;
    const float tx0 = (float)(tx * TILE), ty0 = (float)by0;
    pb.live = px < W && py < H;
    pb.n_visit = pb.live && sub == 0 ? rg.y - rg.x : 0u;
#pragma unroll
    for (int w = 0; w < BL_WORDS / 4; ++w) L.mask[sub * (BL_WORDS / 4) + w][q] = 0u;
    uint32_t lm = quad_live16(__builtin_amdgcn_ballot_w64(pb.live));
    if (lane == 0) L.live[wave] = lm;
    // registers: this chunk's Gaussian, the next chunk's, the pair value of the one after
    float4 n_p = make_float4(0.f, 0.f, 0.f, 0.f);
    float4 n_co = n_p, n_cl = n_p;
    if (rg.x + t < rg.y) {
        const uint32_t f = pval[rg.x + t];
        n_p = xy[f];
        n_co = conic[f];
        n_cl = rgb[f];
    }
    uint32_t n_f = rg.x + BL_CH + t < rg.y ? pval[rg.x + BL_CH + t] : 0u;
    __syncthreads();
    for (uint32_t base = rg.x; base < rg.y; base += BL_CH) {
        // the band's live pixels, bit row * 16 + column (uniform)
        const uint64_t live = (uint64_t)L.live[0] | ((uint64_t)L.live[1] << 16) | ((uint64_t)L.live[2] << 32) |
                              ((uint64_t)L.live[3] << 48);
        if (live == 0) break;
        const float4 gp = n_p, gb = n_co, gc = n_cl;
        const bool valid = base + t < rg.y;
        if (base + BL_CH + t < rg.y) {
            n_p = xy[n_f];
            n_co = conic[n_f];
            n_cl = rgb[n_f];
        }
        n_f = base + 2 * BL_CH + t < rg.y ? pval[base + 2 * BL_CH + t] : 0u;
        L.g[0][t] = gp; L.g[1][t] = gb; L.g[2][t] = gc;
        // 1. selection: this thread's Gaussian over the live pixels of its box in the band
        const float c0 = fmaxf(ceilf((gp.x - gp.z) - tx0), 0.0f), c1 = fminf(floorf((gp.x + gp.z) - tx0), 15.0f);
        const float r0 = fmaxf(ceilf((gp.y - gp.w) - ty0), 0.0f), r1 = fminf(floorf((gp.y + gp.w) - ty0), 3.0f);
        const bool has = valid && c0 <= c1 && r0 <= r1;
        const int ic0 = has ? (int)c0 : 0, ic1 = has ? (int)c1 : -1;
        const int ir0 = has ? (int)r0 : 0, ir1 = has ? (int)r1 : -1;
        const bool small = (ic1 - ic0 + 1) * (ir1 - ir0 + 1) <= BL_SEL_BOX;
        const uint32_t bit = 1u << (t & 31);
        const int word = t >> 5;
        if (small) {
            for (int y = ir0; y <= ir1; ++y) {
                const uint32_t row = (uint32_t)(live >> (y * TILE));
                for (int x = ic0; x <= ic1; ++x)
                    if ((row >> x) & 1u)
                        select_term(L, bit, word, y * TILE + x, tx0 + (float)x, ty0 + (float)y, gp.x, gp.y, gb.x,
                                    gb.y, gb.z, gb.w, n_alpha);
            }
        }
        // the others: one at a time, a band pixel per lane
        uint64_t big = __builtin_amdgcn_ballot_w64(!small);
        const int bx = lane & (TILE - 1), byy = lane / TILE;
        const bool lane_live = (live >> lane) & 1ull;
        while (big != 0) {
            const int j = (int)__builtin_ctzll(big);
            big &= big - 1;
            const int x0 = lane_i(ic0, j), x1 = lane_i(ic1, j), y0 = lane_i(ir0, j), y1 = lane_i(ir1, j);
            if (lane_live && bx >= x0 && bx <= x1 && byy >= y0 && byy <= y1) {
                const int jt = wave * WAVE + j;
                select_term(L, 1u << (jt & 31), jt >> 5, lane, tx0 + (float)bx, ty0 + (float)byy, lane_f(gp.x, j),
                            lane_f(gp.y, j), lane_f(gb.x, j), lane_f(gb.y, j), lane_f(gb.z, j), lane_f(gb.w, j),
                            n_alpha);
            }
        }
        __syncthreads();
        // 2. compositing: the quad's pixel over its selected Gaussians in
        // order, four at a time: sub-lane k evaluates the k-th (exponent and
        // alpha, the costly part), then the quad blends the four in order,
        // each lane taking their alphas from the others (DPP quad
        // broadcasts) and keeping one colour channel (sub-lane k: channel k,
        // none for k = 3), without branches: a term after the stop is not taken
        if (pb.live) {   // uniform over the quad
            const float* const gcol = &L.g[2][0].x;
            for (int w = 0; w < BL_WORDS && pb.live; ++w) {
                uint32_t m = L.mask[w][q];
                while (m != 0u && pb.live) {
                    uint32_t mk = m;   // without its first `sub` bits
                    mk = sub >= 1 ? mk & (mk - 1u) : mk;
                    mk = sub >= 2 ? mk & (mk - 1u) : mk;
                    mk = sub >= 3 ? mk & (mk - 1u) : mk;
#pragma unroll
                    for (int i = 0; i < 4; ++i) m &= m - 1u;
                    // this lane's term: alpha, or -1 where none or out of range
                    float a = -1.0f;
                    const int g = mk != 0u ? w * 32 + (int)__builtin_ctz(mk) : 0;
                    if (mk != 0u) {
                        const float4 P = L.g[0][g], Q = L.g[1][g];
                        const float power = blend_power(P.x, P.y, Q.x, Q.y, Q.z, fpx, fpy);
                        if (power_in_range(power)) a = blend_alpha(power, Q.w);
                    }
                    bool alive = true;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        // every lane of the quad takes part in each broadcast
                        // (a DPP read from an inactive lane gives 0)
                        const float aj = quad_bcast(a, j);
                        const int gj = quad_bcast_i(g, j);
                        const float cj = gcol[4 * gj + sub];
                        const bool take = alive && aj >= 1.0f / 255.0f;
                        const float Tn = pb.T * (1.0f - aj);
                        const bool stop = take && Tn < 0.0001f;
                        const bool add = take && !stop;
                        const float nc = fmaf(cj, aj * pb.T, pb.C0);
                        pb.C0 = add ? nc : pb.C0;
                        pb.T = add ? Tn : pb.T;
                        if (STATS && stop && sub == 0) pb.n_visit = base + (uint32_t)gj + 1u - rg.x;
                        alive = alive && !stop;
                    }
                    pb.live = alive;
                }
            }
        }
#pragma unroll
        for (int w = 0; w < BL_WORDS / 4; ++w) L.mask[sub * (BL_WORDS / 4) + w][q] = 0u;
        lm = quad_live16(__builtin_amdgcn_ballot_w64(pb.live));
        if (lane == 0) L.live[wave] = lm;
        __syncthreads();
    }
    // the pixel's colour from the quad's three channel lanes
    const float c0 = quad_bcast(pb.C0, 0), c1 = quad_bcast(pb.C0, 1), c2 = quad_bcast(pb.C0, 2);
    pb.C0 = c0; pb.C1 = c1; pb.C2 = c2;
}

template <bool STATS>
__device__ __forceinline__ void band_walk_alpha(AlphaLds& L, uint2 rg, const uint32_t* __restrict__ pval,
                                          const float4* __restrict__ xy, const float4* __restrict__ conic,
                                          const float4* __restrict__ rgb, int tx, int ty, int band, int W, int H,
                                          PixelBlend& pb, uint32_t& n_alpha, int& px_out, int& py_out) {
    const int t = (int)threadIdx.x, wave = t / WAVE, lane = (int)__lane_id();
    // the band: columns tx * 16 + [0, 16), rows by0 + [0, 4).  Compositing:
    // wave w takes row w, a quad of lanes per pixel (column lane / 4); the
    // quad's lanes hold the same transmittance, sub-lane k = lane % 4 the
    // pixel's colour channel k (none for k = 3)
    const int by0 = ty * TILE + band * (TILE / BL_BANDS);
    const int col = lane >> 2, sub = lane & 3;
    const int q = wave * TILE + col;   // band pixel of the quad
    const int px = tx * TILE + col, py = by0 + wave;
    px_out = sub == 0 ? px : W;   // one lane of the quad writes the pixel
    py_out = py;
    const float fpx = (float)px, fpy = (float)py;
    const float tx0 = (float)(tx * TILE), ty0 = (float)by0;
    pb.live = px < W && py < H;
    pb.n_visit = pb.live && sub == 0 ? rg.y - rg.x : 0u;
#pragma unroll
    for (int w = 0; w < BL_WORDS / 4; ++w) L.mask[sub * (BL_WORDS / 4) + w][q] = 0u;
    uint32_t lm = quad_live16(__builtin_amdgcn_ballot_w64(pb.live));
    if (lane == 0) L.live[wave] = lm;
    // registers: this chunk's Gaussian, the next chunk's, the pair value of the one after
    float4 n_p = make_float4(0.f, 0.f, 0.f, 0.f);
    float4 n_co = n_p, n_cl = n_p;
    if (rg.x + t < rg.y) {
        const uint32_t f = pval[rg.x + t];
        n_p = xy[f];
        n_co = conic[f];
        n_cl = rgb[f];
    }
    uint32_t n_f = rg.x + BL_CH + t < rg.y ? pval[rg.x + BL_CH + t] : 0u;
    __syncthreads();
    for (uint32_t base = rg.x; base < rg.y; base += BL_CH) {
        // the band's live pixels, bit row * 16 + column (uniform)
        const uint64_t live = (uint64_t)L.live[0] | ((uint64_t)L.live[1] << 16) | ((uint64_t)L.live[2] << 32) |
                              ((uint64_t)L.live[3] << 48);
        if (live == 0) break;
        const float4 gp = n_p, gb = n_co, gc = n_cl;
        const bool valid = base + t < rg.y;
        if (base + BL_CH + t < rg.y) {
            n_p = xy[n_f];
            n_co = conic[n_f];
            n_cl = rgb[n_f];
        }
        n_f = base + 2 * BL_CH + t < rg.y ? pval[base + 2 * BL_CH + t] : 0u;
        L.col[t] = gc;
        // 1. selection: this thread's Gaussian over the live pixels of its box in the band
        const float c0 = fmaxf(ceilf((gp.x - gp.z) - tx0), 0.0f), c1 = fminf(floorf((gp.x + gp.z) - tx0), 15.0f);
        const float r0 = fmaxf(ceilf((gp.y - gp.w) - ty0), 0.0f), r1 = fminf(floorf((gp.y + gp.w) - ty0), 3.0f);
        const bool has = valid && c0 <= c1 && r0 <= r1;
        const int ic0 = has ? (int)c0 : 0, ic1 = has ? (int)c1 : -1;
        const int ir0 = has ? (int)r0 : 0, ir1 = has ? (int)r1 : -1;
        const bool small = (ic1 - ic0 + 1) * (ir1 - ir0 + 1) <= BL_SEL_BOX;
        if (small) {
            for (int y = ir0; y <= ir1; ++y) {
                const uint32_t row = (uint32_t)(live >> (y * TILE));
                for (int x = ic0; x <= ic1; ++x)
                    if ((row >> x) & 1u)
                        select_alpha_term(L, t, y * TILE + x, tx0 + (float)x, ty0 + (float)y, gp.x, gp.y, gb.x, gb.y,
                                    gb.z, gb.w, n_alpha);
            }
        }
        // the others: one at a time, a band pixel per lane
        uint64_t big = __builtin_amdgcn_ballot_w64(!small);
        const int bx = lane & (TILE - 1), byy = lane / TILE;
        const bool lane_live = (live >> lane) & 1ull;
        while (big != 0) {
            const int j = (int)__builtin_ctzll(big);
            big &= big - 1;
            const int x0 = lane_i(ic0, j), x1 = lane_i(ic1, j), y0 = lane_i(ir0, j), y1 = lane_i(ir1, j);
            if (lane_live && bx >= x0 && bx <= x1 && byy >= y0 && byy <= y1) {
                select_alpha_term(L, wave * WAVE + j, lane, tx0 + (float)bx, ty0 + (float)byy, lane_f(gp.x, j),
                            lane_f(gp.y, j), lane_f(gb.x, j), lane_f(gb.y, j), lane_f(gb.z, j), lane_f(gb.w, j),
                            n_alpha);
            }
        }
        __syncthreads();
        // 2. compositing: the quad's pixel over its selected Gaussians in
        // order, four at a time, with the alphas that the selection kept;
        // without branches: a term after the stop is not taken
        if (pb.live) {   // uniform over the quad
            const float* const gcol = &L.col[0].x + sub;   // term j's channel at gcol[4 * j]
            const float* const arow = &L.alpha[q];         // term j's alpha at arow[j * BL_APAD]
            for (int w = 0; w < BL_WORDS && pb.live; ++w) {
                uint32_t m = L.mask[w][q];
                while (m != 0u && pb.live) {
                    uint32_t jj[4];
                    float a[4], cj[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const bool ok = m != 0u;
                        jj[u] = ok ? (uint32_t)(w * 32) + (uint32_t)__builtin_ctz(m) : 0u;
                        m &= m - 1u;
                        const float av = arow[jj[u] * BL_APAD];
                        a[u] = ok ? av : -1.0f;
                        cj[u] = gcol[4 * jj[u]];
                    }
                    bool alive = true;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const bool take = alive && a[u] >= 1.0f / 255.0f;
                        const float Tn = pb.T * (1.0f - a[u]);
                        const bool stop = take && Tn < 0.0001f;
                        const bool add = take && !stop;
                        const float nc = fmaf(cj[u], a[u] * pb.T, pb.C0);
                        pb.C0 = add ? nc : pb.C0;
                        pb.T = add ? Tn : pb.T;
                        if (STATS && stop && sub == 0) pb.n_visit = base + jj[u] + 1u - rg.x;
                        alive = alive && !stop;
                    }
                    pb.live = alive;
                }
            }
        }
#pragma unroll
        for (int w = 0; w < BL_WORDS / 4; ++w) L.mask[sub * (BL_WORDS / 4) + w][q] = 0u;
        lm = quad_live16(__builtin_amdgcn_ballot_w64(pb.live));
        if (lane == 0) L.live[wave] = lm;
        __syncthreads();
    }
    // the pixel's colour from the quad's three channel lanes
    const float c0 = quad_bcast(pb.C0, 0), c1 = quad_bcast(pb.C0, 1), c2 = quad_bcast(pb.C0, 2);
    pb.C0 = c0; pb.C1 = c1; pb.C2 = c2;
}

// Workgroups for n_tiles tiles: four per long tile (at most BL_LONG_CAP of
// them, rounded up to a multiple of 8, plus up to 28 left over by that
// rounding), one per other tile.
__host__ __device__ inline uint32_t blend_long_slots(uint32_t n_tiles) {
    return ((n_tiles < BL_LONG_CAP ? n_tiles : BL_LONG_CAP) + 7u) & ~7u;
}
__host__ __device__ inline uint32_t blend_workgroups(uint32_t n_tiles) {
    return n_tiles + (BL_BANDS - 1) * blend_long_slots(n_tiles) + 4 * 7;
}

// The long tiles (order[n_tiles] of them, at most BL_LONG_CAP) and, among
// them first, those with BL_XLONG pairs or more that the alpha band walk
// takes (order[n_tiles + 1] of them, at most x_cap).
struct BlendSplit {
    uint32_t n_long, n_x;
};
__device__ __forceinline__ BlendSplit blend_split(const uint32_t* __restrict__ order, uint32_t n_tiles,
                                                  uint32_t x_cap) {
    const uint32_t n_long = min(order[n_tiles], blend_long_slots(n_tiles));
    return BlendSplit{n_long, min(min(order[n_tiles + 1], x_cap), n_long)};
}

// Writes the pixel and adds the workgroup's work counters to its tile's.
template <bool STATS>
__device__ __forceinline__ void blend_finish(uint32_t (&st)[2][BL_NT / WAVE], const PixelBlend& pb, uint32_t n_alpha,
                                             int px, int py, int W, int H, uint32_t view, uint32_t tile,
                                             float* __restrict__ image, uint2* __restrict__ stats) {
    if (px < W && py < H) {
        float* o = image + (((size_t)view * H + py) * W + px) * 3;
        o[0] = pb.C0; o[1] = pb.C1; o[2] = pb.C2;
    }
    if (STATS) {
        const uint32_t e = wave_sum(pb.n_visit), al = wave_sum(n_alpha);
        if (__lane_id() == 0) { st[0][threadIdx.x / WAVE] = e; st[1][threadIdx.x / WAVE] = al; }
        __syncthreads();
        if (threadIdx.x == 0) {   // stats cleared before the launch: a long tile's four add up
            uint32_t se = 0, sa = 0;
            for (int i = 0; i < BL_NT / WAVE; ++i) { se += st[0][i]; sa += st[1][i]; }
            atomicAdd(&stats[tile].x, se);
            atomicAdd(&stats[tile].y, sa);
        }
    }
}

// The tiles of `order` but the first n_x: band walk over the long ones,
// strip walk over the others.
template <bool STATS>
__global__ __launch_bounds__(BL_NT) void k_blend(const uint2* __restrict__ ranges, const uint32_t* __restrict__ order,
                                                 const uint32_t* __restrict__ pval, const float4* __restrict__ xy,
                                                 const float4* __restrict__ conic, const float4* __restrict__ rgb,
                                                 int W, int H, int TX, int TY, int n_views, uint32_t x_cap,
                                                 float* __restrict__ image, uint2* __restrict__ stats) {
    __shared__ BlendLds L;
    // Workgroups [0, 4 * n8) serve the long tiles from n_x on (n8: their
    // number rounded up to a multiple of 8), the rest the other tiles in
    // order.  Workgroup ids go round-robin over the eight XCDs, so a long
    // tile's four workgroups are taken 8 ids apart (one XCD).
    const uint32_t n_tiles = (uint32_t)(TX * TY) * (uint32_t)n_views;
    const BlendSplit sp = blend_split(order, n_tiles, x_cap);
    const uint32_t n8 = (sp.n_long - sp.n_x + 7u) & ~7u;
    const uint32_t b = blockIdx.x;
    uint32_t idx;
    int band = -1;
    if (b < 4 * n8) {
        const uint32_t s = b >> 3;
        idx = sp.n_x + (s >> 2) * 8 + (b & 7);
        band = (int)(s & 3);
        if (idx >= sp.n_long) return;
    } else {
        idx = sp.n_long + (b - 4 * n8);
        if (idx >= n_tiles) return;
    }
    const uint32_t tile = order[idx];
    const uint32_t per_view = (uint32_t)(TX * TY);
    const uint32_t view = tile / per_view;
    const uint32_t t = tile - view * per_view;
    const int tx = (int)(t % (uint32_t)TX), ty = (int)(t / (uint32_t)TX);
    const uint2 rg = ranges[tile];
    PixelBlend pb{1.0f, 0.0f, 0.0f, 0.0f, false, 0u};
    uint32_t n_alpha = 0;
    int px, py;
    if (band >= 0)   // uniform over the workgroup
        band_walk<STATS>(L, rg, pval, xy, conic, rgb, tx, ty, band, W, H, pb, n_alpha, px, py);
    else
        strip_walk<STATS>(rg, pval, xy, conic, rgb, tx, ty, W, H, pb, n_alpha, px, py);
    blend_finish<STATS>(L.st, pb, n_alpha, px, py, W, H, view, tile, image, stats);
}

// The first n_x tiles of `order`: the alpha band walk, four workgroups per
// tile (a launch of 4 * x_cap workgroups, x_cap a multiple of 8), beside
// k_blend on another stream.
template <bool STATS>
__global__ __launch_bounds__(BL_NT) void k_blend_x(const uint2* __restrict__ ranges,
                                                   const uint32_t* __restrict__ order,
                                                   const uint32_t* __restrict__ pval, const float4* __restrict__ xy,
                                                   const float4* __restrict__ conic, const float4* __restrict__ rgb,
                                                   int W, int H, int TX, int TY, int n_views, uint32_t x_cap,
                                                   float* __restrict__ image, uint2* __restrict__ stats) {
    __shared__ AlphaLds L;
    const uint32_t n_tiles = (uint32_t)(TX * TY) * (uint32_t)n_views;
    const BlendSplit sp = blend_split(order, n_tiles, x_cap);
    const uint32_t b = blockIdx.x, s = b >> 3;
    const uint32_t idx = (s >> 2) * 8 + (b & 7);
    const int band = (int)(s & 3);
    if (idx >= sp.n_x) return;
    const uint32_t tile = order[idx];
    const uint32_t per_view = (uint32_t)(TX * TY);
    const uint32_t view = tile / per_view;
    const uint32_t t = tile - view * per_view;
    const int tx = (int)(t % (uint32_t)TX), ty = (int)(t / (uint32_t)TX);
    const uint2 rg = ranges[tile];
    PixelBlend pb{1.0f, 0.0f, 0.0f, 0.0f, false, 0u};
    uint32_t n_alpha = 0;
    int px, py;
    band_walk_alpha<STATS>(L, rg, pval, xy, conic, rgb, tx, ty, band, W, H, pb, n_alpha, px, py);
    blend_finish<STATS>(L.st, pb, n_alpha, px, py, W, H, view, tile, image, stats);
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
    a.n_render_dev = nullptr; a.n_rl_dev = nullptr; a.n_views = s.n_views; a.max_total = a.n_total;
    if (a.n_total == 0 || s.n_rl == 0) return;
    hipLaunchKernelGGL(k_preprocess, dim3(nblk(a.n_total, 256)), dim3(256), 0, st, a);
}

void launch_preprocess_dev(hipStream_t st, const SplatArgs& s, const uint32_t* n_render_dev, const uint32_t* n_rl_dev,
                           uint64_t max_total) {
    PreArgs a;
    a.rl = s.rl; a.n_rl = 0; a.pool = s.pool; a.fmt = s.fmt; a.bytes_g = s.fmt == 1 ? 124 : 236;
    a.cams = s.cams; a.W = s.W; a.H = s.H; a.TX = s.TX; a.TY = s.TY;
    a.n_render = 0; a.n_total = 0;
    a.sigma3_tiles = s.sigma3_tiles;
    a.xy = s.xy; a.conic = s.conic; a.rgb = s.rgb; a.depth = s.depth; a.rect = s.rect; a.tiles = s.tiles;
    a.dkey = s.dkey; a.dval = s.dval;
    a.n_render_dev = n_render_dev; a.n_rl_dev = n_rl_dev; a.n_views = s.n_views; a.max_total = max_total;
    if (max_total == 0) return;
    // 8 workgroups of 4 waves per compute unit, striding
    const unsigned nb = (unsigned)std::min<uint64_t>(nblk(max_total, 256), 2048);
    hipLaunchKernelGGL(k_preprocess, dim3(nb), dim3(256), 0, st, a);
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

uint32_t blend_x_cap(uint32_t n_tiles, uint32_t want) {
    const uint32_t c = std::min({want, n_tiles, BL_LONG_CAP});
    return (c + 7u) & ~7u;
}

void launch_blend(hipStream_t st, const uint2* ranges, const uint32_t* order, const uint32_t* pval, const float4* xy,
                  const float4* conic, const float4* rgb, int W, int H, int TX, int TY, int n_views, uint32_t x_cap,
                  float* image, uint2* stats) {
    const uint32_t n_tiles = (uint32_t)(TX * TY * n_views);
    if (!n_tiles) return;
    const uint32_t n_blocks = blend_workgroups(n_tiles);
    if (stats)
        hipLaunchKernelGGL(k_blend<true>, dim3(n_blocks), dim3(BL_NT), 0, st, ranges, order, pval, xy, conic, rgb, W,
                           H, TX, TY, n_views, x_cap, image, stats);
    else
        hipLaunchKernelGGL(k_blend<false>, dim3(n_blocks), dim3(BL_NT), 0, st, ranges, order, pval, xy, conic, rgb, W,
                           H, TX, TY, n_views, x_cap, image, stats);
}

void launch_blend_x(hipStream_t st, const uint2* ranges, const uint32_t* order, const uint32_t* pval,
                    const float4* xy, const float4* conic, const float4* rgb, int W, int H, int TX, int TY,
                    int n_views, uint32_t x_cap, float* image, uint2* stats) {
    const uint32_t n_tiles = (uint32_t)(TX * TY * n_views);
    if (!n_tiles || !x_cap) return;
    const uint32_t n_blocks = BL_BANDS * x_cap;
    if (stats)
        hipLaunchKernelGGL(k_blend_x<true>, dim3(n_blocks), dim3(BL_NT), 0, st, ranges, order, pval, xy, conic, rgb,
                           W, H, TX, TY, n_views, x_cap, image, stats);
    else
        hipLaunchKernelGGL(k_blend_x<false>, dim3(n_blocks), dim3(BL_NT), 0, st, ranges, order, pval, xy, conic, rgb,
                           W, H, TX, TY, n_views, x_cap, image, stats);
}

}  // namespace vm
