// kcommon.h -- device helpers shared by the gfx950 kernels of the VM-3DGS
// frame path (wave64 primitives, the splat math of Kerbl et al. that the
// paper keeps for its renderer, Sec. 4.2).
//
// All kernels are compiled with -ffp-contract=off: every float operation is
// the IEEE operation written here, fused multiply-adds only where fmaf() is
// written.  Decisions that turn floats into integers (tile rectangles, depth
// keys, visibility, alpha thresholds) therefore have one exact definition.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vmk {

constexpr int WAVE = 64;
constexpr int TILE = 16;           // splat tile edge in pixels
constexpr int SUBS = 64;           // sub-slots per physical page (8^2 at most)
constexpr uint32_t NONE32 = 0xffffffffu;
constexpr unsigned long long NONE64 = 0xffffffffffffffffull;

// ---------------------------------------------------------------- wave64
__device__ __forceinline__ uint64_t lanemask_lt() {
    const uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Lanes of this wave whose 8-bit digit equals mine (valid lanes only).
__device__ __forceinline__ uint64_t match_digit8(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

// inclusive scan over the 64 lanes of a wave
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, WAVE);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Exclusive scan across a block of NT threads (NT a multiple of 64); returns
// this thread's exclusive prefix and writes the block total.  Uses `sh`
// (NT/64 words of LDS).  Contains barriers: call from every thread.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
    const int lane = __lane_id();
    const int w = threadIdx.x / WAVE;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == WAVE - 1) sh[w] = inc;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / WAVE; ++i) {
        const uint32_t s = sh[i];
        if (i < w) wbase += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wbase + inc - v;
}

// ---------------------------------------------------------------- math
// exp for the alpha decisions: Cody-Waite reduction n = rint(x log2 e),
// r = x - n ln2 (ln2 = 22713/32768 + tail, so n*head is exact), degree-7
// Taylor polynomial in Horner form with fused multiply-adds, times 2^n.
// Zero below -87 (where e^x is still a normal float).
// vm_exp without its underflow branch: equal to vm_exp for x in [-87, 0]
__device__ __forceinline__ float vm_exp_core(float x) {
    const float kLog2e = (float)(1.0 / 0.69314718055994530942);
    const float kLn2Hi = (float)(22713.0 / 32768.0);
    const float kLn2Lo = (float)(0.69314718055994530942 - 22713.0 / 32768.0);
    const float n = rintf(x * kLog2e);
    float r = fmaf(-n, kLn2Hi, x);
    r = fmaf(-n, kLn2Lo, r);
    float p = (float)(1.0 / 5040.0);
    p = fmaf(p, r, (float)(1.0 / 720.0));
    p = fmaf(p, r, (float)(1.0 / 120.0));
    p = fmaf(p, r, (float)(1.0 / 24.0));
    p = fmaf(p, r, (float)(1.0 / 6.0));
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, 1.0f);
    p = fmaf(p, r, 1.0f);
    const int e = (int)n + 127;
    return p * __int_as_float(e << 23);
}

__device__ __forceinline__ float vm_exp(float x) {
    if (!(x >= -87.0f)) return 0.0f;
    const float kLog2e = (float)(1.0 / 0.69314718055994530942);
    const float kLn2Hi = (float)(22713.0 / 32768.0);
    const float kLn2Lo = (float)(0.69314718055994530942 - 22713.0 / 32768.0);
    const float n = rintf(x * kLog2e);
    float r = fmaf(-n, kLn2Hi, x);
    r = fmaf(-n, kLn2Lo, r);
    float p = (float)(1.0 / 5040.0);
    p = fmaf(p, r, (float)(1.0 / 720.0));
    p = fmaf(p, r, (float)(1.0 / 120.0));
    p = fmaf(p, r, (float)(1.0 / 24.0));
    p = fmaf(p, r, (float)(1.0 / 6.0));
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, 1.0f);
    p = fmaf(p, r, 1.0f);
    const int e = (int)n + 127;  // n in [-126, 0] for the splat's arguments
    return p * __int_as_float(e << 23);
}

// world -> camera: ((r0 x + r1 y) + r2 z) + t
__device__ __forceinline__ float3 view_xform(const float* V, float x, float y, float z) {
    float3 o;
    o.x = ((V[0] * x + V[1] * y) + V[2] * z) + V[3];
    o.y = ((V[4] * x + V[5] * y) + V[6] * z) + V[7];
    o.z = ((V[8] * x + V[9] * y) + V[10] * z) + V[11];
    return o;
}

// Real SH basis to degree 3 (orthonormal; sign convention fixed), applied to
// coefficients c[k*3 + ch], plus the 0.5 offset, clamped at zero.
struct ShConst {
    static constexpr float k0 = 0.28209479177387814f;
    static constexpr float k1 = -0.48860251190291992f;
    static constexpr float k2 = 0.48860251190291992f;
    static constexpr float k3 = -0.48860251190291992f;
    static constexpr float k4 = 1.0925484305920792f;
    static constexpr float k5 = -1.0925484305920792f;
    static constexpr float k6 = 0.31539156525252005f;
    static constexpr float k7 = -1.0925484305920792f;
    static constexpr float k8 = 0.54627421529603959f;
    static constexpr float k9 = -0.59004358992664352f;
    static constexpr float k10 = 2.8906114426405538f;
    static constexpr float k11 = -0.45704579946446572f;
    static constexpr float k12 = 0.3731763325901154f;
    static constexpr float k13 = -0.45704579946446572f;
    static constexpr float k14 = 1.4453057213202769f;
    static constexpr float k15 = -0.59004358992664352f;
};

// ---------------------------------------------------------------- layout
// Page blocks are SoA over the Gaussians of one (sub-)page.
//  fp32 form: 59 float arrays: mean xyz, scale xyz, quat wxyz, opacity, sh[48]
//  half form: mean xyz (3 float arrays), 4 u32 arrays of fp16 pairs
//             (sx,sy) (sz,qw) (qx,qy) (qz,opacity), 24 u32 arrays of bf16
//             pairs (sh[2m], sh[2m+1]).
struct Gauss {
    float m[3], s[3], q[4], o;
    float sh[48];
};

__device__ __forceinline__ float bf16_lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }
__device__ __forceinline__ float f16_lo(uint32_t u) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(u & 0xffffu));
}
__device__ __forceinline__ float f16_hi(uint32_t u) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(u >> 16));
}

}  // namespace vmk
