// Kernels of the page-prefetch network: bf16 matrix products on the gfx950
// matrix cores (v_mfma_f32_32x32x16_bf16, fp32 accumulation) with fused
// epilogues, the logistic loss, bias gradients and Adam.
//
//  k_gemm      C[M][N] = A[M][K] B[K][N] for row-major bf16 A and B, either
//              one read transposed; 256 threads, a 64 x 64 tile of C, four
//              waves of 32 x 32; K in steps of 32 staged through LDS
//              (entries past M, N or K read as zero).
//              Epilogues: + bias, ReLU, bf16 out (hidden layers); + bias,
//              fp32 out (logits); fp32 out (weight gradients); ReLU mask of
//              the layer's input, bf16 out (input gradients).
//  k_bce       per logit: d = (sigmoid(z) - y) / (B K) as bf16, loss terms.
//  k_colsum    bias gradients: column sums of d.
//  k_adam      Adam on the fp32 master weights, bf16 copies for the products.
//
// bf16 here is round-to-nearest-even of the fp32 value (no NaN inputs).
#include "kcommon.h"
#include "vm3dgs_impl.h"

namespace vmk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int GM = 64, GN = 64, GK = 32;
constexpr int LDK = GK + 8;   // LDS row pitch in bf16 (16-byte aligned rows, fewer bank conflicts)

enum Epi { E_BIAS_RELU_BF16 = 0, E_BIAS_F32 = 1, E_F32 = 2, E_MASK_BF16 = 3 };

struct GemmArgs {
    const uint16_t* A; int lda;
    const uint16_t* B; int ldb;
    int M, N, K;
    int m_valid;                 // rows >= m_valid are written as zero (padding of the batch)
    const float* bias;           // E_BIAS_*
    const uint16_t* mask; int ldmask;   // E_MASK_BF16: zero where mask <= 0
    void* C; int ldc;
};

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t sA[GM][LDK];
    __shared__ __attribute__((aligned(16))) uint16_t sB[GN][LDK];   // B tile stored n-major: sB[n][k]
    const int t = threadIdx.x;
    const int m0 = blockIdx.y * GM, n0 = blockIdx.x * GN;
    const int w = t / WAVE, l = t % WAVE;
    const int wm = (w / 2) * 32, wn = (w % 2) * 32;
    f32x16 acc = {};
    for (int k0 = 0; k0 < g.K; k0 += GK) {
        // stage A (64 x 32) and B (32 x 64): 8 elements per thread each
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int e = r * 256 + t;
            int m, k;
            if (TA) { k = e / GM; m = e % GM; } else { m = e / GK; k = e % GK; }
            const int gm = m0 + m, gk = k0 + k;
            uint16_t v = 0;
            if (gm < g.M && gk < g.K) v = TA ? g.A[(size_t)gk * g.lda + gm] : g.A[(size_t)gm * g.lda + gk];
            sA[m][k] = v;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int e = r * 256 + t;
            int n, k;
            if (TB) { n = e / GK; k = e % GK; } else { k = e / GN; n = e % GN; }
            const int gn = n0 + n, gk = k0 + k;
            uint16_t v = 0;
            if (gn < g.N && gk < g.K) v = TB ? g.B[(size_t)gn * g.ldb + gk] : g.B[(size_t)gk * g.ldb + gn];
            sB[n][k] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; kk += 16) {
            const bf16x8 a = *(const bf16x8*)&sA[wm + l % 32][kk + 8 * (l / 32)];
            const bf16x8 b = *(const bf16x8*)&sB[wn + l % 32][kk + 8 * (l / 32)];
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // lane l holds C[wm + 8j + 4(l/32) + i][wn + l%32] in acc[4j + i]
    const int n = n0 + wn + l % 32;
    if (n >= g.N) return;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = m0 + wm + 8 * j + 4 * (l / 32) + i;
            if (m >= g.M) continue;
            float v = acc[4 * j + i];
            const bool live = m < g.m_valid;
            if (EPI == E_BIAS_RELU_BF16) {
                v = v + g.bias[n];
                v = v > 0.0f ? v : 0.0f;
                ((uint16_t*)g.C)[(size_t)m * g.ldc + n] = live ? to_bf16(v) : (uint16_t)0;
            } else if (EPI == E_BIAS_F32) {
                ((float*)g.C)[(size_t)m * g.ldc + n] = live ? v + g.bias[n] : 0.0f;
            } else if (EPI == E_F32) {
                ((float*)g.C)[(size_t)m * g.ldc + n] = v;
            } else {
                const bool on = live && from_bf16(g.mask[(size_t)m * g.ldmask + n]) > 0.0f;
                ((uint16_t*)g.C)[(size_t)m * g.ldc + n] = on ? to_bf16(v) : (uint16_t)0;
            }
        }
}

// fp32 rows -> bf16 rows of a wider (zero-padded) matrix; rows >= n_valid zero
__global__ void k_to_bf16_rows(const float* __restrict__ x, int rows, int cols, int n_valid, uint16_t* __restrict__ y,
                               int ldy) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)rows * ldy) return;
    const int r = (int)(i / ldy), c = (int)(i % ldy);
    y[i] = (r < n_valid && c < cols) ? to_bf16(x[(size_t)r * cols + c]) : (uint16_t)0;
}

// logistic loss of the logits: d = (sigmoid(z) - y) * inv as bf16, and per
// block the sum of softplus(z) - y z
// (rows B .. rows-1 of d are the batch padding and are written as zero)
__global__ __launch_bounds__(256) void k_bce(const float* __restrict__ z, const float* __restrict__ y, int B, int rows,
                                             int K, float inv, uint16_t* __restrict__ d, float* __restrict__ part) {
    __shared__ float sh[256 / WAVE];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float term = 0.0f;
    if (i < (int64_t)rows * K) {
        const int r = (int)(i / K);
        uint16_t dv = 0;
        if (r < B) {
            const float zi = z[i], yi = y[i];
            const float s = 1.0f / (1.0f + expf(-zi));
            dv = to_bf16((s - yi) * inv);
            term = (zi > 0.0f ? zi : 0.0f) + log1pf(expf(-fabsf(zi))) - yi * zi;
        }
        d[i] = dv;
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) term += __shfl_xor(term, o, WAVE);
    if (__lane_id() == 0) sh[threadIdx.x / WAVE] = term;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int k = 0; k < 256 / WAVE; ++k) s += sh[k];
        part[blockIdx.x] = s;
    }
}

// db[n] = sum over the first B rows of d[.][n]
__global__ void k_colsum(const uint16_t* __restrict__ d, int B, int N, int ldd, float* __restrict__ db) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.0f;
    for (int r = 0; r < B; ++r) s += from_bf16(d[(size_t)r * ldd + n]);
    db[n] = s;
}

struct AdamLayer {
    int din, dout, ld_pad;        // bf16 copy: [din_pad][dout], rows >= din stay zero
    int64_t off;                  // offset of W in the parameter vector
    uint16_t* wb;
};

// one layer's weights and bias: index i over din*dout + dout parameters
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, AdamLayer L, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nw = (int64_t)L.din * L.dout;
    if (i >= nw + L.dout) return;
    const int64_t p = L.off + i;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.0f - b1) * gi;
    const float vi = b2 * v[p] + (1.0f - b2) * (gi * gi);
    m[p] = mi;
    v[p] = vi;
    const float wi = w[p] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[p] = wi;
    if (i < nw) L.wb[i] = to_bf16(wi);   // [din][dout] row-major, same index
}

// bf16 copies of a layer's weights from the masters
__global__ void k_w_to_bf16(const float* __restrict__ w, int64_t off, int n, uint16_t* __restrict__ wb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = to_bf16(w[off + i]);
}

// rows idx[i] of src [.][width] into dst [i][width] (training minibatches)
__global__ void k_gather_rows(const float* __restrict__ src, const uint32_t* __restrict__ idx, uint32_t n,
                              uint32_t width, float* __restrict__ dst) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint64_t)n * width) return;
    const uint64_t r = i / width, c = i - r * width;
    dst[i] = src[(uint64_t)idx[r] * width + c];
}

}  // namespace vmk

namespace vm {

void launch_gather_rows(hipStream_t st, const float* src, const uint32_t* idx, uint32_t n, uint32_t width,
                        float* dst) {
    const uint64_t total = (uint64_t)n * width;
    if (total == 0) return;
    hipLaunchKernelGGL(vmk::k_gather_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, src, idx, n, width,
                       dst);
}
using namespace vmk;

static unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <bool TA, bool TB, int EPI>
static void gemm(hipStream_t st, const GemmArgs& g) {
    const dim3 grid((unsigned)((g.N + GN - 1) / GN), (unsigned)((g.M + GM - 1) / GM));
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, st, g);
}

void mlp_forward_dev(hipStream_t st, const MlpDev& d, int B) {
    const int nl = d.n_layers;
    for (int l = 0; l < nl; ++l) {
        GemmArgs g{};
        g.A = d.act[l]; g.lda = d.kpad[l];
        g.B = d.wb[l]; g.ldb = d.dims[l + 1];
        g.M = d.b_pad; g.N = d.dims[l + 1]; g.K = d.kpad[l]; g.m_valid = B;
        g.bias = d.master + d.off[l] + (int64_t)d.dims[l] * d.dims[l + 1];
        if (l + 1 < nl) {
            g.C = d.act[l + 1]; g.ldc = d.kpad[l + 1];
            gemm<false, false, E_BIAS_RELU_BF16>(st, g);
        } else {
            g.C = d.logits; g.ldc = d.dims[nl];
            gemm<false, false, E_BIAS_F32>(st, g);
        }
    }
}

void mlp_input_dev(hipStream_t st, const MlpDev& d, const float* x, int B) {
    const int64_t n = (int64_t)d.b_pad * d.kpad[0];
    hipLaunchKernelGGL(k_to_bf16_rows, dim3(nb(n, 256)), dim3(256), 0, st, x, d.b_pad, d.dims[0], B, d.act[0],
                       d.kpad[0]);
}

void mlp_backward_dev(hipStream_t st, const MlpDev& d, const float* y, int B) {
    const int nl = d.n_layers, K = d.dims[nl];
    const int64_t nz = (int64_t)B * K;
    hipLaunchKernelGGL(k_bce, dim3(nb((int64_t)d.b_pad * K, 256)), dim3(256), 0, st, d.logits, y, B, d.b_pad, K,
                       1.0f / (float)nz, d.dz[nl - 1], d.loss_part);
    for (int l = nl - 1; l >= 0; --l) {
        const int din = d.dims[l], dout = d.dims[l + 1];
        // weight gradient: X^T dZ  ([din][B_pad] x [B_pad][dout])
        GemmArgs g{};
        g.A = d.act[l]; g.lda = d.kpad[l];
        g.B = d.dz[l]; g.ldb = dout;
        g.M = din; g.N = dout; g.K = d.b_pad; g.m_valid = din;
        g.C = d.grad + d.off[l]; g.ldc = dout;
        gemm<true, false, E_F32>(st, g);
        hipLaunchKernelGGL(k_colsum, dim3(nb(dout, 256)), dim3(256), 0, st, d.dz[l], B, dout, dout,
                           d.grad + d.off[l] + (int64_t)din * dout);
        if (l == 0) break;
        // input gradient: dZ W^T through the ReLU of the layer below
        GemmArgs h{};
        h.A = d.dz[l]; h.lda = dout;
        h.B = d.wb[l]; h.ldb = dout;
        h.M = d.b_pad; h.N = din; h.K = dout; h.m_valid = B;
        h.mask = d.act[l]; h.ldmask = d.kpad[l];
        h.C = d.dz[l - 1]; h.ldc = din;
        gemm<false, true, E_MASK_BF16>(st, h);
    }
}

void mlp_adam_dev(hipStream_t st, const MlpDev& d, float lr, float b1, float b2, float eps, int t) {
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    for (int l = 0; l < d.n_layers; ++l) {
        AdamLayer L;
        L.din = d.dims[l]; L.dout = d.dims[l + 1]; L.ld_pad = d.kpad[l]; L.off = d.off[l]; L.wb = d.wb[l];
        const int64_t n = (int64_t)L.din * L.dout + L.dout;
        hipLaunchKernelGGL(k_adam, dim3(nb(n, 256)), dim3(256), 0, st, d.master, d.adam_m, d.adam_v, d.grad, L, lr,
                           b1, b2, eps, c1, c2);
    }
}

void mlp_sync_bf16_dev(hipStream_t st, const MlpDev& d) {
    for (int l = 0; l < d.n_layers; ++l) {
        const int n = d.dims[l] * d.dims[l + 1];
        hipLaunchKernelGGL(k_w_to_bf16, dim3(nb(n, 256)), dim3(256), 0, st, d.master, d.off[l], n, d.wb[l]);
    }
}

}  // namespace vm
