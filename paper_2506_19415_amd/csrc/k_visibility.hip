// k_visibility.hip -- page determination of Sec. 4.1 on gfx950.
//
//  k_frustum       page bounding sphere vs near plane and the four side planes
//  k_rays          per ID-buffer pixel: reciprocal world direction of the
//                  ray through the pixel centre (view depth = ray parameter);
//                  the buffer spans the image widened by a guard band of G
//                  pixels per edge, the frustum planes likewise
//  k_cell_rects    per (view, proxy box of a candidate page): its conservative
//                  pixel rectangle in the ID buffer and area
//  k_raster_items  one thread per (box, pixel) item, balanced over the whole
//                  grid by a prefix sum of the areas: the ray through the
//                  pixel centre against the box (slab test); 64-bit atomicMin
//                  of (depth bits << 32 | page + 1): nearest wins whatever
//                  the order
//  k_reduce        per pixel: nearest depth per page (Sec. 5.1.1 reduction),
//                  one atomic per page per wave
//  k_links         a directly seen page pushes its depth to its linked pages
//  k_requests      LOD level from the projected page radius, request keys
//                  (class, depth, page)
//
// Also the frame's small utility launches: k_fill_multi (the clears at the
// start of a frame, in one launch) and k_readback (the readbacks at a host
// wait, written by the GPU into mapped pinned host memory, in one launch).
#include <algorithm>
#include <stdexcept>

#include "kcommon.h"
#include "vm3dgs_impl.h"

namespace vmk {

using vm::CamK;

__global__ void k_frustum(const float4* __restrict__ sph, int n_pg, const CamK* __restrict__ cams, int n_views,
                          int W, int H, float G, uint8_t* __restrict__ cand, uint32_t* __restrict__ counters) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_pg * n_views) return;
    const int v = (int)(i / n_pg);
    const int p = (int)(i - (int64_t)v * n_pg);
    const CamK& c = cams[v];
    const float4 s = sph[p];
    const float3 q = view_xform(c.V, s.x, s.y, s.z);
    const float r = s.w;
    bool in = q.z + r > c.znear;
    const float tl = (c.cx + G) / c.fx, tr = (((float)W + G) - c.cx) / c.fx;
    const float tt = (c.cy + G) / c.fy, tb = (((float)H + G) - c.cy) / c.fy;
    const float kl = sqrtf(1.0f + tl * tl), kr = sqrtf(1.0f + tr * tr);
    const float kt = sqrtf(1.0f + tt * tt), kb = sqrtf(1.0f + tb * tb);
    in = in && (q.x + tl * q.z >= -(r * kl));
    in = in && (-q.x + tr * q.z >= -(r * kr));
    in = in && (q.y + tt * q.z >= -(r * kt));
    in = in && (-q.y + tb * q.z >= -(r * kb));
    cand[i] = in ? 1 : 0;
    const uint64_t b = __ballot(in);
    if (__lane_id() == 0 && b) atomicAdd(&counters[vm::C_CAND], (uint32_t)__popcll(b));
}

__global__ void k_rays(const CamK* __restrict__ cams, int n_views, int W, int H, float G, int Wv, int Hv,
                       float4* __restrict__ rays) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t npx = (int64_t)Wv * Hv;
    if (i >= npx * n_views) return;
    const int v = (int)(i / npx);
    const int pix = (int)(i - v * npx);
    const int px = pix % Wv, py = pix / Wv;
    const CamK& c = cams[v];
    const float sx = ((float)W + 2.0f * G) / (float)Wv, sy = ((float)H + 2.0f * G) / (float)Hv;
    const float xc = ((float)px + 0.5f) * sx - G, yc = ((float)py + 0.5f) * sy - G;
    const float dcx = (xc - c.cx) / c.fx;
    const float dcy = (yc - c.cy) / c.fy;
    float inv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float d = (c.V[a] * dcx + c.V[4 + a] * dcy) + c.V[8 + a];
        if (d == 0.0f) d = 1e-30f;
        inv[a] = 1.0f / d;
    }
    rays[i] = make_float4(inv[0], inv[1], inv[2], 0.0f);
}

// conservative inclusive pixel rectangle of a world box in the ID buffer
__device__ bool box_rect(const CamK& c, int W, int H, float G, int Wv, int Hv, const float* b, int4* r) {
    float vmin[3] = {INFINITY, INFINITY, INFINITY}, vmax[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float3 p = view_xform(c.V, b[(k & 1) ? 3 : 0], b[(k & 2) ? 4 : 1], b[(k & 4) ? 5 : 2]);
        vmin[0] = fminf(vmin[0], p.x); vmax[0] = fmaxf(vmax[0], p.x);
        vmin[1] = fminf(vmin[1], p.y); vmax[1] = fmaxf(vmax[1], p.y);
        vmin[2] = fminf(vmin[2], p.z); vmax[2] = fmaxf(vmax[2], p.z);
    }
    if (!(vmax[2] > c.znear * 0.5f)) return false;
    const float z0 = fmaxf(vmin[2], c.znear * 0.5f), z1 = vmax[2];
    const float xl = fminf(fminf(vmin[0] / z0, vmin[0] / z1), fminf(vmax[0] / z0, vmax[0] / z1));
    const float xh = fmaxf(fmaxf(vmin[0] / z0, vmin[0] / z1), fmaxf(vmax[0] / z0, vmax[0] / z1));
    const float yl = fminf(fminf(vmin[1] / z0, vmin[1] / z1), fminf(vmax[1] / z0, vmax[1] / z1));
    const float yh = fmaxf(fmaxf(vmin[1] / z0, vmin[1] / z1), fmaxf(vmax[1] / z0, vmax[1] / z1));
    const float sx = ((float)W + 2.0f * G) / (float)Wv, sy = ((float)H + 2.0f * G) / (float)Hv;
    float fx0 = floorf(((c.fx * xl + c.cx) + G) / sx) - 1.0f, fx1 = floorf(((c.fx * xh + c.cx) + G) / sx) + 1.0f;
    float fy0 = floorf(((c.fy * yl + c.cy) + G) / sy) - 1.0f, fy1 = floorf(((c.fy * yh + c.cy) + G) / sy) + 1.0f;
    fx0 = fmaxf(fx0, 0.0f); fy0 = fmaxf(fy0, 0.0f);
    fx1 = fminf(fx1, (float)(Wv - 1)); fy1 = fminf(fy1, (float)(Hv - 1));
    if (!(fx0 <= fx1) || !(fy0 <= fy1)) return false;
    *r = make_int4((int)fx0, (int)fy0, (int)fx1, (int)fy1);
    return true;
}

constexpr int PR_NT = 256;

// per (view, cell): the pixel rectangle of a candidate page's box and its area
__global__ void k_cell_rects(const float4* __restrict__ lo4, const float4* __restrict__ hi4, int64_t nc,
                             const uint8_t* __restrict__ cand, int n_pg, const CamK* __restrict__ cams, int n_views,
                             int W, int H, float G, int Wv, int Hv, int4* __restrict__ rects,
                             uint32_t* __restrict__ area) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc * n_views) return;
    const int v = (int)(i / nc);
    const int64_t c = i - (int64_t)v * nc;
    const float4 l = lo4[c], h = hi4[c];
    const uint32_t page = __float_as_uint(l.w);
    int4 r = make_int4(0, 0, -1, -1);
    uint32_t a = 0;
    if (cand[(int64_t)v * n_pg + page]) {
        const float b[6] = {l.x, l.y, l.z, h.x, h.y, h.z};
        if (box_rect(cams[v], W, H, G, Wv, Hv, b, &r)) a = (uint32_t)((r.z - r.x + 1) * (r.w - r.y + 1));
    }
    rects[i] = r;
    area[i] = a;
}

// one (cell, pixel) item per thread and step: the ray through the pixel centre
// against the cell's box.  Thread 0 brackets the slots holding the block's
// items; each thread then finds its slot by binary search inside the bracket.
__global__ __launch_bounds__(PR_NT) void k_raster_items(const float4* __restrict__ lo4, const float4* __restrict__ hi4,
                                                       int64_t nc, const CamK* __restrict__ cams, int Wv, int Hv,
                                                       const int4* __restrict__ rects, const uint32_t* __restrict__ offs,
                                                       const uint32_t* __restrict__ total_p, int64_t n_slots,
                                                       const float4* __restrict__ rays,
                                                       unsigned long long* __restrict__ idbuf) {
    __shared__ int64_t s_lo, s_hi;
    const uint32_t total = *total_p;      // = offs[n_slots]
    const int64_t npx = (int64_t)Wv * Hv;
    for (uint64_t b0 = (uint64_t)blockIdx.x * PR_NT; b0 < total; b0 += (uint64_t)gridDim.x * PR_NT) {
        if (threadIdx.x == 0) {
            // slot of item x: the first s with offs[s + 1] > x (it has area > 0)
            int64_t lo = 0, hi = n_slots - 1;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (offs[mid + 1] > b0) hi = mid; else lo = mid + 1;
            }
            s_lo = lo;
            const uint64_t last = min((uint64_t)total - 1, b0 + PR_NT - 1);
            int64_t l2 = lo, h2 = n_slots - 1;
            while (l2 < h2) {
                const int64_t mid = (l2 + h2) >> 1;
                if (offs[mid + 1] > last) h2 = mid; else l2 = mid + 1;
            }
            s_hi = l2;
        }
        __syncthreads();
        const uint64_t item = b0 + threadIdx.x;
        if (item < total) {
            int64_t a = s_lo, bnd = s_hi;
            while (a < bnd) {
                const int64_t mid = (a + bnd) >> 1;
                if (offs[mid + 1] > item) bnd = mid; else a = mid + 1;
            }
            const int64_t slot = a;
            const int v = (int)(slot / nc);
            const int64_t c = slot - (int64_t)v * nc;
            const int4 rr = rects[slot];
            const uint32_t w = (uint32_t)(rr.z - rr.x + 1);
            const uint32_t k = (uint32_t)(item - offs[slot]);
            const int px = rr.x + (int)(k % w), py = rr.y + (int)(k / w);
            const CamK& cam = cams[v];
            const float4 inv = rays[v * npx + (int64_t)py * Wv + px];
            const float4 l4 = lo4[c], h4 = hi4[c];
            float ta = (l4.x - cam.pos[0]) * inv.x, tb = (h4.x - cam.pos[0]) * inv.x;
            float t0 = fminf(ta, tb), t1 = fmaxf(ta, tb);
            ta = (l4.y - cam.pos[1]) * inv.y; tb = (h4.y - cam.pos[1]) * inv.y;
            t0 = fmaxf(t0, fminf(ta, tb)); t1 = fminf(t1, fmaxf(ta, tb));
            ta = (l4.z - cam.pos[2]) * inv.z; tb = (h4.z - cam.pos[2]) * inv.z;
            t0 = fmaxf(t0, fminf(ta, tb)); t1 = fminf(t1, fmaxf(ta, tb));
            if (t0 <= t1 && t1 > cam.znear) {
                const float d = fmaxf(t0, cam.znear);
                const unsigned long long key =
                    ((unsigned long long)__float_as_uint(d) << 32) | (unsigned long long)(__float_as_uint(l4.w) + 1u);
                atomicMin(&idbuf[v * npx + (int64_t)py * Wv + px], key);
            }
        }
        __syncthreads();
    }
}

__global__ void k_reduce(const unsigned long long* __restrict__ idbuf, int64_t n, uint32_t* __restrict__ req_direct) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long k = i < n ? idbuf[i] : NONE64;
    const bool valid = k != NONE64;
    const uint32_t page = (uint32_t)(k & 0xffffffffull) - 1u;
    const uint32_t d = (uint32_t)(k >> 32);
    // neighbouring pixels mostly show the same page: one atomic per page per wave
    uint64_t active = __ballot(valid);
    while (active) {
        const int leader = __ffsll((unsigned long long)active) - 1;
        const uint32_t lp = __shfl(page, leader, WAVE);
        const bool mine = valid && page == lp;
        uint32_t m = mine ? d : NONE32;
#pragma unroll
        for (int o = WAVE / 2; o > 0; o >>= 1) m = min(m, (uint32_t)__shfl_xor(m, o, WAVE));
        if ((int)__lane_id() == leader) atomicMin(&req_direct[lp], m);
        active &= ~__ballot(mine);
    }
}

__global__ void k_links(const uint32_t* __restrict__ req_direct, const int32_t* __restrict__ ls,
                        const int32_t* __restrict__ ld, int n_pg, uint32_t* __restrict__ req_link) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_pg) return;
    const uint32_t d = req_direct[q];
    if (d == NONE32) return;
    for (int e = ls[q]; e < ls[q + 1]; ++e) atomicMin(&req_link[ld[e]], d);
}

__global__ void k_requests(const uint32_t* __restrict__ rd, const uint32_t* __restrict__ rl,
                           const float4* __restrict__ sph, int n_pg, int L, float tau, float fy,
                           int8_t* __restrict__ page_level, uint64_t* __restrict__ keys,
                           uint32_t* __restrict__ counters) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    bool req = false, direct = false;
    uint64_t key = 0;
    if (p < n_pg) {
        const uint32_t a = rd[p], b = rl[p];
        const uint32_t d = a < b ? a : b;
        int8_t lvl = -1;
        if (d != NONE32) {
            req = true;
            direct = a != NONE32;
            int l = 0;
            if (L > 1) {
                const float rpx = (fy * sph[p].w) / __uint_as_float(d);
                float thr = tau;
                while (l < L - 1 && !(rpx > thr)) { ++l; thr = thr * 0.5f; }
            }
            lvl = (int8_t)l;
            key = ((uint64_t)(direct ? 0u : 1u) << 61) | ((uint64_t)d << 30) | (uint64_t)p;
        }
        page_level[p] = lvl;
    }
    // wave-aggregated compaction; order is restored by the sort of the keys
    const uint64_t m = __ballot(req);
    const uint64_t md = __ballot(direct);
    const uint64_t mc = __ballot(req && p < n_pg && page_level[p] > 0);
    uint32_t base = 0;
    if (__lane_id() == 0 && m) {
        base = atomicAdd(&counters[vm::C_NREQ], (uint32_t)__popcll(m));
        atomicAdd(&counters[vm::C_DIRECT], (uint32_t)__popcll(md));
        atomicAdd(&counters[vm::C_LINKED], (uint32_t)(__popcll(m) - __popcll(md)));
        if (mc) atomicAdd(&counters[vm::C_NCOARSE], (uint32_t)__popcll(mc));
    }
    base = __shfl(base, 0, WAVE);
    if (req) keys[base + __popcll(m & lanemask_lt())] = key;
}

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// several fills in one launch (the clears at the start of a frame, where the
// GPU would otherwise wait for the host to submit each small kernel)
__global__ void k_fill_multi(vm::FillSegs f) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (int s = 0; s < f.n; ++s) {
        const vm::FillSeg g = f.seg[s];
        for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += stride) {
            if (g.wide) ((unsigned long long*)g.p)[i] = g.v;
            else ((uint32_t*)g.p)[i] = (uint32_t)g.v;
        }
    }
}

// small device-to-host readbacks in one launch, instead of one copy command
// each: 4-byte words where source, destination and size allow, else bytes;
// the system-scope fence makes the writes visible to the host once the
// stream has passed the kernel
__global__ __launch_bounds__(256) void k_readback(vm::ReadSegs r) {
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t i0 = blockIdx.x * blockDim.x + threadIdx.x;
    for (int s = 0; s < r.n; ++s) {
        const vm::ReadSeg g = r.seg[s];
        if ((((uintptr_t)g.src | (uintptr_t)g.dst | (uintptr_t)g.bytes) & 3u) == 0) {
            const uint32_t* a = (const uint32_t*)g.src;
            uint32_t* b = (uint32_t*)g.dst;
            for (uint32_t i = i0; i < g.bytes / 4; i += stride) b[i] = a[i];
        } else {
            const uint8_t* a = (const uint8_t*)g.src;
            uint8_t* b = (uint8_t*)g.dst;
            for (uint32_t i = i0; i < g.bytes; i += stride) b[i] = a[i];
        }
    }
    __threadfence_system();
}

}  // namespace vmk

namespace vm {
using namespace vmk;

static unsigned nblk(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

void launch_fill_u32(hipStream_t st, uint32_t* p, uint64_t n, uint32_t v) {
    if (n) hipLaunchKernelGGL(k_fill_u32, dim3(nblk(n, 256)), dim3(256), 0, st, p, n, v);
}

void launch_fill_u64(hipStream_t st, unsigned long long* p, uint64_t n, unsigned long long v) {
    if (n) hipLaunchKernelGGL(k_fill_u64, dim3(nblk(n, 256)), dim3(256), 0, st, p, n, v);
}

void launch_fill_multi(hipStream_t st, const FillSegs& f) {
    uint64_t mx = 0;
    for (int s = 0; s < f.n; ++s) mx = std::max(mx, f.seg[s].n);
    if (mx) hipLaunchKernelGGL(k_fill_multi, dim3((unsigned)std::min<uint64_t>(nblk(mx, 256), 1024)), dim3(256), 0, st,
                               f);
}

void launch_readback(hipStream_t st, const ReadSegs& r) {
    uint32_t mx = 0;
    for (int s = 0; s < r.n; ++s) mx = std::max(mx, r.seg[s].bytes);
    if (mx) hipLaunchKernelGGL(k_readback, dim3(std::min(nblk(mx / 4 + 1, 256), 64u)), dim3(256), 0, st, r);
}

void visibility_clears(const VisArgs& a, FillSegs& f) {
    const int64_t npx = (int64_t)a.Wv * a.Hv;
    if (f.n + 3 > FillSegs::kMax) throw std::length_error("fill segments exhausted");
    f.seg[f.n++] = FillSeg{a.idbuf, (uint64_t)(npx * a.n_views), NONE64, 1};
    f.seg[f.n++] = FillSeg{a.req_direct, (uint64_t)a.n_pg, NONE32, 0};
    f.seg[f.n++] = FillSeg{a.req_link, (uint64_t)a.n_pg, NONE32, 0};
}

// the ID buffer and the request arrays are cleared beforehand (visibility_clears)
void launch_visibility(hipStream_t st, const VisArgs& a) {
    const int64_t npx = (int64_t)a.Wv * a.Hv;
    hipLaunchKernelGGL(k_frustum, dim3(nblk((uint64_t)a.n_pg * a.n_views, 256)), dim3(256), 0, st, a.spheres, a.n_pg,
                       a.cams, a.n_views, a.W, a.H, a.guard, a.cand, a.counters);
    hipLaunchKernelGGL(k_rays, dim3(nblk(npx * a.n_views, 256)), dim3(256), 0, st, a.cams, a.n_views, a.W, a.H,
                       a.guard, a.Wv, a.Hv, a.rays);
    if (a.nc > 0) {
        const int64_t slots = a.nc * a.n_views;
        hipLaunchKernelGGL(k_cell_rects, dim3(nblk(slots, 256)), dim3(256), 0, st, a.cell_lo, a.cell_hi, a.nc, a.cand,
                           a.n_pg, a.cams, a.n_views, a.W, a.H, a.guard, a.Wv, a.Hv, a.cell_rects, a.cell_area);
        scan_lb(st, *a.sw, a.cell_area, (uint64_t)slots, a.cell_offs, a.cell_offs + slots);
        hipLaunchKernelGGL(k_raster_items, dim3(2048), dim3(PR_NT), 0, st, a.cell_lo, a.cell_hi, a.nc, a.cams, a.Wv,
                           a.Hv, (const int4*)a.cell_rects, (const uint32_t*)a.cell_offs,
                           (const uint32_t*)(a.cell_offs + slots), slots, (const float4*)a.rays, a.idbuf);
    }
    hipLaunchKernelGGL(k_reduce, dim3(nblk(npx * a.n_views, 256)), dim3(256), 0, st,
                       (const unsigned long long*)a.idbuf, npx * a.n_views, a.req_direct);
    if (a.use_links)
        hipLaunchKernelGGL(k_links, dim3(nblk(a.n_pg, 256)), dim3(256), 0, st, (const uint32_t*)a.req_direct,
                           a.link_start, a.link_dst, a.n_pg, a.req_link);
    hipLaunchKernelGGL(k_requests, dim3(nblk(a.n_pg, 256)), dim3(256), 0, st, (const uint32_t*)a.req_direct,
                       (const uint32_t*)a.req_link, a.spheres, a.n_pg, a.L, a.tau, a.fy_max, a.page_level,
                       a.req_keys, a.counters);
}

}  // namespace vm
