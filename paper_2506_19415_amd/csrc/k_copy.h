// k_copy.h -- one chunk of a page copy, done by one workgroup: the GPU reads
// the missed pages from the pinned host store (over PCIe, with many loads in
// flight) and writes them into the pool; the copy commands stay on the
// device.  Offsets and sizes are multiples of 4 bytes (Gaussian records are
// 236 or 124 bytes); 16-byte accesses where the command allows.  A command
// that would leave the store or the pool is skipped and flagged.
#pragma once
#include "kcommon.h"
#include "vm3dgs_impl.h"

namespace vmk {

constexpr int CP_NT = 256;
constexpr uint32_t CP_CHUNK = 16384;

// chunk blk of the copies [first, ...): command first + blk / per, chunk blk % per
__device__ __forceinline__ void copy_chunk(const vm::CopyCmd* __restrict__ cmds, uint32_t first, uint32_t per,
                                          uint32_t blk, const uint8_t* __restrict__ host, uint64_t host_bytes,
                                          uint8_t* __restrict__ pool, uint64_t pool_bytes,
                                          unsigned long long* __restrict__ bytes_done, uint32_t* __restrict__ err) {
    const uint32_t c = first + blk / per;
    const uint32_t ch = blk % per;
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

}  // namespace vmk
