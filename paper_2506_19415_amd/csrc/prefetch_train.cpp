// Training of the learned page prefetch from the method's own page sets
// (C ABI in include/vm3dgs.h).  The paper leaves prefetching to future work
// (Sec. 6); the rows are built here from plain frames of the library: the
// features after frame t, and as labels the clusters of the pages frame t+1
// requested that were not resident after frame t.  Training runs the
// network's own kernels (bf16 matrix products, fp32 Adam) on minibatches
// gathered on the device.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "vm3dgs_impl.h"

using namespace vm;

namespace {

uint64_t splitmix64(uint64_t& s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) hipFree(p);
    }
    hipError_t alloc(size_t bytes) { return hipMalloc(&p, std::max<size_t>(bytes, 4)); }
};

// one path of plain frames: feature rows after every frame but the last, and
// the labels from the next frame's requests against this frame's residency
vm3dgs_status collect_path(vm3dgs* c, const vm3dgs_camera* cams, uint32_t n, const vm3dgs_prefetch_opts& o,
                           int n_pg, int L, float* image, std::vector<float>& x_prev, std::vector<int32_t>& v2p,
                           float* x_out, float* y_out, uint64_t cap, uint64_t& rows) {
    const size_t F = 28 + (size_t)o.hist_bins, K = o.n_clusters;
    vm3dgs_status st = vm3dgs_reset(c);
    if (st != VM3DGS_OK) return st;
    std::vector<uint8_t> res_prev((size_t)n_pg, 0);
    for (uint32_t t = 0; t < n; ++t) {
        vm3dgs_frame_out out{};
        st = vm3dgs_frame(c, &cams[t], 1, image, &out);
        if (st != VM3DGS_OK) return st;
        if (t > 0) {
            if (rows < cap) {
                if (x_out) memcpy(x_out + rows * F, x_prev.data(), sizeof(float) * F);
                if (y_out) {
                    float* y = y_out + rows * K;
                    std::fill(y, y + K, 0.0f);
                    for (uint32_t i = 0; i < out.n_requests; ++i) {
                        const int32_t p = out.requests[i];
                        if (p >= 0 && p < n_pg && !res_prev[(size_t)p])
                            y[(size_t)((int64_t)p * (int64_t)K / n_pg)] = 1.0f;
                    }
                }
            }
            rows++;
        }
        if (t + 1 < n) {
            st = vm3dgs_prefetch_features(c, 1, x_prev.data());
            if (st != VM3DGS_OK) return st;
            const int64_t bytes = (int64_t)v2p.size() * 4;
            if (vm3dgs_debug_get(c, "v2p", v2p.data(), bytes) != bytes) return VM3DGS_E_HIP;
            for (int p = 0; p < n_pg; ++p) {
                uint8_t r = 0;
                for (int l = 0; l < L; ++l) r |= v2p[(size_t)p * L + l] >= 0;
                res_prev[(size_t)p] = r;
            }
        }
    }
    return VM3DGS_OK;
}

}  // namespace

extern "C" {

vm3dgs_status vm3dgs_prefetch_collect(vm3dgs* c, const vm3dgs_dataset* data, float* x_host, float* y_host,
                                      uint64_t cap_rows, uint64_t* rows_out) {
    if (!c) return VM3DGS_E_INVALID_ARG;
    vm3dgs_mlp* net = nullptr;
    vm3dgs_prefetch_opts o{};
    if (!prefetch_stage_of(c, &net, &o) || !data || !data->cams || !data->path_frames || data->n_paths == 0)
        return VM3DGS_E_INVALID_ARG;
    int64_t info[16];
    if (vm3dgs_debug_get(c, "info", info, sizeof info) != (int64_t)sizeof info) return VM3DGS_E_HIP;
    const int n_pg = (int)info[0], L = (int)info[2];
    // the plain method: the network's stage off while collecting
    vm3dgs_status st = vm3dgs_set_prefetch(c, nullptr, &o);
    if (st != VM3DGS_OK) return st;
    // the frames' images go to a buffer of this call (tiles cover the image)
    const int64_t img_px = info[8] * 16 * info[9] * 16;
    DevBuf image;
    if (image.alloc(sizeof(float) * 3 * (size_t)img_px) != hipSuccess) {
        vm3dgs_set_prefetch(c, net, &o);
        return VM3DGS_E_DEVICE_OOM;
    }
    std::vector<float> x_prev(28 + (size_t)o.hist_bins);
    std::vector<int32_t> v2p((size_t)n_pg * L);
    uint64_t rows = 0, first = 0;
    for (uint32_t k = 0; k < data->n_paths && st == VM3DGS_OK; ++k) {
        st = collect_path(c, data->cams + first, data->path_frames[k], o, n_pg, L, (float*)image.p, x_prev, v2p,
                          x_host, y_host, cap_rows, rows);
        first += data->path_frames[k];
    }
    const vm3dgs_status st2 = vm3dgs_set_prefetch(c, net, &o);
    if (st == VM3DGS_OK) st = st2;
    if (st == VM3DGS_OK) st = vm3dgs_reset(c);
    if (rows_out) *rows_out = rows;
    if (st == VM3DGS_OK && (x_host || y_host) && rows > cap_rows) return VM3DGS_E_CAPACITY;
    return st;
}

vm3dgs_status vm3dgs_prefetch_train(vm3dgs* c, const vm3dgs_dataset* data, const vm3dgs_train_opts* opts,
                                    vm3dgs_train_log* log) {
    if (!c || !data || !opts) return VM3DGS_E_INVALID_ARG;
    vm3dgs_mlp* net = nullptr;
    vm3dgs_prefetch_opts o{};
    if (!prefetch_stage_of(c, &net, &o) || !net) return VM3DGS_E_INVALID_ARG;
    if (opts->batch == 0 || (int)opts->batch > mlp_max_batch_of(net) || !(opts->lr > 0.0f) ||
        !(opts->proposal_factor >= 0.0f))
        return VM3DGS_E_INVALID_ARG;
    if (!data->path_frames) return VM3DGS_E_INVALID_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    uint64_t rows = 0;
    for (uint32_t k = 0; k < data->n_paths; ++k) rows += data->path_frames[k] > 0 ? data->path_frames[k] - 1 : 0;
    if (rows == 0 || rows > 0xffffffffull) return VM3DGS_E_INVALID_ARG;
    const size_t F = 28 + (size_t)o.hist_bins, K = o.n_clusters;
    std::vector<float> X, Y;
    try {
        X.resize(rows * F);
        Y.resize(rows * K);
    } catch (const std::bad_alloc&) {
        return VM3DGS_E_HOST_OOM;
    }
    vm3dgs_status st = vm3dgs_prefetch_collect(c, data, X.data(), Y.data(), rows, &rows);
    if (st != VM3DGS_OK) return st;
    double pos = 0.0;
    for (float v : Y) pos += v;
    const double positive_rate = pos / ((double)rows * K);
    const double ms_collect = ms_since(t0);

    const auto t1 = std::chrono::steady_clock::now();
    const hipStream_t ns = mlp_stream_of(net);
    const uint32_t B = opts->batch;
    DevBuf dX, dY, dxb, dyb, didx;
    if (dX.alloc(sizeof(float) * X.size()) != hipSuccess || dY.alloc(sizeof(float) * Y.size()) != hipSuccess ||
        dxb.alloc(sizeof(float) * B * F) != hipSuccess || dyb.alloc(sizeof(float) * B * K) != hipSuccess ||
        didx.alloc(sizeof(uint32_t) * B) != hipSuccess)
        return VM3DGS_E_DEVICE_OOM;
    if (hipMemcpy(dX.p, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dY.p, Y.data(), sizeof(float) * Y.size(), hipMemcpyHostToDevice) != hipSuccess)
        return VM3DGS_E_HIP;
    uint32_t* h_idx = nullptr;
    if (hipHostMalloc((void**)&h_idx, sizeof(uint32_t) * B, hipHostMallocDefault) != hipSuccess)
        return VM3DGS_E_HOST_OOM;
    uint64_t seed = opts->seed;
    std::vector<float> losses;
    float loss_first = NAN, loss_last = NAN;
    for (uint32_t it = 0; it < opts->steps && st == VM3DGS_OK; ++it) {
        // the previous step has read the index buffer once the stream passed it
        if (hipStreamSynchronize(ns) != hipSuccess) { st = VM3DGS_E_HIP; break; }
        for (uint32_t i = 0; i < B; ++i) h_idx[i] = (uint32_t)(splitmix64(seed) % rows);
        if (hipMemcpyAsync(didx.p, h_idx, sizeof(uint32_t) * B, hipMemcpyHostToDevice, ns) != hipSuccess) {
            st = VM3DGS_E_HIP;
            break;
        }
        launch_gather_rows(ns, (const float*)dX.p, (const uint32_t*)didx.p, B, (uint32_t)F, (float*)dxb.p);
        launch_gather_rows(ns, (const float*)dY.p, (const uint32_t*)didx.p, B, (uint32_t)K, (float*)dyb.p);
        const bool want = it == 0 || it + 1 == opts->steps || (opts->log_every && it % opts->log_every == 0);
        float loss = NAN;
        st = vm3dgs_mlp_train_step(net, (const float*)dxb.p, (const float*)dyb.p, B, opts->lr, want ? &loss : nullptr);
        if (want) {
            if (it == 0) loss_first = loss;
            loss_last = loss;
            losses.push_back(loss);
        }
    }
    hipHostFree(h_idx);
    if (st == VM3DGS_OK && hipStreamSynchronize(ns) != hipSuccess) st = VM3DGS_E_HIP;
    if (st != VM3DGS_OK) return st;

    // logit threshold: the network proposes proposal_factor times as many
    // clusters as the labels hold on the training rows
    float thr = o.logit_threshold;
    if (opts->proposal_factor > 0.0f) {
        const uint32_t MB = (uint32_t)mlp_max_batch_of(net);
        DevBuf dz;
        if (dz.alloc(sizeof(float) * (size_t)MB * K) != hipSuccess) return VM3DGS_E_DEVICE_OOM;
        std::vector<float> z(rows * K);
        for (uint64_t r0 = 0; r0 < rows; r0 += MB) {
            const uint32_t nb = (uint32_t)std::min<uint64_t>(MB, rows - r0);
            st = vm3dgs_mlp_forward(net, (const float*)dX.p + r0 * F, nb, (float*)dz.p);
            if (st != VM3DGS_OK) return st;
            if (hipMemcpyAsync(z.data() + r0 * K, dz.p, sizeof(float) * nb * K, hipMemcpyDeviceToHost, ns) !=
                    hipSuccess ||
                hipStreamSynchronize(ns) != hipSuccess)
                return VM3DGS_E_HIP;
        }
        const double q = std::min(std::max(1.0 - opts->proposal_factor * positive_rate, 0.0), 1.0);
        const size_t k = std::min(z.size() - 1, (size_t)std::floor(q * (double)(z.size() - 1)));
        std::nth_element(z.begin(), z.begin() + (ptrdiff_t)k, z.end());
        thr = z[k];
        o.logit_threshold = thr;
        st = vm3dgs_set_prefetch(c, net, &o);
        if (st != VM3DGS_OK) return st;
    }
    if (log) {
        memset(log, 0, sizeof *log);
        log->rows = rows;
        log->positive_rate = (float)positive_rate;
        log->loss_first = loss_first;
        log->loss_last = loss_last;
        log->logit_threshold = thr;
        log->ms_collect = (float)ms_collect;
        log->ms_train = (float)ms_since(t1);
        const size_t n = losses.size(), m = std::min<size_t>(n, 64);
        for (size_t i = 0; i < m; ++i) log->losses[i] = losses[m > 1 ? i * (n - 1) / (m - 1) : 0];
        log->n_losses = (uint32_t)m;
    }
    return VM3DGS_OK;
}

vm3dgs_status vm3dgs_prefetch_load(vm3dgs* c, const char* path) {
    vm3dgs_mlp* net = nullptr;
    if (!c || !prefetch_stage_of(c, &net, nullptr) || !net) return VM3DGS_E_INVALID_ARG;
    return vm3dgs_mlp_load(net, path);
}

}  // extern "C"
