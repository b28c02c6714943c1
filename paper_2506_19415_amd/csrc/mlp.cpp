// Host object of the page-prefetch network (C ABI in include/vm3dgs.h).
// Owns the fp32 master weights, Adam moments, gradients, bf16 weight copies
// and the per-batch activations on the device; every step is a kernel of
// k_mlp.hip on the network's stream.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "vm3dgs_impl.h"

using namespace vm;

struct vm3dgs_mlp {
    MlpDev d;
    int max_batch = 0;
    int64_t n_params = 0;
    int step = 0;
    hipStream_t st = nullptr;
    bool own_st = false;
    std::vector<void*> allocs;
    std::vector<float> h_loss;
    int n_loss_blocks = 0;
    std::string err;
};

namespace {

struct Fail {
    hipError_t e;
    const char* what;
};

#define MCHK(x)                                  \
    do {                                         \
        hipError_t e_ = (x);                     \
        if (e_ != hipSuccess) throw Fail{e_, #x}; \
    } while (0)

template <class T>
T* mal(vm3dgs_mlp* m, size_t n) {
    void* p = nullptr;
    MCHK(hipMalloc(&p, sizeof(T) * std::max<size_t>(n, 1)));
    m->allocs.push_back(p);
    MCHK(hipMemset(p, 0, sizeof(T) * std::max<size_t>(n, 1)));
    return (T*)p;
}

void release(vm3dgs_mlp* m) {
    if (m->st) hipStreamSynchronize(m->st);
    for (void* p : m->allocs) hipFree(p);
    m->allocs.clear();
    if (m->own_st && m->st) hipStreamDestroy(m->st);
    m->st = nullptr;
}

vm3dgs_status fail(vm3dgs_mlp* m, const Fail& f) {
    m->err = std::string("HIP error ") + hipGetErrorString(f.e) + " in " + f.what;
    return VM3DGS_E_HIP;
}

std::string g_mlp_create_error;

}  // namespace

extern "C" {

const char* vm3dgs_mlp_create_error(void) { return g_mlp_create_error.c_str(); }
}  // extern "C"

namespace vm {
const MlpDev* mlp_dev_of(const vm3dgs_mlp* net) { return &net->d; }
int mlp_max_batch_of(const vm3dgs_mlp* net) { return net->max_batch; }
hipStream_t mlp_stream_of(const vm3dgs_mlp* net) { return net->st; }
}  // namespace vm

extern "C" {

vm3dgs_status vm3dgs_mlp_create(const uint32_t* dims, uint32_t n_layers, uint32_t max_batch, void* stream,
                                vm3dgs_mlp** out) {
    g_mlp_create_error.clear();
    if (!out) return VM3DGS_E_INVALID_ARG;
    *out = nullptr;
    if (!dims || n_layers < 1 || n_layers > 8 || max_batch == 0 || max_batch > 65536) {
        g_mlp_create_error = "dims, n_layers (1..8) or max_batch (1..65536) out of range";
        return VM3DGS_E_INVALID_ARG;
    }
    for (uint32_t l = 0; l <= n_layers; ++l)
        if (dims[l] == 0 || dims[l] > 65536) {
            g_mlp_create_error = "every width must be in 1..65536";
            return VM3DGS_E_INVALID_ARG;
        }
    vm3dgs_mlp* m = new vm3dgs_mlp();
    MlpDev& d = m->d;
    d.n_layers = (int)n_layers;
    int64_t off = 0;
    for (uint32_t l = 0; l <= n_layers; ++l) {
        d.dims[l] = (int)dims[l];
        d.kpad[l] = (int)((dims[l] + 31) / 32 * 32);
    }
    for (uint32_t l = 0; l < n_layers; ++l) {
        d.off[l] = off;
        off += (int64_t)dims[l] * dims[l + 1] + dims[l + 1];
    }
    d.off[n_layers] = off;
    m->n_params = off;
    m->max_batch = (int)max_batch;
    d.b_pad = (int)((max_batch + 63) / 64 * 64);
    try {
        if (stream) m->st = (hipStream_t)stream;
        else { MCHK(hipStreamCreateWithFlags(&m->st, hipStreamNonBlocking)); m->own_st = true; }
        d.master = mal<float>(m, (size_t)off);
        d.adam_m = mal<float>(m, (size_t)off);
        d.adam_v = mal<float>(m, (size_t)off);
        d.grad = mal<float>(m, (size_t)off);
        for (uint32_t l = 0; l < n_layers; ++l) {
            d.wb[l] = mal<uint16_t>(m, (size_t)d.kpad[l] * dims[l + 1]);
            d.act[l] = mal<uint16_t>(m, (size_t)d.b_pad * d.kpad[l]);
            d.dz[l] = mal<uint16_t>(m, (size_t)d.b_pad * dims[l + 1]);
        }
        d.logits = mal<float>(m, (size_t)d.b_pad * dims[n_layers]);
        m->n_loss_blocks = (int)(((int64_t)d.b_pad * dims[n_layers] + 255) / 256);
        d.loss_part = mal<float>(m, (size_t)m->n_loss_blocks);
        m->h_loss.resize((size_t)m->n_loss_blocks);
    } catch (const Fail& f) {
        g_mlp_create_error = std::string("HIP error ") + hipGetErrorString(f.e) + " in " + f.what;
        release(m);
        delete m;
        return f.e == hipErrorOutOfMemory ? VM3DGS_E_DEVICE_OOM : VM3DGS_E_HIP;
    }
    *out = m;
    return VM3DGS_OK;
}

void vm3dgs_mlp_destroy(vm3dgs_mlp* m) {
    if (!m) return;
    release(m);
    delete m;
}

const char* vm3dgs_mlp_last_error(const vm3dgs_mlp* m) { return m ? m->err.c_str() : "NULL network"; }

uint64_t vm3dgs_mlp_n_params(const vm3dgs_mlp* m) { return m ? (uint64_t)m->n_params : 0; }

vm3dgs_status vm3dgs_mlp_set_params(vm3dgs_mlp* m, const float* params, uint64_t n) {
    if (!m || !params || n != (uint64_t)m->n_params) return VM3DGS_E_INVALID_ARG;
    try {
        MCHK(hipMemcpyAsync(m->d.master, params, sizeof(float) * n, hipMemcpyHostToDevice, m->st));
        MCHK(hipMemsetAsync(m->d.adam_m, 0, sizeof(float) * n, m->st));
        MCHK(hipMemsetAsync(m->d.adam_v, 0, sizeof(float) * n, m->st));
        mlp_sync_bf16_dev(m->st, m->d);
        MCHK(hipGetLastError());
        MCHK(hipStreamSynchronize(m->st));
        m->step = 0;
    } catch (const Fail& f) {
        return fail(m, f);
    }
    return VM3DGS_OK;
}

vm3dgs_status vm3dgs_mlp_get_state(vm3dgs_mlp* m, float* params, float* adam_m, float* adam_v, uint64_t n,
                                   uint32_t* step) {
    if (!m || n != (uint64_t)m->n_params) return VM3DGS_E_INVALID_ARG;
    try {
        MCHK(hipStreamSynchronize(m->st));
        if (params) MCHK(hipMemcpy(params, m->d.master, sizeof(float) * n, hipMemcpyDeviceToHost));
        if (adam_m) MCHK(hipMemcpy(adam_m, m->d.adam_m, sizeof(float) * n, hipMemcpyDeviceToHost));
        if (adam_v) MCHK(hipMemcpy(adam_v, m->d.adam_v, sizeof(float) * n, hipMemcpyDeviceToHost));
        if (step) *step = (uint32_t)m->step;
    } catch (const Fail& f) {
        return fail(m, f);
    }
    return VM3DGS_OK;
}

vm3dgs_status vm3dgs_mlp_forward(vm3dgs_mlp* m, const float* x, uint32_t batch, float* logits) {
    if (!m || !x || !logits || batch == 0) return VM3DGS_E_INVALID_ARG;
    if (batch > (uint32_t)m->max_batch) { m->err = "batch exceeds max_batch"; return VM3DGS_E_CAPACITY; }
    try {
        mlp_input_dev(m->st, m->d, x, (int)batch);
        mlp_forward_dev(m->st, m->d, (int)batch);
        const int K = m->d.dims[m->d.n_layers];
        MCHK(hipMemcpyAsync(logits, m->d.logits, sizeof(float) * (size_t)batch * K, hipMemcpyDeviceToDevice, m->st));
        MCHK(hipGetLastError());
    } catch (const Fail& f) {
        return fail(m, f);
    }
    return VM3DGS_OK;
}

static float read_loss(vm3dgs_mlp* m, uint32_t batch) {
    const int K = m->d.dims[m->d.n_layers];
    MCHK(hipMemcpyAsync(m->h_loss.data(), m->d.loss_part, sizeof(float) * m->n_loss_blocks, hipMemcpyDeviceToHost,
                        m->st));
    MCHK(hipStreamSynchronize(m->st));
    double s = 0.0;
    for (float v : m->h_loss) s += v;
    return (float)(s / ((double)batch * K));
}

vm3dgs_status vm3dgs_mlp_gradient(vm3dgs_mlp* m, const float* x, const float* y, uint32_t batch, float* grad,
                                  float* loss) {
    if (!m || !x || !y || !grad || batch == 0) return VM3DGS_E_INVALID_ARG;
    if (batch > (uint32_t)m->max_batch) { m->err = "batch exceeds max_batch"; return VM3DGS_E_CAPACITY; }
    try {
        mlp_input_dev(m->st, m->d, x, (int)batch);
        mlp_forward_dev(m->st, m->d, (int)batch);
        mlp_backward_dev(m->st, m->d, y, (int)batch);
        MCHK(hipMemcpyAsync(grad, m->d.grad, sizeof(float) * m->n_params, hipMemcpyDeviceToDevice, m->st));
        MCHK(hipGetLastError());
        if (loss) *loss = read_loss(m, batch);
    } catch (const Fail& f) {
        return fail(m, f);
    }
    return VM3DGS_OK;
}

vm3dgs_status vm3dgs_mlp_train_step(vm3dgs_mlp* m, const float* x, const float* y, uint32_t batch, float lr,
                                    float* loss) {
    if (!m || !x || !y || batch == 0 || !(lr > 0.0f)) return VM3DGS_E_INVALID_ARG;
    if (batch > (uint32_t)m->max_batch) { m->err = "batch exceeds max_batch"; return VM3DGS_E_CAPACITY; }
    try {
        mlp_input_dev(m->st, m->d, x, (int)batch);
        mlp_forward_dev(m->st, m->d, (int)batch);
        mlp_backward_dev(m->st, m->d, y, (int)batch);
        m->step += 1;
        mlp_adam_dev(m->st, m->d, lr, 0.9f, 0.999f, 1e-8f, m->step);
        MCHK(hipGetLastError());
        if (loss) *loss = read_loss(m, batch);
    } catch (const Fail& f) {
        return fail(m, f);
    }
    return VM3DGS_OK;
}

// "VM3DGSNN", uint32 n_layers, uint32 dims[n_layers + 1], float params[n_params]
static const char kMlpMagic[8] = {'V', 'M', '3', 'D', 'G', 'S', 'N', 'N'};

vm3dgs_status vm3dgs_mlp_save(vm3dgs_mlp* m, const char* path) {
    if (!m || !path) return VM3DGS_E_INVALID_ARG;
    std::vector<float> p((size_t)m->n_params);
    const vm3dgs_status st = vm3dgs_mlp_get_state(m, p.data(), nullptr, nullptr, (uint64_t)m->n_params, nullptr);
    if (st != VM3DGS_OK) return st;
    FILE* f = fopen(path, "wb");
    if (!f) { m->err = std::string("cannot open ") + path + " for writing"; return VM3DGS_E_INVALID_ARG; }
    const uint32_t nl = (uint32_t)m->d.n_layers;
    uint32_t dims[9];
    for (int l = 0; l <= m->d.n_layers; ++l) dims[l] = (uint32_t)m->d.dims[l];
    const bool ok = fwrite(kMlpMagic, 1, 8, f) == 8 && fwrite(&nl, 4, 1, f) == 1 &&
                    fwrite(dims, 4, nl + 1, f) == nl + 1 && fwrite(p.data(), 4, p.size(), f) == p.size();
    if (fclose(f) != 0 || !ok) { m->err = std::string("write to ") + path + " failed"; return VM3DGS_E_INVALID_ARG; }
    return VM3DGS_OK;
}

vm3dgs_status vm3dgs_mlp_load(vm3dgs_mlp* m, const char* path) {
    if (!m || !path) return VM3DGS_E_INVALID_ARG;
    FILE* f = fopen(path, "rb");
    if (!f) { m->err = std::string("cannot open ") + path; return VM3DGS_E_INVALID_ARG; }
    char magic[8];
    uint32_t nl = 0, dims[9];
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kMlpMagic, 8) == 0 && fread(&nl, 4, 1, f) == 1 &&
              nl == (uint32_t)m->d.n_layers && fread(dims, 4, nl + 1, f) == nl + 1;
    for (uint32_t l = 0; ok && l <= nl; ++l) ok = dims[l] == (uint32_t)m->d.dims[l];
    std::vector<float> p;
    if (ok) {
        p.resize((size_t)m->n_params);
        ok = fread(p.data(), 4, p.size(), f) == p.size() && fgetc(f) == EOF;
    }
    fclose(f);
    if (!ok) { m->err = std::string(path) + " is not a network of these widths"; return VM3DGS_E_INVALID_ARG; }
    return vm3dgs_mlp_set_params(m, p.data(), (uint64_t)p.size());
}

vm3dgs_status vm3dgs_mlp_sync(vm3dgs_mlp* m) {
    if (!m) return VM3DGS_E_INVALID_ARG;
    return hipStreamSynchronize(m->st) == hipSuccess ? VM3DGS_OK : VM3DGS_E_HIP;
}

}  // extern "C"
