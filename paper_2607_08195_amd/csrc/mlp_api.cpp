// C ABI of the MLP closure (include/mlp.h): weights, forward, backward,
// Adam and minibatch training on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mlp.h"
#include "mlp.h"

struct dsmc_mlp_s {
    hipStream_t stream = nullptr;
    int device = 0;             // the device current at create
    dsmc_allocator alloc{};
    bool has_alloc = false;
    std::vector<void*> owned;
    std::string err;
    float* params = nullptr;    // FP32 master weights
    uint16_t* packed = nullptr; // bf16 operand copies
    float* m = nullptr;         // Adam moments
    float* v = nullptr;
    int step = 0;
    // growable scratch
    float* x = nullptr;
    float* t = nullptr;
    float* y = nullptr;
    int64_t cap_rows = 0;
    float* partial = nullptr;
    float* loss_partial = nullptr;
    int64_t cap_blocks = 0;
    float* grad = nullptr;
    int32_t* idx = nullptr;
    int64_t cap_idx = 0;
    double* loss = nullptr;
    int64_t cap_loss = 0;
};

namespace {

using namespace dsmcx;

std::string g_mlp_error;

dsmc_status mfail(dsmc_mlp n, dsmc_status s, const std::string& msg) {
    if (n) n->err = msg; else g_mlp_error = msg;
    return s;
}

#define MLP_TRY(net, call)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) return mfail(net, DSMC_E_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

void* mlp_alloc(dsmc_mlp n, size_t bytes) {
    if (bytes == 0) bytes = 16;
    void* p = nullptr;
    if (n->has_alloc) p = n->alloc.alloc(bytes, n->alloc.user);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (p) n->owned.push_back(p);
    return p;
}

void mlp_free(dsmc_mlp n, void* p) {
    if (!p) return;
    auto it = std::find(n->owned.begin(), n->owned.end(), p);
    if (it != n->owned.end()) n->owned.erase(it);
    if (n->has_alloc) n->alloc.free(p, n->alloc.user); else hipFree(p);
}

template <class T>
bool grow(dsmc_mlp n, T*& p, int64_t& cap, int64_t need) {
    if (need <= cap && p) return true;
    if (hipStreamSynchronize(n->stream) != hipSuccess) return false;
    mlp_free(n, p);
    const int64_t c = std::max<int64_t>(need, 2 * cap);
    p = (T*)mlp_alloc(n, sizeof(T) * (size_t)c);
    cap = p ? c : 0;
    return p != nullptr;
}

dsmc_status ensure_rows(dsmc_mlp n, int64_t rows) {
    if (rows > n->cap_rows || !n->x) {
        if (hipStreamSynchronize(n->stream) != hipSuccess) return mfail(n, DSMC_E_DEVICE, "stream synchronize failed");
        mlp_free(n, n->x);
        mlp_free(n, n->t);
        mlp_free(n, n->y);
        const int64_t c = std::max<int64_t>(rows, 2 * n->cap_rows);
        n->x = (float*)mlp_alloc(n, sizeof(float) * kMlpIn * (size_t)c);
        n->t = (float*)mlp_alloc(n, sizeof(float) * kMlpOut * (size_t)c);
        n->y = (float*)mlp_alloc(n, sizeof(float) * kMlpOut * (size_t)c);
        if (!n->x || !n->t || !n->y) {
            n->cap_rows = 0;
            return mfail(n, DSMC_E_OOM, "device allocation failed");
        }
        n->cap_rows = c;
    }
    return DSMC_OK;
}

dsmc_status ensure_blocks(dsmc_mlp n, int64_t blocks) {
    if (blocks > n->cap_blocks || !n->partial) {
        if (hipStreamSynchronize(n->stream) != hipSuccess) return mfail(n, DSMC_E_DEVICE, "stream synchronize failed");
        mlp_free(n, n->partial);
        mlp_free(n, n->loss_partial);
        const int64_t c = std::max<int64_t>(blocks, 2 * n->cap_blocks);
        n->partial = (float*)mlp_alloc(n, sizeof(float) * kMlpParams * (size_t)c);
        n->loss_partial = (float*)mlp_alloc(n, sizeof(float) * (size_t)c);
        if (!n->partial || !n->loss_partial) {
            n->cap_blocks = 0;
            return mfail(n, DSMC_E_OOM, "device allocation failed");
        }
        n->cap_blocks = c;
    }
    return DSMC_OK;
}

MlpDev view(dsmc_mlp n) { return mlp_dev_view(n->params, n->packed); }

// Scratch of dsmc_mlp_backward_noalloc, one copy per device for the life of
// the process: the per-block gradient partials of at most
// DSMC_MLP_NOALLOC_MAX_ROWS rows ([blocks][kMlpParams] floats) followed by
// the per-block loss partials.  Every block writes its whole partial, so
// nothing has to start at zero.
constexpr int64_t kNoAllocBlocks = DSMC_MLP_NOALLOC_MAX_ROWS / kMlpTile;
constexpr size_t kNoAllocLossOffset = ((sizeof(float) * kMlpParams * kNoAllocBlocks + 255) / 256) * 256;
constexpr size_t kNoAllocBytes = kNoAllocLossOffset + sizeof(float) * kNoAllocBlocks;
static_assert(DSMC_MLP_NOALLOC_MAX_ROWS % kMlpTile == 0, "whole tiles");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

// The device address of this device's scratch (host code must not use the
// array's own name: it is a host-side stand-in).  Called by dsmc_mlp_create
// with the network's device current.
dsmc_status bind_scratch(dsmc_mlp n) {
    if (n->device < 0 || n->device >= kMaxDevices) return mfail(n, DSMC_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[n->device]) return DSMC_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return mfail(n, DSMC_E_DEVICE, std::string("hipGetSymbolAddress of the scratch failed: ") + hipGetErrorString(e));
    g_scratch_ptr[n->device] = ptr;
    return DSMC_OK;
}

}  // namespace

namespace dsmcx {
// Device view of a network for the coupling step (its arrays stay valid
// while the network lives).
MlpDev mlp_handle_view(dsmc_mlp n) { return view(n); }
}  // namespace dsmcx

extern "C" {

dsmc_status dsmc_mlp_create(dsmc_mlp* out, void* hip_stream, const dsmc_allocator* allocator) {
    if (!out) return mfail(nullptr, DSMC_E_INVALID, "out is NULL");
    *out = nullptr;
    dsmc_mlp n = new dsmc_mlp_s();
    n->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&n->device) != hipSuccess) {
        delete n;
        return mfail(nullptr, DSMC_E_DEVICE, "no current device");
    }
    if (bind_scratch(n) != DSMC_OK) {
        std::string m = n->err;
        delete n;
        return mfail(nullptr, DSMC_E_DEVICE, m);
    }
    if (allocator) {
        if (!allocator->alloc || !allocator->free) {
            delete n;
            return mfail(nullptr, DSMC_E_INVALID, "allocator callbacks missing");
        }
        n->alloc = *allocator;
        n->has_alloc = true;
    }
    n->params = (float*)mlp_alloc(n, sizeof(float) * kMlpParams);
    n->packed = (uint16_t*)mlp_alloc(n, sizeof(uint16_t) * kMlpPackTotal);
    n->m = (float*)mlp_alloc(n, sizeof(float) * kMlpParams);
    n->v = (float*)mlp_alloc(n, sizeof(float) * kMlpParams);
    n->grad = (float*)mlp_alloc(n, sizeof(float) * kMlpParams);
    if (!n->params || !n->packed || !n->m || !n->v || !n->grad) {
        dsmc_mlp_destroy(n);
        return mfail(nullptr, DSMC_E_OOM, "device allocation failed");
    }
    std::vector<float> z(kMlpParams, 0.f);
    if (dsmc_mlp_set_weights(n, z.data()) != DSMC_OK) {
        std::string m = n->err;
        dsmc_mlp_destroy(n);
        return mfail(nullptr, DSMC_E_DEVICE, m);
    }
    *out = n;
    return DSMC_OK;
}

dsmc_status dsmc_mlp_set_weights(dsmc_mlp n, const float* p) {
    if (!n || !p) return mfail(n, DSMC_E_INVALID, "bad arguments");
    std::vector<float> z(kMlpParams, 0.f);
    MLP_TRY(n, hipMemcpyAsync(n->params, p, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, n->stream));
    MLP_TRY(n, hipMemcpyAsync(n->m, z.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice, n->stream));
    MLP_TRY(n, hipMemcpyAsync(n->v, z.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice, n->stream));
    launch_mlp_pack(n->stream, n->params, n->packed);
    MLP_TRY(n, hipGetLastError());
    MLP_TRY(n, hipStreamSynchronize(n->stream));
    n->step = 0;
    return DSMC_OK;
}

dsmc_status dsmc_mlp_init_weights(dsmc_mlp n, uint64_t seed) {
    if (!n) return mfail(n, DSMC_E_INVALID, "bad arguments");
    std::vector<float> z(kMlpParams, 0.f);
    launch_mlp_init(n->stream, n->params, RngKey{(uint32_t)(seed & 0xFFFFFFFFu), 1u});
    MLP_TRY(n, hipMemcpyAsync(n->m, z.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice, n->stream));
    MLP_TRY(n, hipMemcpyAsync(n->v, z.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice, n->stream));
    launch_mlp_pack(n->stream, n->params, n->packed);
    MLP_TRY(n, hipGetLastError());
    MLP_TRY(n, hipStreamSynchronize(n->stream));
    n->step = 0;
    return DSMC_OK;
}

dsmc_status dsmc_mlp_get_weights(dsmc_mlp n, float* p) {
    if (!n || !p) return mfail(n, DSMC_E_INVALID, "bad arguments");
    MLP_TRY(n, hipStreamSynchronize(n->stream));
    MLP_TRY(n, hipMemcpy(p, n->params, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    return DSMC_OK;
}

dsmc_status dsmc_mlp_forward(dsmc_mlp n, const float* x, int64_t rows, float* y, int32_t on_device) {
    if (!n || rows < 0 || (rows > 0 && (!x || !y))) return mfail(n, DSMC_E_INVALID, "bad arguments");
    if (rows == 0) return DSMC_OK;
    if (rows >= ((int64_t)1 << 31)) return mfail(n, DSMC_E_INVALID, "too many rows");
    const float* dx = x;
    float* dy = y;
    if (!on_device) {
        dsmc_status st = ensure_rows(n, rows);
        if (st != DSMC_OK) return st;
        MLP_TRY(n, hipMemcpyAsync(n->x, x, sizeof(float) * kMlpIn * rows, hipMemcpyHostToDevice, n->stream));
        dx = n->x;
        dy = n->y;
    }
    launch_mlp_forward(n->stream, view(n), dx, nullptr, rows, dy);
    MLP_TRY(n, hipGetLastError());
    if (!on_device)
        MLP_TRY(n, hipMemcpyAsync(y, dy, sizeof(float) * kMlpOut * rows, hipMemcpyDeviceToHost, n->stream));
    MLP_TRY(n, hipStreamSynchronize(n->stream));
    return DSMC_OK;
}

dsmc_status dsmc_mlp_backward(dsmc_mlp n, const float* x, const float* t, int64_t rows, float* grad, double* loss) {
    if (!n || rows <= 0 || !x || !t || !grad) return mfail(n, DSMC_E_INVALID, "bad arguments");
    if (rows >= ((int64_t)1 << 31)) return mfail(n, DSMC_E_INVALID, "too many rows");
    dsmc_status st = ensure_rows(n, rows);
    if (st == DSMC_OK) st = ensure_blocks(n, mlp_blocks(rows));
    if (st != DSMC_OK) return st;
    if (!grow(n, n->loss, n->cap_loss, 1)) return mfail(n, DSMC_E_OOM, "device allocation failed");
    MLP_TRY(n, hipMemcpyAsync(n->x, x, sizeof(float) * kMlpIn * rows, hipMemcpyHostToDevice, n->stream));
    MLP_TRY(n, hipMemcpyAsync(n->t, t, sizeof(float) * kMlpOut * rows, hipMemcpyHostToDevice, n->stream));
    launch_mlp_grad(n->stream, view(n), n->x, n->t, nullptr, rows, n->partial, n->loss_partial);
    launch_mlp_reduce(n->stream, n->partial, n->loss_partial, mlp_blocks(rows), n->grad, n->loss);
    MLP_TRY(n, hipGetLastError());
    MLP_TRY(n, hipMemcpyAsync(grad, n->grad, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, n->stream));
    double l = 0;
    MLP_TRY(n, hipMemcpyAsync(&l, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    MLP_TRY(n, hipStreamSynchronize(n->stream));
    if (loss) *loss = l / ((double)rows * kMlpOut);
    return DSMC_OK;
}

dsmc_status dsmc_mlp_backward_noalloc(dsmc_mlp n, const float* x, const float* t, int64_t rows, float* grad,
                                      double* loss) {
    if (!n || !x || !t || !grad || !loss) return mfail(n, DSMC_E_INVALID, "bad arguments");
    if (rows <= 0 || rows > DSMC_MLP_NOALLOC_MAX_ROWS)
        return mfail(n, DSMC_E_INVALID, "rows must be between 1 and DSMC_MLP_NOALLOC_MAX_ROWS (" +
                                            std::to_string(DSMC_MLP_NOALLOC_MAX_ROWS) + ")");
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        base = g_scratch_ptr[n->device];
    }
    if (!base) return mfail(n, DSMC_E_DEVICE, "the scratch of this device has no address");
    float* partial = (float*)base;
    float* loss_partial = (float*)((unsigned char*)base + kNoAllocLossOffset);
    launch_mlp_grad(n->stream, view(n), x, t, nullptr, rows, partial, loss_partial);
    launch_mlp_reduce(n->stream, partial, loss_partial, mlp_blocks(rows), grad, loss, (double)rows * kMlpOut);
    MLP_TRY(n, hipGetLastError());
    return DSMC_OK;
}

dsmc_status dsmc_mlp_adam_step(dsmc_mlp n, const float* grad, float lr, float b1, float b2, float eps) {
    if (!n || !grad) return mfail(n, DSMC_E_INVALID, "bad arguments");
    MLP_TRY(n, hipMemcpyAsync(n->grad, grad, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, n->stream));
    n->step += 1;
    launch_mlp_adam(n->stream, n->params, n->grad, n->m, n->v, n->step, lr, b1, b2, eps);
    launch_mlp_pack(n->stream, n->params, n->packed);
    MLP_TRY(n, hipGetLastError());
    MLP_TRY(n, hipStreamSynchronize(n->stream));
    return DSMC_OK;
}

dsmc_status dsmc_mlp_train(dsmc_mlp n, const float* x, const float* t, int64_t rows,
                           const dsmc_mlp_train_params* p, dsmc_mlp_train_report* rep) {
    if (!n || !p || rows <= 0 || !x || !t || p->steps < 0 || p->batch < 0)
        return mfail(n, DSMC_E_INVALID, "bad arguments");
    if (rows >= ((int64_t)1 << 31)) return mfail(n, DSMC_E_INVALID, "too many rows");
    const bool full = p->batch == 0 || p->batch >= rows;
    const int64_t b = full ? rows : p->batch;
    dsmc_status st = ensure_rows(n, rows);
    if (st == DSMC_OK) st = ensure_blocks(n, mlp_blocks(b));
    if (st != DSMC_OK) return st;
    if (!grow(n, n->loss, n->cap_loss, std::max(1, p->steps))) return mfail(n, DSMC_E_OOM, "device allocation failed");
    if (!full && !grow(n, n->idx, n->cap_idx, b)) return mfail(n, DSMC_E_OOM, "device allocation failed");
    MLP_TRY(n, hipMemcpyAsync(n->x, x, sizeof(float) * kMlpIn * rows, hipMemcpyHostToDevice, n->stream));
    MLP_TRY(n, hipMemcpyAsync(n->t, t, sizeof(float) * kMlpOut * rows, hipMemcpyHostToDevice, n->stream));
    const RngKey key{(uint32_t)(p->seed & 0xFFFFFFFFu), 0u};
    for (int s = 0; s < p->steps; ++s) {
        if (!full) launch_mlp_batch(n->stream, key, (uint32_t)s, rows, b, n->idx);
        launch_mlp_grad(n->stream, view(n), n->x, n->t, full ? nullptr : n->idx, b, n->partial, n->loss_partial);
        launch_mlp_reduce(n->stream, n->partial, n->loss_partial, mlp_blocks(b), n->grad, n->loss + s);
        n->step += 1;
        launch_mlp_adam(n->stream, n->params, n->grad, n->m, n->v, n->step, p->lr, p->beta1, p->beta2, p->eps);
        launch_mlp_pack(n->stream, n->params, n->packed);
    }
    MLP_TRY(n, hipGetLastError());
    MLP_TRY(n, hipStreamSynchronize(n->stream));
    if (rep) {
        rep->steps = p->steps;
        rep->loss_first = rep->loss_last = 0.0;
        if (p->steps > 0) {
            double l0 = 0, l1 = 0;
            MLP_TRY(n, hipMemcpy(&l0, n->loss, sizeof(double), hipMemcpyDeviceToHost));
            MLP_TRY(n, hipMemcpy(&l1, n->loss + (p->steps - 1), sizeof(double), hipMemcpyDeviceToHost));
            rep->loss_first = l0 / ((double)b * kMlpOut);
            rep->loss_last = l1 / ((double)b * kMlpOut);
        }
    }
    return DSMC_OK;
}

const char* dsmc_mlp_last_error(dsmc_mlp n) { return n ? n->err.c_str() : g_mlp_error.c_str(); }

void dsmc_mlp_destroy(dsmc_mlp n) {
    if (!n) return;
    hipStreamSynchronize(n->stream);
    for (void* p : n->owned) {
        if (n->has_alloc) n->alloc.free(p, n->alloc.user); else hipFree(p);
    }
    delete n;
}

}  // extern "C"
