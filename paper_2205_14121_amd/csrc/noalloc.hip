// Controller forward pass for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid allocation): the same
// kernels as aimts_ctrl_forward (moving-average filter, z-score, two-layer GRU encoder,
// latent, fully connected head; Sec. 3.3, Table 2), with the bfloat16 weight copy and
// the activations in a file-scope device array instead of a context's workspace.
//
// Each GPU holds its own copy of `scratch` from module load until the process ends.
// Host code never uses the array's name as a device address: its address on the
// current device is looked up once per device with hipGetSymbolAddress and kept in
// g_scratch_ptr.  Every call on one GPU shares that GPU's array, so calls that overlap
// on one GPU (two streams, two threads) race.  Nothing in it needs to start at zero:
// every buffer the forward pass reads is written earlier in the same call.
#include <cstdio>
#include <mutex>
#include <string>

#include "../../include/aimts.h"
#include "common.h"
#include "ctrl.h"

namespace aimts {
namespace {

constexpr int kStaticMaxBatch = AIMTS_CTRL_STATIC_MAX_BATCH;
constexpr int kMaxDevices = 64;

// Byte offsets of the forward-pass buffers inside the array (256-byte aligned).
struct StaticLayout {
    size_t wbf, xt, hs0, hs1, c0, c1, lat, act, logits, seq_loss, total;
};

constexpr size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

constexpr StaticLayout static_layout()
{
    StaticLayout L{};
    const size_t B = kStaticMaxBatch;
    size_t o = 0;
    auto take = [&o](size_t bytes) { const size_t r = o; o += align256(bytes); return r; };
    L.wbf = take(sizeof(uint16_t) * (size_t)ctrl_layout().total);
    L.xt = take(sizeof(float) * B * kT * kF);
    L.hs0 = take(sizeof(float) * B * kT * kH);
    L.hs1 = take(sizeof(float) * B * kT * kH);
    L.c0 = take(sizeof(float) * B * kT * 4 * kH);
    L.c1 = take(sizeof(float) * B * kT * 4 * kH);
    L.lat = take(sizeof(float) * B * kLat);
    L.act = take(sizeof(float) * B * 56);
    L.logits = take(sizeof(float) * B * kNout);
    L.seq_loss = take(sizeof(float) * 2 * B);
    L.total = o;
    return L;
}

constexpr size_t kScratchBytes = static_layout().total;  // 40.7 MiB at 256 windows

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
aimts_status scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        set_context_free_error("aimts_ctrl_forward_static: no usable current HIP device");
        return AIMTS_E_HIP;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            std::string msg = std::string("aimts_ctrl_forward_static: hipGetSymbolAddress failed: ") +
                              hipGetErrorString(e);
            set_context_free_error(msg.c_str());
            return AIMTS_E_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return AIMTS_OK;
}

}  // namespace
}  // namespace aimts

using namespace aimts;

extern "C" aimts_status aimts_ctrl_forward_static(const float *d_params, int64_t n_params, const float *d_windows,
                                                  int32_t batch, float *d_latent, float *d_logits, void *hip_stream)
{
    if (!d_params || !d_windows) {
        set_context_free_error("aimts_ctrl_forward_static: parameters and windows are required");
        return AIMTS_E_INVALID;
    }
    if (n_params != ctrl_num_params()) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "aimts_ctrl_forward_static: expected %lld parameters",
                      (long long)ctrl_num_params());
        set_context_free_error(buf);
        return AIMTS_E_INVALID;
    }
    if (batch < 1 || batch > kStaticMaxBatch) {
        char buf[160];
        std::snprintf(buf, sizeof buf,
                      "aimts_ctrl_forward_static: batch %d outside [1, %d] (the static scratch holds %d windows)",
                      batch, kStaticMaxBatch, kStaticMaxBatch);
        set_context_free_error(buf);
        return AIMTS_E_INVALID;
    }
    (void)hipGetLastError();
    void *base = nullptr;
    aimts_status st = scratch_address(&base);
    if (st) return st;
    constexpr StaticLayout L = static_layout();
    char *b = static_cast<char *>(base);
    CtrlState c{};
    c.max_batch = kStaticMaxBatch;
    c.np = ctrl_num_params();
    c.have_weights = true;
    c.master = const_cast<float *>(d_params);  // read only: the z-score statistics
    c.wbf = reinterpret_cast<uint16_t *>(b + L.wbf);
    c.xt = reinterpret_cast<float *>(b + L.xt);
    c.hs[0] = reinterpret_cast<float *>(b + L.hs0);
    c.hs[1] = reinterpret_cast<float *>(b + L.hs1);
    c.cache[0] = reinterpret_cast<float *>(b + L.c0);
    c.cache[1] = reinterpret_cast<float *>(b + L.c1);
    c.lat = reinterpret_cast<float *>(b + L.lat);
    c.act = reinterpret_cast<float *>(b + L.act);
    c.logits = reinterpret_cast<float *>(b + L.logits);
    c.seq_loss = reinterpret_cast<float *>(b + L.seq_loss);
    hipStream_t s = (hipStream_t)hip_stream;
    ctrl_round_weights(d_params, c.wbf, s);
    ctrl_forward(c, d_windows, batch, s, nullptr, false);
    ctrl_copy_outputs(c, batch, d_latent, d_logits, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        std::string msg = std::string("aimts_ctrl_forward_static: ") + hipGetErrorString(e);
        set_context_free_error(msg.c_str());
        return AIMTS_E_HIP;
    }
    return AIMTS_OK;
}
