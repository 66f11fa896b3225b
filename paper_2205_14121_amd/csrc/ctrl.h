// Learned MTS controller (AI inference pipeline of Table 2): device state and entry
// points.  Parameters are one float32 master vector (layout in include/aimts.h); the
// kernels read a bfloat16 copy of it and keep activations and accumulators in float32.
#pragma once

#include <stdint.h>

#include "../../include/aimts.h"
#include "common.h"

namespace aimts {

constexpr int kH = 64, kF = 8, kT = 64, kLat = 16, kG = 3 * kH, kNout = 9, kMA = 5;
constexpr int kCtrlSplit = 64;  // row chunks of the weight-gradient contractions

// Offsets (in floats) of every tensor in the parameter vector.
struct CtrlLayout {
    int64_t enc0_wih, enc0_whh, enc0_bih, enc0_bhh;
    int64_t enc1_wih, enc1_whh, enc1_bih, enc1_bhh;
    int64_t lat_w, lat_b;
    int64_t dec0_wih, dec0_whh, dec0_bih, dec0_bhh;
    int64_t dec1_wih, dec1_whh, dec1_bih, dec1_bhh;
    int64_t out_w, out_b;
    int64_t h1_w, h1_b, h2_w, h2_b, h3_w, h3_b, h4_w, h4_b;
    int64_t norm_mean, norm_std;
    int64_t total;
    int64_t head_begin, head_end;  // the head's parameters are one contiguous range
    int64_t ae_end;                // autoencoder parameters are [0, ae_end)
};

__host__ __device__ constexpr CtrlLayout ctrl_layout()
{
    CtrlLayout L{};
    int64_t o = 0;
    auto take = [&](int64_t n) { int64_t r = o; o += n; return r; };
    L.enc0_wih = take(kG * kF); L.enc0_whh = take(kG * kH); L.enc0_bih = take(kG); L.enc0_bhh = take(kG);
    L.enc1_wih = take(kG * kH); L.enc1_whh = take(kG * kH); L.enc1_bih = take(kG); L.enc1_bhh = take(kG);
    L.lat_w = take(kLat * kH); L.lat_b = take(kLat);
    L.dec0_wih = take(kG * kLat); L.dec0_whh = take(kG * kH); L.dec0_bih = take(kG); L.dec0_bhh = take(kG);
    L.dec1_wih = take(kG * kH); L.dec1_whh = take(kG * kH); L.dec1_bih = take(kG); L.dec1_bhh = take(kG);
    L.out_w = take(kF * kH); L.out_b = take(kF);
    L.ae_end = o;
    L.head_begin = o;
    L.h1_w = take(32 * kLat); L.h1_b = take(32);
    L.h2_w = take(16 * 32); L.h2_b = take(16);
    L.h3_w = take(8 * 16); L.h3_b = take(8);
    L.h4_w = take(kNout * 8); L.h4_b = take(kNout);
    L.head_end = o;
    L.norm_mean = take(kF); L.norm_std = take(kF);
    L.total = o;
    return L;
}

struct CtrlState {
    int32_t max_batch = 0;
    int64_t P = 0;
    int64_t np = 0;
    bool have_weights = false;
    int64_t adam_t[2] = {0, 0};
    float *master = nullptr;     // [np] float32 master parameters
    uint16_t *wbf = nullptr;     // [np] bfloat16 compute copy
    float *adam_m = nullptr, *adam_v = nullptr, *grad = nullptr;  // [np]
    // activations, batch-major, sized for max(max_batch, P)
    float *xt = nullptr;         // [B][T][F] denoised input
    float *hs[4] = {};           // layer outputs [B][T][H]: enc0, enc1, dec0, dec1
    float *cache[4] = {};        // per step r, z, n, ghn: [B][T][4H]
    float *lat = nullptr;        // [B][LAT]
    float *recon = nullptr;      // [B][T][F]
    float *act = nullptr;        // head activations [B][32 + 16 + 8] (pre-activation)
    float *logits = nullptr;     // [B][NOUT]
    float *dgi[4] = {}, *dgh[4] = {};  // gate gradients [B][T][G]
    float *dlat = nullptr;       // [B][LAT]
    float *dre = nullptr;        // [B][T][F] d loss / d recon
    float *seq_loss = nullptr;   // [B][2] squared error, cross-entropy
    float *wg_scratch = nullptr; // split-row partial sums of the weight gradients
    float *head_part = nullptr;  // [B][head params] per-sequence head gradients
    float *loss = nullptr;       // scalar
    float *windows = nullptr;    // [P][T][F] inference windows gathered from the ring
    int32_t *decision = nullptr; // k, hold, fallback
    int32_t *pratio = nullptr;   // [P] ratio predicted for each platelet at the last decision
};

int64_t ctrl_num_params();

template <typename Take>
void ctrl_carve(CtrlState &c, int32_t max_batch, int64_t P, Take take)
{
    const CtrlLayout L = ctrl_layout();
    const int64_t B = max_batch > P ? max_batch : P;
    c.max_batch = max_batch;
    c.P = P;
    c.np = L.total;
    c.master = (float *)take(sizeof(float) * L.total);
    c.wbf = (uint16_t *)take(sizeof(uint16_t) * L.total);
    c.adam_m = (float *)take(sizeof(float) * L.total);
    c.adam_v = (float *)take(sizeof(float) * L.total);
    c.grad = (float *)take(sizeof(float) * L.total);
    c.xt = (float *)take(sizeof(float) * B * kT * kF);
    for (int l = 0; l < 4; ++l) {
        c.hs[l] = (float *)take(sizeof(float) * B * kT * kH);
        c.cache[l] = (float *)take(sizeof(float) * B * kT * 4 * kH);
        c.dgi[l] = (float *)take(sizeof(float) * B * kT * kG);
        c.dgh[l] = (float *)take(sizeof(float) * B * kT * kG);
    }
    c.lat = (float *)take(sizeof(float) * B * kLat);
    c.recon = (float *)take(sizeof(float) * B * kT * kF);
    c.act = (float *)take(sizeof(float) * B * 56);
    c.logits = (float *)take(sizeof(float) * B * kNout);
    c.dlat = (float *)take(sizeof(float) * B * kLat);
    c.dre = (float *)take(sizeof(float) * B * kT * kF);
    c.seq_loss = (float *)take(sizeof(float) * 2 * B);
    c.wg_scratch = (float *)take(sizeof(float) * kCtrlSplit * kG * kH);
    c.head_part = (float *)take(sizeof(float) * B * (L.head_end - L.head_begin));
    c.loss = (float *)take(sizeof(float) * 4);
    c.windows = (float *)take(sizeof(float) * (P > 0 ? P : 1) * kT * kF);
    c.decision = (int32_t *)take(sizeof(int32_t) * 4);
    c.pratio = (int32_t *)take(sizeof(int32_t) * (P > 0 ? P : 1));
}

void ctrl_init(CtrlState &c, hipStream_t st);
void ctrl_after_set(CtrlState &c, hipStream_t st);
// bfloat16 copy (round to nearest even) of a float32 parameter vector
void ctrl_round_weights(const float *params, uint16_t *wbf, hipStream_t st);
// decode = false skips the decoder (inference: latent and logits only)
void ctrl_forward(CtrlState &c, const float *windows, int B, hipStream_t st, const int32_t *labels,
                  bool decode = true);
void ctrl_copy_outputs(CtrlState &c, int B, float *d_latent, float *d_logits, hipStream_t st);
void ctrl_backward(CtrlState &c, const int32_t *labels, int B, int phase, hipStream_t st);
void ctrl_copy_grads(CtrlState &c, float *d_grads, hipStream_t st);
void ctrl_adam(CtrlState &c, int phase, float lr, hipStream_t st);
aimts_status ctrl_infer_ring(CtrlState &c, const Dev &s, const float *ring, int head, int32_t *k, int32_t *hold,
                             int *fallback, hipStream_t st);

}  // namespace aimts
