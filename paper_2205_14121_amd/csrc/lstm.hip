// The paper's own AI inference pipeline (Sec. 3.3, Table 2), in its sizes: windows of
// 50 points of 6 platelet measurements; two-stage denoising (a causal 5-point moving
// average, then a one-level Haar wavelet transform whose detail coefficients are
// soft-thresholded at the universal threshold (median |d| / 0.6745) sqrt(2 ln T) of
// Donoho and Johnstone, and transformed back) and a z-score with stored statistics; a
// 2-layer LSTM autoencoder with 16 and 4 units whose 8 latents are the last hidden and
// cell states of the 4-unit layer, with a mirrored decoder (4 and 16 units, read-out
// 16 -> 6) for training; a fully connected network 8 -> 32 -> 16 -> 8 -> 1 (ReLU between
// layers) predicting log2 of the MTS ratio.  The autoencoder and the FCN are trained
// separately (Sec. 3.3), by BPTT and Adam.
//
// Context-free: parameters, windows and outputs are caller-owned device buffers, and
// the activations live in a caller-provided workspace.  One workgroup of 64 lanes per
// window: an LSTM step gives one lane to each gate row (4H <= 64) and then one lane to
// each unit.  Everything is float32.  Weight gradients are summed per window, then over
// the windows in index order, so results do not depend on scheduling.
#include <cmath>
#include <cstdio>

#include "../../include/aimts.h"
#include "common.h"

namespace aimts {
namespace lstmnet {

constexpr int T = 50, F = 6, H1 = 16, H2 = 4, LAT = 2 * H2, MA = 5;
constexpr int kBS = 64;

// Offsets (floats) of every tensor in the parameter vector; the order of the
// declaration in include/aimts.h.
struct Layout {
    int64_t e0_wih, e0_whh, e0_bih, e0_bhh, e1_wih, e1_whh, e1_bih, e1_bhh;
    int64_t d0_wih, d0_whh, d0_bih, d0_bhh, d1_wih, d1_whh, d1_bih, d1_bhh;
    int64_t out_w, out_b, fc1_w, fc1_b, fc2_w, fc2_b, fc3_w, fc3_b, fc4_w, fc4_b;
    int64_t norm_mean, norm_std, total, ae_end, fcn_begin, fcn_end;
};

__host__ __device__ constexpr Layout layout()
{
    Layout L{};
    int64_t o = 0;
    auto take = [&](int64_t n) { int64_t r = o; o += n; return r; };
    L.e0_wih = take(4 * H1 * F); L.e0_whh = take(4 * H1 * H1); L.e0_bih = take(4 * H1); L.e0_bhh = take(4 * H1);
    L.e1_wih = take(4 * H2 * H1); L.e1_whh = take(4 * H2 * H2); L.e1_bih = take(4 * H2); L.e1_bhh = take(4 * H2);
    L.d0_wih = take(4 * H2 * LAT); L.d0_whh = take(4 * H2 * H2); L.d0_bih = take(4 * H2); L.d0_bhh = take(4 * H2);
    L.d1_wih = take(4 * H1 * H2); L.d1_whh = take(4 * H1 * H1); L.d1_bih = take(4 * H1); L.d1_bhh = take(4 * H1);
    L.out_w = take(F * H1); L.out_b = take(F);
    L.ae_end = o;
    L.fcn_begin = o;
    L.fc1_w = take(32 * LAT); L.fc1_b = take(32); L.fc2_w = take(16 * 32); L.fc2_b = take(16);
    L.fc3_w = take(8 * 16); L.fc3_b = take(8); L.fc4_w = take(8); L.fc4_b = take(1);
    L.fcn_end = o;
    L.norm_mean = take(F); L.norm_std = take(F);
    L.total = o;
    return L;
}
constexpr int64_t NP = layout().total;

// Per-window scratch (floats): the denoised input, each LSTM layer's cache (hidden
// states, cell states, tanh of the cell states, gates i f g o after their
// nonlinearities), the latent, the reconstruction, the FCN's pre-activations.
struct Cache {
    int64_t xt, lat, recon, fcn, total;
    int64_t layer[4];  // enc0, enc1, dec0, dec1: [T][H] h, [T][H] c, [T][H] tanh c, [T][4H] gates
};

__host__ __device__ constexpr int64_t layer_floats(int h) { return (int64_t)T * 7 * h; }

__host__ __device__ constexpr Cache cache_layout()
{
    Cache C{};
    int64_t o = 0;
    auto take = [&](int64_t n) { int64_t r = o; o += (n + 15) / 16 * 16; return r; };
    C.xt = take(T * F);
    C.layer[0] = take(layer_floats(H1));
    C.layer[1] = take(layer_floats(H2));
    C.layer[2] = take(layer_floats(H2));
    C.layer[3] = take(layer_floats(H1));
    C.lat = take(LAT);
    C.recon = take(T * F);
    C.fcn = take(32 + 16 + 8 + 1);
    C.total = o;
    return C;
}
constexpr int64_t kWinFloats = cache_layout().total;
constexpr int64_t kPartFloats = (NP + 63) / 64 * 64;  // per-window partial gradients

__host__ __device__ constexpr size_t workspace_bytes(int64_t B)
{
    return sizeof(float) * (size_t)B * (size_t)(kWinFloats + kPartFloats + 2);
}

__device__ __forceinline__ float sigm(float a) { return 1.0f / (1.0f + expf(-a)); }

__device__ __forceinline__ void block_sync() { __syncthreads(); }

// ---------------------------------------------------------------------------
// Step 2: denoising of one window [T][F] in LDS (in: raw; out: z-scored)
// ---------------------------------------------------------------------------
__device__ void denoise_window(const float *P, const float *raw, float *ma, float *out, float *scr)
{
    const Layout L = layout();
    const int tid = threadIdx.x;
    for (int q = tid; q < T * F; q += kBS) {
        const int t = q / F, f = q - t * F;
        const int lo = t - MA + 1 < 0 ? 0 : t - MA + 1;
        float s = 0.0f;
        for (int u = lo; u <= t; ++u) s += raw[u * F + f];
        ma[q] = s / (float)(t - lo + 1);
    }
    block_sync();
    // one-level Haar transform per feature; soft thresholding of the details
    constexpr int K = T / 2;
    const float is2 = 0.70710678118654752f;
    if (tid < F) {
        const int f = tid;
        float *ad = scr + f * K;  // |d| sorted ascending (insertion sort of 25 values)
        for (int k = 0; k < K; ++k) {
            const float d = (ma[(2 * k) * F + f] - ma[(2 * k + 1) * F + f]) * is2;
            const float v = fabsf(d);
            int p = k;
            while (p > 0 && ad[p - 1] > v) {
                ad[p] = ad[p - 1];
                --p;
            }
            ad[p] = v;
        }
        const float lam = ad[K / 2] / 0.6745f * 2.79714962f;  // sqrt(2 ln 50)
        for (int k = 0; k < K; ++k) {
            const float x0 = ma[(2 * k) * F + f], x1 = ma[(2 * k + 1) * F + f];
            const float a = (x0 + x1) * is2;
            const float d = (x0 - x1) * is2;
            const float m = fabsf(d) - lam;
            const float ds = m > 0.0f ? copysignf(m, d) : 0.0f;
            out[(2 * k) * F + f] = (a + ds) * is2;
            out[(2 * k + 1) * F + f] = (a - ds) * is2;
        }
    }
    block_sync();
    for (int q = tid; q < T * F; q += kBS) {
        const int f = q % F;
        out[q] = (out[q] - P[L.norm_mean + f]) / P[L.norm_std + f];
    }
    block_sync();
}

// ---------------------------------------------------------------------------
// One LSTM layer over T steps: input in[t][nin] (LDS; stride 0 repeats one vector),
// hidden states to hs[t][H] (LDS), cache to global memory.
// ---------------------------------------------------------------------------
__device__ void lstm_layer(const float *P, int64_t wih, int64_t whh, int64_t bih, int64_t bhh, int nin, int H,
                           const float *in, int in_stride, float *hs, float *cache, float *gate, float *hc)
{
    const int tid = threadIdx.x, G = 4 * H;
    float *ch = cache, *cc = cache + T * H, *ctc = cache + 2 * T * H, *cg = cache + 3 * T * H;
    float *h = hc, *c = hc + 16;
    if (tid < H) {
        h[tid] = 0.0f;
        c[tid] = 0.0f;
    }
    block_sync();
    for (int t = 0; t < T; ++t) {
        if (tid < G) {
            const float *x = in + t * in_stride;
            float a = P[bih + tid] + P[bhh + tid];
            for (int k = 0; k < nin; ++k) a += P[wih + tid * nin + k] * x[k];
            for (int j = 0; j < H; ++j) a += P[whh + tid * H + j] * h[j];
            const int kind = tid / H;  // 0 i, 1 f, 2 g, 3 o
            const float g = kind == 2 ? tanhf(a) : sigm(a);
            gate[tid] = g;
            cg[t * G + tid] = g;
        }
        block_sync();
        if (tid < H) {
            const float ig = gate[tid], fg = gate[H + tid], gg = gate[2 * H + tid], og = gate[3 * H + tid];
            const float cn = fg * c[tid] + ig * gg;
            const float tc = tanhf(cn);
            const float hn = og * tc;
            c[tid] = cn;
            h[tid] = hn;
            hs[t * H + tid] = hn;
            ch[t * H + tid] = hn;
            cc[t * H + tid] = cn;
            ctc[t * H + tid] = tc;
        }
        block_sync();
    }
}

// Forward pass of one window; decode = false skips the decoder (inference).
__device__ void forward_window(const float *P, const float *win, float *wc, bool decode, float *lat_out,
                               float *pred_out, float *recon_out)
{
    const Layout L = layout();
    const Cache C = cache_layout();
    __shared__ float raw[T * F], ma[T * F], xt[T * F], scr[F * (T / 2)];
    __shared__ float h0[T * H1], h1[T * H2], gate[64], hc[32], lat[LAT], fc[64];
    const int tid = threadIdx.x;
    for (int q = tid; q < T * F; q += kBS) raw[q] = win[q];
    block_sync();
    denoise_window(P, raw, ma, xt, scr);
    for (int q = tid; q < T * F; q += kBS) wc[C.xt + q] = xt[q];
    lstm_layer(P, L.e0_wih, L.e0_whh, L.e0_bih, L.e0_bhh, F, H1, xt, F, h0, wc + C.layer[0], gate, hc);
    lstm_layer(P, L.e1_wih, L.e1_whh, L.e1_bih, L.e1_bhh, H1, H2, h0, H1, h1, wc + C.layer[1], gate, hc);
    if (tid < H2) {
        lat[tid] = hc[tid];            // h_T
        lat[H2 + tid] = hc[16 + tid];  // c_T
    }
    block_sync();
    if (tid < LAT) {
        wc[C.lat + tid] = lat[tid];
        if (lat_out) lat_out[tid] = lat[tid];
    }
    // FCN 8 -> 32 -> 16 -> 8 -> 1 (pre-activations cached)
    float *a1 = fc, *a2 = fc + 32, *a3 = fc + 48;
    if (tid < 32) {
        float a = P[L.fc1_b + tid];
        for (int k = 0; k < LAT; ++k) a += P[L.fc1_w + tid * LAT + k] * lat[k];
        a1[tid] = a;
    }
    block_sync();
    if (tid < 16) {
        float a = P[L.fc2_b + tid];
        for (int k = 0; k < 32; ++k) a += P[L.fc2_w + tid * 32 + k] * fmaxf(a1[k], 0.0f);
        a2[tid] = a;
    }
    block_sync();
    if (tid < 8) {
        float a = P[L.fc3_b + tid];
        for (int k = 0; k < 16; ++k) a += P[L.fc3_w + tid * 16 + k] * fmaxf(a2[k], 0.0f);
        a3[tid] = a;
    }
    block_sync();
    if (tid == 0) {
        float y = P[L.fc4_b];
        for (int k = 0; k < 8; ++k) y += P[L.fc4_w + k] * fmaxf(a3[k], 0.0f);
        fc[56] = y;
        if (pred_out) *pred_out = y;
    }
    block_sync();
    for (int q = tid; q < 57; q += kBS) wc[C.fcn + q] = fc[q];
    if (!decode) return;
    __shared__ float d0[T * H2], d1[T * H1];
    lstm_layer(P, L.d0_wih, L.d0_whh, L.d0_bih, L.d0_bhh, LAT, H2, lat, 0, d0, wc + C.layer[2], gate, hc);
    lstm_layer(P, L.d1_wih, L.d1_whh, L.d1_bih, L.d1_bhh, H2, H1, d0, H2, d1, wc + C.layer[3], gate, hc);
    for (int q = tid; q < T * F; q += kBS) {
        const int t = q / F, o = q - t * F;
        float r = P[L.out_b + o];
        for (int j = 0; j < H1; ++j) r += P[L.out_w + o * H1 + j] * d1[t * H1 + j];
        wc[C.recon + q] = r;
        if (recon_out) recon_out[q] = r;
    }
    block_sync();
}

__global__ __launch_bounds__(kBS) void k_lstm_fwd(const float *P, const float *windows, int B, float *ws, int decode,
                                                  float *lat, float *pred, float *recon)
{
    const int b = blockIdx.x;
    if (b >= B) return;
    forward_window(P, windows + (int64_t)b * T * F, ws + (int64_t)b * kWinFloats, decode != 0,
                   lat ? lat + (int64_t)b * LAT : nullptr, pred ? pred + b : nullptr,
                   recon ? recon + (int64_t)b * T * F : nullptr);
}

__global__ __launch_bounds__(kBS) void k_lstm_filter(const float *P, const float *windows, int B, float *out)
{
    __shared__ float raw[T * F], ma[T * F], xt[T * F], scr[F * (T / 2)];
    const int b = blockIdx.x;
    if (b >= B) return;
    for (int q = threadIdx.x; q < T * F; q += kBS) raw[q] = windows[(int64_t)b * T * F + q];
    block_sync();
    denoise_window(P, raw, ma, xt, scr);
    for (int q = threadIdx.x; q < T * F; q += kBS) out[(int64_t)b * T * F + q] = xt[q];
}

// ---------------------------------------------------------------------------
// Backward pass of one LSTM layer (BPTT), from the cache of the forward pass.
// dh_in[t][H]: dL/dh_t from above (LDS, may be null), dcT[H]: dL/dc_T (LDS, may be
// null), x[t][nin] the layer's input (LDS; stride 0 repeats one vector).  Adds the
// weight gradients into g (this window's partial gradient vector, zeroed beforehand)
// and writes dx[t][nin] (LDS) unless dx is null.
// ---------------------------------------------------------------------------
__device__ void lstm_layer_bwd(const float *P, float *g, int64_t wih, int64_t whh, int64_t bih, int64_t bhh, int nin,
                               int H, const float *cache, const float *x, int x_stride, const float *dh_in,
                               const float *dcT, float *dx, float *da, float *st)
{
    const int tid = threadIdx.x, G = 4 * H;
    const float *ch = cache, *cc = cache + T * H, *ctc = cache + 2 * T * H, *cg = cache + 3 * T * H;
    float *dh = st, *dc = st + 16;
    if (tid < H) {
        dh[tid] = 0.0f;
        dc[tid] = dcT ? dcT[tid] : 0.0f;
    }
    // each gate row's gradients accumulate in its lane's registers over the steps
    float gw_ih[16], gw_hh[16], gb = 0.0f;
#pragma unroll
    for (int k = 0; k < 16; ++k) gw_ih[k] = gw_hh[k] = 0.0f;
    block_sync();
    for (int t = T - 1; t >= 0; --t) {
        if (tid < H) {
            const float dht = dh[tid] + (dh_in ? dh_in[t * H + tid] : 0.0f);
            const float ig = cg[t * G + tid], fg = cg[t * G + H + tid], gg = cg[t * G + 2 * H + tid],
                        og = cg[t * G + 3 * H + tid];
            const float tc = ctc[t * H + tid];
            const float cp = t > 0 ? cc[(t - 1) * H + tid] : 0.0f;
            const float dct = dc[tid] + dht * og * (1.0f - tc * tc);
            da[tid] = dct * gg * ig * (1.0f - ig);
            da[H + tid] = dct * cp * fg * (1.0f - fg);
            da[2 * H + tid] = dct * ig * (1.0f - gg * gg);
            da[3 * H + tid] = dht * tc * og * (1.0f - og);
            dc[tid] = dct * fg;
        }
        block_sync();
        if (tid < G) {
            const float a = da[tid];
            const float *xt = x + t * x_stride;
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (k < nin) gw_ih[k] += a * xt[k];
            if (t > 0) {
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    if (j < H) gw_hh[j] += a * ch[(t - 1) * H + j];
            }
            gb += a;
        }
        if (dx && tid < nin) {
            float s = 0.0f;
            for (int q = 0; q < G; ++q) s += da[q] * P[wih + q * nin + tid];
            dx[t * nin + tid] = s;
        }
        float nh = 0.0f;
        if (tid < H)
            for (int q = 0; q < G; ++q) nh += da[q] * P[whh + q * H + tid];
        block_sync();
        if (tid < H) dh[tid] = nh;
        block_sync();
    }
    if (tid < G) {
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (k < nin) g[wih + tid * nin + k] += gw_ih[k];
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (j < H) g[whh + tid * H + j] += gw_hh[j];
        g[bih + tid] += gb;
        g[bhh + tid] += gb;
    }
    block_sync();
}

// Gradients of one window.  phase 0: reconstruction MSE (autoencoder parameters);
// phase 1: MSE of the predicted log2 ratio (FCN parameters).  B: the batch size (the
// losses are means over it); target: this window's label.
__global__ __launch_bounds__(kBS) void k_lstm_bwd(const float *P, const float *windows, const float *targets, int B,
                                                  int phase, float *ws)
{
    const Layout L = layout();
    const Cache C = cache_layout();
    const int b = blockIdx.x;
    if (b >= B) return;
    const int tid = threadIdx.x;
    float *wc = ws + (int64_t)b * kWinFloats;
    float *g = ws + (int64_t)B * kWinFloats + (int64_t)b * kPartFloats;
    float *sl = ws + (int64_t)B * (kWinFloats + kPartFloats) + 2 * b;  // this window's loss terms
    forward_window(P, windows + (int64_t)b * T * F, wc, phase == 0, nullptr, nullptr, nullptr);
    for (int64_t q = tid; q < NP; q += kBS) g[q] = 0.0f;
    block_sync();
    if (phase == 1) {
        const float *a1 = wc + C.fcn, *a2 = a1 + 32, *a3 = a1 + 48;
        const float y = a1[56];
        const float dy = 2.0f * (y - targets[b]) / (float)B;
        __shared__ float d3[8], d2[16], d1[32];
        if (tid == 0) {
            sl[0] = 0.0f;
            sl[1] = (y - targets[b]) * (y - targets[b]);
            g[L.fc4_b] = dy;
        }
        if (tid < 8) {
            g[L.fc4_w + tid] = dy * fmaxf(a3[tid], 0.0f);
            d3[tid] = a3[tid] > 0.0f ? dy * P[L.fc4_w + tid] : 0.0f;
        }
        block_sync();
        if (tid < 16) {
            float s = 0.0f;
            for (int j = 0; j < 8; ++j) s += d3[j] * P[L.fc3_w + j * 16 + tid];
            d2[tid] = a2[tid] > 0.0f ? s : 0.0f;
        }
        for (int q = tid; q < 8 * 16; q += kBS) g[L.fc3_w + q] = d3[q / 16] * fmaxf(a2[q % 16], 0.0f);
        if (tid < 8) g[L.fc3_b + tid] = d3[tid];
        block_sync();
        if (tid < 32) {
            float s = 0.0f;
            for (int j = 0; j < 16; ++j) s += d2[j] * P[L.fc2_w + j * 32 + tid];
            d1[tid] = a1[tid] > 0.0f ? s : 0.0f;
        }
        for (int q = tid; q < 16 * 32; q += kBS) g[L.fc2_w + q] = d2[q / 32] * fmaxf(a1[q % 32], 0.0f);
        if (tid < 16) g[L.fc2_b + tid] = d2[tid];
        block_sync();
        for (int q = tid; q < 32 * LAT; q += kBS) g[L.fc1_w + q] = d1[q / LAT] * wc[C.lat + q % LAT];
        if (tid < 32) g[L.fc1_b + tid] = d1[tid];
        return;
    }
    // autoencoder: d loss / d recon, read-out, decoder, latent, encoder
    __shared__ float dre[T * F], dd1[T * H1], dd0[T * H2], dh0[T * H1], xin[T * H1], da[64], st[32], dlat[LAT];
    const float scale = 2.0f / (float)((int64_t)B * T * F);
    float se = 0.0f;
    for (int q = tid; q < T * F; q += kBS) {
        const float e = wc[C.recon + q] - wc[C.xt + q];
        dre[q] = scale * e;
        se += e * e;
    }
    // the window's squared error, summed in a fixed order through LDS
    da[tid] = se;
    block_sync();
    if (tid == 0) {
        float s = 0.0f;
        for (int q = 0; q < kBS; ++q) s += da[q];
        sl[0] = s;
        sl[1] = 0.0f;
    }
    block_sync();
    const float *d1h = wc + C.layer[3];  // decoder layer 1 hidden states [T][H1]
    for (int q = tid; q < F * H1; q += kBS) {
        const int o = q / H1, j = q - o * H1;
        float s = 0.0f;
        for (int t = 0; t < T; ++t) s += dre[t * F + o] * d1h[t * H1 + j];
        g[L.out_w + q] = s;
    }
    if (tid < F) {
        float s = 0.0f;
        for (int t = 0; t < T; ++t) s += dre[t * F + tid];
        g[L.out_b + tid] = s;
    }
    for (int q = tid; q < T * H1; q += kBS) {
        const int t = q / H1, j = q - t * H1;
        float s = 0.0f;
        for (int o = 0; o < F; ++o) s += dre[t * F + o] * P[L.out_w + o * H1 + j];
        dd1[q] = s;
    }
    // decoder layer 1: input = decoder layer 0's hidden states
    const float *d0h = wc + C.layer[2];
    for (int q = tid; q < T * H2; q += kBS) xin[q] = d0h[q];
    block_sync();
    lstm_layer_bwd(P, g, L.d1_wih, L.d1_whh, L.d1_bih, L.d1_bhh, H2, H1, wc + C.layer[3], xin, H2, dd1, nullptr, dd0,
                   da, st);
    // decoder layer 0: input = the latent at every step
    __shared__ float latv[LAT], dzin[T * LAT];
    if (tid < LAT) latv[tid] = wc[C.lat + tid];
    block_sync();
    lstm_layer_bwd(P, g, L.d0_wih, L.d0_whh, L.d0_bih, L.d0_bhh, LAT, H2, wc + C.layer[2], latv, 0, dd0, nullptr, dzin,
                   da, st);
    if (tid < LAT) {
        float s = 0.0f;
        for (int t = 0; t < T; ++t) s += dzin[t * LAT + tid];
        dlat[tid] = s;
    }
    block_sync();
    // encoder layer 1: dL/dh_T = dlat[0:4], dL/dc_T = dlat[4:8]; input = encoder layer 0's states
    __shared__ float dh1[T * H2];
    for (int q = tid; q < T * H2; q += kBS) dh1[q] = (q / H2 == T - 1) ? dlat[q % H2] : 0.0f;
    const float *e0h = wc + C.layer[0];
    for (int q = tid; q < T * H1; q += kBS) xin[q] = e0h[q];
    block_sync();
    lstm_layer_bwd(P, g, L.e1_wih, L.e1_whh, L.e1_bih, L.e1_bhh, H1, H2, wc + C.layer[1], xin, H1, dh1, dlat + H2, dh0,
                   da, st);
    // encoder layer 0: input = the denoised window
    for (int q = tid; q < T * F; q += kBS) xin[q] = wc[C.xt + q];
    block_sync();
    lstm_layer_bwd(P, g, L.e0_wih, L.e0_whh, L.e0_bih, L.e0_bhh, F, H1, wc + C.layer[0], xin, F, dh0, nullptr, nullptr,
                   da, st);
}

// Sum of the per-window partial gradients in window order; zero outside the phase's
// parameters.  Also the loss: the mean over the batch.
__global__ void k_lstm_reduce(const float *ws, int B, int phase, float *grad, float *loss)
{
    const Layout L = layout();
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t beg = phase == 0 ? 0 : L.fcn_begin, end = phase == 0 ? L.ae_end : L.fcn_end;
    const float *part = ws + (int64_t)B * kWinFloats;
    if (q < NP) {
        float s = 0.0f;
        if (q >= beg && q < end)
            for (int b = 0; b < B; ++b) s += part[(int64_t)b * kPartFloats + q];
        grad[q] = s;
    }
    if (q == 0 && loss) {
        const float *sl = ws + (int64_t)B * (kWinFloats + kPartFloats);
        float s = 0.0f;
        for (int b = 0; b < B; ++b) s += sl[2 * b + phase];
        *loss = phase == 0 ? s / (float)((int64_t)B * T * F) : s / (float)B;
    }
}

// Adam (Kingma & Ba), bias-corrected, on the phase's parameters.
__global__ void k_lstm_adam(float *p, float *m, float *v, const float *g, int64_t beg, int64_t end, float lr, float c1,
                            float c2)
{
    const int64_t q = beg + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= end) return;
    const float gq = g[q];
    const float mq = 0.9f * m[q] + 0.1f * gq;
    const float vq = 0.999f * v[q] + 0.001f * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + 1e-8f);
}

aimts_status fail(const char *msg)
{
    set_context_free_error(msg);
    return AIMTS_E_INVALID;
}

aimts_status hip_status(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return AIMTS_OK;
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    set_context_free_error(buf);
    return AIMTS_E_HIP;
}

}  // namespace lstmnet
}  // namespace aimts

using namespace aimts::lstmnet;

extern "C" {

aimts_status aimts_lstm_num_params(int64_t *n)
{
    if (!n) return AIMTS_E_INVALID;
    *n = NP;
    return AIMTS_OK;
}

aimts_status aimts_lstm_workspace_size(int32_t max_batch, size_t *bytes)
{
    if (!bytes || max_batch < 1) return fail("aimts_lstm_workspace_size: max_batch must be >= 1");
    *bytes = workspace_bytes(max_batch);
    return AIMTS_OK;
}

aimts_status aimts_lstm_filter(const float *d_params, const float *d_windows, int32_t batch, float *d_out,
                               void *hip_stream)
{
    if (!d_params || !d_windows || !d_out || batch < 1) return fail("aimts_lstm_filter: null buffer or batch < 1");
    hipLaunchKernelGGL(k_lstm_filter, dim3(batch), dim3(kBS), 0, (hipStream_t)hip_stream, d_params, d_windows, batch,
                       d_out);
    return hip_status("aimts_lstm_filter");
}

aimts_status aimts_lstm_forward(const float *d_params, const float *d_windows, int32_t batch, float *d_latent,
                                float *d_pred, float *d_recon, void *d_workspace, size_t bytes, void *hip_stream)
{
    if (!d_params || !d_windows || batch < 1 || !d_workspace) return fail("aimts_lstm_forward: null buffer or batch < 1");
    if (bytes < workspace_bytes(batch)) {
        aimts::set_context_free_error("aimts_lstm_forward: workspace too small for the batch");
        return AIMTS_E_NOMEM;
    }
    hipLaunchKernelGGL(k_lstm_fwd, dim3(batch), dim3(kBS), 0, (hipStream_t)hip_stream, d_params, d_windows, batch,
                       (float *)d_workspace, d_recon ? 1 : 0, d_latent, d_pred, d_recon);
    return hip_status("aimts_lstm_forward");
}

aimts_status aimts_lstm_backward(const float *d_params, const float *d_windows, const float *d_targets, int32_t batch,
                                 int32_t phase, float *d_grad, float *d_loss, void *d_workspace, size_t bytes,
                                 void *hip_stream)
{
    if (!d_params || !d_windows || !d_grad || batch < 1 || !d_workspace || (phase == 1 && !d_targets))
        return fail("aimts_lstm_backward: null buffer, batch < 1 or no targets for phase 1");
    if (phase != 0 && phase != 1) return fail("aimts_lstm_backward: phase must be 0 (autoencoder) or 1 (FCN)");
    if (bytes < workspace_bytes(batch)) {
        aimts::set_context_free_error("aimts_lstm_backward: workspace too small for the batch");
        return AIMTS_E_NOMEM;
    }
    const hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_lstm_bwd, dim3(batch), dim3(kBS), 0, st, d_params, d_windows, d_targets, batch, phase,
                       (float *)d_workspace);
    hipLaunchKernelGGL(k_lstm_reduce, dim3((unsigned)((NP + 255) / 256)), dim3(256), 0, st,
                       (const float *)d_workspace, batch, phase, d_grad, d_loss);
    return hip_status("aimts_lstm_backward");
}

aimts_status aimts_lstm_adam(float *d_params, float *d_m, float *d_v, const float *d_grad, int32_t phase, int64_t step,
                             float lr, void *hip_stream)
{
    if (!d_params || !d_m || !d_v || !d_grad || step < 1 || !(lr > 0.0f))
        return fail("aimts_lstm_adam: null buffer, step < 1 or lr <= 0");
    if (phase != 0 && phase != 1) return fail("aimts_lstm_adam: phase must be 0 or 1");
    const Layout L = layout();
    const int64_t beg = phase == 0 ? 0 : L.fcn_begin, end = phase == 0 ? L.ae_end : L.fcn_end;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)step)), c2 = (float)(1.0 - std::pow(0.999, (double)step));
    hipLaunchKernelGGL(k_lstm_adam, dim3((unsigned)((end - beg + 255) / 256)), dim3(256), 0, (hipStream_t)hip_stream,
                       d_params, d_m, d_v, d_grad, beg, end, lr, c1, c2);
    return hip_status("aimts_lstm_adam");
}

}  // extern "C"
