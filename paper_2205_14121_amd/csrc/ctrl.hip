// Learned MTS controller kernels: the AI inference pipeline of Table 2 (denoise ->
// autoencoder latent -> fully connected head -> ratio and hold), and its training
// (backpropagation through time, Adam), all on the device.
//
// Precision: parameters are read as bfloat16 (rounded from the float32 master copy);
// activations, gradients and every accumulation are float32.
//
// Kernels:
//   k_fwd      one workgroup per window: moving average + z-score, 2-layer GRU encoder,
//              latent, 2-layer GRU decoder, read-out, head.  Each layer's weights are
//              staged in LDS (transposed, so a thread's gate row is read with unit
//              stride across the wavefront).  Per-step gate values are cached for BPTT.
//   k_bwd_ae   one workgroup per window: BPTT through decoder and encoder; stores the
//              gate-preactivation gradients of every step.
//   k_wgrad    weight gradients as contractions over (window, step) rows, split over
//              row chunks with a fixed-order reduction (deterministic).
//   k_bwd_head per-window head gradients, reduced over windows in order.
//   k_adam     bias-corrected Adam on the phase's parameters, refreshing the bf16 copy.
#include <cmath>

#include "ctrl.h"

namespace aimts {

int64_t ctrl_num_params() { return ctrl_layout().total; }

namespace {

constexpr int kBS = 256;
constexpr int kSplit = kCtrlSplit;

__device__ __forceinline__ float bf(uint16_t w) { return __uint_as_float((uint32_t)w << 16); }

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float sigm(float a) { return 1.0f / (1.0f + expf(-a)); }

__global__ void k_round_bf16(const float *m, uint16_t *w, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[i] = to_bf16(m[i]);
}

__global__ void k_zero_f32(float *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// LDS images of one GRU layer: W_ih^T [nin][G], W_hh^T [H][G] (bf16), biases.
struct GruLds {
    uint16_t wih[kH * kG];
    uint16_t whh[kH * kG];
    float bih[kG], bhh[kG];
};

__device__ void load_gru_T(GruLds &L, const uint16_t *w, int64_t o_wih, int64_t o_whh, int64_t o_bih,
                           int64_t o_bhh, int nin)
{
    for (int e = threadIdx.x; e < kG * nin; e += kBS) {
        const int g = e / nin, u = e % nin;
        L.wih[u * kG + g] = w[o_wih + e];
    }
    for (int e = threadIdx.x; e < kG * kH; e += kBS) {
        const int g = e / kH, u = e % kH;
        L.whh[u * kG + g] = w[o_whh + e];
    }
    for (int e = threadIdx.x; e < kG; e += kBS) {
        L.bih[e] = bf(w[o_bih + e]);
        L.bhh[e] = bf(w[o_bhh + e]);
    }
    __syncthreads();
}

// Run one GRU layer over kT steps.  in(t, u) gives the input; outputs go to out_lds
// [T][H] and to the global hs/cache of this window.
template <typename In>
__device__ void gru_layer(const GruLds &L, int nin, In in, float *out_lds, float *hs_g, float *cache_g, float *gi,
                          float *gh, float *h)
{
    if (threadIdx.x < kH) h[threadIdx.x] = 0.0f;
    __syncthreads();
    for (int t = 0; t < kT; ++t) {
        if (threadIdx.x < kG) {
            const int g = threadIdx.x;
            float a = L.bih[g], c = L.bhh[g];
            for (int u = 0; u < nin; ++u) a += bf(L.wih[u * kG + g]) * in(t, u);
            for (int u = 0; u < kH; ++u) c += bf(L.whh[u * kG + g]) * h[u];
            gi[g] = a;
            gh[g] = c;
        }
        __syncthreads();
        if (threadIdx.x < kH) {
            const int u = threadIdx.x;
            const float r = sigm(gi[u] + gh[u]);
            const float z = sigm(gi[kH + u] + gh[kH + u]);
            const float n = tanhf(gi[2 * kH + u] + r * gh[2 * kH + u]);
            const float hn = (1.0f - z) * n + z * h[u];
            out_lds[t * kH + u] = hn;
            hs_g[t * kH + u] = hn;
            float *cc = cache_g + (int64_t)t * 4 * kH;
            cc[u] = r;
            cc[kH + u] = z;
            cc[2 * kH + u] = n;
            cc[3 * kH + u] = gh[2 * kH + u];
        }
        __syncthreads();
        if (threadIdx.x < kH) h[threadIdx.x] = out_lds[t * kH + threadIdx.x];
        __syncthreads();
    }
}

struct FwdLds {
    GruLds w;
    float x[kT * kF];
    float a[kT * kH];
    float b[kT * kH];
    float gi[kG], gh[kG], h[kH];
    float lat[kLat];
    float head[64];
    float red[kBS];
};

// decode = 0 (inference only): the decoder and the reconstruction are skipped; the
// latent, head activations and logits are the same as with decode = 1.
__global__ __launch_bounds__(kBS) void k_fwd(CtrlState c, const float *windows, const int32_t *labels, int B,
                                            int decode)
{
    __shared__ FwdLds S;
    const int b = blockIdx.x;
    const CtrlLayout L = ctrl_layout();
    const uint16_t *w = c.wbf;
    const float *raw = windows + (int64_t)b * kT * kF;
    // 1. denoise: causal moving average over kMA points, then z-score
    for (int e = threadIdx.x; e < kT * kF; e += kBS) {
        const int t = e / kF, f = e % kF;
        const int lo = t - kMA + 1 < 0 ? 0 : t - kMA + 1;
        float s = 0.0f;
        for (int q = lo; q <= t; ++q) s += raw[q * kF + f];
        const float ma = s / (float)(t - lo + 1);
        const float v = (ma - c.master[L.norm_mean + f]) / c.master[L.norm_std + f];
        S.x[e] = v;
        c.xt[(int64_t)b * kT * kF + e] = v;
    }
    __syncthreads();
    const int64_t hoff = (int64_t)b * kT * kH, coff = (int64_t)b * kT * 4 * kH;
    // 2. encoder
    load_gru_T(S.w, w, L.enc0_wih, L.enc0_whh, L.enc0_bih, L.enc0_bhh, kF);
    gru_layer(S.w, kF, [&](int t, int u) { return S.x[t * kF + u]; }, S.a, c.hs[0] + hoff, c.cache[0] + coff, S.gi,
              S.gh, S.h);
    load_gru_T(S.w, w, L.enc1_wih, L.enc1_whh, L.enc1_bih, L.enc1_bhh, kH);
    gru_layer(S.w, kH, [&](int t, int u) { return S.a[t * kH + u]; }, S.b, c.hs[1] + hoff, c.cache[1] + coff, S.gi,
              S.gh, S.h);
    // 3. latent from the last top-layer state
    if (threadIdx.x < kLat) {
        const int j = threadIdx.x;
        float s = bf(w[L.lat_b + j]);
        for (int u = 0; u < kH; ++u) s += bf(w[L.lat_w + j * kH + u]) * S.b[(kT - 1) * kH + u];
        S.lat[j] = s;
        c.lat[b * kLat + j] = s;
    }
    __syncthreads();
    // 4. decoder, fed the latent at every step
    if (decode) {
        load_gru_T(S.w, w, L.dec0_wih, L.dec0_whh, L.dec0_bih, L.dec0_bhh, kLat);
        gru_layer(S.w, kLat, [&](int, int u) { return S.lat[u]; }, S.a, c.hs[2] + hoff, c.cache[2] + coff, S.gi, S.gh,
                  S.h);
        load_gru_T(S.w, w, L.dec1_wih, L.dec1_whh, L.dec1_bih, L.dec1_bhh, kH);
        gru_layer(S.w, kH, [&](int t, int u) { return S.a[t * kH + u]; }, S.b, c.hs[3] + hoff, c.cache[3] + coff, S.gi,
                  S.gh, S.h);
        // 5. read-out and reconstruction error
        float err = 0.0f;
        for (int e = threadIdx.x; e < kT * kF; e += kBS) {
            const int t = e / kF, f = e % kF;
            float s = bf(w[L.out_b + f]);
            for (int u = 0; u < kH; ++u) s += bf(w[L.out_w + f * kH + u]) * S.b[t * kH + u];
            c.recon[(int64_t)b * kT * kF + e] = s;
            const float d = s - S.x[e];
            err += d * d;
        }
        S.red[threadIdx.x] = err;
        __syncthreads();
        for (int s = kBS / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) S.red[threadIdx.x] += S.red[threadIdx.x + s];
            __syncthreads();
        }
    } else {
        if (threadIdx.x == 0) S.red[0] = 0.0f;
        __syncthreads();
    }
    // 6. head: 16 -> 32 -> 16 -> 8 (ReLU) -> 9
    if (threadIdx.x == 0) {
        float *act = c.act + (int64_t)b * 56;
        float a1[32], a2[16], a3[8];
        for (int j = 0; j < 32; ++j) {
            float s = bf(w[L.h1_b + j]);
            for (int u = 0; u < kLat; ++u) s += bf(w[L.h1_w + j * kLat + u]) * S.lat[u];
            a1[j] = s;
            act[j] = s;
        }
        for (int j = 0; j < 16; ++j) {
            float s = bf(w[L.h2_b + j]);
            for (int u = 0; u < 32; ++u) s += bf(w[L.h2_w + j * 32 + u]) * fmaxf(a1[u], 0.0f);
            a2[j] = s;
            act[32 + j] = s;
        }
        for (int j = 0; j < 8; ++j) {
            float s = bf(w[L.h3_b + j]);
            for (int u = 0; u < 16; ++u) s += bf(w[L.h3_w + j * 16 + u]) * fmaxf(a2[u], 0.0f);
            a3[j] = s;
            act[48 + j] = s;
        }
        float lg[kNout];
        for (int j = 0; j < kNout; ++j) {
            float s = bf(w[L.h4_b + j]);
            for (int u = 0; u < 8; ++u) s += bf(w[L.h4_w + j * 8 + u]) * fmaxf(a3[u], 0.0f);
            lg[j] = s;
            c.logits[b * kNout + j] = s;
        }
        float ce = 0.0f;
        if (labels) {
            // cross-entropy of the ratio group (5) and the hold group (4)
            for (int grp = 0; grp < 2; ++grp) {
                const int o = grp == 0 ? 0 : 5, n = grp == 0 ? 5 : 4;
                float mx = lg[o];
                for (int j = 1; j < n; ++j) mx = fmaxf(mx, lg[o + j]);
                float se = 0.0f;
                for (int j = 0; j < n; ++j) se += expf(lg[o + j] - mx);
                ce += mx + logf(se) - lg[o + labels[2 * b + grp]];
            }
        }
        c.seq_loss[2 * b] = S.red[0];
        c.seq_loss[2 * b + 1] = ce;
    }
}

// ---------------------------------------------------------------------------
// Backward through the autoencoder (phase 0)
// ---------------------------------------------------------------------------
struct BwdLds {
    uint16_t wih[kG * kH];   // W_ih [G][nin] (row-major, as stored)
    uint16_t whh[kG * kH];   // W_hh [G][H]
    float dx[kT * kH];       // gradient w.r.t. the layer input, per step
    float dtop[kT * kH];     // gradient arriving from above, per step
    float dgi[kG], dgh[kG], dh[kH];
    float dlat[kLat];
};

__device__ void load_gru_rowmajor(BwdLds &S, const uint16_t *w, int64_t o_wih, int64_t o_whh, int nin)
{
    for (int e = threadIdx.x; e < kG * nin; e += kBS) S.wih[e] = w[o_wih + e];
    for (int e = threadIdx.x; e < kG * kH; e += kBS) S.whh[e] = w[o_whh + e];
    __syncthreads();
}

// BPTT of one layer.  dtop[t] is dL/dh_t from above; writes dgi/dgh per step to
// global and, if want_dx, dL/d input_t into S.dx (accumulating over t into dx[0] when
// the input is the same vector at every step).
__device__ void gru_layer_bwd(BwdLds &S, int nin, const float *hs_g, const float *cache_g, float *dgi_g,
                              float *dgh_g, int dx_mode /*0 none, 1 per step, 2 summed*/)
{
    if (threadIdx.x < kH) S.dh[threadIdx.x] = 0.0f;
    if (dx_mode == 2)
        for (int e = threadIdx.x; e < nin; e += kBS) S.dx[e] = 0.0f;
    __syncthreads();
    for (int t = kT - 1; t >= 0; --t) {
        if (threadIdx.x < kH) {
            const int u = threadIdx.x;
            const float *cc = cache_g + (int64_t)t * 4 * kH;
            const float r = cc[u], z = cc[kH + u], n = cc[2 * kH + u], ghn = cc[3 * kH + u];
            const float hp = t > 0 ? hs_g[(t - 1) * kH + u] : 0.0f;
            const float dh = S.dh[u] + S.dtop[t * kH + u];
            const float dn = dh * (1.0f - z);
            const float dz = dh * (hp - n);
            const float dan = dn * (1.0f - n * n);
            const float dar = dan * ghn * r * (1.0f - r);
            const float daz = dz * z * (1.0f - z);
            S.dgi[u] = dar;
            S.dgi[kH + u] = daz;
            S.dgi[2 * kH + u] = dan;
            S.dgh[u] = dar;
            S.dgh[kH + u] = daz;
            S.dgh[2 * kH + u] = dan * r;
            S.dh[u] = dh * z;  // direct path; the recurrent path is added below
        }
        __syncthreads();
        for (int g = threadIdx.x; g < kG; g += kBS) {
            dgi_g[(int64_t)t * kG + g] = S.dgi[g];
            dgh_g[(int64_t)t * kG + g] = S.dgh[g];
        }
        if (threadIdx.x < kH) {
            const int u = threadIdx.x;
            float s = 0.0f;
            for (int g = 0; g < kG; ++g) s += S.dgh[g] * bf(S.whh[g * kH + u]);
            S.dh[u] += s;
        }
        if (dx_mode != 0) {
            const int u = (int)threadIdx.x - kH;  // threads kH .. kH + nin - 1 form the input gradient
            if (u >= 0 && u < nin) {
                float s = 0.0f;
                for (int g = 0; g < kG; ++g) s += S.dgi[g] * bf(S.wih[g * nin + u]);
                if (dx_mode == 1) S.dx[t * nin + u] = s;
                else S.dx[u] += s;
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBS) void k_bwd_ae(CtrlState c, int B)
{
    __shared__ BwdLds S;
    const int b = blockIdx.x;
    const CtrlLayout L = ctrl_layout();
    const uint16_t *w = c.wbf;
    const int64_t hoff = (int64_t)b * kT * kH, coff = (int64_t)b * kT * 4 * kH, goff = (int64_t)b * kT * kG;
    const float scale = 2.0f / ((float)B * kT * kF);
    // d recon and d(top decoder state) = dre . out_w
    for (int e = threadIdx.x; e < kT * kF; e += kBS) {
        const int64_t q = (int64_t)b * kT * kF + e;
        c.dre[q] = scale * (c.recon[q] - c.xt[q]);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kT * kH; e += kBS) {
        const int t = e / kH, u = e % kH;
        float s = 0.0f;
        for (int f = 0; f < kF; ++f) s += c.dre[(int64_t)b * kT * kF + t * kF + f] * bf(w[L.out_w + f * kH + u]);
        S.dtop[e] = s;
    }
    __syncthreads();
    // decoder layer 1 -> gradient into decoder layer 0 outputs
    load_gru_rowmajor(S, w, L.dec1_wih, L.dec1_whh, kH);
    gru_layer_bwd(S, kH, c.hs[3] + hoff, c.cache[3] + coff, c.dgi[3] + goff, c.dgh[3] + goff, 1);
    for (int e = threadIdx.x; e < kT * kH; e += kBS) S.dtop[e] = S.dx[e];
    __syncthreads();
    // decoder layer 0: its input is the latent at every step -> summed input gradient
    load_gru_rowmajor(S, w, L.dec0_wih, L.dec0_whh, kLat);
    gru_layer_bwd(S, kLat, c.hs[2] + hoff, c.cache[2] + coff, c.dgi[2] + goff, c.dgh[2] + goff, 2);
    if (threadIdx.x < kLat) {
        S.dlat[threadIdx.x] = S.dx[threadIdx.x];
        c.dlat[b * kLat + threadIdx.x] = S.dx[threadIdx.x];
    }
    __syncthreads();
    // latent -> last encoder state
    for (int e = threadIdx.x; e < kT * kH; e += kBS) S.dtop[e] = 0.0f;
    __syncthreads();
    if (threadIdx.x < kH) {
        const int u = threadIdx.x;
        float s = 0.0f;
        for (int j = 0; j < kLat; ++j) s += S.dlat[j] * bf(w[L.lat_w + j * kH + u]);
        S.dtop[(kT - 1) * kH + u] = s;
    }
    __syncthreads();
    load_gru_rowmajor(S, w, L.enc1_wih, L.enc1_whh, kH);
    gru_layer_bwd(S, kH, c.hs[1] + hoff, c.cache[1] + coff, c.dgi[1] + goff, c.dgh[1] + goff, 1);
    for (int e = threadIdx.x; e < kT * kH; e += kBS) S.dtop[e] = S.dx[e];
    __syncthreads();
    load_gru_rowmajor(S, w, L.enc0_wih, L.enc0_whh, kF);
    gru_layer_bwd(S, kF, c.hs[0] + hoff, c.cache[0] + coff, c.dgi[0] + goff, c.dgh[0] + goff, 0);
}

// out[m][k] (+)= sum over rows r of A[r][m] * X(r)[k], split over kSplit row chunks.
// X row of (window b, step t): mode 0 -> X[(b*T + t)], mode 1 -> X[(b*T + t - 1)] or 0
// at t = 0, mode 2 -> X[b] (same vector at every step).
__global__ __launch_bounds__(kBS) void k_wgrad(const float *A, int lda, const float *X, int ldx, int mode, int M,
                                               int K, int64_t R, float *partial)
{
    __shared__ float As[16][64];
    __shared__ float Xs[16][64];
    const int m0 = blockIdx.x * 64, k0 = blockIdx.y * 64, split = blockIdx.z;
    const int64_t r_beg = R * split / kSplit, r_end = R * (split + 1) / kSplit;
    const int tm = threadIdx.x / 16, tk = threadIdx.x % 16;  // 4x4 outputs per thread
    float acc[4][4] = {};
    for (int64_t r0 = r_beg; r0 < r_end; r0 += 16) {
        for (int e = threadIdx.x; e < 16 * 64; e += kBS) {
            const int rr = e / 64, cc = e % 64;
            const int64_t r = r0 + rr;
            float av = 0.0f, xv = 0.0f;
            if (r < r_end) {
                if (m0 + cc < M) av = A[r * lda + m0 + cc];
                if (k0 + cc < K) {
                    const int64_t bb = r / kT, t = r % kT;
                    if (mode == 0) xv = X[r * ldx + k0 + cc];
                    else if (mode == 1) xv = t > 0 ? X[(r - 1) * ldx + k0 + cc] : 0.0f;
                    else xv = X[bb * ldx + k0 + cc];
                }
            }
            As[rr][cc] = av;
            Xs[rr][cc] = xv;
        }
        __syncthreads();
        for (int rr = 0; rr < 16; ++rr)
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) acc[i][j] += As[rr][tm * 4 + i] * Xs[rr][tk * 4 + j];
        __syncthreads();
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            const int m = m0 + tm * 4 + i, k = k0 + tk * 4 + j;
            if (m < M && k < K) partial[((int64_t)split * M + m) * K + k] = acc[i][j];
        }
}

// out[e] = sum over splits of partial[s][e]   (fixed order)
__global__ void k_split_reduce(const float *partial, int64_t n, float *out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float s = 0.0f;
    for (int q = 0; q < kSplit; ++q) s += partial[q * n + e];
    out[e] = s;
}

// out[m] = sum over rows of A[r][m]  (bias gradients), fixed order per column
__global__ void k_colsum(const float *A, int lda, int M, int64_t R, float *out)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    float s = 0.0f;
    for (int64_t r = 0; r < R; ++r) s += A[r * lda + m];
    out[m] = s;
}

// ---------------------------------------------------------------------------
// Head backward (phase 1): one thread per window, then an ordered reduction.
// ---------------------------------------------------------------------------
__global__ void k_bwd_head(CtrlState c, const int32_t *labels, int B)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const CtrlLayout L = ctrl_layout();
    const uint16_t *w = c.wbf;
    const float *act = c.act + (int64_t)b * 56;
    const float *lg = c.logits + (int64_t)b * kNout;
    const float *lat = c.lat + (int64_t)b * kLat;
    float *gp = c.head_part + (int64_t)b * (L.head_end - L.head_begin);
    auto G = [&](int64_t off) { return gp + (off - L.head_begin); };
    float dlg[kNout];
    for (int grp = 0; grp < 2; ++grp) {
        const int o = grp == 0 ? 0 : 5, n = grp == 0 ? 5 : 4;
        float mx = lg[o];
        for (int j = 1; j < n; ++j) mx = fmaxf(mx, lg[o + j]);
        float se = 0.0f;
        for (int j = 0; j < n; ++j) se += expf(lg[o + j] - mx);
        for (int j = 0; j < n; ++j) dlg[o + j] = (expf(lg[o + j] - mx) / se - (j == labels[2 * b + grp] ? 1.0f : 0.0f)) / B;
    }
    float r3[8], d3[8], r2[16], d2[16], r1[32], d1[32];
    for (int j = 0; j < 8; ++j) r3[j] = fmaxf(act[48 + j], 0.0f);
    for (int j = 0; j < 16; ++j) r2[j] = fmaxf(act[32 + j], 0.0f);
    for (int j = 0; j < 32; ++j) r1[j] = fmaxf(act[j], 0.0f);
    for (int j = 0; j < kNout; ++j) {
        *G(L.h4_b + j) = dlg[j];
        for (int u = 0; u < 8; ++u) *G(L.h4_w + j * 8 + u) = dlg[j] * r3[u];
    }
    for (int u = 0; u < 8; ++u) {
        float s = 0.0f;
        for (int j = 0; j < kNout; ++j) s += dlg[j] * bf(w[L.h4_w + j * 8 + u]);
        d3[u] = act[48 + u] > 0.0f ? s : 0.0f;
        *G(L.h3_b + u) = d3[u];
        for (int q = 0; q < 16; ++q) *G(L.h3_w + u * 16 + q) = d3[u] * r2[q];
    }
    for (int u = 0; u < 16; ++u) {
        float s = 0.0f;
        for (int j = 0; j < 8; ++j) s += d3[j] * bf(w[L.h3_w + j * 16 + u]);
        d2[u] = act[32 + u] > 0.0f ? s : 0.0f;
        *G(L.h2_b + u) = d2[u];
        for (int q = 0; q < 32; ++q) *G(L.h2_w + u * 32 + q) = d2[u] * r1[q];
    }
    for (int u = 0; u < 32; ++u) {
        float s = 0.0f;
        for (int j = 0; j < 16; ++j) s += d2[j] * bf(w[L.h2_w + j * 32 + u]);
        d1[u] = act[u] > 0.0f ? s : 0.0f;
        *G(L.h1_b + u) = d1[u];
        for (int q = 0; q < kLat; ++q) *G(L.h1_w + u * kLat + q) = d1[u] * lat[q];
    }
}

__global__ void k_head_reduce(const float *part, int64_t nh, int B, float *out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nh) return;
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += part[(int64_t)b * nh + e];
    out[e] = s;
}

// loss: phase 0 = sum of squared errors / (B T F); phase 1 = mean cross-entropy
__global__ void k_loss(const float *seq_loss, int B, int phase, float *loss)
{
    if (threadIdx.x != 0) return;
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += seq_loss[2 * b + phase];
    *loss = phase == 0 ? s / ((float)B * kT * kF) : s / (float)B;
}

__global__ void k_adam(float *p, uint16_t *wbf, float *m, float *v, const float *g, int64_t beg, int64_t end, float lr,
                       float bc1, float bc2)
{
    const int64_t i = beg + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= end) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
    p[i] = pi;
    wbf[i] = to_bf16(pi);
}

// Gather each platelet's last kT feature rows (oldest first) from the ring.
__global__ void k_gather_windows(const float *ring, int head, int64_t P, float *win)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * kT * kF) return;
    const int64_t p = e / (kT * kF), r = (e / kF) % kT, f = e % kF;
    win[e] = ring[(p * kT + (head + r) % kT) * kF + f];
}

// Ratio and hold per platelet by argmax; the system takes the minimum over platelets.
// A platelet with any non-finite logit takes the fallback ratio 4 (and hold 16).
__global__ void k_decide(const float *logits, int64_t P, int32_t *out, int32_t *pratio)
{
    if (threadIdx.x != 0) return;
    const int ratios[5] = {1, 2, 4, 8, 16};
    const int holds[4] = {16, 32, 64, 128};
    int k = 1 << 30, h = 1 << 30, fb = 0;
    for (int64_t p = 0; p < P; ++p) {
        const float *lg = logits + p * kNout;
        bool ok = true;
        for (int j = 0; j < kNout; ++j) ok = ok && isfinite(lg[j]);
        int kr = 4, hr = 16;
        if (ok) {
            int a = 0;
            for (int j = 1; j < 5; ++j) if (lg[j] > lg[a]) a = j;
            int bh = 0;
            for (int j = 1; j < 4; ++j) if (lg[5 + j] > lg[5 + bh]) bh = j;
            kr = ratios[a];
            hr = holds[bh];
        } else {
            fb = 1;
        }
        pratio[p] = kr;
        k = kr < k ? kr : k;
        h = hr < h ? hr : h;
    }
    out[0] = k;
    out[1] = h;
    out[2] = fb;
}

void wgrad(CtrlState &c, const float *A, int lda, const float *X, int ldx, int mode, int M, int K, int64_t R,
           float *out_w, float *out_b, float *scratch, hipStream_t st)
{
    dim3 grid((unsigned)((M + 63) / 64), (unsigned)((K + 63) / 64), kSplit);
    hipLaunchKernelGGL(k_wgrad, grid, dim3(kBS), 0, st, A, lda, X, ldx, mode, M, K, R, scratch);
    hipLaunchKernelGGL(k_split_reduce, dim3(nblocks((int64_t)M * K, 256)), dim3(256), 0, st, (const float *)scratch,
                       (int64_t)M * K, out_w);
    if (out_b) hipLaunchKernelGGL(k_colsum, dim3(nblocks(M, 64)), dim3(64), 0, st, A, lda, M, R, out_b);
}

}  // namespace

void ctrl_init(CtrlState &c, hipStream_t st)
{
    c.have_weights = false;
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(4), 0, st, c.loss, (int64_t)4);
}

void ctrl_after_set(CtrlState &c, hipStream_t st)
{
    const int64_t n = c.np;
    hipLaunchKernelGGL(k_round_bf16, dim3(nblocks(n, 256)), dim3(256), 0, st, c.master, c.wbf, n);
    hipLaunchKernelGGL(k_zero_f32, dim3(nblocks(n, 256)), dim3(256), 0, st, c.adam_m, n);
    hipLaunchKernelGGL(k_zero_f32, dim3(nblocks(n, 256)), dim3(256), 0, st, c.adam_v, n);
    c.adam_t[0] = c.adam_t[1] = 0;
    c.have_weights = true;
}

void ctrl_round_weights(const float *params, uint16_t *wbf, hipStream_t st)
{
    const int64_t n = ctrl_num_params();
    hipLaunchKernelGGL(k_round_bf16, dim3(nblocks(n, 256)), dim3(256), 0, st, params, wbf, n);
}

void ctrl_forward(CtrlState &c, const float *windows, int B, hipStream_t st, const int32_t *labels, bool decode)
{
    hipLaunchKernelGGL(k_fwd, dim3(B), dim3(kBS), 0, st, c, windows, labels, B, decode ? 1 : 0);
}

void ctrl_copy_outputs(CtrlState &c, int B, float *d_latent, float *d_logits, hipStream_t st)
{
    if (d_latent) (void)hipMemcpyAsync(d_latent, c.lat, sizeof(float) * B * kLat, hipMemcpyDeviceToDevice, st);
    if (d_logits) (void)hipMemcpyAsync(d_logits, c.logits, sizeof(float) * B * kNout, hipMemcpyDeviceToDevice, st);
}

void ctrl_backward(CtrlState &c, const int32_t *labels, int B, int phase, hipStream_t st)
{
    const CtrlLayout L = ctrl_layout();
    hipLaunchKernelGGL(k_zero_f32, dim3(nblocks(c.np, 256)), dim3(256), 0, st, c.grad, c.np);
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(64), 0, st, (const float *)c.seq_loss, B, phase, c.loss);
    if (phase == 1) {
        const int64_t nh = L.head_end - L.head_begin;
        hipLaunchKernelGGL(k_bwd_head, dim3(nblocks(B, 64)), dim3(64), 0, st, c, labels, B);
        hipLaunchKernelGGL(k_head_reduce, dim3(nblocks(nh, 256)), dim3(256), 0, st, (const float *)c.head_part, nh, B,
                           c.grad + L.head_begin);
        return;
    }
    hipLaunchKernelGGL(k_bwd_ae, dim3(B), dim3(kBS), 0, st, c, B);
    const int64_t R = (int64_t)B * kT;
    float *scratch = c.wg_scratch;
    float *g = c.grad;
    // read-out
    wgrad(c, c.dre, kF, c.hs[3], kH, 0, kF, kH, R, g + L.out_w, g + L.out_b, scratch, st);
    // GRU layers: input weights (mode by input kind) and recurrent weights (previous state)
    struct LayerRef { int l; int64_t wih, whh, bih, bhh; const float *in; int ldin; int mode; int nin; };
    const LayerRef layers[4] = {
        {0, L.enc0_wih, L.enc0_whh, L.enc0_bih, L.enc0_bhh, c.xt, kF, 0, kF},
        {1, L.enc1_wih, L.enc1_whh, L.enc1_bih, L.enc1_bhh, c.hs[0], kH, 0, kH},
        {2, L.dec0_wih, L.dec0_whh, L.dec0_bih, L.dec0_bhh, c.lat, kLat, 2, kLat},
        {3, L.dec1_wih, L.dec1_whh, L.dec1_bih, L.dec1_bhh, c.hs[2], kH, 0, kH},
    };
    for (const LayerRef &q : layers) {
        wgrad(c, c.dgi[q.l], kG, q.in, q.ldin, q.mode, kG, q.nin, R, g + q.wih, g + q.bih, scratch, st);
        wgrad(c, c.dgh[q.l], kG, c.hs[q.l], kH, 1, kG, kH, R, g + q.whh, g + q.bhh, scratch, st);
    }
    // latent: rows are windows; the encoder's last state is row T-1 of hs[1]
    wgrad(c, c.dlat, kLat, c.hs[1] + (kT - 1) * kH, kT * kH, 0, kLat, kH, B, g + L.lat_w, g + L.lat_b, scratch, st);
}

void ctrl_copy_grads(CtrlState &c, float *d_grads, hipStream_t st)
{
    (void)hipMemcpyAsync(d_grads, c.grad, sizeof(float) * c.np, hipMemcpyDeviceToDevice, st);
}

void ctrl_adam(CtrlState &c, int phase, float lr, hipStream_t st)
{
    const CtrlLayout L = ctrl_layout();
    const int64_t beg = phase == 0 ? 0 : L.head_begin, end = phase == 0 ? L.ae_end : L.head_end;
    const int64_t t = ++c.adam_t[phase];
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)t));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)t));
    hipLaunchKernelGGL(k_adam, dim3(nblocks(end - beg, 256)), dim3(256), 0, st, c.master, c.wbf, c.adam_m, c.adam_v,
                       (const float *)c.grad, beg, end, lr, bc1, bc2);
}

aimts_status ctrl_infer_ring(CtrlState &c, const Dev &s, const float *ring, int head, int32_t *k, int32_t *hold,
                             int *fallback, hipStream_t st)
{
    const int64_t P = s.P;
    hipLaunchKernelGGL(k_gather_windows, dim3(nblocks(P * kT * kF, 256)), dim3(256), 0, st, ring, head, P, c.windows);
    ctrl_forward(c, c.windows, (int)P, st, nullptr, false);
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(64), 0, st, (const float *)c.logits, P, c.decision, c.pratio);
    int32_t out[4] = {4, 16, 0, 0};
    hipError_t e = hipMemcpyAsync(out, c.decision, sizeof(int32_t) * 3, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return AIMTS_E_HIP;
    *k = out[0];
    *hold = out[1];
    *fallback = out[2];
    return AIMTS_OK;
}

}  // namespace aimts
