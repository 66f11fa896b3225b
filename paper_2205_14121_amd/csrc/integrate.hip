// Two-group RESPA velocity Verlet (Sec. 3.3, MSM pseudocode Table 1): half kicks at
// entry and exit of each level, drifts at the inner step.
//
// Fluid particles that are not inner members feel no inner force, so their velocity is
// constant through the inner loop except at a wall bounce.  open_kick_lazy_drift gives
// them the outer half kick and then all k inner drifts in registers in one pass: the
// same k additions and wall/periodic tests as drifting k times, for one read and one
// write of x and v instead of k.  The members (beads and fluid near beads) get their
// first inner half kick and drift in the same pass; the later kicks and drifts are fused
// into the inner force kernel.
#include "common.h"

namespace aimts {

namespace {

__device__ __forceinline__ double fo_at(const Dev &s, int k, int64_t t)
{
    return s.fp32 ? (double)((const float *)s.fo)[k * s.N + t] : ((const double *)s.fo)[k * s.N + t];
}

// Largest of a non-negative value over the wavefront (every lane must call it).
__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Raises the float held as bits in *slot to the largest v of the 256-thread block
// (every thread must call it; v >= 0).  The maximum over all blocks lands in one word,
// so each block first reads it and only issues the atomic when it would raise it:
// device-scope atomics on one address serialise, and with most blocks above the floor
// one atomic per wavefront costs more than the kernel's own memory traffic.  The word
// only grows between resets (made by an earlier kernel), so a read can only
// under-estimate it and never skips a needed update.
__device__ __forceinline__ void block_max_commit(uint32_t *slot, float v, float floor)
{
    __shared__ float part[4];
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float b = fmaxf(fmaxf(part[0], part[1]), fmaxf(part[2], part[3]));
        if (b > floor) {
            const uint32_t cur = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__float_as_uint(b) > cur) atomicMax(slot, __float_as_uint(b));
        }
    }
}

// Opening outer half kick of every mobile particle.  A non-member then takes all k inner
// drifts in registers; a member takes the opening inner half kick of the first inner
// step and its drift, written to (xw, vw) (which may be the particle arrays themselves:
// each thread reads and writes its own particle only), and keeps its largest
// displacement since the rebuild in dmax.  Wall particles are copied into (xa, va), the
// members' second state buffer.
__global__ void k_open_lazy(Dev s, double h_out, int k, double dt, double *xa, double *va, LevelStep ls, double *xw,
                            double *vw)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float pmax = 0.0f;  // largest k-drift path of a non-member
    bool bad = false;
    const int ty = t < s.N ? ptype(s, s.id[t]) : -1;
    const int64_t N = s.N;
    if (ty == 1) {  // frozen walls are never integrated; the members' second buffer holds them too
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xa[c * N + t] = s.x[c * N + t];
            va[c * N + t] = s.v[c * N + t];
        }
    } else if (ty >= 0) {
        const double mi = s.minv[ty];
        double v0 = s.v[t], v1 = s.v[N + t], v2 = s.v[2 * N + t];
        v0 += h_out * fo_at(s, 0, t) * mi;
        v1 += h_out * fo_at(s, 1, t) * mi;
        v2 += h_out * fo_at(s, 2, t) * mi;
        double x0 = s.x[t], x1 = s.x[N + t], x2 = s.x[2 * N + t];
        const int32_t m = s.mos[t];
        if (m < 0) {
            // the k drifts move the particle by at most k dt |v| (a bounce only turns it round)
            const double path = (double)k * dt * sqrt(v0 * v0 + v1 * v1 + v2 * v2);
            for (int q = 0; q < k; ++q) drift_one(s, x0, x1, x2, v0, v1, v2, dt);
            s.x[t] = x0;
            s.x[N + t] = x1;
            s.x[2 * N + t] = x2;
            s.v[t] = v0;
            s.v[N + t] = v1;
            s.v[2 * N + t] = v2;
            if (!isfinite(path)) bad = true;
            else pmax = (float)(path * 1.000001);
        } else {
            const int64_t C = s.cap_members;
            if (s.nlev == 3) {
                // three-level mode: every level opens, outermost first (interface M, flowing
                // sublevel P1, aggregating sublevel P2), each with its own half step
                const double hh[3] = {ls.hm, ls.h1, ls.h2};
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    v0 += hh[l] * s.fi[(3 * l) * C + m] * mi;
                    v1 += hh[l] * s.fi[(3 * l + 1) * C + m] * mi;
                    v2 += hh[l] * s.fi[(3 * l + 2) * C + m] * mi;
                }
            } else {
                v0 += ls.h2 * s.fi[m] * mi;
                v1 += ls.h2 * s.fi[C + m] * mi;
                v2 += ls.h2 * s.fi[2 * C + m] * mi;
            }
            drift_one(s, x0, x1, x2, v0, v1, v2, dt);
            xw[t] = x0;
            xw[N + t] = x1;
            xw[2 * N + t] = x2;
            vw[t] = v0;
            vw[N + t] = v1;
            vw[2 * N + t] = v2;
            const double e0 = min_image(s, 0, x0 - s.xref[m]);
            const double e1 = min_image(s, 1, x1 - s.xref[C + m]);
            const double e2 = min_image(s, 2, x2 - s.xref[2 * C + m]);
            const double disp = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
            if (!isfinite(disp)) {
                bad = true;
            } else {
                const float d = (float)(disp * 1.000001);  // rounded up
                if (d > s.dmax[m]) s.dmax[m] = d;
            }
        }
    }
    if (s.nb > 0) block_max_commit(&s.maxdisp[0], pmax, (float)s.disp_floor);
    if (bad) atomicOr(s.err, kErrNonFinite);
}

__global__ void k_outer_kick(Dev s, double h)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= s.N) return;
    const int ty = ptype(s, s.id[t]);
    if (ty == 1) return;
    const double mi = s.minv[ty];
    const int64_t N = s.N;
    const double v0 = s.v[t] + h * fo_at(s, 0, t) * mi;
    const double v1 = s.v[N + t] + h * fo_at(s, 1, t) * mi;
    const double v2 = s.v[2 * N + t] + h * fo_at(s, 2, t) * mi;
    s.v[t] = v0;
    s.v[N + t] = v1;
    s.v[2 * N + t] = v2;
    if (!isfinite(v0 + v1 + v2)) atomicOr(s.err, kErrNonFinite);
}

}  // namespace

void open_kick_lazy_drift(const Dev &s, double h_out, int k, double dt_in, double *xa, double *va,
                          const LevelStep &ls, double *xw, double *vw, hipStream_t st)
{
    hipLaunchKernelGGL(k_open_lazy, dim3(nblocks(s.N, 256)), dim3(256), 0, st, s, h_out, k, dt_in, xa, va, ls, xw, vw);
}

void outer_kick(const Dev &s, double h_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_outer_kick, dim3(nblocks(s.N, 256)), dim3(256), 0, st, s, h_out);
}

}  // namespace aimts
