// Two-group RESPA velocity Verlet (Sec. 3.3, MSM pseudocode Table 1): half kicks at
// entry and exit of each level, drifts at the inner step.
//
// Fluid particles that are not inner members feel no inner force, so their velocity is
// constant through the inner loop except at a wall bounce.  open_kick_lazy_drift gives
// them the outer half kick and then all k inner drifts in registers in one pass: the
// same k additions and wall/periodic tests as drifting k times, for one read and one
// write of x and v instead of k.  The members (beads and fluid near beads) are drifted
// by the inner loop kernels.
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

__global__ void k_open_lazy(Dev s, double h_out, int k, double dt)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float pmax = 0.0f;  // largest k-drift path of a non-member
    bool bad = false;
    const int ty = t < s.N ? ptype(s, s.id[t]) : 1;
    if (ty != 1) {  // frozen walls are never integrated
        const double mi = s.minv[ty];
        const int64_t N = s.N;
        double v0 = s.v[t], v1 = s.v[N + t], v2 = s.v[2 * N + t];
        v0 += h_out * fo_at(s, 0, t) * mi;
        v1 += h_out * fo_at(s, 1, t) * mi;
        v2 += h_out * fo_at(s, 2, t) * mi;
        if (s.mos[t] < 0) {
            double x0 = s.x[t], x1 = s.x[N + t], x2 = s.x[2 * N + t];
            // the k drifts move the particle by at most k dt |v| (a bounce only turns it round)
            const double path = (double)k * dt * sqrt(v0 * v0 + v1 * v1 + v2 * v2);
            for (int q = 0; q < k; ++q) drift_one(s, x0, x1, x2, v0, v1, v2, dt);
            s.x[t] = x0;
            s.x[N + t] = x1;
            s.x[2 * N + t] = x2;
            if (!isfinite(path)) bad = true;
            else pmax = (float)(path * 1.000001);
        }
        s.v[t] = v0;
        s.v[N + t] = v1;
        s.v[2 * N + t] = v2;
    }
    if (s.nb > 0) block_max_commit(&s.maxdisp[0], pmax, (float)s.disp_floor);
    if (bad) atomicOr(s.err, kErrNonFinite);
}

// Largest two of the union of two pairs (a1 >= a2, b1 >= b2).
__device__ __forceinline__ void top2_merge(float &a1, float &a2, float b1, float b2)
{
    a2 = fmaxf(fminf(a1, b1), fmaxf(a2, b2));
    a1 = fmaxf(a1, b1);
}

// nkicks = 1: opening half kick of the first inner step; 2: closing half kick of the
// previous inner step followed by the opening half kick of this one.  Each member keeps
// its largest displacement since the rebuild in dmax; the last drift of the outer step
// also leaves, per wavefront, the two largest of them (all members, beads only) for the
// skin check of the next rebuild.
__global__ void k_inner_kick_drift(Dev s, double h, int nkicks, double dt, int last)
{
    float dm = 0.0f;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (m < *s.n_members) {
        const int32_t t = s.member_slot[m];
        const int64_t N = s.N, C = s.cap_members;
        const double mi = s.minv[ptype(s, s.id[t])];
        double v0 = s.v[t], v1 = s.v[N + t], v2 = s.v[2 * N + t];
        const double a0 = s.fi[m], a1 = s.fi[C + m], a2 = s.fi[2 * C + m];
        for (int q = 0; q < nkicks; ++q) {
            v0 += h * a0 * mi;
            v1 += h * a1 * mi;
            v2 += h * a2 * mi;
        }
        double x0 = s.x[t], x1 = s.x[N + t], x2 = s.x[2 * N + t];
        drift_one(s, x0, x1, x2, v0, v1, v2, dt);
        s.x[t] = x0;
        s.x[N + t] = x1;
        s.x[2 * N + t] = x2;
        s.v[t] = v0;
        s.v[N + t] = v1;
        s.v[2 * N + t] = v2;
        const double e0 = min_image(s, 0, x0 - s.xref[m]);
        const double e1 = min_image(s, 1, x1 - s.xref[C + m]);
        const double e2 = min_image(s, 2, x2 - s.xref[2 * C + m]);
        const double disp = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
        if (!isfinite(disp)) {
            bad = true;
        } else {
            const float d = (float)(disp * 1.000001);  // rounded up
            dm = s.dmax[m];
            if (d > dm) {
                dm = d;
                s.dmax[m] = d;
            }
        }
    }
    if (last) {  // uniform over the grid
        float a1 = dm, a2 = 0.0f, b1 = m < s.nb ? dm : 0.0f, b2 = 0.0f;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const float c1 = __shfl_xor(a1, o, 64), c2 = __shfl_xor(a2, o, 64);
            const float e1 = __shfl_xor(b1, o, 64), e2 = __shfl_xor(b2, o, 64);
            top2_merge(a1, a2, c1, c2);
            top2_merge(b1, b2, e1, e2);
        }
        if ((threadIdx.x & 63) == 0) s.dpart[m >> 6] = make_float4(a1, a2, b1, b2);
    }
    if (bad) atomicOr(s.err, kErrNonFinite);
}

__global__ void k_inner_kick(Dev s, double h)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= *s.n_members) return;
    const int32_t t = s.member_slot[m];
    const int64_t N = s.N, C = s.cap_members;
    const double mi = s.minv[ptype(s, s.id[t])];
    s.v[t] += h * s.fi[m] * mi;
    s.v[N + t] += h * s.fi[C + m] * mi;
    s.v[2 * N + t] += h * s.fi[2 * C + m] * mi;
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

void open_kick_lazy_drift(const Dev &s, double h_out, int k, double dt_in, hipStream_t st)
{
    hipLaunchKernelGGL(k_open_lazy, dim3(nblocks(s.N, 256)), dim3(256), 0, st, s, h_out, k, dt_in);
}

void inner_kick_drift(const Dev &s, double h_in, int nkicks, double dt_in, bool last, hipStream_t st)
{
    if (s.cap_members > 0)
        hipLaunchKernelGGL(k_inner_kick_drift, dim3(nblocks(s.cap_members, 256)), dim3(256), 0, st, s, h_in, nkicks,
                           dt_in, last ? 1 : 0);
}

void inner_kick(const Dev &s, double h_in, hipStream_t st)
{
    if (s.cap_members > 0)
        hipLaunchKernelGGL(k_inner_kick, dim3(nblocks(s.cap_members, 256)), dim3(256), 0, st, s, h_in);
}

void outer_kick(const Dev &s, double h_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_outer_kick, dim3(nblocks(s.N, 256)), dim3(256), 0, st, s, h_out);
}

}  // namespace aimts
