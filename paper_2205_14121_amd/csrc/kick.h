// Per-slot pieces of the outer-level kicks (Sec. 3.3, MSM pseudocode Table 1: the half
// kicks at entry and exit of the outer level), shared by the kernels that apply them, so
// that a kick gives the same bits whichever kernel applies it.
#pragma once

#include "common.h"

namespace aimts {

__device__ __forceinline__ double outer_force(const Dev &s, int c, int64_t t)
{
    return s.fp32 ? (double)((const float *)s.fo)[c * s.N + t] : ((const double *)s.fo)[c * s.N + t];
}

// v + h f / m with one fixed rounding sequence: h f rounded, then one fused multiply-add.
__device__ __forceinline__ double kick_add(double v, double h, double f, double mi) { return __fma_rn(h * f, mi, v); }

// Outer half kick of slot t (of mass inverse mi) applied to (v0, v1, v2).
__device__ __forceinline__ void outer_half_kick(const Dev &s, int64_t t, double h, double mi, double &v0, double &v1,
                                                double &v2)
{
    v0 = kick_add(v0, h, outer_force(s, 0, t), mi);
    v1 = kick_add(v1, h, outer_force(s, 1, t), mi);
    v2 = kick_add(v2, h, outer_force(s, 2, t), mi);
}

// Largest of a non-negative value over the wavefront (every lane must call it).
__device__ __forceinline__ float wave_max_f(float v)
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
    v = wave_max_f(v);
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

// What the opening of an outer step does to one mobile slot t of type ty, from its
// velocity (v0, v1, v2) before the opening outer half kick h_out: the kick, then for a
// fluid particle that is no inner member all k inner drifts in registers (its velocity
// is constant through the inner loop but at a wall bounce), written back in place; for a
// member the opening inner half kick(s) of the first inner step (ls: of every level in
// three-level mode) and its drift, written to (xw, vw) (which may be the particle arrays
// themselves: each slot is read and written by its own thread only), with its largest
// displacement since the rebuild kept in dmax.  pmax collects a non-member's path bound
// k dt |v| (a bounce only turns it round); bad flags a non-finite result.
__device__ __forceinline__ void open_slot(const Dev &s, int64_t t, int ty, double v0, double v1, double v2,
                                          double h_out, int k, double dt, const LevelStep &ls, double *xw, double *vw,
                                          float &pmax, bool &bad)
{
    const int64_t N = s.N;
    const double mi = s.minv[ty];
    outer_half_kick(s, t, h_out, mi, v0, v1, v2);
    double x0 = s.x[t], x1 = s.x[N + t], x2 = s.x[2 * N + t];
    const int32_t m = s.mos[t];
    if (m < 0) {
        const double path = (double)k * dt * sqrt(v0 * v0 + v1 * v1 + v2 * v2);
        for (int q = 0; q < k; ++q) drift_one(s, x0, x1, x2, v0, v1, v2, dt);
        s.x[t] = x0;
        s.x[N + t] = x1;
        s.x[2 * N + t] = x2;
        s.v[t] = v0;
        s.v[N + t] = v1;
        s.v[2 * N + t] = v2;
        if (!isfinite(path)) bad = true;
        else pmax = fmaxf(pmax, (float)(path * 1.000001));
        return;
    }
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

// The opening of an outer step: the arguments of open_slot, and where wall particles
// are copied (xa, va: the members' second state buffer, which holds them too).
struct OuterOpen {
    double h_out;
    int k;
    double dt;
    double *xa, *va, *xw, *vw;
    LevelStep ls;
};

}  // namespace aimts
