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
#include "kick.h"

namespace aimts {

namespace {

// Opening outer half kick of every mobile particle, the lazy drifts of the non-members
// and the members' first inner kick and drift (open_slot); wall particles are copied
// into (xa, va), the members' second state buffer.
__global__ void k_open_lazy(Dev s, OuterOpen op)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float pmax = 0.0f;  // largest k-drift path of a non-member
    bool bad = false;
    const int ty = t < s.N ? ptype(s, s.id[t]) : -1;
    const int64_t N = s.N;
    if (ty == 1) {  // frozen walls are never integrated; the members' second buffer holds them too
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            op.xa[c * N + t] = s.x[c * N + t];
            op.va[c * N + t] = s.v[c * N + t];
        }
    } else if (ty >= 0) {
        open_slot(s, t, ty, s.v[t], s.v[N + t], s.v[2 * N + t], op.h_out, op.k, op.dt, op.ls, op.xw, op.vw, pmax,
                  bad);
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
    const int64_t N = s.N;
    double v0 = s.v[t], v1 = s.v[N + t], v2 = s.v[2 * N + t];
    outer_half_kick(s, t, h, s.minv[ty], v0, v1, v2);
    s.v[t] = v0;
    s.v[N + t] = v1;
    s.v[2 * N + t] = v2;
    if (!isfinite(v0 + v1 + v2)) atomicOr(s.err, kErrNonFinite);
}

}  // namespace

void open_kick_lazy_drift(const Dev &s, double h_out, int k, double dt_in, double *xa, double *va,
                          const LevelStep &ls, double *xw, double *vw, hipStream_t st)
{
    const OuterOpen op{h_out, k, dt_in, xa, va, xw, vw, ls};
    hipLaunchKernelGGL(k_open_lazy, dim3(nblocks(s.N, 256)), dim3(256), 0, st, s, op);
}

void outer_kick(const Dev &s, double h_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_outer_kick, dim3(nblocks(s.N, 256)), dim3(256), 0, st, s, h_out);
}

}  // namespace aimts
