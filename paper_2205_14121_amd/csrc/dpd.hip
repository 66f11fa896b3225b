// Outer force group: DPD conservative + dissipative + random pair forces (Sec. 3.2,
// Eq. 1) between fluid particles and between fluid and frozen wall particles, plus the
// body force on the fluid (F^E of Eq. 1).
//
// One thread per fluid slot gathers over the 27 cells around it.  Because a cell's
// fluid/wall slots come before its beads, the candidate range of a cell is
// [cell_start, cell_start + cell_nonbead): beads never enter this loop.  The periodic
// image of a neighbour cell is applied once per cell as a shift of the home position,
// so the candidate loop is three subtractions and a distance test.  Each accepted pair
// runs one Philox4x32-10 block keyed on (min id, max id, evaluation counter); the pair
// is evaluated from both ends (no atomics, deterministic, exactly antisymmetric).
//
// R = double: all arithmetic in float64.  R = float: the separation is formed in
// float64, rounded, and everything after that (including the Gaussian, from the same
// 32-bit words) is float32 with float32 accumulation.
#include "common.h"

namespace aimts {

namespace {

template <typename R>
__global__ __launch_bounds__(256) void k_dpd(Dev s, uint64_t count, double inv_sqrt_dt, R *f)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.N) return;
    const int64_t N = s.N;
    const uint32_t idi = s.id[i];
    R f0 = R(0), f1 = R(0), f2 = R(0);
    if (idi < (uint64_t)s.nf) {
        const double x0 = s.x[i], x1 = s.x[N + i], x2 = s.x[2 * N + i];
        const double v0 = s.v[i], v1 = s.v[N + i], v2 = s.v[2 * N + i];
        const int cx = cell_coord(s, 0, x0), cy = cell_coord(s, 1, x1), cz = cell_coord(s, 2, x2);
        const R a = (R)s.a, gam = (R)s.gamma, sig = (R)s.sigma, inv_rc = (R)s.inv_rc, rc2 = (R)s.rc2;
        const R isdt = (R)inv_sqrt_dt;
        for (int dy = -1; dy <= 1; ++dy) {
            int iy = cy + dy;
            double sy = 0.0;
            if (iy < 0 || iy >= s.nc[1]) {
                if (!s.per[1]) continue;
                sy = iy < 0 ? s.L[1] : -s.L[1];   // image of the neighbour cell lies at -sy
                iy = iy < 0 ? iy + s.nc[1] : iy - s.nc[1];
            }
            const double hy = x1 + sy;
            for (int dx = -1; dx <= 1; ++dx) {
                int ix = cx + dx;
                double sx = 0.0;
                if (ix < 0 || ix >= s.nc[0]) {
                    if (!s.per[0]) continue;
                    sx = ix < 0 ? s.L[0] : -s.L[0];
                    ix = ix < 0 ? ix + s.nc[0] : ix - s.nc[0];
                }
                const double hx = x0 + sx;
                for (int dz = -1; dz <= 1; ++dz) {
                    int iz = cz + dz;
                    double sz = 0.0;
                    if (iz < 0 || iz >= s.nc[2]) {
                        if (!s.per[2]) continue;
                        sz = iz < 0 ? s.L[2] : -s.L[2];
                        iz = iz < 0 ? iz + s.nc[2] : iz - s.nc[2];
                    }
                    const double hz = x2 + sz;
                    const int64_t c = cell_index(s, ix, iy, iz);
                    const int32_t beg = s.cell_start[c];
                    const int32_t end = beg + s.cell_nonbead[c];
                    for (int32_t j = beg; j < end; ++j) {
                        const R d0 = (R)(hx - s.x[j]);
                        const R d1 = (R)(hy - s.x[N + j]);
                        const R d2 = (R)(hz - s.x[2 * N + j]);
                        const R r2 = d0 * d0 + d1 * d1 + d2 * d2;
                        if (r2 < rc2 && j != i && r2 > R(0)) {
                            const R rinv = R(1) / sqrt(r2);
                            const R r = r2 * rinv;
                            const R w = R(1) - r * inv_rc;
                            const R ev = (d0 * (R)(v0 - s.v[j]) + d1 * (R)(v1 - s.v[N + j]) +
                                          d2 * (R)(v2 - s.v[2 * N + j])) * rinv;
                            uint32_t w0, w1;
                            pair_words(idi, s.id[j], count, s.key0, s.key1, w0, w1);
                            R z;
                            if constexpr (sizeof(R) == 8) z = gauss64(w0, w1);
                            else z = gauss32(w0, w1);
                            const R fs = (a * w - gam * w * w * ev + sig * w * z * isdt) * rinv;
                            f0 += fs * d0;
                            f1 += fs * d1;
                            f2 += fs * d2;
                        }
                    }
                }
            }
        }
        f0 += (R)s.g[0];
        f1 += (R)s.g[1];
        f2 += (R)s.g[2];
    }
    f[i] = f0;
    f[N + i] = f1;
    f[2 * N + i] = f2;
}

}  // namespace

void outer_forces(const Dev &s, uint64_t count, double dt_outer, hipStream_t st)
{
    const int bs = 256;
    const double isdt = 1.0 / sqrt(dt_outer);
    if (s.fp32)
        hipLaunchKernelGGL(k_dpd<float>, dim3(nblocks(s.N, bs)), dim3(bs), 0, st, s, count, isdt, (float *)s.fo);
    else
        hipLaunchKernelGGL(k_dpd<double>, dim3(nblocks(s.N, bs)), dim3(bs), 0, st, s, count, isdt, (double *)s.fo);
}

}  // namespace aimts
