// k_voronoi.hip -- tessellation patterns of the pattern generator (Sec. 3.4):
// every node takes the eps value of its nearest seed (a polycrystal of
// crystallites with their own critical temperature, Fig. 2c), under the
// Euclidean, absolute (city-block) or maximum distance.
#include "kernels.h"

namespace tdgl {

// Seeds staged per work-group through LDS in chunks of this many.
constexpr int kVorChunk = 512;

// Per-axis separation of node coordinate x = i h from seed coordinate c:
// |x - c| on an open axis; on a periodic axis of length L the smallest of
// |d|, |d - L|, |d + L| with d = x - c (the nearest image for seeds in the
// box).  Double precision, no contraction.
__device__ __forceinline__ double vor_sep(double x, double c, double L, bool per) {
    const double d = x - c;
    double a = fabs(d);
    if (per) a = fmin(a, fmin(fabs(d - L), fabs(d + L)));
    return a;
}

// One thread per node; seeds are scanned in index order and a strictly
// smaller distance replaces the current one, so equal distances go to the
// lowest seed index.  metric 0: (dx^2 + dy^2) + dz^2, 1: (|dx| + |dy|) + |dz|,
// 2: max(max(|dx|, |dy|), |dz|); an axis not in `axes` (bit a for axis a)
// contributes 0.  A seed with a non-finite coordinate is skipped; a node
// with no finite distance keeps its eps.
__global__ __launch_bounds__(256) void k_voronoi(const Inst *__restrict__ insts, int inst,
                                                 const double *__restrict__ seeds,
                                                 const float *__restrict__ values, int ns, int metric,
                                                 int axes) {
#pragma clang fp contract(off)
    __shared__ double sc[3][kVorChunk];
    __shared__ unsigned char ok[kVorChunk];
    const Inst &I = insts[inst];
    const long m = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const bool live = m < I.N;
    const long mm = live ? m : 0;
    const int i = (int)(mm % I.nx);
    const int j = (int)((mm / I.nx) % I.ny);
    const int k = (int)(mm / ((long)I.nx * I.ny));
    const double x = (double)i * I.hx, y = (double)j * I.hy, z = (double)k * I.hz;
    const double Lx = (double)I.nx * I.hx, Ly = (double)I.ny * I.hy, Lz = (double)I.nz * I.hz;
    const bool px = I.per[0], py = I.per[1], pz = I.per[2];
    const bool ux = axes & 1, uy = axes & 2, uz = axes & 4;
    double best = INFINITY;
    int arg = -1;
    for (int s0 = 0; s0 < ns; s0 += kVorChunk) {
        const int cnt = min(kVorChunk, ns - s0);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
            sc[0][t] = seeds[3 * (long)(s0 + t)];
            sc[1][t] = seeds[3 * (long)(s0 + t) + 1];
            sc[2][t] = seeds[3 * (long)(s0 + t) + 2];
            ok[t] = isfinite(sc[0][t]) && isfinite(sc[1][t]) && isfinite(sc[2][t]);
        }
        __syncthreads();
        for (int t = 0; t < cnt; ++t) {
            if (!ok[t]) continue;
            const double dx = ux ? vor_sep(x, sc[0][t], Lx, px) : 0.0;
            const double dy = uy ? vor_sep(y, sc[1][t], Ly, py) : 0.0;
            const double dz = uz ? vor_sep(z, sc[2][t], Lz, pz) : 0.0;
            double d;
            if (metric == 0)
                d = (dx * dx + dy * dy) + dz * dz;
            else if (metric == 1)
                d = (dx + dy) + dz;
            else
                d = fmax(fmax(dx, dy), dz);
            if (d < best) {
                best = d;
                arg = s0 + t;
            }
        }
    }
    if (live && arg >= 0) I.eps[m] = values[arg];
}

}  // namespace tdgl
