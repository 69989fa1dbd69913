// k_mg.hip -- multigrid solver for the scalar potential on gfx950.
//
// The Poisson equation of Sec. 3.2, Delta_h mu = f (7-point stencil, plain
// wrap on periodic axes, Neumann reflection at open faces), is solved by
// V-cycles.  The smoother is the paper's pseudo-time relaxation: one
// Crank-Nicolson pseudo-step of d mu / d tau = Delta mu - f solved by a
// single Jacobi iteration is a damped Jacobi sweep,
//     mu <- mu + omega (f - A mu) / D,
// with omega = 2 h_tau S / (1 + h_tau S) set by the pseudo time step.
//
// Level operators are the finite-volume form of the stencil,
//     (A mu)_m = sum_a ap_a (mu_{m+a} - mu_m) + am_a (mu_{m-a} - mu_m),
// which is exactly Delta_h on the finest level (the boundary coefficient of
// an open face is twice the interior one, the Neumann ghost).  Periodic axes
// are coarsened by two; open axes keep nodes {0, 2, 4, ...} and the last node,
// so any node count coarsens, at the price of a non-uniform coarse spacing.
// Transfers are linear interpolation and its volume-weighted transpose.
//
// Kernels map one thread to one (x, y) column of a 64 x 4 tile and march
// through a chunk of z planes, keeping the z neighbours in registers.
#include "kernels.h"
#include "stencil.h"

namespace tdgl {

struct MGCols {
    int lv, x, y, k0, k1;
    bool valid;
};

__device__ __forceinline__ MGCols mg_map(const MGLevel &L, int lb) {
    MGCols c;
    int t = lb;
    const int tx = t % L.tiles_x;
    t /= L.tiles_x;
    const int ty = t % L.tiles_y;
    const int tz = t / L.tiles_y;
    c.x = tx * MTX + (threadIdx.x & (MTX - 1));
    c.y = ty * MTY + (threadIdx.x / MTX);
    c.k0 = tz * L.chunk;
    c.k1 = min(c.k0 + L.chunk, L.nz);
    c.valid = (c.x < L.nx) && (c.y < L.ny);
    return c;
}

__device__ __forceinline__ int wrapi(int i, int n, int per) {
    if (i < 0) return per ? i + n : 0;
    if (i >= n) return per ? i - n : n - 1;
    return i;
}

// Poisson residual rows: the solve of this step ended at cycle c (or an
// earlier one) when row c is below max(mu_tol, mu_rtol * row 0).  Row c is
// written by the finest residual of cycle c.  Read by whole wavefronts
// (uniform control flow, full waves).
__device__ __forceinline__ float mg_threshold(const Inst &I) {
    return fmaxf(I.mu_tol, I.mu_rtol * row_max_wave(I.mures, I.rstride, 0));
}
__device__ __forceinline__ bool mg_done(const Inst &I, int c) {
    if (c >= I.mu_max_cycles) return true;
    return row_max_wave(I.mures, I.rstride, c) < mg_threshold(I);
}

// Shared column context: coefficient values of the column and its x/y
// neighbour indices.
struct ColCoef {
    float apx, amx, apy, amy;
    int xm, xp, ym, yp;
};

__device__ __forceinline__ ColCoef col_coef(const MGLevel &L, int x, int y) {
    ColCoef c;
    c.apx = L.ap[0][x];
    c.amx = L.am[0][x];
    c.apy = L.ap[1][y];
    c.amy = L.am[1][y];
    c.xm = wrapi(x - 1, L.nx, L.per[0]);
    c.xp = wrapi(x + 1, L.nx, L.per[0]);
    c.ym = wrapi(y - 1, L.ny, L.per[1]);
    c.yp = wrapi(y + 1, L.ny, L.per[1]);
    return c;
}

// Damped Jacobi sweep dst = src + omega (rhs - A src) / D on level lv.
// Level 0 subtracts the weighted mean of f from its right side (projection
// onto the range of the singular operator).
__global__ __launch_bounds__(256) void k_mg_smooth(const Inst *__restrict__ insts,
                                                   const int *__restrict__ prefix, int ninst,
                                                   int lv, int isrc, int idst, int cyc,
                                                   float omega) {
    const int ii = find_inst(prefix, ninst, blockIdx.x);
    const Inst &I = insts[ii];
    if (mg_done(I, cyc)) return;
    const MGLevel &L = I.lev[lv];
    const MGCols q = mg_map(L, blockIdx.x - prefix[ii]);
    if (!q.valid) return;
    const float *__restrict__ src = L.mu[isrc];
    float *__restrict__ dst = L.mu[idst];
    const float fm = (lv == 0) ? (float)I.st->f_mean : 0.f;
    const ColCoef c = col_coef(L, q.x, q.y);
    const long nxy = (long)L.nx * L.ny;
    const long col = (long)q.y * L.nx + q.x;
    const int zper = L.per[2];
    const int km = wrapi(q.k0 - 1, L.nz, zper);
    float mprev = src[km * nxy + col];
    float mc = src[q.k0 * nxy + col];
    for (int k = q.k0; k < q.k1; ++k) {
        const int kp = wrapi(k + 1, L.nz, zper);
        const float mnext = src[kp * nxy + col];
        const long pb = k * nxy;
        const float apz = L.ap[2][k], amz = L.am[2][k];
        const float Amu = c.apx * (src[pb + q.y * (long)L.nx + c.xp] - mc) +
                          c.amx * (src[pb + q.y * (long)L.nx + c.xm] - mc) +
                          c.apy * (src[pb + c.yp * (long)L.nx + q.x] - mc) +
                          c.amy * (src[pb + c.ym * (long)L.nx + q.x] - mc) +
                          apz * (mnext - mc) + amz * (mprev - mc);
        const float D = -(c.apx + c.amx + c.apy + c.amy + apz + amz);
        const float rhs = L.rhs[pb + col] - fm;
        dst[pb + col] = (D != 0.f) ? mc + omega * (rhs - Amu) / D : mc;
        mprev = mc;
        mc = mnext;
    }
}

// Residual r = rhs - A mu evaluated in double precision from the stored
// single-precision iterate.  On level 0 it also reduces max |r| into the
// cycle's convergence word and, when the previous cycle had already
// converged, does nothing.
__global__ __launch_bounds__(256) void k_mg_residual(const Inst *__restrict__ insts,
                                                     const int *__restrict__ prefix, int ninst,
                                                     int lv, int isrc, int cyc) {
    __shared__ float red[4];
    const int ii = find_inst(prefix, ninst, blockIdx.x);
    const Inst &I = insts[ii];
    if (I.fft) return;  // spectral instances (level 0 is launched over all driven ones)
    if (lv == 0) {
        if (cyc > 0 && mg_done(I, cyc - 1)) return;
    } else if (mg_done(I, cyc)) {
        return;
    }
    const MGLevel &L = I.lev[lv];
    const MGCols q = mg_map(L, blockIdx.x - prefix[ii]);
    float rmax = 0.f;
    if (q.valid) {
        const float *__restrict__ src = L.mu[isrc];
        const double fm = (lv == 0) ? I.st->f_mean : 0.0;
        const ColCoef c = col_coef(L, q.x, q.y);
        const long nxy = (long)L.nx * L.ny;
        const long col = (long)q.y * L.nx + q.x;
        const int zper = L.per[2];
        double mprev = src[wrapi(q.k0 - 1, L.nz, zper) * nxy + col];
        double mc = src[q.k0 * nxy + col];
        for (int k = q.k0; k < q.k1; ++k) {
            const double mnext = src[wrapi(k + 1, L.nz, zper) * nxy + col];
            const long pb = k * nxy;
            const double Amu =
                (double)c.apx * ((double)src[pb + q.y * (long)L.nx + c.xp] - mc) +
                (double)c.amx * ((double)src[pb + q.y * (long)L.nx + c.xm] - mc) +
                (double)c.apy * ((double)src[pb + c.yp * (long)L.nx + q.x] - mc) +
                (double)c.amy * ((double)src[pb + c.ym * (long)L.nx + q.x] - mc) +
                (double)L.ap[2][k] * (mnext - mc) + (double)L.am[2][k] * (mprev - mc);
            const double r = ((double)L.rhs[pb + col] - fm) - Amu;
            L.r[pb + col] = (float)r;
            const float ra = (float)fabs(r);
            rmax = (ra > rmax || ra != ra) ? ra : rmax;
            mprev = mc;
            mc = mnext;
        }
    }
    if (lv == 0) wg_max_to<256>(row_slot(I.mures, I.rstride, cyc, blockIdx.x), rmax, red);
}

// Restriction of the residual of level lv to the right side of level lv+1
// (volume-weighted transpose of linear interpolation, up to three fine
// indices per axis), followed by the first smoothing sweep of the coarse
// correction from a zero initial guess: e = omega rhs / D.
__global__ __launch_bounds__(256) void k_mg_restrict(const Inst *__restrict__ insts,
                                                     const int *__restrict__ prefix, int ninst,
                                                     int lv, int cyc, float omega) {
    const int ii = find_inst(prefix, ninst, blockIdx.x);
    const Inst &I = insts[ii];
    if (mg_done(I, cyc)) return;
    const MGLevel &F = I.lev[lv];
    const MGLevel &C = I.lev[lv + 1];
    const MGCols q = mg_map(C, blockIdx.x - prefix[ii]);
    if (!q.valid) return;
    int fx[3], fy[3];
    float wx[3], wy[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        fx[a] = F.rk[0][3 * q.x + a];
        wx[a] = F.rw[0][3 * q.x + a];
        fy[a] = F.rk[1][3 * q.y + a];
        wy[a] = F.rw[1][3 * q.y + a];
    }
    const float Dxy = C.ap[0][q.x] + C.am[0][q.x] + C.ap[1][q.y] + C.am[1][q.y];
    const long fnxy = (long)F.nx * F.ny;
    const long cnxy = (long)C.nx * C.ny;
    for (int K = q.k0; K < q.k1; ++K) {
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float wz = F.rw[2][3 * K + c];
            const long pb = (long)F.rk[2][3 * K + c] * fnxy;
#pragma unroll
            for (int b2 = 0; b2 < 3; ++b2) {
                const long rb = pb + (long)fy[b2] * F.nx;
                const float wzy = wz * wy[b2];
#pragma unroll
                for (int a = 0; a < 3; ++a) s += wzy * wx[a] * F.r[rb + fx[a]];
            }
        }
        const long m = K * cnxy + (long)q.y * C.nx + q.x;
        C.rhs[m] = s;
        const float D = -(Dxy + C.ap[2][K] + C.am[2][K]);
        C.mu[0][m] = (D != 0.f) ? omega * s / D : 0.f;
    }
}

// Coarse-to-fine correction mu_f += P e_c (linear interpolation per axis).
__global__ __launch_bounds__(256) void k_mg_prolong(const Inst *__restrict__ insts,
                                                    const int *__restrict__ prefix, int ninst,
                                                    int lv, int ifine, int cyc) {
    const int ii = find_inst(prefix, ninst, blockIdx.x);
    const Inst &I = insts[ii];
    if (mg_done(I, cyc)) return;
    // the coarsest level keeps its result in buffer 0, other levels in 1
    const int icoarse = (lv + 1 == I.nlev - 1) ? 0 : 1;
    const MGLevel &F = I.lev[lv];
    const MGLevel &C = I.lev[lv + 1];
    const MGCols q = mg_map(F, blockIdx.x - prefix[ii]);
    if (!q.valid) return;
    const int kx0 = F.pk[0][2 * q.x], kx1 = F.pk[0][2 * q.x + 1];
    const float wx0 = F.pw[0][2 * q.x], wx1 = F.pw[0][2 * q.x + 1];
    const int ky0 = F.pk[1][2 * q.y], ky1 = F.pk[1][2 * q.y + 1];
    const float wy0 = F.pw[1][2 * q.y], wy1 = F.pw[1][2 * q.y + 1];
    const float *__restrict__ ec = C.mu[icoarse];
    float *__restrict__ mf = F.mu[ifine];
    const long cnxy = (long)C.nx * C.ny, fnxy = (long)F.nx * F.ny;
    for (int k = q.k0; k < q.k1; ++k) {
        const int kz0 = F.pk[2][2 * k], kz1 = F.pk[2][2 * k + 1];
        const float wz0 = F.pw[2][2 * k], wz1 = F.pw[2][2 * k + 1];
        const long b0 = kz0 * cnxy, b1 = kz1 * cnxy;
        const float e =
            wz0 * (wy0 * (wx0 * ec[b0 + (long)ky0 * C.nx + kx0] + wx1 * ec[b0 + (long)ky0 * C.nx + kx1]) +
                   wy1 * (wx0 * ec[b0 + (long)ky1 * C.nx + kx0] + wx1 * ec[b0 + (long)ky1 * C.nx + kx1])) +
            wz1 * (wy0 * (wx0 * ec[b1 + (long)ky0 * C.nx + kx0] + wx1 * ec[b1 + (long)ky0 * C.nx + kx1]) +
                   wy1 * (wx0 * ec[b1 + (long)ky1 * C.nx + kx0] + wx1 * ec[b1 + (long)ky1 * C.nx + kx1]));
        mf[k * fnxy + (long)q.y * F.nx + q.x] += e;
    }
}

// Coarsest level: one work-group per instance iterates Jacobi sweeps in
// double precision (in the level's two buffers) until the residual falls
// below 1e-6 of the right side or 4000 sweeps, after projecting the right
// side onto the range (zero volume-weighted mean) and shifting the result to
// zero mean.  Result in mu[0].  The level may be the finest one (tiny grids):
// then its right side is f minus its weighted mean and the iterate starts
// from the stored mu.
__global__ __launch_bounds__(CO_THREADS) void k_mg_coarsest(const Inst *__restrict__ insts,
                                                            int ninst, int cyc) {
    __shared__ double red[CO_THREADS / 64];
    __shared__ double sh_mean, sh_rmax;
    const Inst &I = insts[blockIdx.x];
    if (!I.driven || I.fft || mg_done(I, cyc)) return;
    const int lv = I.nlev - 1;
    const MGLevel &L = I.lev[lv];
    const int N = L.N;
    const double fm = (lv == 0) ? I.st->f_mean : 0.0;
    // volume-weighted mean of the right side
    double s = 0.0;
    for (int m = threadIdx.x; m < N; m += CO_THREADS) {
        const int x = m % L.nx, y = (m / L.nx) % L.ny, z = m / (L.nx * L.ny);
        const double V = (double)L.vol[0][x] * L.vol[1][y] * L.vol[2][z];
        s += V * ((double)L.rhs[m] - fm);
    }
    s = wg_sum<CO_THREADS>(s, red);
    if (threadIdx.x == 0) sh_mean = s / L.vsum;
    __syncthreads();
    const double rmean = sh_mean;
    double rnorm = 0.0;
    for (int m = threadIdx.x; m < N; m += CO_THREADS)
        rnorm = fmax(rnorm, fabs((double)L.rhs[m] - fm - rmean));
    // max over the group
    for (int o = 32; o > 0; o >>= 1) rnorm = fmax(rnorm, __shfl_xor(rnorm, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rnorm;
    __syncthreads();
    if (threadIdx.x == 0) {
        double mx = 0.0;
        for (int i = 0; i < CO_THREADS / 64; ++i) mx = fmax(mx, red[i]);
        sh_rmax = mx;
    }
    __syncthreads();
    const double thr = 1e-6 * sh_rmax;
    float *a = L.mu[0], *bq = L.mu[1];
    if (lv != 0)
        for (int m = threadIdx.x; m < N; m += CO_THREADS) a[m] = 0.f;
    __syncthreads();
    for (int it = 0; it < 4000; ++it) {
        double rloc = 0.0;
        for (int m = threadIdx.x; m < N; m += CO_THREADS) {
            const int x = m % L.nx, y = (m / L.nx) % L.ny, z = m / (L.nx * L.ny);
            const int xm = wrapi(x - 1, L.nx, L.per[0]), xp = wrapi(x + 1, L.nx, L.per[0]);
            const int ym = wrapi(y - 1, L.ny, L.per[1]), yp = wrapi(y + 1, L.ny, L.per[1]);
            const int zm = wrapi(z - 1, L.nz, L.per[2]), zp = wrapi(z + 1, L.nz, L.per[2]);
            const double mc = a[m];
            const long nx = L.nx, nxy = (long)L.nx * L.ny;
            const double Amu = (double)L.ap[0][x] * (a[z * nxy + y * nx + xp] - mc) +
                               (double)L.am[0][x] * (a[z * nxy + y * nx + xm] - mc) +
                               (double)L.ap[1][y] * (a[z * nxy + yp * nx + x] - mc) +
                               (double)L.am[1][y] * (a[z * nxy + ym * nx + x] - mc) +
                               (double)L.ap[2][z] * (a[zp * nxy + y * nx + x] - mc) +
                               (double)L.am[2][z] * (a[zm * nxy + y * nx + x] - mc);
            const double D = -((double)L.ap[0][x] + L.am[0][x] + L.ap[1][y] + L.am[1][y] +
                               L.ap[2][z] + L.am[2][z]);
            const double r = ((double)L.rhs[m] - fm - rmean) - Amu;
            rloc = fmax(rloc, fabs(r));
            bq[m] = (D != 0.0) ? (float)(mc + 0.9 * r / D) : (float)mc;
        }
        for (int o = 32; o > 0; o >>= 1) rloc = fmax(rloc, __shfl_xor(rloc, o, 64));
        __syncthreads();
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rloc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double mx = 0.0;
            for (int i = 0; i < CO_THREADS / 64; ++i) mx = fmax(mx, red[i]);
            sh_rmax = mx;
        }
        __syncthreads();
        // swap roles
        float *t = a;
        a = bq;
        bq = t;
        if (sh_rmax <= thr) break;
        __syncthreads();
    }
    // shift to zero weighted mean and leave the result in mu[0]
    double sm = 0.0;
    for (int m = threadIdx.x; m < N; m += CO_THREADS) {
        const int x = m % L.nx, y = (m / L.nx) % L.ny, z = m / (L.nx * L.ny);
        sm += (double)L.vol[0][x] * L.vol[1][y] * L.vol[2][z] * a[m];
    }
    sm = wg_sum<CO_THREADS>(sm, red);
    if (threadIdx.x == 0) sh_mean = sm / L.vsum;
    __syncthreads();
    const float mmean = (float)sh_mean;
    for (int m = threadIdx.x; m < N; m += CO_THREADS) {
        const float v = a[m] - mmean;
        L.mu[0][m] = v;
    }
}

// End of a Poisson solve: number of cycles and final residual; clears the
// cycle words.  One thread per instance.
__global__ __launch_bounds__(FIN_THREADS) void k_mg_finalize(const Inst *__restrict__ insts, int ninst,
                                                               int count_step) {
    // one work-group per instance: the first wavefront scans the rows, then
    // all threads clear them
    const int ii = blockIdx.x;
    if (ii >= ninst) return;
    const Inst &I = insts[ii];
    if (!I.driven || I.fft) return;
    DevState *st = I.st;
    if (threadIdx.x < 64) {
        int cycles = I.mu_max_cycles, capped = 1;
        const float thr = mg_threshold(I);
        float last = row_max_wave(I.mures, I.rstride, I.mu_max_cycles - 1);
        for (int c = 0; c < I.mu_max_cycles; ++c) {
            const float r = row_max_wave(I.mures, I.rstride, c);
            if (r < thr) { cycles = c; capped = 0; last = r; break; }
        }
        if (threadIdx.x == 0) {
            st->mu_cycles = cycles;
            st->mu_capped = capped;
            st->mu_last_res = last;
            if (count_step) {
                st->acc_mu_cycles += cycles;
                st->acc_mu_capped += capped;
            }
        }
    }
    __syncthreads();
    const int words = I.mu_max_cycles * NSLOT;
    for (int w = threadIdx.x; w < words; w += FIN_THREADS) I.mures[(size_t)w * I.rstride] = 0u;
}

// Partial sums of V mu (which = 0) or V f (which = 1) on level 0 for the
// weighted mean.
__global__ __launch_bounds__(256) void k_mu_mean_partial(const Inst *__restrict__ insts,
                                                         const int *__restrict__ prefix, int ninst,
                                                         int which) {
    __shared__ double red[4];
    const int ii = find_inst(prefix, ninst, blockIdx.x);
    const Inst &I = insts[ii];
    const MGLevel &L = I.lev[0];
    const int lb = blockIdx.x - prefix[ii];
    const MGCols q = mg_map(L, lb);
    double acc = 0.0;
    if (q.valid) {
        const double vxy = (double)L.vol[0][q.x] * L.vol[1][q.y];
        const long nxy = (long)L.nx * L.ny, col = (long)q.y * L.nx + q.x;
        const gf1 *src = (const gf1 *)(which ? L.rhs : L.mu[0]);
        const gf1 *volz = (const gf1 *)L.vol[2];
        // eight planes' loads in flight before they are summed in plane order
        constexpr int KB = 8;
        int k = q.k0;
        for (; k + KB <= q.k1; k += KB) {
            float v[KB], wv[KB];
#pragma unroll
            for (int c = 0; c < KB; ++c) {
                v[c] = src[(k + c) * nxy + col];
                wv[c] = volz[k + c];
            }
#pragma unroll
            for (int c = 0; c < KB; ++c) acc += vxy * wv[c] * (double)v[c];
        }
        for (; k < q.k1; ++k) acc += vxy * volz[k] * (double)src[k * nxy + col];
    }
    const double s = wg_sum<256>(acc, red);
    if (threadIdx.x == 0) I.part[lb] = s;
}

}  // namespace tdgl
