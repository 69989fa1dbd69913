// k_gl.hip -- stencil kernels of the implicit TDGL step on gfx950.
//
// All four stencil passes over psi share one 2.5D tiling: a work-group owns a
// 64 x 16 tile of (x, y) columns and marches through a chunk of z planes.
// Plane k of the tile plus a one-cell halo is staged in LDS (double
// buffered, one barrier per plane) for the x and y neighbours; the z
// neighbours stay in registers as the march advances.  Every HBM array is
// read once per pass in coalesced 512-byte rows (one float2 row per
// wavefront); halo rows come from L2.
//
//   MODE_FIRST  assemble b, M_mm of Eq. GL_linearized / Eq. b and perform
//               the first Jacobi iteration (Eq. final) from psi^(0) = psi^-,
//               writing b/M_mm, (ht/2)/M_mm and psi^(1);
//   MODE_SWEEP  one Jacobi iteration psi^(l+1) = b/M + (ht/2)/M * NS(psi^(l));
//   MODE_RHS    right side of the Poisson equation (Sec. 3.2);
//   MODE_ENERGY free-energy density summed in FP64.
// FIRST and SWEEP also reduce max_m |r_m|^2 of their input iterate
// (Eq. convergence) through r = M_mm (psi^(l+1) - psi^(l)).
#include "kernels.h"

namespace tdgl {

// Value of psi at (gx, gy) of plane k as the 7-point stencil sees it, for
// gx in [-1, nx] and gy in [-1, ny]: interior nodes are loaded, one-cell
// ghosts follow the boundary rules of Sec. 3.3 -- plain wrap on a periodic
// x axis, the quasi-periodic phase jump psi_{i,-1,k} = P_{i,k} psi_{i,ny-1,k}
// on a periodic y axis, and the Neumann ghost (U^* psi_{-1} = U psi_1) on an
// open face.  Anything else (corners, beyond a ragged tile) is zero.
__device__ __forceinline__ float2 psi_at(const Inst &I, const float2 *__restrict__ src,
                                         int gx, int gy, int k) {
    const int nx = I.nx, ny = I.ny;
    const long plane = (long)k * nx * ny;
    const bool xin = (unsigned)gx < (unsigned)nx, yin = (unsigned)gy < (unsigned)ny;
    if (xin && yin) return src[plane + (long)gy * nx + gx];
    if (xin) {
        if (gy == -1) {
            if (I.per[1]) return cmul(I.P[(long)k * nx + gx], src[plane + (long)(ny - 1) * nx + gx]);
            return ny >= 2 ? src[plane + (long)nx + gx] : make_float2(0.f, 0.f);
        }
        if (gy == ny) {
            if (I.per[1]) return cmulc(I.P[(long)k * nx + gx], src[plane + gx]);
            return ny >= 2 ? src[plane + (long)(ny - 2) * nx + gx] : make_float2(0.f, 0.f);
        }
        return make_float2(0.f, 0.f);
    }
    if (yin) {
        const long row = plane + (long)gy * nx;
        if (gx == -1) {
            if (I.per[0]) return src[row + nx - 1];
            if (nx < 2) return make_float2(0.f, 0.f);
            float2 u = I.ux[gy];
            return cmul(cmul(u, u), src[row + 1]);
        }
        if (gx == nx) {
            if (I.per[0]) return src[row];
            if (nx < 2) return make_float2(0.f, 0.f);
            float2 u = I.ux[gy];
            return cmulc(cmul(u, u), src[row + nx - 2]);
        }
    }
    return make_float2(0.f, 0.f);
}

// z neighbour plane index of plane p in direction d (+1/-1), or -1 if none.
__device__ __forceinline__ int zplane(const Inst &I, int p, int d) {
    int q = p + d;
    if (q >= 0 && q < I.nz) return q;
    if (!I.per[2]) return -1;
    return q < 0 ? I.nz - 1 : 0;
}

// Own cell value of a thread for plane p (p may be -1: none -> 0).
__device__ __forceinline__ float2 own_at(const Inst &I, const float2 *__restrict__ src, int x,
                                         int y, int p) {
    if (p < 0) return make_float2(0.f, 0.f);
    if (x < I.nx && y < I.ny) return src[((long)p * I.ny + y) * I.nx + x];
    return psi_at(I, src, x, y, p);
}

// Halo cell handled by thread t (t < HALO) of the tile at (x0, y0):
// rows y0-1 and y0+TY (64 cells each), columns x0-1 and x0+TX (16 each).
__device__ __forceinline__ void halo_cell(int t, int x0, int y0, int &gx, int &gy, int &lx, int &ly) {
    if (t < TX) { gx = x0 + t; gy = y0 - 1; lx = t + 1; ly = 0; }
    else if (t < 2 * TX) { gx = x0 + t - TX; gy = y0 + TY; lx = t - TX + 1; ly = TY + 1; }
    else if (t < 2 * TX + TY) { gx = x0 - 1; gy = y0 + t - 2 * TX; lx = 0; ly = t - 2 * TX + 1; }
    else { gx = x0 + TX; gy = y0 + t - 2 * TX - TY; lx = TX + 1; ly = t - 2 * TX - TY + 1; }
}

template <int MODE>
__global__ __launch_bounds__(WG) void k_stencil(const Inst *__restrict__ insts,
                                                const int *__restrict__ prefix, int ninst, int l) {
    __shared__ float2 lds[2][LDY][LDX];
    __shared__ double red[WG / 64];

    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int ii = find_inst(prefix, ninst, b);
    const Inst &I = insts[ii];
    DevState *st = I.st;
    if (MODE == MODE_SWEEP) {
        // The previous sweep's input residual met the tolerance (or this
        // instance's cap is reached): its solve is complete and the launch
        // is a no-op for it.
        if (l >= I.max_iter) return;
        const float prev = row_max(I.res, I.rstride, l - 1);
        if (prev < I.tol) return;
    }
    if ((MODE == MODE_RHS) && !I.driven) return;

    int t = b - prefix[ii];
    const int txi = t % I.tiles_x;
    t /= I.tiles_x;
    const int tyi = t % I.tiles_y;
    const int tzi = t / I.tiles_y;
    const int x0 = txi * TX, y0 = tyi * TY;
    const int k0 = tzi * I.chunk;
    const int k1 = min(k0 + I.chunk, I.nz);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int x = x0 + lane;
    const int nx = I.nx, ny = I.ny;
    const long NXY = (long)nx * ny;

    const int cur = st->cur;
    const float2 *__restrict__ src =
        (MODE == MODE_FIRST || MODE == MODE_RHS || MODE == MODE_ENERGY) ? I.psi[cur]
                                                                        : I.psi[cur ^ (l & 1)];
    float2 *__restrict__ dst = I.psi[cur ^ ((l + 1) & 1)];

    const float cx = I.cx, cy = I.cy, cz = I.cz;
    float2 ux[ROWS], uz[ROWS];
    bool vy[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int y = y0 + w * ROWS + r;
        vy[r] = (x < nx) && (y < ny);
        ux[r] = (y < ny) ? I.ux[y] : make_float2(1.f, 0.f);
        uz[r] = (y < ny) ? I.uz[y] : make_float2(1.f, 0.f);
    }

    // halo bookkeeping
    const bool hthr = threadIdx.x < HALO;
    int hgx = 0, hgy = 0, hlx = 0, hly = 0;
    if (hthr) halo_cell(threadIdx.x, x0, y0, hgx, hgy, hlx, hly);

    // prologue: registers for planes k0-1, k0, k0+1; LDS buffer 0 = plane k0
    float2 pm[ROWS], pc[ROWS], pn[ROWS];
    {
        const int pp = zplane(I, k0, -1), pq = zplane(I, k0, +1);
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int y = y0 + w * ROWS + r;
            pc[r] = own_at(I, src, x, y, k0);
            pm[r] = own_at(I, src, x, y, pp);
            pn[r] = own_at(I, src, x, y, pq);
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) lds[0][1 + w * ROWS + r][1 + lane] = pc[r];
        if (hthr) lds[0][hly][hlx] = psi_at(I, src, hgx, hgy, k0);
    }
    float2 hv = make_float2(0.f, 0.f);
    if (hthr && k0 + 1 < k1) hv = psi_at(I, src, hgx, hgy, k0 + 1);

    const float ht2 = I.ht2, S2 = I.S2, u = I.u;
    const bool zper = I.per[2] != 0;
    const float mu_mean = (MODE == MODE_FIRST && I.driven) ? (float)st->mu_mean : 0.f;
    float rmax = 0.f;
    double acc = 0.0;

    for (int k = k0; k < k1; ++k) {
        const int buf = (k - k0) & 1;
        const long pbase = (long)k * NXY;
        // issue this plane's streams and the next planes' loads early
        float2 bh[ROWS], dh[ROWS];
        float ep[ROWS], mu[ROWS];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const long m = pbase + (long)(y0 + w * ROWS + r) * nx + x;
            if (MODE == MODE_SWEEP) {
                bh[r] = vy[r] ? I.bh[m] : make_float2(0.f, 0.f);
                dh[r] = vy[r] ? I.dh[m] : make_float2(0.f, 0.f);
            }
            if (MODE == MODE_FIRST || MODE == MODE_ENERGY) ep[r] = vy[r] ? I.eps[m] : 0.f;
            if (MODE == MODE_FIRST) mu[r] = (vy[r] && I.driven) ? I.mu[m] - mu_mean : 0.f;
        }
        float2 pnn[ROWS];
        float2 hvn = make_float2(0.f, 0.f);
        if (k + 1 < k1) {
            const int pq = zplane(I, k + 1, +1);
#pragma unroll
            for (int r = 0; r < ROWS; ++r) pnn[r] = own_at(I, src, x, y0 + w * ROWS + r, pq);
            if (hthr && k + 2 < k1) hvn = psi_at(I, src, hgx, hgy, k + 2);
        }
        __syncthreads();  // plane k staged; the other buffer is free
        if (k + 1 < k1) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) lds[buf ^ 1][1 + w * ROWS + r][1 + lane] = pn[r];
            if (hthr) lds[buf ^ 1][hly][hlx] = hv;
        }
        const bool zm = (k > 0) || zper, zp = (k < I.nz - 1) || zper;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int ly = 1 + w * ROWS + r;
            const float2 c = pc[r];
            const float2 xm = lds[buf][ly][lane], xp = lds[buf][ly][lane + 2];
            const float2 ym = lds[buf][ly - 1][lane + 1], yp = lds[buf][ly + 1][lane + 1];
            if (!vy[r]) continue;
            const long m = pbase + (long)(y0 + w * ROWS + r) * nx + x;
            if (MODE == MODE_ENERGY) {
                // forward edges only; an edge beyond an open face does not exist.
                const float a2 = cabs2(c);
                const int y = y0 + w * ROWS + r;
                const bool fx = I.per[0] || x < nx - 1, fy = I.per[1] || y < ny - 1;
                const float wxn = (!I.per[0] && nx > 1 && (x == 0 || x == nx - 1)) ? 0.5f : 1.f;
                const float wyn = (!I.per[1] && ny > 1 && (y == 0 || y == ny - 1)) ? 0.5f : 1.f;
                const float wzn = (!zper && I.nz > 1 && (k == 0 || k == I.nz - 1)) ? 0.5f : 1.f;
                double e = (double)(wxn * wyn * wzn) * (double)(-ep[r] * a2 + 0.5f * a2 * a2);
                if (fx) e += (double)(wyn * wzn * cx) * (double)cabs2(csub(cmul(ux[r], xp), c));
                if (fy) e += (double)(wxn * wzn * cy) * (double)cabs2(csub(yp, c));
                if (zp)
                    e += (double)(wxn * wyn * cz) * (double)cabs2(csub(cmul(uz[r], pn[r]), c));
                acc += e;
                continue;
            }
            // off-diagonal neighbour sum NS of the covariant Laplacian
            // (Eq. LaplUV_xz), open faces doubling the inner neighbour.
            float2 zt;
            if (zm && zp) zt = cadd(cmul(uz[r], pn[r]), cmulc(uz[r], pm[r]));
            else if (zp) zt = cscale(2.f, cmul(uz[r], pn[r]));
            else if (zm) zt = cscale(2.f, cmulc(uz[r], pm[r]));
            else zt = make_float2(0.f, 0.f);
            const float2 xt = cadd(cmul(ux[r], xp), cmulc(ux[r], xm));
            const float2 yt = cadd(yp, ym);
            const float2 ns = make_float2(cx * xt.x + cy * yt.x + cz * zt.x,
                                          cx * xt.y + cy * yt.y + cz * zt.y);
            if (MODE == MODE_RHS) {
                // f = sum_a (1/h_a^2) Im[psi^* (U psi_+ + U^* psi_-)] = Im[psi^* NS]
                const float f = c.x * ns.y - c.y * ns.x;
                I.f[m] = f;
                acc += (double)f * (double)node_w(I, x, y0 + w * ROWS + r, k);
                continue;
            }
            float2 nw;
            if (MODE == MODE_FIRST) {
                // b = psi^- + ht/2 [ (eps - i u mu) psi^- - |psi^-|^2 psi^- + L psi^- ]
                // M = 1 + ht/2 [ |psi^-|^2 + 2S + i u mu - eps ]
                const float a2 = cabs2(c);
                const float e = ep[r], um = u * mu[r];
                const float2 lap = make_float2(ns.x - S2 * c.x, ns.y - S2 * c.y);
                const float2 src_t = make_float2(e * c.x + um * c.y - a2 * c.x + lap.x,
                                                 e * c.y - um * c.x - a2 * c.y + lap.y);
                const float2 bb = make_float2(c.x + ht2 * src_t.x, c.y + ht2 * src_t.y);
                const float2 M = make_float2(1.f + ht2 * (a2 + S2 - e), ht2 * um);
                const float inv = 1.f / cabs2(M);
                const float2 Mi = make_float2(M.x * inv, -M.y * inv);
                const float2 bhv = cmul(bb, Mi);
                const float2 dhv = cscale(ht2, Mi);
                I.bh[m] = bhv;
                I.dh[m] = dhv;
                nw = cadd(bhv, cmul(dhv, ns));
                const float2 d = csub(nw, c);
                const float r2 = cabs2(M) * cabs2(d);
                rmax = (r2 > rmax || r2 != r2) ? r2 : rmax;
            } else {
                nw = cadd(bh[r], cmul(dh[r], ns));
                const float2 d = csub(nw, c);
                const float r2 = cabs2(d) * (ht2 * ht2) / cabs2(dh[r]);
                rmax = (r2 > rmax || r2 != r2) ? r2 : rmax;
            }
            dst[m] = nw;
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            pm[r] = pc[r];
            pc[r] = pn[r];
            if (k + 1 < k1) pn[r] = pnn[r];
        }
        hv = hvn;
    }

    if (MODE == MODE_FIRST || MODE == MODE_SWEEP) {
        __syncthreads();
        wg_max_to<WG>(row_slot(I.res, I.rstride, l, b), rmax, reinterpret_cast<float *>(red));
    } else {
        const double s = wg_sum<WG>(acc, red);
        if (threadIdx.x == 0) I.part[b - prefix[ii]] = s;
    }
}

template __global__ void k_stencil<MODE_FIRST>(const Inst *, const int *, int, int);
template __global__ void k_stencil<MODE_SWEEP>(const Inst *, const int *, int, int);
template __global__ void k_stencil<MODE_RHS>(const Inst *, const int *, int, int);
template __global__ void k_stencil<MODE_ENERGY>(const Inst *, const int *, int, int);

}  // namespace tdgl
