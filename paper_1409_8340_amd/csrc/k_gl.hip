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
//   MODE_ENERGY free-energy density summed in FP64;
//   MODE_NS     the neighbour sum NS(x) of an arbitrary complex field x (the
//               off-diagonal part of the covariant Laplacian; used by the
//               adjoint).
// FIRST and SWEEP also reduce max_m |r_m|^2 of their input iterate
// (Eq. convergence) through r = M_mm (psi^(l+1) - psi^(l)).
#include "kernels.h"
#include "stencil.h"

#include <hip/hip_cooperative_groups.h>

namespace tdgl {

// MODE selects the pass; R is the number of consecutive rows a thread owns
// (tile 64 x 4R: a larger R streams more per thread, a smaller one keeps
// more waves resident; the autotuner picks R and the z chunk).
// One pass of MODE over tile b of the batched grid (see k_stencil); used by
// the ordinary launch (one tile per work-group) and by the persistent Jacobi
// solve (tiles in a grid-stride loop).  pub (sweeps of a host-driven solve,
// else null): the work-group of each instance's first tile hands the row
// l - 1 it has read to the host, tagged seq.
template <int MODE, int R, bool NT, bool YZ>
__device__ __forceinline__ void stencil_tile(const Inst *__restrict__ insts, const int *__restrict__ prefix,
                                             int ninst, int l, const float2 *ext_in, float2 *ext_out, int b,
                                             unsigned long long *pub, unsigned seq) {
    constexpr int ROWS = R;
    constexpr int TYv = 4 * R;
    constexpr int HALOv = 2 * TX + 2 * TYv;
    __shared__ float2 lds[2][TYv + 2][LDX];
    __shared__ double red[WG / 64];

    const int ii = find_inst(prefix, ninst, b);
    const Inst &I = insts[ii];
    DevState *st = I.st;
    // l = -1 (sweep only): a timing pass for the tile autotuner -- reads the
    // current psi, writes the spare buffer, skips the convergence test and
    // records no residual, so the solver state is left as it was.
    // l = -2: the corrective sweep of two-sweep mode -- when the solve ended
    // on an even iterate, recompute it from the odd one in psi[cur ^ 1] into
    // psi[cur] (no residual row).  The assemble pass takes l = -1 as a
    // timing pass too: b/M and (ht/2)/M (dead between steps) and the spare
    // psi buffer are written, no residual row.
    const bool timing = (MODE == MODE_SWEEP || is_first_mode(MODE)) && l == -1;
    const bool fixp = (MODE == MODE_SWEEP) && l == -2;
    if (fixp && !st->fix) return;
    if (timing) l = 0;
    if (fixp) l = 1;
    if (MODE == MODE_SWEEP && !timing && !fixp) {
        // The previous sweep's input residual met the tolerance (or this
        // instance's cap is reached): its solve is complete and the launch
        // is a no-op for it.
        if (l >= I.max_iter) return;
        const float prev = row_max_wave(I.res, I.rstride, l - 1);
        if (pub && b == prefix[ii] && threadIdx.x == 0) publish(pub + (size_t)(l - 1) * ninst + ii, seq, prev);
        if (prev < I.tol) return;
    }
    if ((MODE == MODE_RHS) && !I.driven) return;

    // the Poisson right side with four rows per thread has a 64 x 16 tiling
    // of its own (the same as the stencil's when the context's rows are 4)
    constexpr bool own4 = (MODE == MODE_RHS) && (ROWS == 4);
    const int tiles_y = own4 ? I.tiles_y4 : I.tiles_y;
    const int chunk = own4 ? I.chunk4 : I.chunk;
    int t = b - prefix[ii];
    const int txi = t % I.tiles_x;
    t /= I.tiles_x;
    const int tyi = t % tiles_y;
    const int tzi = t / tiles_y;
    const int x0 = txi * TX, y0 = tyi * TYv;
    const int k0 = tzi * chunk;
    const int k1 = min(k0 + chunk, I.nz);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int x = x0 + lane;
    const int nx = I.nx, ny = I.ny, nz = I.nz;
    const unsigned NXY = (unsigned)nx * (unsigned)ny;

    const int cur = st->cur;
    const gf2 *__restrict__ src =
        (const gf2 *)((MODE == MODE_NS) ? ext_in : (MODE == MODE_SWEEP) ? I.psi[cur ^ (l & 1)] : I.psi[cur]);
    gf2 *__restrict__ nsout = (gf2 *)ext_out;
    gf2 *__restrict__ dst = (gf2 *)I.psi[cur ^ ((l + 1) & 1)];
    const gf2 *__restrict__ Pt = (const gf2 *)I.P;
    const gf2 *__restrict__ bhp = (const gf2 *)I.bh;
    const gf2 *__restrict__ dhp = (const gf2 *)I.dh;
    gf2 *__restrict__ bhw = (gf2 *)I.bh;
    gf2 *__restrict__ dhw = (gf2 *)I.dh;
    const gf1 *__restrict__ epsp = (const gf1 *)I.eps;
    const gf1 *__restrict__ mup = (const gf1 *)I.mu;
    gf1 *__restrict__ fw = (gf1 *)I.f;

    const float cx = I.cx, cy = I.cy, cz = I.cz;
    float2 ux[ROWS], uz[ROWS];
    bool vy[ROWS];
    CellSrc own[ROWS];
    bool all_plain = true;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int y = y0 + w * ROWS + r;
        vy[r] = (x < nx) && (y < ny);
        ux[r] = (y < ny) ? I.ux[y] : make_float2(1.f, 0.f);
        uz[r] = (y < ny) ? I.uz[y] : make_float2(1.f, 0.f);
        own[r] = cell_src(I, x, y);
        all_plain = all_plain && own[r].mode == SRC_PLAIN;
    }
    const bool hthr = threadIdx.x < HALOv;
    int hgx = 0, hgy = 0, hlx = 0, hly = 0;
    CellSrc hs{0, SRC_ZERO, 0, make_float2(1.f, 0.f)};
    if (hthr) {
        halo_cell<TYv>(threadIdx.x, x0, y0, hgx, hgy, hlx, hly);
        hs = cell_src(I, hgx, hgy);
    }
    auto own_plane = [&](int p, float2 *out) {
        // own cells of plane p (p = -1: no such plane -> zeros)
        if (p < 0) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) out[r] = make_float2(0.f, 0.f);
            return;
        }
        const unsigned pb = (unsigned)p * NXY;
        if (all_plain) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) out[r] = ld2(src, pb + (unsigned)own[r].off);
        } else {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) out[r] = fetch<YZ>(src, Pt, pb, p, nx, own[r], I.wz);
        }
    };

    // prologue: registers for planes k0-1, k0, k0+1; LDS buffer 0 = plane k0
    float2 pm[ROWS], pc[ROWS], pn[ROWS];
    own_plane(zplane(I, k0, -1), pm);
    own_plane(k0, pc);
    own_plane(zplane(I, k0, +1), pn);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) lds[0][1 + w * ROWS + r][1 + lane] = pc[r];
    if (hthr) lds[0][hly][hlx] = fetch<YZ>(src, Pt, (unsigned)k0 * NXY, k0, nx, hs, I.wz);
    float2 hv = make_float2(0.f, 0.f);
    if (hthr && k0 + 1 < k1) hv = fetch<YZ>(src, Pt, (unsigned)(k0 + 1) * NXY, k0 + 1, nx, hs, I.wz);

    // per-plane streams of the first plane
    float2 bh[ROWS], dh[ROWS];
    float ep[ROWS], mu[ROWS];
    const float mu_mean = (is_first_mode(MODE) && I.driven) ? (float)st->mu_mean : 0.f;
    auto load_streams = [&](int k, float2 *bh_, float2 *dh_, float *ep_, float *mu_) {
        const unsigned pb = (unsigned)k * NXY;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const unsigned m = pb + (unsigned)own[r].off;
            if (MODE == MODE_SWEEP) {
                bh_[r] = vy[r] ? (NT ? ld2nt(bhp, m) : ld2(bhp, m)) : make_float2(0.f, 0.f);
                dh_[r] = vy[r] ? (NT ? ld2nt(dhp, m) : ld2(dhp, m)) : make_float2(0.f, 0.f);
            }
            if (is_first_mode(MODE) || MODE == MODE_ENERGY)
                ep_[r] = vy[r] ? (NT ? __builtin_nontemporal_load(&epsp[m]) : float(epsp[m])) : 0.f;
            if (is_first_mode(MODE))
                mu_[r] = (vy[r] && I.driven) ? (NT ? __builtin_nontemporal_load(&mup[m]) : float(mup[m])) - mu_mean : 0.f;
        }
    };
    load_streams(k0, bh, dh, ep, mu);

    const float ht2 = I.ht2, S2 = I.S2, u = I.u;
    const bool zper = I.per[2] != 0;
    // a yz field on a periodic z axis: the z neighbours across the wrap
    // carry the seam phase, psi_{-1} = zs psi_{nz-1} and psi_{nz} =
    // conj(zs) psi_0 (zs = 1 for any other field)
    const float2 zsx = (YZ && zper) ? I.zs[min(x, nx - 1)] : make_float2(1.f, 0.f);
    // Langevin draws of this step (assemble only): step counter before the step
    const bool noise = (MODE == MODE_FIRSTN) && I.zeta_max > 0.f;
    const unsigned long long nstep = noise ? (unsigned long long)st->n : 0ull;
    float rmax = 0.f;
    double acc = 0.0;
    // assemble under a two-sweep tiling: slots in the side copies of b/M and
    // (ht/2)/M of this thread's first row at z = 0 (-1: its column x is not
    // beside a tile column); row r adds 2 r, plane k adds 2 ny k
    int eL = -1, eR = -1;
    if (is_first_mode(MODE) && I.edge) edge_slots(I, x, y0 + w * ROWS, 0, eL, eR);
    const unsigned eplane = 2u * (unsigned)ny;

    for (int k = k0; k < k1; ++k) {
        const int buf = (k - k0) & 1;
        const unsigned pbase = (unsigned)k * NXY;
        // issue the next planes' loads before the barrier
        float2 pnn[ROWS], bhn[ROWS], dhn[ROWS];
        float epn[ROWS], mun[ROWS];
        float2 hvn = make_float2(0.f, 0.f);
        if (k + 1 < k1) {
            own_plane(zplane(I, k + 1, +1), pnn);
            load_streams(k + 1, bhn, dhn, epn, mun);
            if (hthr && k + 2 < k1) hvn = fetch<YZ>(src, Pt, (unsigned)(k + 2) * NXY, k + 2, nx, hs, I.wz);
        }
        __syncthreads();  // plane k staged; the other buffer is free
        if (k + 1 < k1) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) lds[buf ^ 1][1 + w * ROWS + r][1 + lane] = pn[r];
            if (hthr) lds[buf ^ 1][hly][hlx] = hv;
        }
        const bool zm = (k > 0) || zper, zp = (k < nz - 1) || zper;
        float2 pmk[ROWS], pnk[ROWS];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            pmk[r] = pm[r];
            pnk[r] = pn[r];
        }
        if (YZ && zper) {
            if (k == 0) {
#pragma unroll
                for (int r = 0; r < ROWS; ++r) pmk[r] = xcmul(zsx, pm[r]);
            }
            if (k == nz - 1) {
#pragma unroll
                for (int r = 0; r < ROWS; ++r) pnk[r] = xcmulc(zsx, pn[r]);
            }
        }
        // x links of this plane (a yz-plane field adds the factor wz[k])
        float2 uxk[ROWS];
        if (YZ) {
            const float2 wk = I.wz[k];
#pragma unroll
            for (int r = 0; r < ROWS; ++r) uxk[r] = xcmul(ux[r], wk);
        } else {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) uxk[r] = ux[r];
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int ly = 1 + w * ROWS + r;
            const float2 c = pc[r];
            const float2 xm = lds[buf][ly][lane], xp = lds[buf][ly][lane + 2];
            const float2 ym = lds[buf][ly - 1][lane + 1], yp = lds[buf][ly + 1][lane + 1];
            if (!vy[r]) continue;
            const unsigned m = pbase + (unsigned)own[r].off;
            if (MODE == MODE_ENERGY) {
                // forward edges only; an edge beyond an open face does not exist.
                const float a2 = cabs2(c);
                const int y = y0 + w * ROWS + r;
                const bool fx = I.per[0] || x < nx - 1, fy = I.per[1] || y < ny - 1;
                const float wxn = (!I.per[0] && nx > 1 && (x == 0 || x == nx - 1)) ? 0.5f : 1.f;
                const float wyn = (!I.per[1] && ny > 1 && (y == 0 || y == ny - 1)) ? 0.5f : 1.f;
                const float wzn = (!zper && nz > 1 && (k == 0 || k == nz - 1)) ? 0.5f : 1.f;
                double e = (double)(wxn * wyn * wzn) * (double)(-ep[r] * a2 + 0.5f * a2 * a2);
                if (fx) e += (double)(wyn * wzn * cx) * (double)cabs2(csub(cmul(uxk[r], xp), c));
                if (fy) e += (double)(wxn * wzn * cy) * (double)cabs2(csub(yp, c));
                if (zp) e += (double)(wxn * wyn * cz) * (double)cabs2(csub(cmul(uz[r], pnk[r]), c));
                acc += e;
                continue;
            }
            // off-diagonal neighbour sum NS of the covariant Laplacian
            // (Eq. LaplUV_xz), open faces doubling the inner neighbour.
            const float2 ns = nsum(uxk[r], uz[r], xm, xp, ym, yp, pmk[r], pnk[r], zm, zp, cx, cy, cz);
            if (MODE == MODE_NS) {
                st2(nsout, m, ns);
                continue;
            }
            if (MODE == MODE_RHS) {
                // f = sum_a (1/h_a^2) Im[psi^* (U psi_+ + U^* psi_-)] = Im[psi^* NS]
                const float f = rhs_node(c, ns);
                fw[m] = f;
                acc += (double)f * (double)node_w(I, x, y0 + w * ROWS + r, k);
                continue;
            }
            float2 nw;
            if (is_first_mode(MODE)) {
                float2 bhv, dhv;
                float r2;
                const float2 zz = noise ? langevin2(I, m, nstep) : make_float2(0.f, 0.f);
                assemble_node(c, ep[r], u * mu[r], ns, S2, ht2, noise, zz, bhv, dhv, nw, r2);
                if (NT) {
                    st2nt(bhw, m, bhv);
                    st2nt(dhw, m, dhv);
                } else {
                    st2(bhw, m, bhv);
                    st2(dhw, m, dhv);
                }
                // side copies for the two-sweep super-tiles (one 16-byte
                // global store each)
                if (eL >= 0) st4(I.edge, (unsigned)eL + 2u * r + eplane * k, bhv, dhv);
                if (eR >= 0) st4(I.edge, (unsigned)eR + 2u * r + eplane * k, bhv, dhv);
                rmax = (r2 > rmax || r2 != r2) ? r2 : rmax;
            } else {
                nw = jacobi(bh[r], dh[r], ns);
                const float r2 = resid2(nw, c, dh[r], ht2);
                rmax = (r2 > rmax || r2 != r2) ? r2 : rmax;
            }
            if (NT) st2nt(dst, m, nw);
            else st2(dst, m, nw);
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            pm[r] = pc[r];
            pc[r] = pn[r];
            if (k + 1 < k1) {
                pn[r] = pnn[r];
                bh[r] = bhn[r];
                dh[r] = dhn[r];
                ep[r] = epn[r];
                mu[r] = mun[r];
            }
        }
        hv = hvn;
    }

    if (MODE == MODE_NS) {
        return;
    } else if (is_first_mode(MODE) || MODE == MODE_SWEEP) {
        if (timing || fixp) return;
        __syncthreads();
        wg_max_to<WG>(row_slot(I.res, I.rstride, l, b), rmax, reinterpret_cast<float *>(red));
    } else {
        const double s = wg_sum<WG>(acc, red);
        if (threadIdx.x == 0) I.part[b - prefix[ii]] = s;
    }
}

template <int MODE, int R, bool NT, bool YZ>
__global__ __launch_bounds__(WG) void k_stencil(const Inst *__restrict__ insts,
                                                const int *__restrict__ prefix, int ninst, int l,
                                                const float2 *ext_in, float2 *ext_out, unsigned long long *pub,
                                                unsigned seq) {
    stencil_tile<MODE, R, NT, YZ>(insts, prefix, ninst, l, ext_in, ext_out, xcd_remap(blockIdx.x, gridDim.x), pub,
                              seq);
}

// The whole Jacobi solve of every instance in one cooperative launch: sweeps
// l = l0, l0+1, ... over all tiles (grid-stride loop, XCD-aware order), a
// grid-wide barrier between sweeps, and the convergence words read after
// the barrier -- the same words by every work-group, so the decision to go
// on is uniform.  A sweep does what the separate launch l does (tiles of an
// instance whose solve has ended exit at once); the loop ends once no
// instance's solve is open or at lcap.  The barrier releases this
// work-group's stores at device scope before it arrives and acquires the
// others' after it leaves (one L2 write-back and invalidate per work-group
// and sweep).  l0 = -1: lcap timing sweeps (l = -1 each, no convergence
// test, state untouched) for the tile autotuner.
template <int R, bool NT>
__global__ __launch_bounds__(WG) void k_jacobi_persist(const Inst *__restrict__ insts,
                                                       const int *__restrict__ prefix, int ninst, int l0,
                                                       int lcap, int ntiles) {
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    __shared__ int go;
    const bool timing = l0 < 0;
    const int l_begin = timing ? 0 : l0;
    for (int l = l_begin; l < lcap; ++l) {
        if (!timing) {
            if (threadIdx.x < 64) {
                int open = 0;
                for (int i = 0; i < ninst && !open; ++i) {
                    const Inst &I = insts[i];
                    if (l < I.max_iter && !(row_max_wave(I.res, I.rstride, l - 1) < I.tol)) open = 1;
                }
                if (threadIdx.x == 0) go = open;
            }
            __syncthreads();
            if (!go) break;
        }
        for (int t = blockIdx.x; t < ntiles; t += gridDim.x)
            stencil_tile<MODE_SWEEP, R, NT, false>(insts, prefix, ninst, timing ? -1 : l, nullptr, nullptr,
                                            xcd_remap(t, ntiles), nullptr, 0u);
        grid.sync();
    }
}

#define TDGL_INST(M, R, NT, YZ)                                                                            \
    template __global__ void k_stencil<M, R, NT, YZ>(const Inst *, const int *, int, int, const float2 *, float2 *, \
                                                     unsigned long long *, unsigned);
// YZ: a yz-plane field in the context (per-plane x-link factor)
#define TDGL_INST_R(R)                      \
    TDGL_INST(MODE_FIRST, R, false, false)  \
    TDGL_INST(MODE_FIRST, R, true, false)   \
    TDGL_INST(MODE_FIRSTN, R, false, false) \
    TDGL_INST(MODE_FIRSTN, R, true, false)  \
    TDGL_INST(MODE_SWEEP, R, false, false)  \
    TDGL_INST(MODE_SWEEP, R, true, false)   \
    TDGL_INST(MODE_RHS, R, false, false)    \
    TDGL_INST(MODE_ENERGY, R, false, false) \
    TDGL_INST(MODE_NS, R, false, false)     \
    TDGL_INST(MODE_FIRST, R, false, true)   \
    TDGL_INST(MODE_FIRST, R, true, true)    \
    TDGL_INST(MODE_FIRSTN, R, false, true)  \
    TDGL_INST(MODE_FIRSTN, R, true, true)   \
    TDGL_INST(MODE_SWEEP, R, false, true)   \
    TDGL_INST(MODE_SWEEP, R, true, true)    \
    TDGL_INST(MODE_RHS, R, false, true)     \
    TDGL_INST(MODE_ENERGY, R, false, true)  \
    TDGL_INST(MODE_NS, R, false, true)
TDGL_INST_R(1)
TDGL_INST_R(2)
TDGL_INST_R(4)
#define TDGL_INSTP(R, NT) \
    template __global__ void k_jacobi_persist<R, NT>(const Inst *, const int *, int, int, int, int);
TDGL_INSTP(1, false)
TDGL_INSTP(1, true)
TDGL_INSTP(2, false)
TDGL_INSTP(2, true)
TDGL_INSTP(4, false)
TDGL_INSTP(4, true)
#undef TDGL_INSTP
#undef TDGL_INST_R
#undef TDGL_INST

}  // namespace tdgl
