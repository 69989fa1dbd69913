// k_gl2.hip -- two Jacobi iterations (Eq. final) per pass over HBM.
//
// The single-sweep kernel reads psi^(l), b/M and (ht/2)/M and writes
// psi^(l+1) for every node: 32 bytes per node and iteration.  Here one pass
// takes psi^(l) to psi^(l+2): a work-group computes psi^(l+1) on its tile
// and on the one-cell ring around it, then psi^(l+2) on the tile, reading
// the three input streams once and writing psi^(l+2) once.
//
// The z march of the tiled kernel is kept, with a lag of one plane: in the
// step for plane v the group computes psi^(l+1) on plane v (tile + ring) and
// psi^(l+2) on plane v - 1.  psi^(l) of plane v with its one-cell halo sits
// in LDS as in the single sweep; psi^(l+1) of planes v-1 and v (tile + ring)
// in a second double-buffered LDS array; the z neighbours of the tile's own
// nodes in registers.
//
// Ring values of psi^(l+1) belong to neighbouring tiles (or to ghost nodes):
// each one is the boundary rule of its slot (wrap, quasi-periodic phase,
// Neumann mirror) applied to the Jacobi update of the real source node,
// computed from global memory with the same arithmetic as the tile path, so
// every iterate is bit-identical to two single sweeps.
//
// Residuals: the group reduces max |r|^2 of psi^(l) (row l) and of psi^(l+1)
// (row l+1), exactly as two single sweeps would.  Buffers: the pairs start
// either at l = 1 (from the assemble kernel's psi^(1)) or at l = 2 (after one
// single sweep); pass l reads psi[cur ^ pair_src(l)] and writes the other
// one, so the iterates the pairs store alternate between the two buffers.
// When the solve ends on the first sweep of a pair (or on a cap inside one),
// a corrective single sweep recomputes that iterate from the stored one
// before it (see k_solve_finalize and the single-sweep kernel's fix pass).
#include "kernels.h"
#include "stencil.h"

namespace tdgl {

namespace {

// x link of row y on plane p: the row's table entry, times the plane factor
// wz[p] of a yz-plane field (YZ), computed as the single-sweep kernel does.
template <bool YZ>
__device__ __forceinline__ float2 xlink(const Inst &I, float2 u, int p) {
    return YZ ? xcmul(u, I.wz[p]) : u;
}

// Jacobi update of the real node (sx, sy) of plane p from global memory,
// in the domain's coordinates: the neighbours follow cell_src / zplane like
// the tile path's LDS and register values do.
template <bool YZ>
__device__ __forceinline__ float2 node_update(const Inst &I, const gf2 *__restrict__ src,
                                              const gf2 *__restrict__ Pt, const gf2 *__restrict__ bhp,
                                              const gf2 *__restrict__ dhp, int sx, int sy, int p,
                                              unsigned NXY, bool zper) {
    const int nx = I.nx, nz = I.nz;
    const unsigned pb = (unsigned)p * NXY;
    const unsigned so = (unsigned)(sy * nx + sx);
    const float2 xm = fetch<YZ>(src, Pt, pb, p, nx, cell_src(I, sx - 1, sy), I.wz);
    const float2 xp = fetch<YZ>(src, Pt, pb, p, nx, cell_src(I, sx + 1, sy), I.wz);
    const float2 ym = fetch<YZ>(src, Pt, pb, p, nx, cell_src(I, sx, sy - 1), I.wz);
    const float2 yp = fetch<YZ>(src, Pt, pb, p, nx, cell_src(I, sx, sy + 1), I.wz);
    const int pm = zplane(I, p, -1), pp = zplane(I, p, +1);
    const float2 zmv = pm >= 0 ? ld2(src, (unsigned)pm * NXY + so) : make_float2(0.f, 0.f);
    const float2 zpv = pp >= 0 ? ld2(src, (unsigned)pp * NXY + so) : make_float2(0.f, 0.f);
    const bool zm = (p > 0) || zper, zp = (p < nz - 1) || zper;
    const float2 ns = nsum(xlink<YZ>(I, I.ux[sy], p), I.uz[sy], xm, xp, ym, yp, zmv, zpv, zm, zp, I.cx, I.cy, I.cz);
    return jacobi(ld2(bhp, pb + so), ld2(dhp, pb + so), ns);
}

// The open-x ghost factor of slot s on plane p: s.fac (U^2 or its
// conjugate), times wz[p]^2 (or its conjugate) for a yz-plane field, as
// fetch<YZ> applies it.
template <bool YZ>
__device__ __forceinline__ float2 fac_at(const Inst &I, const CellSrc &s, int p) {
    if (!YZ) return s.fac;
    float2 w2 = xcmul(I.wz[p], I.wz[p]);
    if (s.px) w2.y = -w2.y;
    return xcmul(s.fac, w2);
}

// Value of the slot described by s (its boundary rule relative to the real
// node s.off) in plane p, given that node's update v: the same operations
// fetch() applies to a stored value.
template <bool YZ>
__device__ __forceinline__ float2 apply_src(const Inst &I, const gf2 *__restrict__ Pt, int p, int nx,
                                            const CellSrc &s, float2 v) {
    if (s.mode == SRC_PLAIN) return v;
    if (s.mode == SRC_ZERO) return make_float2(0.f, 0.f);
    if (s.mode == SRC_FAC) return xcmul(fac_at<YZ>(I, s, p), v);
    const float2 ph = ld2(Pt, (unsigned)p * nx + s.px);
    return s.mode == SRC_P ? xcmul(ph, v) : xcmulc(ph, v);
}

template <bool YZ>
__device__ __forceinline__ float2 slot_update(const Inst &I, const gf2 *__restrict__ src,
                                              const gf2 *__restrict__ Pt, const gf2 *__restrict__ bhp,
                                              const gf2 *__restrict__ dhp, const CellSrc &s, int p,
                                              unsigned NXY, bool zper) {
    if (s.mode == SRC_ZERO) return make_float2(0.f, 0.f);
    const int sy = s.off / I.nx, sx = s.off - sy * I.nx;
    return apply_src<YZ>(I, Pt, p, I.nx, s, node_update<YZ>(I, src, Pt, bhp, dhp, sx, sy, p, NXY, zper));
}

}  // namespace

// Slot h of the two-node halo of a TX x TYv tile at (x0, y0): rows y0-2,
// y0-1 and y0+TYv, y0+TYv+1 (TX + 4 wide), then columns x0-2, x0-1, x0+TX,
// x0+TX+1 of the tile's rows.  (lx, ly): index in the (TX+4) x (TYv+4) LDS
// plane.
template <int TYv>
__device__ __forceinline__ void halo2_cell(int h, int x0, int y0, int &gx, int &gy, int &lx, int &ly) {
    constexpr int LX = TX + 4;
    if (h < 4 * LX) {
        const int rr = h / LX, c = h - rr * LX;
        ly = rr < 2 ? rr : TYv + rr;
        lx = c;
    } else {
        const int q = h - 4 * LX, cc = q / TYv, r = q - cc * TYv;
        lx = cc < 2 ? cc : TX + cc;
        ly = r + 2;
    }
    gx = x0 + lx - 2;
    gy = y0 + ly - 2;
}

template <int R, bool NT, bool YZ>
__global__ __launch_bounds__(WG) void k_sweep2(const Inst *__restrict__ insts, const int *__restrict__ prefix,
                                               int ninst, int l, unsigned long long *pub, unsigned seq) {
    constexpr int TYv = 4 * R;
    constexpr int LX = TX + 4, LY = TYv + 4;
    constexpr int NH2 = LX * LY - TX * TYv;   // two-node halo slots of psi^(l)
    constexpr int HALOv = 2 * TX + 2 * TYv;   // one-node ring of psi^(l+1)
    static_assert(NH2 <= 2 * WG, "two halo slots per thread at most");
    __shared__ float2 la[4][LY][LX];          // psi^(l) planes v-1 .. v+2, two-node halo
    __shared__ float2 lb[2][TYv + 2][LDX];    // psi^(l+1) planes v-1, v: tile + ring
    __shared__ float red[WG / 64];

    // work-groups over the instance's non-interior (x, y) tiles, bchunk
    // planes each (prefix: blocks per instance); the first is tile (0, 0)
    // from plane 0, which hands the rows over
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int ii = find_inst(prefix, ninst, b);
    const Inst &I = insts[ii];
    const DevState *st = I.st;
    const int q = b - prefix[ii];
    const int nzb = (I.nz + I.bchunk - 1) / I.bchunk;
    const int xyi = q / nzb, zsub = q - xyi * nzb;
    const int tile = I.btile[xyi];
    const int txi = tile % I.tiles_x, tyi = tile / I.tiles_x;
    const int x0 = txi * TX, y0 = tyi * TYv;
    // l < 0: timing pass of the autotuner (psi[cur] -> psi[cur ^ 1], no
    // residual rows, no convergence test)
    const bool timing = l < 0;
    if (!timing) {
        // the solve has ended on psi^(l) or psi^(l-1): nothing to do (a row
        // that a skipped pass never wrote reads 0, so an earlier end shows
        // here too), and the buffer of psi^(l-1) must survive for the
        // corrective sweep
        if (l >= I.max_iter) return;
        const float p1 = row_max_wave(I.res, I.rstride, l - 1);
        const float p2 = (l >= 2) ? row_max_wave(I.res, I.rstride, l - 2) : 1.f;
        // hand rows l - 1 and l - 2 (written by the previous pass) to the host
        if (pub && q == 0 && threadIdx.x == 0) {
            publish(pub + (size_t)(l - 1) * ninst + ii, seq, p1);
            if (l >= 2) publish(pub + (size_t)(l - 2) * ninst + ii, seq, p2);
        }
        if (p1 < I.tol) return;
        if (l >= 2 && p2 < I.tol) return;
    }
    const bool rec2 = !timing && (l + 1 < I.max_iter);

    const int k0 = zsub * I.bchunk;
    const int k1 = min(k0 + I.bchunk, I.nz);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int x = x0 + lane;
    const int nx = I.nx, ny = I.ny, nz = I.nz;
    const unsigned NXY = (unsigned)nx * (unsigned)ny;
    const bool zper = I.per[2] != 0;

    const int cur = st->cur;
    const int xs = timing ? 0 : pair_src(l);
    const gf2 *__restrict__ src = (const gf2 *)I.psi[cur ^ xs];
    gf2 *__restrict__ dst = (gf2 *)I.psi[cur ^ xs ^ 1];
    const gf2 *__restrict__ Pt = (const gf2 *)I.P;
    const gf2 *__restrict__ bhp = (const gf2 *)I.bh;
    const gf2 *__restrict__ dhp = (const gf2 *)I.dh;
    const float cx = I.cx, cy = I.cy, cz = I.cz, ht2 = I.ht2;

    // own nodes
    float2 ux[R], uz[R];
    bool vy[R];
    CellSrc own[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int y = y0 + w * R + r;
        vy[r] = (x < nx) && (y < ny);
        ux[r] = (y < ny) ? I.ux[y] : make_float2(1.f, 0.f);
        uz[r] = (y < ny) ? I.uz[y] : make_float2(1.f, 0.f);
        // the two-node rules: a ring slot's tile path may read an own slot
        // two nodes beyond the grid in a ragged tile
        own[r] = cell_src2(I, x, y);
    }
    // two-node halo slots of psi^(l) this thread stages (h = tid, tid + WG)
    CellSrc h2s[2];
    int h2lx[2], h2ly[2];
    bool h2on[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int h = threadIdx.x + q * WG;
        h2on[q] = h < NH2;
        int gx = 0, gy = 0;
        h2lx[q] = h2ly[q] = 0;
        h2s[q] = CellSrc{0, SRC_ZERO, 0, make_float2(1.f, 0.f)};
        if (h2on[q]) {
            halo2_cell<TYv>(h, x0, y0, gx, gy, h2lx[q], h2ly[q]);
            h2s[q] = cell_src2(I, gx, gy);
        }
    }
    // ring slot of psi^(l+1) (index spread over the wavefronts).  Ring
    // values follow their slot's boundary rule from a real source node.
    // Tile path: the source's neighbourhood is in the LDS planes (in-range
    // nodes, x wraps taken at the slot's own position, open-face mirrors at
    // the mirror node); global path: slots carrying the quasi-periodic y
    // phase, computed from global memory.
    const int hidx = lane * 4 + w;
    const bool hthr = hidx < HALOv;
    int rlx = 0, rly = 0;               // slot in lb
    int rmode = 0;                      // 0: zero, 1: tile path, 2: global path
    int tlx = 0, tly = 0;               // tile-path source in la
    unsigned rso = 0;                   // source node's in-plane offset
    float2 rux = make_float2(1.f, 0.f), ruz = make_float2(1.f, 0.f), rfac = make_float2(1.f, 0.f);
    CellSrc rs{0, SRC_ZERO, 0, make_float2(1.f, 0.f)};
    if (hthr) {
        int gx, gy;
        halo_cell<TYv>(hidx, x0, y0, gx, gy, rlx, rly);
        rs = cell_src(I, gx, gy);
        if (rs.mode == SRC_P || rs.mode == SRC_PCONJ) {
            rmode = 2;
        } else if (rs.mode != SRC_ZERO) {
            rmode = 1;
            rso = (unsigned)rs.off;
            const int sy = rs.off / nx, sx = rs.off - sy * nx;
            const bool xwrap = (gx < 0 || gx >= nx) && I.per[0];
            tlx = (xwrap ? gx : sx) - x0 + 2;
            tly = sy - y0 + 2;
            rux = I.ux[sy];
            ruz = I.uz[sy];
            rfac = rs.mode == SRC_FAC ? rs.fac : make_float2(1.f, 0.f);
        }
    }

    // virtual plane v -> stored plane (-1: none)
    auto pz = [&](int v) -> int {
        if (v >= 0 && v < nz) return v;
        if (!zper) return -1;
        return ((v % nz) + nz) % nz;
    };
    // psi^(l) of plane p: own values and halo values into registers
    auto load_a = [&](int p, float2 *ao, float2 *hv) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            ao[r] = (p < 0) ? make_float2(0.f, 0.f) : fetch<YZ>(src, Pt, (unsigned)p * NXY, p, nx, own[r], I.wz);
#pragma unroll
        for (int q = 0; q < 2; ++q)
            hv[q] = (p < 0 || !h2on[q]) ? make_float2(0.f, 0.f)
                                        : fetch<YZ>(src, Pt, (unsigned)p * NXY, p, nx, h2s[q], I.wz);
    };
    auto stage_a = [&](int v, const float2 *ao, const float2 *hv) {
        float2 (*L)[LX] = la[v & 3];
#pragma unroll
        for (int r = 0; r < R; ++r) L[2 + w * R + r][2 + lane] = ao[r];
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (h2on[q]) L[h2ly[q]][h2lx[q]] = hv[q];
    };
    auto load_bd = [&](int p, float2 *bh_, float2 *dh_, float2 &rbh, float2 &rdh) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (p >= 0 && vy[r]) {
                const unsigned m = (unsigned)p * NXY + (unsigned)own[r].off;
                bh_[r] = NT ? ld2nt(bhp, m) : ld2(bhp, m);
                dh_[r] = NT ? ld2nt(dhp, m) : ld2(dhp, m);
            } else {
                bh_[r] = make_float2(0.f, 0.f);
                dh_[r] = make_float2(1.f, 0.f);
            }
        }
        if (p >= 0 && rmode == 1) {
            rbh = ld2(bhp, (unsigned)p * NXY + rso);
            rdh = ld2(dhp, (unsigned)p * NXY + rso);
        } else {
            rbh = make_float2(0.f, 0.f);
            rdh = make_float2(1.f, 0.f);
        }
    };

    // psi^(l+1) planes vb0 .. k1 feed psi^(l+2) on k0 .. k1-1; psi^(l) is
    // needed on vb0-1 .. k1+1
    const int vb0 = (pz(k0 - 1) >= 0) ? k0 - 1 : k0;
    const int ve = k1;
    auto needed_a = [&](int v) { return v >= vb0 - 1 && v <= k1 + 1 && pz(v) >= 0; };

    {
        float2 ao[R], hv[2];
        for (int v = vb0 - 1; v <= vb0 + 1; ++v)
            if (needed_a(v)) {
                load_a(pz(v), ao, hv);
                stage_a(v, ao, hv);
            }
    }
    float2 an2[R], hn2[2];  // psi^(l) of plane v + 2 (staged in step v)
    load_a(needed_a(vb0 + 2) ? pz(vb0 + 2) : -1, an2, hn2);
    float2 bhc[R], dhc[R], rbhc, rdhc;  // b/M, (ht/2)/M of plane v (own, ring source)
    load_bd(pz(vb0), bhc, dhc, rbhc, rdhc);
    float2 b2[R], b1[R], bhq[R], dhq[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        b2[r] = b1[r] = make_float2(0.f, 0.f);
        bhq[r] = make_float2(0.f, 0.f);
        dhq[r] = make_float2(1.f, 0.f);
    }

    float rmax1 = 0.f, rmax2 = 0.f;
    for (int v = vb0; v <= ve; ++v) {
        const int p = pz(v);
        const bool stageA = (p >= 0);
        const bool stageB = (v - 1 >= k0) && (v - 1 < k1);
        // next loads, issued before the barrier
        float2 an3[R], hn3[2], bhn[R], dhn[R], rbhn, rdhn;
        load_a(needed_a(v + 3) ? pz(v + 3) : -1, an3, hn3);
        load_bd(v + 1 <= k1 ? pz(v + 1) : -1, bhn, dhn, rbhn, rdhn);
        __syncthreads();  // planes v-1 .. v+1 of psi^(l) and plane v-1 of psi^(l+1) complete
        if (needed_a(v + 2)) stage_a(v + 2, an2, hn2);
        float2 b0[R];
        if (stageA) {
            const float2 (*L)[LX] = la[v & 3];
            const float2 (*Lm)[LX] = la[(v + 3) & 3];  // plane v - 1
            const float2 (*Lp)[LX] = la[(v + 1) & 3];  // plane v + 1
            const int lq = v & 1;
            const bool zm = (p > 0) || zper, zp = (p < nz - 1) || zper;
            // psi^(l+1) on the tile
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int ly = 2 + w * R + r, lx = 2 + lane;
                if (vy[r]) {
                    const float2 c = L[ly][lx];
                    const float2 ns = nsum(xlink<YZ>(I, ux[r], p), uz[r], L[ly][lx - 1], L[ly][lx + 1], L[ly - 1][lx],
                                           L[ly + 1][lx], Lm[ly][lx], Lp[ly][lx], zm, zp, cx, cy, cz);
                    b0[r] = jacobi(bhc[r], dhc[r], ns);
                    const float r2 = resid2(b0[r], c, dhc[r], ht2);
                    rmax1 = (r2 > rmax1 || r2 != r2) ? r2 : rmax1;
                } else {
                    // a node outside the grid in a ragged tile: its ghost value
                    b0[r] = slot_update<YZ>(I, src, Pt, bhp, dhp, own[r], p, NXY, zper);
                }
                lb[lq][ly - 1][lx - 1] = b0[r];
            }
            // ... and on the ring
            if (hthr) {
                float2 val = make_float2(0.f, 0.f);
                if (rmode == 1) {
                    const float2 ns = nsum(xlink<YZ>(I, rux, p), ruz, L[tly][tlx - 1], L[tly][tlx + 1],
                                           L[tly - 1][tlx], L[tly + 1][tlx], Lm[tly][tlx], Lp[tly][tlx], zm, zp, cx,
                                           cy, cz);
                    val = jacobi(rbhc, rdhc, ns);
                    if (rs.mode == SRC_FAC) val = xcmul(YZ ? fac_at<YZ>(I, rs, p) : rfac, val);
                } else if (rmode == 2) {
                    val = slot_update<YZ>(I, src, Pt, bhp, dhp, rs, p, NXY, zper);
                }
                lb[lq][rly][rlx] = val;
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) b0[r] = make_float2(0.f, 0.f);
        }
        if (stageB) {
            // psi^(l+2) on plane k = v - 1 from psi^(l+1) of planes k-1, k, k+1
            const int k = v - 1;
            const int pk = pz(k);
            const int lq = k & 1;
            const bool zm = (pk > 0) || zper, zp = (pk < nz - 1) || zper;
            const unsigned pbase = (unsigned)pk * NXY;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int ly = 1 + w * R + r;
                if (!vy[r]) continue;
                const float2 ns = nsum(xlink<YZ>(I, ux[r], pk), uz[r], lb[lq][ly][lane], lb[lq][ly][lane + 2],
                                       lb[lq][ly - 1][lane + 1], lb[lq][ly + 1][lane + 1], b2[r], b0[r], zm, zp, cx,
                                       cy, cz);
                const float2 c2 = jacobi(bhq[r], dhq[r], ns);
                const float r2 = resid2(c2, b1[r], dhq[r], ht2);
                rmax2 = (r2 > rmax2 || r2 != r2) ? r2 : rmax2;
                const unsigned m = pbase + (unsigned)own[r].off;
                if (NT) st2nt(dst, m, c2);
                else st2(dst, m, c2);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            an2[r] = an3[r];
            b2[r] = b1[r];
            b1[r] = b0[r];
            bhq[r] = bhc[r];
            dhq[r] = dhc[r];
            bhc[r] = bhn[r];
            dhc[r] = dhn[r];
        }
        hn2[0] = hn3[0];
        hn2[1] = hn3[1];
        rbhc = rbhn;
        rdhc = rdhn;
    }
    if (timing) return;
    __syncthreads();
    wg_max_to<WG>(row_slot(I.res, I.rstride, l, b), rmax1, red);
    if (rec2) {
        __syncthreads();
        wg_max_to<WG>(row_slot(I.res, I.rstride, l + 1, b), rmax2, red);
    }
}

// Pre-pass of a two-sweep pass on a seam2 instance: psi^(l+1) of rows ny-1
// and 0 of every plane, i.e. the Jacobi updates of the real nodes behind the
// ring slots that the super-tiles on the quasi-periodic y seam hold beyond
// it (row -1 is row ny-1 times P, row ny is row 0 times conj P).  Same
// function and operands as k_sweep2's slot update, so the same bits; the
// super-tile kernel then applies the phase.  out[(p 2 + r) nx + x], r = 0
// for row ny-1, 1 for row 0.  Exits like the pass when the solve has ended.
template <bool YZ>
__global__ __launch_bounds__(256) void k_seam_ring(const Inst *__restrict__ insts, const int *__restrict__ prefix,
                                                   int ninst, int l) {
    const int b = blockIdx.x;
    const int ii = find_inst(prefix, ninst, b);
    const Inst &I = insts[ii];
    const bool timing = l < 0;
    if (!timing) {
        if (l >= I.max_iter) return;
        if (row_max_wave(I.res, I.rstride, l - 1) < I.tol) return;
        if (l >= 2 && row_max_wave(I.res, I.rstride, l - 2) < I.tol) return;
    }
    const int nx = I.nx, ny = I.ny, nz = I.nz;
    const int t = (b - prefix[ii]) * 256 + (int)threadIdx.x;
    if (t >= 2 * nz * nx) return;
    const int x = t % nx, pr = t / nx, r = pr & 1, p = pr >> 1;
    const int cur = I.st->cur;
    const int xs = timing ? 0 : pair_src(l);
    const gf2 *__restrict__ src = (const gf2 *)I.psi[cur ^ xs];
    I.sring[t] = node_update<YZ>(I, src, (const gf2 *)I.P, (const gf2 *)I.bh, (const gf2 *)I.dh, x,
                                 r == 0 ? ny - 1 : 0, p, (unsigned)nx * (unsigned)ny, I.per[2] != 0);
}

// The two-sweep pass on interior super-tiles (tile_interior2 with the
// height TY): the tile, its two-node halo of psi^(l) and its ring of psi^(l+1)
// are real nodes with real neighbours (or their plain images across a
// periodic x wrap), so every load is a plain load at a fixed in-plane
// offset, issued unconditionally (a plane outside the grid reads a real
// plane whose values are never used).  With no loads under branches the
// prefetched planes stay in flight across the barrier.  The update
// arithmetic is that of k_sweep2's tile path (same functions, same
// operands), so both kernels give the same bits; k_sweep2 takes the 64 x 4R
// tiles of the other super-tiles.  NT: the new iterate is stored
// non-temporally; b/M and (ht/2)/M stay cacheable, since the neighbours'
// rings read them again.
template <int R, bool NT, bool YZ, int TY>
__global__ __launch_bounds__(WG * sweep2i_mult(R, TY), 4) void k_sweep2i(const Inst *__restrict__ insts,
                                                               const int *__restrict__ prefix, int ninst, int l,
                                                               unsigned long long *pub, unsigned seq) {
    constexpr int M = sweep2i_mult(R, TY);
    constexpr int WGI = WG * M;
    constexpr int TYv = TY;
    constexpr int LX = TX + 4, LY = TYv + 4;
    constexpr int NH2 = LX * LY - TX * TYv;
    constexpr int NQ = (NH2 + WGI - 1) / WGI;  // two-node halo slots per thread
    constexpr int HALOv = 2 * TX + 2 * TYv;
    static_assert(HALOv % 4 == 0 && HALOv / 4 <= 64, "ring slots packed into four wavefronts");
    __shared__ float2 la[4][LY][LX];          // psi^(l) planes v-1 .. v+2, two-node halo
    __shared__ float2 lb[2][TYv + 2][LDX];    // psi^(l+1) planes v-1, v: tile + ring
    __shared__ float red[WGI / 64];

    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int ii = find_inst(prefix, ninst, b);
    const Inst &I = insts[ii];
    const int nx = I.nx, ny = I.ny, nz = I.nz;
    // blocks: tiles_x x sweep2i_rows x tiles_z2 super-tiles
    const bool seam2 = I.seam2 != 0;
    const int nsy = sweep2i_rows(ny, R, TY, seam2);
    int t = b - prefix[ii];
    const bool first = t == 0;
    const int txi = t % I.tiles_x;
    t /= I.tiles_x;
    const int tyr = t % nsy;
    const int tzi = t / nsy;
    // seam2: the two seam rows (a little slower: their halo rows beyond the
    // seam carry the phase) are taken first, so that they do not finish
    // last: row order 0, nsy - 1, 1, 2, ..., nsy - 2
    const int tyi = (!seam2 || tyr == 0) ? tyr : (tyr == 1 ? nsy - 1 : tyr - 1);
    const int x0 = txi * TX, y0 = sweep2i_y0(tyi, R, TY, seam2);
    const bool xper = I.per[0] != 0;
    const bool timing = l < 0;
    if (!timing) {
        if (l >= I.max_iter) return;
        const float p1 = row_max_wave(I.res, I.rstride, l - 1);
        const float p2 = (l >= 2) ? row_max_wave(I.res, I.rstride, l - 2) : 1.f;
        // an instance with no boundary tiles hands rows l - 1 and l - 2 to
        // the host from here (else the boundary kernel does)
        if (pub && I.nbt == 0 && first && threadIdx.x == 0) {
            publish(pub + (size_t)(l - 1) * ninst + ii, seq, p1);
            if (l >= 2) publish(pub + (size_t)(l - 2) * ninst + ii, seq, p2);
        }
        if (p1 < I.tol) return;
        if (l >= 2 && p2 < I.tol) return;
    }
    if (!tile_interior2(x0, y0, TYv, nx, ny, xper, seam2)) return;
    // a super-tile on the quasi-periodic y seam (seam2): its y halo rows
    // beyond the grid are the wrapped rows times the phase P (or conj P),
    // and its ring slots there are the wrapped nodes' updates (made by
    // k_seam_ring before the pass) with that phase, as cell_src2 /
    // slot_update give them to the general kernel
    const bool seam = seam2 && (y0 == 0 || y0 + TYv == ny);
    const gf2 *__restrict__ Pt = (const gf2 *)I.P;
    const bool rec2 = !timing && (l + 1 < I.max_iter);
    const int k0 = tzi * I.chunk2;
    const int k1 = min(k0 + I.chunk2, nz);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int x = x0 + lane;
    const unsigned NXY = (unsigned)nx * (unsigned)ny;
    const bool zper = I.per[2] != 0;

    const int cur = I.st->cur;
    const int xs = timing ? 0 : pair_src(l);
    const gf2 *__restrict__ src = (const gf2 *)I.psi[cur ^ xs];
    gf2 *__restrict__ dst = (gf2 *)I.psi[cur ^ xs ^ 1];
    const gf2 *__restrict__ bhp = (const gf2 *)I.bh;
    const gf2 *__restrict__ dhp = (const gf2 *)I.dh;
    const float cx = I.cx, cy = I.cy, cz = I.cz, ht2 = I.ht2;

    // own nodes
    float2 ux[R], uz[R];
    unsigned oo[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int y = y0 + w * R + r;
        ux[r] = I.ux[y];
        uz[r] = I.uz[y];
        oo[r] = (unsigned)(y * nx + x);
    }
    // two-node halo slots this thread stages (h = tid + q WGI); h2m: 0
    // plain, SRC_P / SRC_PCONJ across the seam, with the phase's x index
    // in h2x (its table entry is loaded with the slot, for every tile)
    unsigned h2o[NQ];
    int h2l[NQ], h2m[NQ], h2x[NQ];
    bool h2on[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int h = threadIdx.x + q * WGI;
        h2on[q] = h < NH2;
        h2o[q] = oo[0];
        h2l[q] = 0;
        h2m[q] = SRC_PLAIN;
        h2x[q] = 0;
        if (h2on[q]) {
            int gx, gy, lx, ly;
            halo2_cell<TYv>(h, x0, y0, gx, gy, lx, ly);
            const int sx = xper ? ((gx % nx) + nx) % nx : gx;
            int sy = gy;
            if (gy < 0) { sy = gy + ny; h2m[q] = SRC_P; h2x[q] = sx; }
            else if (gy >= ny) { sy = gy - ny; h2m[q] = SRC_PCONJ; h2x[q] = sx; }
            h2o[q] = (unsigned)(sy * nx + sx);
            h2l[q] = ly * LX + lx;
        }
    }
    // ring slot of psi^(l+1): a real node (or its plain x image) whose
    // neighbourhood is in la around the slot's own position.  The slots sit
    // in the first HALOv / 4 lanes of wavefronts 0..3 (one per SIMD), so the
    // other wavefronts skip the ring update as a whole.
    const int hidx = w * (HALOv / 4) + lane;
    const bool hthr = w < 4 && lane < HALOv / 4;
    int rlx = 0, rly = 0, tlx = 2, tly = 2;
    // the slot's b/M and (ht/2)/M: offsets from bh and from dh and the
    // plane stride (a slot beside the tile reads the side copies, where the
    // 16 rows of a side lie in one run)
    unsigned rob = oo[0], rod = oo[0], rst = NXY;
    float2 rux = make_float2(1.f, 0.f), ruz = make_float2(1.f, 0.f);
    // ring slot beyond the seam (a row slot at y = -1 or ny): its real
    // node's update comes from k_seam_ring, at sring[(p 2) nx + rsr], times
    // P (row -1) or conj P (row ny) at its x, cell_src2's rule for the slot
    bool rcross = false, rtop = false;
    unsigned rsr = 0, rsx = 0;
    if (hthr) {
        int gx, gy;
        halo_cell<TYv>(hidx, x0, y0, gx, gy, rlx, rly);
        const int sx = xper ? ((gx % nx) + nx) % nx : gx;
        rcross = gy < 0 || gy >= ny;
        rtop = gy < 0;
        const int sy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
        rsx = (unsigned)sx;
        rsr = (unsigned)((gy < 0 ? 0 : nx) + sx);
        rob = rod = (unsigned)(sy * nx + sx);
        if (I.edge && gy >= y0 && gy < y0 + TYv) {
            const unsigned e = (gx < x0 ? 0u : I.edge_r) +
                               2u * ((unsigned)txi * (unsigned)nz * (unsigned)ny + (unsigned)gy);
            rob = I.edge_ob + e;
            rod = I.edge_od + e + 1u;
            rst = 2u * (unsigned)ny;
        }
        tlx = gx - x0 + 2;
        tly = gy - y0 + 2;
        rux = I.ux[sy];
        ruz = I.uz[sy];
    }

    auto pz = [&](int v) -> int {
        if (v >= 0 && v < nz) return v;
        if (!zper) return -1;
        return ((v % nz) + nz) % nz;
    };
    // (the phase entries are loaded by every tile, with the other loads and
    // unconditionally, so that no load sits under a branch; only seam tiles
    // use them)
    // A load whose values are not used (p < 0: a plane beyond an open face,
    // or a padding step after the run) reads the tile's first node from
    // every lane, one line per wavefront, rather than a whole plane whose
    // lines have long left L2.
    const unsigned o0 = (unsigned)(y0 * nx + x0);
    auto load_a = [&](int p, float2 *ao, float2 *hv, float2 *ph) {
        const int pp = p < 0 ? 0 : p;
        const unsigned msk = p < 0 ? 0u : ~0u;
        const unsigned pb = p < 0 ? o0 : (unsigned)pp * NXY;
#pragma unroll
        for (int r = 0; r < R; ++r) ao[r] = ld2(src, pb + (oo[r] & msk));
#pragma unroll
        for (int q = 0; q < NQ; ++q) hv[q] = ld2(src, pb + (h2o[q] & msk));
#pragma unroll
        for (int q = 0; q < NQ; ++q) ph[q] = ld2(Pt, (unsigned)pp * nx + (h2x[q] & msk));
    };
    auto stage_a = [&](int v, const float2 *ao, const float2 *hv, const float2 *ph) {
        float2 (*L)[LX] = la[v & 3];
        float2 *Lf = &la[v & 3][0][0];
#pragma unroll
        for (int r = 0; r < R; ++r) L[2 + w * R + r][2 + lane] = ao[r];
        if (seam) {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                if (h2on[q])
                    Lf[h2l[q]] = h2m[q] == SRC_P ? xcmul(ph[q], hv[q])
                                                 : (h2m[q] == SRC_PCONJ ? xcmulc(ph[q], hv[q]) : hv[q]);
        } else {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                if (h2on[q]) Lf[h2l[q]] = hv[q];
        }
    };
    auto load_bd = [&](int p, float2 *bh_, float2 *dh_, float2 &rbh, float2 &rdh) {
        const unsigned msk = p < 0 ? 0u : ~0u;
        const unsigned pb = p < 0 ? o0 : (unsigned)p * NXY;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            bh_[r] = ld2(bhp, pb + (oo[r] & msk));
            dh_[r] = ld2(dhp, pb + (oo[r] & msk));
        }
        const unsigned rp = p < 0 ? o0 : (unsigned)p * rst;
        rbh = ld2(bhp, rp + (rob & msk));
        rdh = ld2(dhp, rp + (rod & msk));
    };

    const int vb0 = (pz(k0 - 1) >= 0) ? k0 - 1 : k0;
    const int ve = k1;
    auto needed_a = [&](int v) { return v >= vb0 - 1 && v <= k1 + 1 && pz(v) >= 0; };

    {
        float2 ao[R], hv[NQ], ph[NQ];
        for (int v = vb0 - 1; v <= vb0 + 1; ++v)
            if (needed_a(v)) {
                load_a(pz(v), ao, hv, ph);
                stage_a(v, ao, hv, ph);
            }
    }
    // three register sets for the prefetched planes, rotating every plane
    // (the loop body runs three times per trip): psi^(l) of plane q sits in
    // set q mod 3 from two steps before it is staged, b/M of plane q from
    // two steps before its sweep, so that two planes of loads are in flight
    // across each barrier and no register a load is still filling is ever
    // copied.  Sets are indexed relative to vb0.
    float2 aS0[R], hS0[NQ], aS1[R], hS1[NQ], aS2[R], hS2[NQ];  // psi^(l)
    float2 pS0[NQ], pS1[NQ], pS2[NQ];                         // seam phases of the halo slots
    float2 bT0[R], dT0[R], bT1[R], dT1[R], bT2[R], dT2[R];     // b/M, (ht/2)/M
    float2 rbT0, rdT0, rbT1, rdT1, rbT2, rdT2;                  // ... at the ring source
    load_a(needed_a(vb0 + 2) ? pz(vb0 + 2) : -1, aS2, hS2, pS2);
    load_a(needed_a(vb0 + 3) ? pz(vb0 + 3) : -1, aS0, hS0, pS0);
    load_bd(pz(vb0), bT0, dT0, rbT0, rdT0);
    load_bd(vb0 + 1 <= k1 ? pz(vb0 + 1) : -1, bT1, dT1, rbT1, rdT1);
    float2 b2[R], b1[R];
#pragma unroll
    for (int r = 0; r < R; ++r) b2[r] = b1[r] = make_float2(0.f, 0.f);

    float rmax1 = 0.f, rmax2 = 0.f;
    // plane v: stage psi^(l) of v + 2 (an2), sweep 1 on v with b/M of v
    // (bhc), sweep 2 on v - 1 with b/M of v - 1 (bh2, the set plane v + 2's
    // b/M is loaded into afterwards); loads of plane v + 4 into an4.  v > ve:
    // a padding step (loads only) that makes the trip count a multiple of
    // three.
    auto body = [&](int v, float2 (&an2)[R], float2 (&hn2)[NQ], float2 (&pn2)[NQ], float2 (&an4)[R],
                    float2 (&hn4)[NQ], float2 (&pn4)[NQ], float2 (&bhc)[R], float2 (&dhc)[R], float2 &rbhc,
                    float2 &rdhc, float2 (&bh2)[R], float2 (&dh2)[R], float2 &rbh2,
                    float2 &rdh2) __attribute__((always_inline)) {
        const bool live = v <= ve;
        const int p = pz(v);
        const bool stageA = live && (p >= 0);
        const bool stageB = live && (v - 1 >= k0) && (v - 1 < k1);
        load_a(needed_a(v + 4) ? pz(v + 4) : -1, an4, hn4, pn4);
        __syncthreads();
        if (live && needed_a(v + 2)) stage_a(v + 2, an2, hn2, pn2);
        float2 b0[R];
        if (stageA) {
            const float2 (*L)[LX] = la[v & 3];
            const float2 (*Lm)[LX] = la[(v + 3) & 3];
            const float2 (*Lp)[LX] = la[(v + 1) & 3];
            const int lq = v & 1;
            const bool zm = (p > 0) || zper, zp = (p < nz - 1) || zper;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int ly = 2 + w * R + r, lx = 2 + lane;
                const float2 c = L[ly][lx];
                const float2 ns = nsum(xlink<YZ>(I, ux[r], p), uz[r], L[ly][lx - 1], L[ly][lx + 1], L[ly - 1][lx],
                                       L[ly + 1][lx], Lm[ly][lx], Lp[ly][lx], zm, zp, cx, cy, cz);
                b0[r] = jacobi(bhc[r], dhc[r], ns);
                const float r2 = resid2(b0[r], c, dhc[r], ht2);
                rmax1 = (r2 > rmax1 || r2 != r2) ? r2 : rmax1;
                lb[lq][ly - 1][lx - 1] = b0[r];
            }
            if (hthr) {
                if (seam && rcross) {
                    const float2 v = ld2((const gf2 *)I.sring, (unsigned)p * 2u * (unsigned)nx + rsr);
                    const float2 ph = ld2(Pt, (unsigned)p * nx + rsx);
                    lb[lq][rly][rlx] = rtop ? xcmul(ph, v) : xcmulc(ph, v);
                } else {
                    const float2 ns = nsum(xlink<YZ>(I, rux, p), ruz, L[tly][tlx - 1], L[tly][tlx + 1],
                                           L[tly - 1][tlx], L[tly + 1][tlx], Lm[tly][tlx], Lp[tly][tlx], zm, zp, cx,
                                           cy, cz);
                    lb[lq][rly][rlx] = jacobi(rbhc, rdhc, ns);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) b0[r] = make_float2(0.f, 0.f);
        }
        if (stageB) {
            const int k = v - 1;
            const int pk = pz(k);
            const int lq = k & 1;
            const bool zm = (pk > 0) || zper, zp = (pk < nz - 1) || zper;
            const unsigned pbase = (unsigned)pk * NXY;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int ly = 1 + w * R + r;
                const float2 ns = nsum(xlink<YZ>(I, ux[r], pk), uz[r], lb[lq][ly][lane], lb[lq][ly][lane + 2],
                                       lb[lq][ly - 1][lane + 1], lb[lq][ly + 1][lane + 1], b2[r], b0[r], zm, zp, cx,
                                       cy, cz);
                const float2 c2 = jacobi(bh2[r], dh2[r], ns);
                const float r2 = resid2(c2, b1[r], dh2[r], ht2);
                rmax2 = (r2 > rmax2 || r2 != r2) ? r2 : rmax2;
                if (NT) st2nt(dst, pbase + oo[r], c2);
                else st2(dst, pbase + oo[r], c2);
            }
        }
        load_bd(v + 2 <= k1 ? pz(v + 2) : -1, bh2, dh2, rbh2, rdh2);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            b2[r] = b1[r];
            b1[r] = b0[r];
        }
    };
    for (int v = vb0; v <= ve; v += 3) {
        body(v, aS2, hS2, pS2, aS1, hS1, pS1, bT0, dT0, rbT0, rdT0, bT2, dT2, rbT2, rdT2);
        body(v + 1, aS0, hS0, pS0, aS2, hS2, pS2, bT1, dT1, rbT1, rdT1, bT0, dT0, rbT0, rdT0);
        body(v + 2, aS1, hS1, pS1, aS0, hS0, pS0, bT2, dT2, rbT2, rdT2, bT1, dT1, rbT1, rdT1);
    }
    if (timing) return;
    __syncthreads();
    wg_max_to<WGI>(row_slot(I.res, I.rstride, l, b), rmax1, red);
    if (rec2) {
        __syncthreads();
        wg_max_to<WGI>(row_slot(I.res, I.rstride, l + 1, b), rmax2, red);
    }
}

template __global__ void k_seam_ring<false>(const Inst *, const int *, int, int);
template __global__ void k_seam_ring<true>(const Inst *, const int *, int, int);

#define TDGL_INST2I(R, NT, YZ, TY)                                                                        \
    template __global__ void k_sweep2i<R, NT, YZ, TY>(const Inst *, const int *, int, int, unsigned long long *, \
                                                      unsigned);
#define TDGL_INST2(R, NT, YZ)                                                                           \
    template __global__ void k_sweep2<R, NT, YZ>(const Inst *, const int *, int, int, unsigned long long *,  \
                                                 unsigned);                                                 \
    TDGL_INST2I(R, NT, YZ, 16)
TDGL_INST2(1, false, false)
TDGL_INST2(1, true, false)
TDGL_INST2(2, false, false)
TDGL_INST2(2, true, false)
TDGL_INST2(4, false, false)
TDGL_INST2(4, true, false)
TDGL_INST2(1, false, true)
TDGL_INST2(1, true, true)
TDGL_INST2(2, false, true)
TDGL_INST2(2, true, true)
TDGL_INST2(4, false, true)
TDGL_INST2(4, true, true)
// 32-row super-tiles: R = 2 and 4 (R = 1 would need 2048 threads)
TDGL_INST2I(2, false, false, 32)
TDGL_INST2I(2, true, false, 32)
TDGL_INST2I(4, false, false, 32)
TDGL_INST2I(4, true, false, 32)
TDGL_INST2I(2, false, true, 32)
TDGL_INST2I(2, true, true, 32)
TDGL_INST2I(4, false, true, 32)
TDGL_INST2I(4, true, true, 32)
#undef TDGL_INST2
#undef TDGL_INST2I

}  // namespace tdgl
