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
// (row l+1), exactly as two single sweeps would.  Buffers: pass l (odd, the
// first from psi^(1)) reads psi[cur ^ ((l + 1) / 2 & 1)] and writes the
// other one.  When the solve ends on psi^(l+1) -- the first sweep of a pair
// converged, or an even cap -- a corrective single sweep recomputes it from
// psi^(l) (see k_solve_finalize and the single-sweep kernel's fix pass).
#include "kernels.h"
#include "stencil.h"

namespace tdgl {

namespace {

// Jacobi update of the real node (sx, sy) of plane p from global memory,
// in the domain's coordinates: the neighbours follow cell_src / zplane like
// the tile path's LDS and register values do.
__device__ __forceinline__ float2 node_update(const Inst &I, const gf2 *__restrict__ src,
                                              const gf2 *__restrict__ Pt, const gf2 *__restrict__ bhp,
                                              const gf2 *__restrict__ dhp, int sx, int sy, int p,
                                              unsigned NXY, bool zper) {
    const int nx = I.nx, nz = I.nz;
    const unsigned pb = (unsigned)p * NXY;
    const unsigned so = (unsigned)(sy * nx + sx);
    const float2 xm = fetch(src, Pt, pb, p, nx, cell_src(I, sx - 1, sy));
    const float2 xp = fetch(src, Pt, pb, p, nx, cell_src(I, sx + 1, sy));
    const float2 ym = fetch(src, Pt, pb, p, nx, cell_src(I, sx, sy - 1));
    const float2 yp = fetch(src, Pt, pb, p, nx, cell_src(I, sx, sy + 1));
    const int pm = zplane(I, p, -1), pp = zplane(I, p, +1);
    const float2 zmv = pm >= 0 ? ld2(src, (unsigned)pm * NXY + so) : make_float2(0.f, 0.f);
    const float2 zpv = pp >= 0 ? ld2(src, (unsigned)pp * NXY + so) : make_float2(0.f, 0.f);
    const bool zm = (p > 0) || zper, zp = (p < nz - 1) || zper;
    const float2 ns = nsum(I.ux[sy], I.uz[sy], xm, xp, ym, yp, zmv, zpv, zm, zp, I.cx, I.cy, I.cz);
    return jacobi(ld2(bhp, pb + so), ld2(dhp, pb + so), ns);
}

// Value of the slot described by s (its boundary rule relative to the real
// node s.off) in plane p, given that node's update v: the same operations
// fetch() applies to a stored value.
__device__ __forceinline__ float2 apply_src(const gf2 *__restrict__ Pt, int p, int nx, const CellSrc &s,
                                            float2 v) {
    if (s.mode == SRC_PLAIN) return v;
    if (s.mode == SRC_ZERO) return make_float2(0.f, 0.f);
    if (s.mode == SRC_FAC) return xcmul(s.fac, v);
    const float2 ph = ld2(Pt, (unsigned)p * nx + s.px);
    return s.mode == SRC_P ? xcmul(ph, v) : xcmulc(ph, v);
}

__device__ __forceinline__ float2 slot_update(const Inst &I, const gf2 *__restrict__ src,
                                              const gf2 *__restrict__ Pt, const gf2 *__restrict__ bhp,
                                              const gf2 *__restrict__ dhp, const CellSrc &s, int p,
                                              unsigned NXY, bool zper) {
    if (s.mode == SRC_ZERO) return make_float2(0.f, 0.f);
    const int sy = s.off / I.nx, sx = s.off - sy * I.nx;
    return apply_src(Pt, p, I.nx, s, node_update(I, src, Pt, bhp, dhp, sx, sy, p, NXY, zper));
}

}  // namespace

template <int R, bool NT>
__global__ __launch_bounds__(WG) void k_sweep2(const Inst *__restrict__ insts, const int *__restrict__ prefix,
                                               int ninst, int l) {
    constexpr int TYv = 4 * R;
    constexpr int HALOv = 2 * TX + 2 * TYv;
    __shared__ float2 la[2][TYv + 2][LDX];  // psi^(l) of one plane, one-cell halo
    __shared__ float2 lb[2][TYv + 2][LDX];  // psi^(l+1) of one plane, tile + ring
    __shared__ float red[WG / 64];

    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int ii = find_inst(prefix, ninst, b);
    const Inst &I = insts[ii];
    const DevState *st = I.st;
    // l < 0: timing pass of the autotuner (psi[cur] -> psi[cur ^ 1], no
    // residual rows, no convergence test)
    const bool timing = l < 0;
    if (!timing) {
        // the solve has ended on psi^(l) or psi^(l-1): nothing to do (a row
        // that a skipped pass never wrote reads 0, so an earlier end shows
        // here too), and the buffer of psi^(l-1) must survive for the
        // corrective sweep
        if (l >= I.max_iter) return;
        if (row_max(I.res, I.rstride, l - 1) < I.tol) return;
        if (l >= 2 && row_max(I.res, I.rstride, l - 2) < I.tol) return;
    }
    const bool rec2 = !timing && (l + 1 < I.max_iter);

    int t = b - prefix[ii];
    const int txi = t % I.tiles_x;
    t /= I.tiles_x;
    const int tyi = t % I.tiles_y;
    const int tzi = t / I.tiles_y;
    const int x0 = txi * TX, y0 = tyi * TYv;
    const int k0 = tzi * I.chunk;
    const int k1 = min(k0 + I.chunk, I.nz);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int x = x0 + lane;
    const int nx = I.nx, ny = I.ny, nz = I.nz;
    const unsigned NXY = (unsigned)nx * (unsigned)ny;
    const bool zper = I.per[2] != 0;

    const int cur = st->cur;
    const int xs = timing ? 0 : (((l + 1) >> 1) & 1);
    const gf2 *__restrict__ src = (const gf2 *)I.psi[cur ^ xs];
    gf2 *__restrict__ dst = (gf2 *)I.psi[cur ^ xs ^ 1];
    const gf2 *__restrict__ Pt = (const gf2 *)I.P;
    const gf2 *__restrict__ bhp = (const gf2 *)I.bh;
    const gf2 *__restrict__ dhp = (const gf2 *)I.dh;
    const float cx = I.cx, cy = I.cy, cz = I.cz, ht2 = I.ht2;

    float2 ux[R], uz[R];
    bool vy[R];
    CellSrc own[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int y = y0 + w * R + r;
        vy[r] = (x < nx) && (y < ny);
        ux[r] = (y < ny) ? I.ux[y] : make_float2(1.f, 0.f);
        uz[r] = (y < ny) ? I.uz[y] : make_float2(1.f, 0.f);
        own[r] = cell_src(I, x, y);
    }
    // halo / ring slot of this thread; the slot index is spread over the
    // wavefronts so that the ring's extra updates balance between them
    const int hidx = lane * 4 + w;
    const bool hthr = hidx < HALOv;
    int hgx = 0, hgy = 0, hlx = 0, hly = 0;
    CellSrc hs{0, SRC_ZERO, 0, make_float2(1.f, 0.f)};
    if (hthr) {
        halo_cell<TYv>(hidx, x0, y0, hgx, hgy, hlx, hly);
        hs = cell_src(I, hgx, hgy);
    }

    // virtual plane v -> stored plane (-1: none)
    auto pz = [&](int v) -> int {
        if (v >= 0 && v < nz) return v;
        if (!zper) return -1;
        return ((v % nz) + nz) % nz;
    };
    auto own_plane = [&](int p, float2 *out) {
#pragma unroll
        for (int r = 0; r < R; ++r) out[r] = (p < 0) ? make_float2(0.f, 0.f) : fetch(src, Pt, (unsigned)p * NXY, p, nx, own[r]);
    };
    auto load_bd = [&](int p, float2 *bh_, float2 *dh_) {
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
    };

    // psi^(l+1) planes v-1 .. k1 feed psi^(l+2) on k0 .. k1-1
    const int vb0 = (pz(k0 - 1) >= 0) ? k0 - 1 : k0;
    const int ve = k1;  // last step (psi^(l+1) only if that plane exists)

    float2 am[R], ac[R], an[R];  // psi^(l) own: planes v-1, v, v+1
    float2 b2[R], b1[R];         // psi^(l+1) own: planes v-2, v-1
    float2 bhc[R], dhc[R];       // b/M, (ht/2)/M of plane v
    float2 bhq[R], dhq[R];       // ... of plane v-1
    own_plane(pz(vb0 - 1), am);
    own_plane(pz(vb0), ac);
    own_plane(pz(vb0 + 1), an);
    load_bd(pz(vb0), bhc, dhc);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        b2[r] = b1[r] = make_float2(0.f, 0.f);
        bhq[r] = make_float2(0.f, 0.f);
        dhq[r] = make_float2(1.f, 0.f);
    }
    {
        const int p = pz(vb0);
        if (p >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) la[vb0 & 1][1 + w * R + r][1 + lane] = ac[r];
            if (hthr) la[vb0 & 1][hly][hlx] = fetch(src, Pt, (unsigned)p * NXY, p, nx, hs);
        }
    }
    float2 hv = make_float2(0.f, 0.f);
    if (hthr && pz(vb0 + 1) >= 0) hv = fetch(src, Pt, (unsigned)pz(vb0 + 1) * NXY, pz(vb0 + 1), nx, hs);

    float rmax1 = 0.f, rmax2 = 0.f;
    for (int v = vb0; v <= ve; ++v) {
        const int p = pz(v);
        const bool stageA = (p >= 0) && v <= k1;
        const bool stageB = (v - 1 >= k0) && (v - 1 < k1);
        const int pn1 = pz(v + 1), pn2 = pz(v + 2);
        // next planes' loads, issued before the barrier
        float2 ann[R], bhn[R], dhn[R];
        float2 hvn = make_float2(0.f, 0.f);
        own_plane(v + 2 <= k1 + 1 ? pn2 : -1, ann);
        load_bd(v + 1 <= k1 ? pn1 : -1, bhn, dhn);
        if (hthr && v + 2 <= k1 && pn2 >= 0) hvn = fetch(src, Pt, (unsigned)pn2 * NXY, pn2, nx, hs);
        __syncthreads();  // la[v] and lb[v - 1] complete; the other buffers are free
        if (v + 1 <= k1 && pn1 >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) la[(v + 1) & 1][1 + w * R + r][1 + lane] = an[r];
            if (hthr) la[(v + 1) & 1][hly][hlx] = hv;
        }
        float2 b0[R];
        if (stageA) {
            // psi^(l+1) on plane v: own nodes from LDS ...
            const int lb_ = v & 1;
            const bool zm = (p > 0) || zper, zp = (p < nz - 1) || zper;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int ly = 1 + w * R + r;
                const float2 xm = la[lb_][ly][lane], xp = la[lb_][ly][lane + 2];
                const float2 ym = la[lb_][ly - 1][lane + 1], yp = la[lb_][ly + 1][lane + 1];
                if (vy[r]) {
                    const float2 ns = nsum(ux[r], uz[r], xm, xp, ym, yp, am[r], an[r], zm, zp, cx, cy, cz);
                    b0[r] = jacobi(bhc[r], dhc[r], ns);
                    const float r2 = resid2(b0[r], ac[r], dhc[r], ht2);
                    rmax1 = (r2 > rmax1 || r2 != r2) ? r2 : rmax1;
                } else {
                    // a node outside the grid in a ragged tile: its ghost value
                    b0[r] = slot_update(I, src, Pt, bhp, dhp, own[r], p, NXY, zper);
                }
                lb[lb_][ly][1 + lane] = b0[r];
            }
            // ... and the ring from the source nodes' updates
            if (hthr) lb[lb_][hly][hlx] = slot_update(I, src, Pt, bhp, dhp, hs, p, NXY, zper);
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
                const float2 xm = lb[lq][ly][lane], xp = lb[lq][ly][lane + 2];
                const float2 ym = lb[lq][ly - 1][lane + 1], yp = lb[lq][ly + 1][lane + 1];
                if (!vy[r]) continue;
                const float2 ns = nsum(ux[r], uz[r], xm, xp, ym, yp, b2[r], b0[r], zm, zp, cx, cy, cz);
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
            am[r] = ac[r];
            ac[r] = an[r];
            an[r] = ann[r];
            b2[r] = b1[r];
            b1[r] = b0[r];
            bhq[r] = bhc[r];
            dhq[r] = dhc[r];
            bhc[r] = bhn[r];
            dhc[r] = dhn[r];
        }
        hv = hvn;
    }
    if (timing) return;
    __syncthreads();
    wg_max_to<WG>(row_slot(I.res, I.rstride, l, b), rmax1, red);
    if (rec2) {
        __syncthreads();
        wg_max_to<WG>(row_slot(I.res, I.rstride, l + 1, b), rmax2, red);
    }
}

#define TDGL_INST2(R, NT) \
    template __global__ void k_sweep2<R, NT>(const Inst *, const int *, int, int);
TDGL_INST2(1, false)
TDGL_INST2(1, true)
TDGL_INST2(2, false)
TDGL_INST2(2, true)
TDGL_INST2(4, false)
TDGL_INST2(4, true)
#undef TDGL_INST2

}  // namespace tdgl
