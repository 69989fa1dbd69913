// stencil.h -- device helpers shared by the stencil kernels (k_gl.hip,
// k_gl2.hip): global-address-space vector loads and stores, the boundary
// description of a halo slot and the halo-slot mapping of a tile.
#pragma once
#include "kernels.h"

namespace tdgl {

// Global-address-space views: pointers read out of the descriptor are
// generic, which would make every access a FLAT instruction.  A FLAT load
// also counts against the LDS wait counter, so a kernel that mixes LDS or
// cross-lane operations with FLAT loads in flight waits for the loads at
// every LDS wait; through these views the loads are global instructions.
// Complex values move as native two-float vectors.
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) v2f gf2;
typedef __attribute__((address_space(1))) float gf1;
typedef __attribute__((address_space(1))) double gd1;
__device__ __forceinline__ float2 ld2(const gf2 *p, unsigned i) {
    const v2f v = p[i];
    return make_float2(v.x, v.y);
}
// Streams read or written once per pass (b/M, (ht/2)/M, eps, mu, the new
// iterate) can bypass the caches' retention with non-temporal hints, so that
// L2 keeps the psi rows the neighbouring tiles re-read as halos.  That pays
// when the arrays do not fit the last-level cache; for grids that stay
// cache-resident between sweeps the hints cost time, so they are a template
// option (NT) chosen per context.
__device__ __forceinline__ float2 ld2nt(const gf2 *p, unsigned i) {
    const v2f v = __builtin_nontemporal_load(&p[i]);
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void st2nt(gf2 *p, unsigned i, float2 a) {
    v2f v;
    v.x = a.x;
    v.y = a.y;
    __builtin_nontemporal_store(v, &p[i]);
}
__device__ __forceinline__ void st2(gf2 *p, unsigned i, float2 a) {
    v2f v;
    v.x = a.x;
    v.y = a.y;
    p[i] = v;
}
// Two complex values at p[i], p[i + 1] (i even, p 16-byte aligned) as one
// 16-byte global store.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) v4f gf4;
__device__ __forceinline__ void st4(float2 *p, unsigned i, float2 a, float2 b) {
    v4f v;
    v.x = a.x;
    v.y = a.y;
    v.z = b.x;
    v.w = b.y;
    ((gf4 *)p)[i >> 1] = v;
}

// The Jacobi update below is written with explicit fused multiply-adds and
// with contraction of the remaining products and sums switched off, so that
// no compiler contraction choice -- which can differ between the places the
// code is inlined into -- changes a bit: every kernel that recomputes a value
// (the two-sweep kernel's ring) gets the same one.
__device__ __forceinline__ float2 xcmul(float2 a, float2 b) {  // a b
#pragma clang fp contract(off)
    return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 xcmulc(float2 a, float2 b) {  // conj(a) b
#pragma clang fp contract(off)
    return make_float2(__builtin_fmaf(a.x, b.x, a.y * b.y), __builtin_fmaf(a.x, b.y, -(a.y * b.x)));
}
__device__ __forceinline__ float2 xcadd(float2 a, float2 b) {
#pragma clang fp contract(off)
    return make_float2(a.x + b.x, a.y + b.y);
}

// Where the value of one LDS slot comes from in every plane.  The slot at
// (gx, gy), gx in [-1, nx], gy in [-1, ny], holds psi as the 7-point stencil
// sees it: interior nodes are loaded; one-cell ghosts follow the boundary
// rules of Sec. 3.3 -- plain wrap on a periodic x axis, the quasi-periodic
// phase jump psi_{i,-1,k} = P_{i,k} psi_{i,ny-1,k} (and psi_{i,ny,k} =
// P*_{i,k} psi_{i,0,k}) on a periodic y axis, and the Neumann ghost
// U^* psi_{-1} = U psi_1 on an open face.  Corners and slots beyond a ragged
// tile are zero.  The description does not depend on the plane, so it is
// computed once per thread.
enum { SRC_PLAIN = 0, SRC_P = 1, SRC_PCONJ = 2, SRC_FAC = 3, SRC_ZERO = 4 };
struct CellSrc {
    int off;      // element offset within a plane
    int mode;
    int px;       // x index of the phase P_{px,k}; SRC_FAC: 0 at x = -1, 1 at x = nx
    float2 fac;   // constant factor (open-x ghost)
};

__device__ __forceinline__ CellSrc cell_src(const Inst &I, int gx, int gy) {
    const int nx = I.nx, ny = I.ny;
    const bool xin = (unsigned)gx < (unsigned)nx, yin = (unsigned)gy < (unsigned)ny;
    CellSrc s{0, SRC_ZERO, 0, make_float2(1.f, 0.f)};
    if (xin && yin) { s.off = gy * nx + gx; s.mode = SRC_PLAIN; return s; }
    if (xin) {
        if (gy == -1) {
            if (I.per[1]) { s.off = (ny - 1) * nx + gx; s.mode = SRC_P; s.px = gx; }
            else if (ny >= 2) { s.off = nx + gx; s.mode = SRC_PLAIN; }
        } else if (gy == ny) {
            if (I.per[1]) { s.off = gx; s.mode = SRC_PCONJ; s.px = gx; }
            else if (ny >= 2) { s.off = (ny - 2) * nx + gx; s.mode = SRC_PLAIN; }
        }
        return s;
    }
    if (yin) {
        const float2 u = I.ux[gy];
        if (gx == -1) {
            if (I.per[0]) { s.off = gy * nx + nx - 1; s.mode = SRC_PLAIN; }
            else if (nx >= 2) { s.off = gy * nx + 1; s.mode = SRC_FAC; s.fac = xcmul(u, u); }
        } else if (gx == nx) {
            if (I.per[0]) { s.off = gy * nx; s.mode = SRC_PLAIN; }
            else if (nx >= 2) {
                const float2 u2 = xcmul(u, u);
                s.off = gy * nx + nx - 2; s.mode = SRC_FAC; s.fac = make_float2(u2.x, -u2.y); s.px = 1;
            }
        }
    }
    return s;
}

// YZ: the x link of plane k carries the factor wz[k] (yz-plane field), so
// the open-x ghost factor U^2 (or its conjugate) gains wz[k]^2.
template <bool YZ = false>
__device__ __forceinline__ float2 fetch(const gf2 *__restrict__ src, const gf2 *__restrict__ P,
                                        unsigned pbase, int k, int nx, const CellSrc &s,
                                        const float2 *__restrict__ wz = nullptr) {
    if (s.mode == SRC_PLAIN) return ld2(src, pbase + (unsigned)s.off);
    if (s.mode == SRC_ZERO) return make_float2(0.f, 0.f);
    const float2 v = ld2(src, pbase + (unsigned)s.off);
    if (s.mode == SRC_FAC) {
        if (YZ) {
            float2 w2 = xcmul(wz[k], wz[k]);
            if (s.px) w2.y = -w2.y;
            return xcmul(xcmul(s.fac, w2), v);
        }
        return xcmul(s.fac, v);
    }
    const float2 ph = ld2(P, (unsigned)k * nx + s.px);
    return s.mode == SRC_P ? xcmul(ph, v) : xcmulc(ph, v);
}

// Like cell_src, for slots up to two nodes outside the grid and the corners
// of the one-node ring, as the two-sweep kernel's two-node halo needs them:
// each axis maps on its own (periodic: wrap at any distance, the y wrap
// with its phase P; open: the Neumann mirror at distance one, nothing
// beyond).  A corner that would need both an x mirror and a y ghost is
// never read and is left ZERO.  On the slots cell_src covers, both agree.
__device__ __forceinline__ CellSrc cell_src2(const Inst &I, int gx, int gy) {
    const int nx = I.nx, ny = I.ny;
    CellSrc s{0, SRC_ZERO, 0, make_float2(1.f, 0.f)};
    int sx = gx, sy = gy, xmir = 0, ymode = SRC_PLAIN;
    if (gx < 0 || gx >= nx) {
        if (I.per[0]) sx = ((gx % nx) + nx) % nx;
        else if (nx >= 2 && gx == -1) { sx = 1; xmir = -1; }
        else if (nx >= 2 && gx == nx) { sx = nx - 2; xmir = 1; }
        else return s;
    }
    if (gy < 0 || gy >= ny) {
        if (xmir) return s;
        if (I.per[1]) { sy = ((gy % ny) + ny) % ny; ymode = gy < 0 ? SRC_P : SRC_PCONJ; }
        else if (ny >= 2 && gy == -1) sy = 1;
        else if (ny >= 2 && gy == ny) sy = ny - 2;
        else return s;
    }
    s.off = sy * nx + sx;
    if (xmir) {
        const float2 u2 = xcmul(I.ux[sy], I.ux[sy]);
        s.mode = SRC_FAC;
        s.fac = xmir < 0 ? u2 : make_float2(u2.x, -u2.y);
        s.px = xmir > 0 ? 1 : 0;
    } else if (ymode != SRC_PLAIN) {
        s.mode = ymode;
        s.px = sx;
    } else {
        s.mode = SRC_PLAIN;
    }
    return s;
}

// z neighbour plane index of plane p in direction d (+1/-1), or -1 if none.
__device__ __forceinline__ int zplane(const Inst &I, int p, int d) {
    int q = p + d;
    if (q >= 0 && q < I.nz) return q;
    if (!I.per[2]) return -1;
    return q < 0 ? I.nz - 1 : 0;
}

// Halo cell handled by thread t (t < 2 TX + 2 TYv) of a TX x TYv tile at
// (x0, y0): rows y0-1 and y0+TYv (TX cells each), columns x0-1 and x0+TX.
template <int TYv>
__device__ __forceinline__ void halo_cell(int t, int x0, int y0, int &gx, int &gy, int &lx, int &ly) {
    if (t < TX) { gx = x0 + t; gy = y0 - 1; lx = t + 1; ly = 0; }
    else if (t < 2 * TX) { gx = x0 + t - TX; gy = y0 + TYv; lx = t - TX + 1; ly = TYv + 1; }
    else if (t < 2 * TX + TYv) { gx = x0 - 1; gy = y0 + t - 2 * TX; lx = 0; ly = t - 2 * TX + 1; }
    else { gx = x0 + TX; gy = y0 + t - 2 * TX - TYv; lx = TX + 1; ly = t - 2 * TX - TYv + 1; }
}

// Off-diagonal neighbour sum NS of the covariant Laplacian at one node
// (Eq. LaplUV_xz): x and z links of the node's row, in-plane neighbours as
// the stencil sees them (ghosts by the boundary rules), z neighbours with
// the open-face doubling (zm / zp: whether the plane below / above exists).
// Every stencil kernel goes through this one function.
__device__ __forceinline__ float2 nsum(float2 ux, float2 uz, float2 xm, float2 xp, float2 ym, float2 yp,
                                       float2 zmv, float2 zpv, bool zm, bool zp, float cx, float cy, float cz) {
#pragma clang fp contract(off)
    float2 zt;
    if (zm && zp) {
        zt = xcadd(xcmul(uz, zpv), xcmulc(uz, zmv));
    } else if (zp) {
        zt = xcmul(uz, zpv);
        zt = make_float2(2.f * zt.x, 2.f * zt.y);
    } else if (zm) {
        zt = xcmulc(uz, zmv);
        zt = make_float2(2.f * zt.x, 2.f * zt.y);
    } else {
        zt = make_float2(0.f, 0.f);
    }
    const float2 xt = xcadd(xcmul(ux, xp), xcmulc(ux, xm));
    const float2 yt = xcadd(yp, ym);
    return make_float2(__builtin_fmaf(cx, xt.x, __builtin_fmaf(cy, yt.x, cz * zt.x)),
                       __builtin_fmaf(cx, xt.y, __builtin_fmaf(cy, yt.y, cz * zt.y)));
}

// One Jacobi iterate (Eq. final): b/M + (ht/2)/M * NS.
__device__ __forceinline__ float2 jacobi(float2 bh, float2 dh, float2 ns) { return xcadd(bh, xcmul(dh, ns)); }

// |r|^2 of the iterate's input, r = M (new - old), |M|^2 = (ht/2)^2 / |(ht/2)/M|^2.
// The quotient uses the hardware reciprocal (1 ulp) instead of an IEEE
// division: the value only meets the stop threshold and the reported
// residual, and the division was a tenth of the hot loop's instructions.
__device__ __forceinline__ float resid2(float2 nw, float2 old, float2 dh, float ht2) {
#pragma clang fp contract(off)
    const float dx = nw.x - old.x, dy = nw.y - old.y;
    const float d2 = __builtin_fmaf(dx, dx, dy * dy);
    const float m2 = __builtin_fmaf(dh.x, dh.x, dh.y * dh.y);
    return (d2 * (ht2 * ht2)) * __builtin_amdgcn_rcpf(m2);
}

// Assemble at one node (Eq. GL_linearized, Eq. b, with |psi|^2 lagged):
//   b   = psi^- + ht/2 [ (eps - i u mu) psi^- - |psi^-|^2 psi^- + L psi^- + 2 zeta ]
//   M   = 1 + ht/2 [ |psi^-|^2 + 2S + i u mu - eps ]
// returns b/M, (ht/2)/M, the first iterate b/M + (ht/2)/M NS(psi^-) and
// |r|^2 of psi^(0) = psi^-.  Contraction-proof like jacobi(), so that every
// tiling of the grid gives the same bits.
__device__ __forceinline__ void assemble_node(float2 c, float e, float um, float2 ns, float S2, float ht2,
                                              bool noise, float2 zz, float2 &bhv, float2 &dhv, float2 &nw,
                                              float &r2) {
#pragma clang fp contract(off)
    const float a2 = __builtin_fmaf(c.x, c.x, c.y * c.y);
    const float2 lap = make_float2(__builtin_fmaf(-S2, c.x, ns.x), __builtin_fmaf(-S2, c.y, ns.y));
    const float ea = e - a2;
    float2 st = make_float2(__builtin_fmaf(ea, c.x, __builtin_fmaf(um, c.y, lap.x)),
                            __builtin_fmaf(ea, c.y, __builtin_fmaf(-um, c.x, lap.y)));
    if (noise) st = make_float2(st.x + zz.x, st.y + zz.y);  // + 2 zeta (Eq. b)
    const float2 bb = make_float2(__builtin_fmaf(ht2, st.x, c.x), __builtin_fmaf(ht2, st.y, c.y));
    const float2 M = make_float2(__builtin_fmaf(ht2, (a2 + S2) - e, 1.f), ht2 * um);
    const float m2 = __builtin_fmaf(M.x, M.x, M.y * M.y);
    const float inv = 1.f / m2;
    const float2 Mi = make_float2(M.x * inv, -(M.y * inv));
    bhv = xcmul(bb, Mi);
    dhv = make_float2(ht2 * Mi.x, ht2 * Mi.y);
    nw = jacobi(bhv, dhv, ns);
    const float dx = nw.x - c.x, dy = nw.y - c.y;
    r2 = m2 * __builtin_fmaf(dx, dx, dy * dy);
}

// Right side of the Poisson equation at one node: Im[psi^* NS(psi)].
__device__ __forceinline__ float rhs_node(float2 c, float2 ns) {
#pragma clang fp contract(off)
    return __builtin_fmaf(c.x, ns.y, -(c.y * ns.x));
}

}  // namespace tdgl
