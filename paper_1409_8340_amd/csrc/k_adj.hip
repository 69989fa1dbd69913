// k_adj.hip -- kernels of the adjoint (reverse-mode) derivative of the
// time-averaged voltage with respect to eps(r).
//
// One implicit step maps (psi^-, mu^-, K^-) to (psi, mu, K): the
// Crank-Nicolson solve M psi = b of Sec. 3.1, J_av of Sec. 3.1.1, the K
// update of Eq. K_ODE and the Poisson solve of Sec. 3.2.  Its reverse, for a
// real loss L and complex adjoints zbar = dL/dRe z + i dL/dIm z:
//   fbar   = W G(W^-1 mubar)                  (Delta_h is W-self-adjoint)
//   psibar += -i fbar NS(psi) + i W NS(W^-1 fbar psi)
//   Kbar   += sum fbar dIm[psi^* NS psi]/dK,  Ebar = dt Kbar + dL/dE,
//   Jbar = -Ebar,  psibar += -i Jbar T psi / (N hx),  Kbar += Jbar dJ/dK
//   lambda = M^-H psibar, solved as M~ nu = W^-1 psibar with M~ = conj(diag)
//            - (ht/2) NS (the forward Jacobi sweep with other b/M, (ht/2)/M)
//   epsbar += (ht/2) Re[conj(lambda)(psi^- + psi)]
//   mubar^- = (u ht/2) Im[conj(lambda)(psi^- + psi)]
//   Kbar   += (ht/2) Re sum conj(lambda) dNS/dK (psi^- + psi)
//   psibar^- = conj(alpha) lambda + beta conj(lambda) + (ht/2) W L(W^-1 lambda)
// with alpha = 1 + (ht/2)(eps - i u mu^-) - ht |psi^-|^2 - (ht/2) conj(psi^-) psi
// and  beta  = -(ht/2) psi^-^2 - (ht/2) psi^- psi   (|psi^-|^2 psi^- is not
// holomorphic, hence the conj(lambda) term).  Sums over x edges use
// summation by parts so that every K term is a sum over edges (m, m+x).
// The kernels act on instance 0 of a one-instance context; flat kernels use
// a grid-stride loop over the nodes and write per-block partials.
#include "kernels.h"
#include "stencil.h"

namespace tdgl {

__device__ __forceinline__ void node_ijk(const Inst &I, int m, int &i, int &j, int &k) {
    i = m % I.nx;
    const int r = m / I.nx;
    j = r % I.ny;
    k = r / I.ny;
}

__device__ __forceinline__ float node_wm(const Inst &I, int m) {
    int i, j, k;
    node_ijk(I, m, i, j, k);
    return node_w(I, i, j, k);
}

#define FLAT_LOOP(m) \
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < I.N; m += gridDim.x * blockDim.x)

// State save / restore.  raw = 1 (checkpoints): psi, mu as stored and
// dK[0] = K, dK[1] = weighted mean of mu, dK[2] = step counter (it keys the
// Langevin draws), so that a restored step replays bit for bit.  raw = 0 (states the reverse sweep reads): mu with its
// weighted mean removed, as the step uses it, and dK[0] = K.
__global__ void k_adj_save(const Inst *__restrict__ insts, float2 *dpsi, float *dmu, double *dK, int raw) {
    const Inst &I = insts[0];
    const float2 *psi = I.psi[I.st->cur];
    const float mean = raw ? 0.f : (float)I.st->mu_mean;
    FLAT_LOOP(m) {
        dpsi[m] = psi[m];
        dmu[m] = I.mu[m] - mean;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        dK[0] = I.st->K;
        if (raw) {
            dK[1] = I.st->mu_mean;
            dK[2] = I.st->n;  // the step counter keys the Langevin draws of the replay
        }
    }
}

// Restores a raw = 1 save.
__global__ void k_adj_load(const Inst *__restrict__ insts, const float2 *spsi, const float *smu,
                           const double *sK) {
    const Inst &I = insts[0];
    float2 *psi = I.psi[I.st->cur];
    FLAT_LOOP(m) {
        psi[m] = spsi[m];
        I.mu[m] = smu[m];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        I.st->K = sK[0];
        I.st->mu_mean = sK[1];
        I.st->n = sK[2];
    }
}

__global__ void k_adj_logE(const Inst *__restrict__ insts, double *Elog, int n) {
    if (threadIdx.x == 0) Elog[n] = insts[0].st->E_last;
}

// Vbar = (1/W) sum_{n = wb}^{nsteps-1} E_n, summed in step order by one
// thread (the same additions, in the same order, as a sequential host loop).
__global__ void k_adj_vbar(const double *Elog, int wb, int nsteps, double *vbar) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double acc = 0.0;
    for (int n = wb; n < nsteps; ++n) acc += Elog[n];
    *vbar = acc / (double)(nsteps - wb);
}

__global__ void k_adj_zero(AdjState *adj) {
    if (threadIdx.x == 0) { adj->Kbar = 0.0; adj->Jbar = 0.0; adj->scale = 1.0; }
}

// Poisson transpose, right side: f = W^-1 mubar; the iterative solve starts
// from zero so that the result does not depend on what the buffer held.
__global__ void k_adj_prep_f(const Inst *__restrict__ insts, const float *mubar) {
    const Inst &I = insts[0];
    FLAT_LOOP(m) {
        I.f[m] = mubar[m] / node_wm(I, m);
        I.mu[m] = 0.f;
    }
}

// g = W^-1 fbar psi = (mu - mean) psi, with mu the Poisson-transpose output
__global__ void k_adj_g(const Inst *__restrict__ insts, const float2 *psin, float2 *g) {
    const Inst &I = insts[0];
    const float mean = (float)I.st->mu_mean;
    FLAT_LOOP(m) g[m] = cscale(I.mu[m] - mean, psin[m]);
}

// psibar += -i fbar NS(psi) + i W NS(g)
__global__ void k_adj_facc(const Inst *__restrict__ insts, float2 *psibar, const float2 *ns_psi,
                           const float2 *ns_g) {
    const Inst &I = insts[0];
    const float mean = (float)I.st->mu_mean;
    FLAT_LOOP(m) {
        const float w = node_wm(I, m);
        const float fb = w * (I.mu[m] - mean);
        const float2 a = ns_psi[m], c = ns_g[m];
        // -i fb a + i w c
        psibar[m] = cadd(psibar[m], make_float2(fb * a.y - w * c.y, -fb * a.x + w * c.x));
    }
}

// partials of sum_m (fbar_m - fbar_{m+x}) Re[conj(psi_m) U_j psi_{m+x}]  (x periodic)
__global__ __launch_bounds__(256) void k_adj_edge_f(const Inst *__restrict__ insts, const float2 *psin) {
    __shared__ double red[4];
    const Inst &I = insts[0];
    const float mean = (float)I.st->mu_mean;
    double acc = 0.0;
    FLAT_LOOP(m) {
        int i, j, k;
        node_ijk(I, m, i, j, k);
        const int mp = (i == I.nx - 1) ? m - (I.nx - 1) : m + 1;
        const float fb0 = node_w(I, i, j, k) * (I.mu[m] - mean);
        const float fb1 = node_w(I, (i == I.nx - 1) ? 0 : i + 1, j, k) * (I.mu[mp] - mean);
        const float2 up = cmul(xcmul(I.ux[j], I.wz[k]), psin[mp]);
        acc += (double)(fb0 - fb1) * (double)(psin[m].x * up.x + psin[m].y * up.y);
    }
    const double s = wg_sum<256>(acc, red);
    if (threadIdx.x == 0) I.part[blockIdx.x] = s;
}

// psibar += -i Jbar (T psi) / (N hx); partials of sum Re[conj(psi_m) U_j psi_{m+x}]
__global__ __launch_bounds__(256) void k_adj_jterm(const Inst *__restrict__ insts, float2 *psibar,
                                                   const float2 *psin, const AdjState *adj) {
    __shared__ double red[4];
    const Inst &I = insts[0];
    const float c = (float)(-adj->Jbar / ((double)I.N * I.hx));
    double acc = 0.0;
    FLAT_LOOP(m) {
        int i, j, k;
        node_ijk(I, m, i, j, k);
        const int mp = (i == I.nx - 1) ? m - (I.nx - 1) : m + 1;
        const int mm = (i == 0) ? m + (I.nx - 1) : m - 1;
        const float2 u = xcmul(I.ux[j], I.wz[k]);
        const float2 up = cmul(u, psin[mp]);
        const float2 t = csub(up, cmulc(u, psin[mm]));
        // c * (i t)
        psibar[m] = cadd(psibar[m], make_float2(-c * t.y, c * t.x));
        acc += (double)(psin[m].x * up.x + psin[m].y * up.y);
    }
    const double s = wg_sum<256>(acc, red);
    if (threadIdx.x == 0) I.part[blockIdx.x] = s;
}

// partial maxima of |psibar| / w
__global__ __launch_bounds__(256) void k_adj_maxabs(const Inst *__restrict__ insts, const float2 *psibar) {
    __shared__ double red[4];
    const Inst &I = insts[0];
    double mx = 0.0;
    FLAT_LOOP(m) mx = fmax(mx, (double)(sqrtf(cabs2(psibar[m])) / node_wm(I, m)));
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) I.part[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Adjoint system of step n: M~ nu = W^-1 psibar / scale with M from
// (psi^-, mu^-, eps).  Writes b/M~ and (ht/2)/M~.  The solve starts warm
// from the previous reverse steps' solutions: lamW holds scale' nu' of the
// last one (zero before the first) and lamW_old that of the one before, so
// nu^(0) = lamW / scale, or, with extrap, the linear extrapolation
// (2 lamW - lamW_old) / scale in reverse time (about a third fewer sweeps
// at 128 x 128 x 32; the stop rule is unchanged).  No sweep has
// produced that iterate, so it is stored as iterate 1 and convergence row 0
// is marked open (+inf): sweep 1 then measures the residual of nu^(0) and
// the solve proceeds as usual, one iteration index later.
__global__ __launch_bounds__(256) void k_adj_assemble(const Inst *__restrict__ insts, const float2 *psibar,
                                                      const float2 *psim, const float *mum,
                                                      const float2 *lamW, const float2 *lamW_old, int extrap,
                                                      const AdjState *adj) {
    __shared__ float red[4];
    const Inst &I = insts[0];
    const float inv_s = (float)(1.0 / adj->scale);
    const float ht2 = I.ht2, S2 = I.S2, u = I.u;
    float2 *nu1 = I.psi[I.st->cur ^ 1];
    FLAT_LOOP(m) {
        const float2 p = psim[m];
        const float a2 = cabs2(p);
        const float e = I.eps[m], um = u * mum[m];
        // conj(M_mm) with M = 1 + ht/2 (|p|^2 + 2S + i u mu - eps)
        const float2 Mc = make_float2(1.f + ht2 * (a2 + S2 - e), -ht2 * um);
        const float inv = 1.f / cabs2(Mc);
        const float2 Mi = make_float2(Mc.x * inv, -Mc.y * inv);
        const float2 rhs = cscale(inv_s / node_wm(I, m), psibar[m]);
        const float2 bhv = cmul(rhs, Mi), dhv = cscale(ht2, Mi);
        I.bh[m] = bhv;
        I.dh[m] = dhv;
        if (I.edge) {
            // side copies for the two-sweep super-tiles
            const int x = (int)(m % I.nx), t = (int)(m / I.nx);
            int el, er;
            edge_slots(I, x, t % I.ny, t / I.ny, el, er);
            if (el >= 0) {
                I.edge[el] = bhv;
                I.edge[el + 1] = dhv;
            }
            if (er >= 0) {
                I.edge[er] = bhv;
                I.edge[er + 1] = dhv;
            }
        }
        const float2 w0 = lamW[m];
        float2 g = w0;
        if (extrap) {
            const float2 w1 = lamW_old[m];
            g = make_float2(2.f * w0.x - w1.x, 2.f * w0.y - w1.y);
        }
        nu1[m] = cscale(inv_s, g);
    }
    wg_max_to<256>(row_slot(I.res, I.rstride, 0, blockIdx.x), __int_as_float(0x7f800000), red);
}

// lamW = lambda / W = scale * nu (also the next reverse step's warm start)
__global__ void k_adj_scale_nu(const Inst *__restrict__ insts, const AdjState *adj, float2 *tmp) {
    const Inst &I = insts[0];
    const float s = (float)adj->scale;
    const float2 *nu = I.psi[I.st->cur];
    FLAT_LOOP(m) tmp[m] = cscale(s, nu[m]);
}

// epsbar, mubar^- and psibar^- from lambda = W scale nu.
__global__ void k_adj_sources(const Inst *__restrict__ insts, float2 *psibar, float *mubar, float *epsbar,
                              const float2 *psim, const float2 *psin, const float *mum,
                              const float2 *ns_l, const AdjState *adj) {
    const Inst &I = insts[0];
    const float s = (float)adj->scale;
    const float ht2 = I.ht2, u = I.u, S2 = I.S2;
    const float2 *nu = I.psi[I.st->cur];
    FLAT_LOOP(m) {
        const float w = node_wm(I, m);
        const float2 lam = cscale(w * s, nu[m]);
        const float2 p = psim[m], q = psin[m];
        const float2 sm = cadd(p, q);
        const float2 cl_s = cmulc(lam, sm);  // conj(lambda) * (psi^- + psi)
        epsbar[m] += ht2 * cl_s.x;
        mubar[m] = u * ht2 * cl_s.y;
        const float a2 = cabs2(p);
        const float e = I.eps[m], um = u * mum[m];
        // alpha = 1 + ht/2 (eps - i u mu) - ht |p|^2 - ht/2 conj(p) q
        const float2 cpq = cmulc(p, q);
        const float2 alpha = make_float2(1.f + ht2 * e - 2.f * ht2 * a2 - ht2 * cpq.x, -ht2 * um - ht2 * cpq.y);
        // beta = -ht/2 p^2 - ht/2 p q
        const float2 p2 = cmul(p, p), pq = cmul(p, q);
        const float2 beta = make_float2(-ht2 * (p2.x + pq.x), -ht2 * (p2.y + pq.y));
        const float2 t1 = cmulc(alpha, lam);                                  // conj(alpha) lambda
        const float2 t2 = cmul(beta, make_float2(lam.x, -lam.y));             // beta conj(lambda)
        const float2 lh = make_float2(w * ns_l[m].x - S2 * lam.x, w * ns_l[m].y - S2 * lam.y);
        psibar[m] = make_float2(t1.x + t2.x + ht2 * lh.x, t1.y + t2.y + ht2 * lh.y);
    }
}

// partials of Re[i sum_m (conj(lambda_m) U_j s_{m+x} - conj(lambda_{m+x} U_j) s_m)],
// s = psi^- + psi
__global__ __launch_bounds__(256) void k_adj_edge_s(const Inst *__restrict__ insts, const float2 *psim,
                                                    const float2 *psin, const AdjState *adj) {
    __shared__ double red[4];
    const Inst &I = insts[0];
    const float sc = (float)adj->scale;
    const float2 *nu = I.psi[I.st->cur];
    double acc = 0.0;
    FLAT_LOOP(m) {
        int i, j, k;
        node_ijk(I, m, i, j, k);
        const int ip = (i == I.nx - 1) ? 0 : i + 1;
        const int mp = (i == I.nx - 1) ? m - (I.nx - 1) : m + 1;
        const float2 l0 = cscale(node_w(I, i, j, k) * sc, nu[m]);
        const float2 l1 = cscale(node_w(I, ip, j, k) * sc, nu[mp]);
        const float2 u = xcmul(I.ux[j], I.wz[k]);
        const float2 s0 = cadd(psim[m], psin[m]), s1 = cadd(psim[mp], psin[mp]);
        const float2 a = cmulc(l0, cmul(u, s1));   // conj(lambda_m) U s_{m+x}
        const float2 bb = cmulc(cmul(l1, u), s0);  // conj(lambda_{m+x} U) s_m
        // Re[i (a - bb)] = -(a - bb).y
        acc += -(double)(a.y - bb.y);
    }
    const double s = wg_sum<256>(acc, red);
    if (threadIdx.x == 0) I.part[blockIdx.x] = s;
}

// Combine the partials of one flat kernel into the adjoint scalars.
//   which 0: Kbar += S / hx; then Jbar = -(dt Kbar + ew)
//   which 1: Kbar += Jbar S / N
//   which 2: Kbar += (ht/2) S / hx
//   which 3: scale = max partial (1 when zero)
__global__ __launch_bounds__(256) void k_adj_reduce(const Inst *__restrict__ insts, int nparts, int which,
                                                    double ew, AdjState *adj) {
    __shared__ double red[4];
    const Inst &I = insts[0];
    if (which == 3) {
        double mx = 0.0;
        for (int t = threadIdx.x; t < nparts; t += blockDim.x) mx = fmax(mx, I.part[t]);
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
        __syncthreads();
        if (threadIdx.x == 0) {
            const double s = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
            adj->scale = s > 0.0 ? s : 1.0;
        }
        return;
    }
    double a = 0.0;
    for (int t = threadIdx.x; t < nparts; t += blockDim.x) a += I.part[t];
    const double S = wg_sum<256>(a, red);
    if (threadIdx.x == 0) {
        if (which == 0) {
            adj->Kbar += S / I.hx;
            adj->Jbar = -(I.dt * adj->Kbar + ew);
        } else if (which == 1) {
            adj->Kbar += adj->Jbar * S / (double)I.N;
        } else {
            adj->Kbar += (double)I.ht2 * S / I.hx;
        }
    }
}

#undef FLAT_LOOP

}  // namespace tdgl
