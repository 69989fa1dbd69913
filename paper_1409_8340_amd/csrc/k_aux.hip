// k_aux.hip -- link tables, reductions, the K update and small state
// kernels of libtdgl.
#include "kernels.h"
#include "stencil.h"

namespace tdgl {

// exp(i phi) in double precision with the argument reduced to [-pi, pi]
// first, rounded to complex64.
__device__ __forceinline__ float2 expi(double phi) {
    const double twopi = 6.283185307179586476925286766559;
    phi -= twopi * rint(phi / twopi);
    double s, c;
    sincos(phi, &s, &c);
    return make_float2((float)c, (float)s);
}

// y offset of the x links: ybar_j = j hy - y_ref with y_ref = Ly/2 for the
// xz-plane field (Eq. A_xz) and 0 for the yz-plane field (see k_links).
__device__ __forceinline__ double link_yref(const Inst &I, const DevState *st) {
    const double Ly = I.per[1] ? I.ny * I.hy : (I.ny - 1) * I.hy;
    return st->yz ? 0.0 : 0.5 * Ly;
}

// Link tables of one instance.  xz-plane field, Landau gauge (Eq. A_xz,
// Eq. link_variables, Sec. 3.3.1):
//   ux[j] = exp(+i hx (K + Bz ybar_j)),  uz[j] = exp(-i hz Bx ybar_j),
//   P[k*nx + i] = exp(i (i hx Ly Bz - k hz Ly Bx)),  wz[k] = 1,
// with ybar_j = j hy - Ly/2 and Ly the system size along y.
// yz-plane field (Eq. B_yz): the vector potential A = (-y Bz + z By, 0, 0)
// (curl A = (0, By, Bz)), which puts the whole field on the x links:
//   ux[j] = exp(+i hx (K + Bz j hy)),  wz[k] = exp(-i hx By k hz),
//   uz[j] = 1,  P[k*nx + i] = exp(i xbar_i Ly Bz),  xbar_i = i hx - Lx/2,
// so the x link of node (i, j, k) is ux[j] wz[k].  It differs from the
// paper's gauge of Eq. A_yz by the gauge transformation
//   psi_paper = exp(i (j hy Bz - k hz By) xbar_i) psi
// (same flux through every plaquette and the same phase around every
// periodic loop; z must be open when By != 0).
// One work-group per instance (grid = ninst); `which` = 1 refreshes ux only.
// Kp (the adjoint's replay): K = *Kp is stored in the state first and the
// links are those at it.
__global__ void k_links(const Inst *__restrict__ insts, int which, const double *Kp) {
    const Inst &I = insts[blockIdx.x];
    DevState *st = I.st;
    const double Ly = I.per[1] ? I.ny * I.hy : (I.ny - 1) * I.hy;
    const double Lx = I.per[0] ? I.nx * I.hx : (I.nx - 1) * I.hx;
    const double Kn = Kp ? *Kp : st->K;
    if (Kp && threadIdx.x == 0) st->K = Kn;
    const double K = I.driven ? Kn : 0.0, Bx = st->Bx, Bz = st->Bz, By = st->By;
    const bool yz = st->yz != 0;
    const double yref = link_yref(I, st);
    for (int j = threadIdx.x; j < I.ny; j += blockDim.x) {
        const double yb = j * I.hy - yref;
        I.ux[j] = expi(I.hx * (K + Bz * yb));
        if (which == 0) I.uz[j] = yz ? make_float2(1.f, 0.f) : expi(-I.hz * Bx * yb);
    }
    if (which == 0) {
        for (int k = threadIdx.x; k < I.nz; k += blockDim.x)
            I.wz[k] = yz ? expi(-I.hx * By * (k * I.hz)) : make_float2(1.f, 0.f);
        // the z wrap of a yz field on a periodic z axis: A_x grows by Lz By
        // across it, a gauge shift by xbar Lz By (xbar = i hx - Lx/2)
        const double Lz = I.nz * I.hz;
        const bool zseam = yz && I.per[2] && By != 0.0;
        for (int i = threadIdx.x; i < I.nx; i += blockDim.x)
            I.zs[i] = zseam ? expi(-(i * I.hx - 0.5 * Lx) * Lz * By) : make_float2(1.f, 0.f);
        const long n = (long)I.nx * I.nz;
        for (long t = threadIdx.x; t < n; t += blockDim.x) {
            const int i = (int)(t % I.nx), k = (int)(t / I.nx);
            I.P[t] = yz ? expi((i * I.hx - 0.5 * Lx) * Ly * Bz) : expi(i * I.hx * Ly * Bz - k * I.hz * Ly * Bx);
        }
    }
}

// End of a Jacobi solve: the first sweep l whose input residual met tol ends
// the solve with that sweep's output (Eq. convergence); otherwise the cap,
// which is the instance's max_iter or the nl sweeps launched, whichever is
// smaller.  fused: 0 -- single sweeps; 1 -- the sweeps after the first ran
// as two-sweep passes from l = 1; 2 -- one single sweep (l = 1), then
// two-sweep passes from l = 2.
// Updates the psi buffer index and step counters and clears the residual
// words for the next step.
__global__ __launch_bounds__(FIN_THREADS) void k_solve_finalize(const Inst *__restrict__ insts, int ninst,
                                                                  int count_step, int nl, int fused,
                                                                  unsigned long long *pub, unsigned seq) {
    // one work-group per instance: the first wavefront scans the rows, then
    // all threads clear them.  pub (host-driven solves): the iteration count
    // and the last tested residual go to the host at pub[ii] and
    // pub[ninst + ii], tagged seq.
    const int ii = blockIdx.x;
    if (ii >= ninst) return;
    const Inst &I = insts[ii];
    DevState *st = I.st;
    if (threadIdx.x < 64) {
        const int cap = min(I.max_iter, nl);
        int sweeps = cap, capped = 1;
        float last = 0.f;
        for (int l = 0; l < cap; ++l) {
            last = row_max_wave(I.res, I.rstride, l);
            if (last < I.tol) { sweeps = l + 1; capped = 0; break; }
        }
        if (threadIdx.x == 0) {
            st->sweeps = sweeps;
            st->capped = capped;
            if (!fused) {
                st->cur ^= (sweeps & 1);
                st->fix = 0;
            } else {
                // the iterates the passes store: psi^(1) and, from the
                // pairs, those of the parity of the pairs' end (odd from
                // l = 1, even from l = 2), psi^(s) in cur ^ pair_src(s) --
                // a pair's output is the next pair's input; any other s is
                // recomputed from psi^(s-1) into the other buffer by the
                // corrective sweep
                const int ps = (fused == 1) ? 1 : 0;  // parity of the stored iterates
                const bool stored = (sweeps == 1) || ((sweeps & 1) == ps);
                const int so = stored ? sweeps : sweeps - 1;
                const int bo = st->cur ^ (so == 1 ? 1 : pair_src(so));
                st->fix = stored ? 0 : 1;
                st->cur = stored ? bo : (bo ^ 1);
            }
            if (count_step) {
                st->t += I.dt;
                st->n += 1.0;
                st->acc_sweeps += sweeps;
                st->acc_passes += pass_count(fused, sweeps);
                st->acc_capped += capped;
                st->acc_sw_min = min(st->acc_sw_min, sweeps);
                st->acc_sw_max = max(st->acc_sw_max, sweeps);
            }
            // keep the last tested residual
            st->last_res2 = last;
            if (pub) {
                publish(pub + ii, seq, __int_as_float(sweeps));
                publish(pub + ninst + ii, seq, last);
            }
        }
    }
    __syncthreads();
    // clear the words for the next step
    const int words = I.max_iter * NSLOT;
    for (int w = threadIdx.x; w < words; w += FIN_THREADS) I.res[(size_t)w * I.rstride] = 0u;
}

// Partial sums of Im[psi_m^* U_x(j) psi_{m+x}] (periodic x) for J_av
// (Sec. 3.1.1; the symmetric form of the paper equals twice this one-sided
// sum when x is periodic).  Flat mapping: CPT consecutive cells per thread.
__global__ __launch_bounds__(256) void k_jav_partial(const Inst *__restrict__ insts,
                                                     const int *__restrict__ prefix, int ninst) {
    constexpr int JB = 8;
    __shared__ double red[4];
    __shared__ float2 first[JB][4];  // lane 0 of every wavefront, per cell of a batch
    const int b = blockIdx.x;
    const int ii = find_inst(prefix, ninst, b);
    const Inst &I = insts[ii];
    const int lb = b - prefix[ii];
    const gf2 *__restrict__ psi = (const gf2 *)I.psi[I.st->cur];
    const gf2 *__restrict__ uxg = (const gf2 *)I.ux;
    const gf2 *__restrict__ wzg = (const gf2 *)I.wz;
    double acc = 0.0;
    const int nx = I.nx, ny = I.ny;
    const bool yz = I.st->yz != 0;
    // cells m = base + c 256 + tid, c = 0 .. fcpt-1, summed in that order;
    // their x, y and z indices follow from one division for c = 0 and then
    // by stepping 256 cells at a time.  The 256 threads hold 256
    // consecutive cells, so psi_{m+x} is the next lane's psi_m (a shuffle),
    // the next wavefront's first cell for lane 63 (through LDS), and is
    // loaded only at the end of an x row (the periodic wrap) and for the
    // block's last cell of a batch.  With nx a multiple of 64 a wavefront's
    // cells lie in one row, whose x link it reads once.  Every load of a
    // batch of JB cells is issued before any is used (a cell past the end
    // loads cell 0 and adds nothing).
    static_assert(JAV_CPT % JB == 0 && JAV_CPT_MAX % JB == 0, "whole batches");
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const bool rows64 = (nx & 63) == 0;
    const int cpt = I.fcpt;
    int m = (int)((long)lb * 256 * cpt) + (int)threadIdx.x;
    int i = m % nx, j = (m / nx) % ny, k = m / (nx * ny);
    const int N = (int)I.N;
    for (int c0 = 0; c0 < cpt; c0 += JB) {
        int mq[JB], iq[JB], jq[JB], kq[JB];
#pragma unroll
        for (int q = 0; q < JB; ++q) {
            mq[q] = m;
            iq[q] = i;
            jq[q] = j < ny ? j : 0;
            kq[q] = m < N ? k : 0;
            m += 256;
            i += 256;
            while (i >= nx) {
                i -= nx;
                if (++j == ny) {
                    j = 0;
                    ++k;
                }
            }
        }
        float2 a[JB], nb[JB], u[JB];
#pragma unroll
        for (int q = 0; q < JB; ++q) a[q] = ld2(psi, mq[q] < N ? mq[q] : 0);
        // loaded neighbours: the x wrap, and the cell after the block's last
        // one in the batch's last step
#pragma unroll
        for (int q = 0; q < JB; ++q) {
            const bool wrap = iq[q] == nx - 1;
            const bool own = (wrap || (threadIdx.x == 255 && q == JB - 1)) && mq[q] < N;
            nb[q] = own ? ld2(psi, wrap ? mq[q] - (nx - 1) : mq[q] + 1) : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int q = 0; q < JB; ++q) u[q] = ld2(uxg, rows64 ? __builtin_amdgcn_readfirstlane(jq[q]) : jq[q]);
        if (yz) {
#pragma unroll
            for (int q = 0; q < JB; ++q) u[q] = xcmul(u[q], ld2(wzg, kq[q]));
        }
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < JB; ++q) first[q][w] = a[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < JB; ++q) {
            float2 p;
            p.x = __shfl_down(a[q].x, 1, 64);
            p.y = __shfl_down(a[q].y, 1, 64);
            if (lane == 63) {
                // the next wavefront's first cell; after wavefront 3, the
                // first cell of the next step (loaded for the last step)
                if (w < 3) p = first[q][w + 1];
                else if (q < JB - 1) p = first[q + 1][0];
                else p = nb[q];
            }
            if (iq[q] == nx - 1) p = nb[q];
            if (mq[q] < N) {
                const float2 up = cmul(u[q], p);
                acc += (double)(a[q].x * up.y - a[q].y * up.x);
            }
        }
        __syncthreads();
    }
    const double s = wg_sum<256>(acc, red);
    if (threadIdx.x == 0) I.part[lb] = s;
}

// Deterministic fixed-order sum of `n` partials by one 256-thread work-group.
__device__ double wg_reduce_parts(const double *__restrict__ part, int n, double *red) {
    // each thread sums its partials t, t + 256, ... in that order, with
    // eight loads in flight before they are added
    constexpr int B = 8;
    double a = 0.0;
    int t = threadIdx.x;
    for (; t + (B - 1) * 256 < n; t += B * 256) {
        double v[B];
#pragma unroll
        for (int c = 0; c < B; ++c) v[c] = part[t + c * 256];
#pragma unroll
        for (int c = 0; c < B; ++c) a += v[c];
    }
    for (; t < n; t += 256) a += part[t];
    return wg_sum<256>(a, red);
}

// K update (Eq. K_ODE with dA/dt = 0, explicit Euler in real time dt):
//   J_av = sum / (N hx), E = J_ext - J_av, K += dt E, V_sum += E,
//   K -> K - (2 pi / hx) floor(K hx / 2 pi)  (phase rewind, Sec. 2.2),
// then the x-link table is rebuilt for the new K.  One work-group per
// instance; undriven instances are left alone.
__global__ __launch_bounds__(256) void k_kupdate(const Inst *__restrict__ insts,
                                                 const int *__restrict__ nparts) {
    __shared__ double red[4];
    __shared__ double Ks;
    const Inst &I = insts[blockIdx.x];
    if (!I.driven) return;
    DevState *st = I.st;
    const double s = wg_reduce_parts(I.part, nparts[blockIdx.x], red);
    if (threadIdx.x == 0) {
        const double twopi = 6.283185307179586476925286766559;
        const double J = s / ((double)I.N * I.hx);
        const double E = st->Jext - J;
        double K = st->K + I.dt * E;
        if (st->in_window) { st->V_sum += E; st->n_avg += 1.0; }
        K = K - (twopi / I.hx) * floor(K * I.hx / twopi);
        st->K = K;
        st->E_last = E;
        st->J_last = J;
        Ks = K;
    }
    __syncthreads();
    const double yref = link_yref(I, st);
    for (int j = threadIdx.x; j < I.ny; j += blockDim.x) {
        const double yb = j * I.hy - yref;
        I.ux[j] = expi(I.hx * (Ks + st->Bz * yb));
    }
}

// Reduce an instance's partials into a DevState field: dst = scale * sum.
// field: 0 = f_mean (from node-weighted sums), 1 = mu_mean, 2 = F,
// 3 = psi2 (mean |psi|^2), 4 = f_mean (from volume-weighted sums).
__global__ __launch_bounds__(256) void k_reduce_to_state(const Inst *__restrict__ insts,
                                                         const int *__restrict__ nparts, int field,
                                                         int driven_only) {
    __shared__ double red[4];
    const Inst &I = insts[blockIdx.x];
    if (driven_only && !I.driven) return;
    const double s = wg_reduce_parts(I.part, nparts[blockIdx.x], red);
    if (threadIdx.x == 0) {
        DevState *st = I.st;
        if (field == 0) st->f_mean = s / I.w_sum;
        else if (field == 1) st->mu_mean = s / I.lev[0].vsum;
        else if (field == 4) st->f_mean = s / I.lev[0].vsum;
        else if (field == 2) st->F = s * I.hx * I.hy * I.hz;
        else st->psi2 = s / (double)I.N;
    }
}

// Partial sums of |psi|^2 (flat mapping).
__global__ __launch_bounds__(256) void k_psi2_partial(const Inst *__restrict__ insts,
                                                      const int *__restrict__ prefix, int ninst) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    const int ii = find_inst(prefix, ninst, b);
    const Inst &I = insts[ii];
    const int lb = b - prefix[ii];
    const float2 *__restrict__ psi = I.psi[I.st->cur];
    double acc = 0.0;
    const long base = (long)lb * 256 * I.fcpt;
    for (int c = 0; c < I.fcpt; ++c) {
        const long m = base + (long)c * 256 + threadIdx.x;
        if (m < I.N) acc += (double)cabs2(psi[m]);
    }
    const double s = wg_sum<256>(acc, red);
    if (threadIdx.x == 0) I.part[lb] = s;
}

// ---------------------------------------------------------------------------
// state and copy helpers
__global__ void k_fill_c(float2 *p, long n, float re, float im) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        p[i] = make_float2(re, im);
}
__global__ void k_fill_f(float *p, long n, float v) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u(unsigned *p, long n, unsigned v) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        p[i] = v;
}

// psi in/out through the current buffer index (known only on the device).
__global__ void k_psi_io(const Inst *__restrict__ insts, int inst, float2 *ext, int to_ext) {
    const Inst &I = insts[inst];
    float2 *psi = I.psi[I.st->cur];
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < I.N; i += (long)gridDim.x * blockDim.x) {
        if (to_ext) ext[i] = psi[i];
        else psi[i] = ext[i];
    }
}

// mu out with the weighted mean removed; mu in (stored as given, mean 0 set).
__global__ void k_mu_io(const Inst *__restrict__ insts, int inst, float *ext, int to_ext) {
    const Inst &I = insts[inst];
    const float mean = (float)I.st->mu_mean;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < I.N; i += (long)gridDim.x * blockDim.x) {
        if (to_ext) ext[i] = I.mu[i] - mean;
        else I.mu[i] = ext[i];
    }
}

// Clears the device step-statistics accumulators of every instance.
__global__ void k_acc_reset(const Inst *__restrict__ insts, int ninst) {
    const int ii = blockIdx.x * blockDim.x + threadIdx.x;
    if (ii >= ninst) return;
    DevState *st = insts[ii].st;
    st->acc_sweeps = 0.0;
    st->acc_capped = 0.0;
    st->acc_mu_cycles = 0.0;
    st->acc_mu_capped = 0.0;
    st->acc_passes = 0.0;
    st->acc_sw_min = 1 << 30;
    st->acc_sw_max = 0;
}

// Scalar state writes, ordered on the stream.
__global__ void k_state_set(const Inst *__restrict__ insts, int inst, int field, double v) {
    DevState *st = insts[inst].st;
    switch (field) {
        case 0: st->K = v; break;
        case 1: st->t = v; break;
        case 2: st->V_sum = v; break;
        case 3: st->n = v; break;
        case 4: st->n_avg = v; break;
        case 5: st->E_last = v; break;
        case 6: st->J_last = v; break;
        case 7: st->Jext = v; break;
        case 8: st->Bx = v; break;
        case 9: st->Bz = v; break;
        case 10: st->mu_mean = v; break;
        case 11: st->in_window = (int)v; break;
        case 12: st->cur = (int)v; break;
        case 13: st->By = v; break;
        case 14: st->yz = (int)v; break;
        default: break;
    }
}

}  // namespace tdgl
