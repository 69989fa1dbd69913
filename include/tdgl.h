/*
 * tdgl.h -- C ABI of libtdgl, an MI355X (gfx950) solver for the implicit
 * time step of the time-dependent Ginzburg-Landau equations in the form of
 * Sadovskyy, Koshelev, Phillips, Karpeyev and Glatz, "Stable large-scale
 * solver for Ginzburg-Landau equations for superconductors"
 * (arXiv:1409.8340).
 *
 * Model (reduced units of Sec. 2.1: lengths in xi_0, time in t_0, field in
 * H_c2(0), current in J_0):
 *     u (d/dt + i mu~) psi~ = eps(r) psi~ - |psi~|^2 psi~ + (grad - i A~)^2 psi~
 * (Eq. GL_external_current, noise term zero) with a uniform field in the xz
 * plane in the Landau gauge A = ybar [-Bz, 0, Bx] (Sec. 2.3, Eq. A_xz),
 * A~ = A - [K, 0, 0], the current phase K(t) driven by Eq. K_ODE and the
 * scalar potential mu~ from the Poisson equation of Sec. 2.2.
 *
 * Conventions shared by every entry point
 *   - A context holds one or more independent instances ("batch").  Calls
 *     that act on one instance take its index `inst` (0 for a single one).
 *   - Every array argument is a DEVICE pointer into memory the caller owns,
 *     on the device that was current at tdgl_create.  Scalars and the small
 *     structs below are host memory.
 *   - Grid arrays are laid out x fastest: element m = i + nx*(j + ny*k)
 *     (Sec. 3).  Complex values are interleaved single precision
 *     (re, im) pairs, i.e. the layout of float2 / torch.complex64.
 *   - The library allocates no device memory.  All device state lives in a
 *     caller-supplied workspace of tdgl_plan() bytes (256-byte aligned) that
 *     must outlive the context.  It allocates a few hundred bytes of pinned
 *     host memory per context for convergence polling.
 *   - Work is enqueued on the stream given at tdgl_create.  Calls return
 *     after enqueueing unless documented as synchronising.
 *   - Every function returns a tdgl_status.  On failure nothing is enqueued
 *     and tdgl_last_error() (per calling thread) describes the problem.  No
 *     exception or abort crosses this interface.
 */
#ifndef TDGL_H
#define TDGL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int tdgl_status;
#define TDGL_OK 0
#define TDGL_EINVAL 1    /* invalid argument or parameter combination      */
#define TDGL_EWS 2       /* workspace missing, misaligned or too small      */
#define TDGL_ENOCONV 3   /* strict mode: a solve hit its iteration cap      */
#define TDGL_EDEVICE 4   /* HIP runtime error (message names the call)      */
#define TDGL_ESTATE 5    /* call not valid in the context's current state   */

#define TDGL_PERIODIC 0  /* periodic; quasi-periodic y when the field needs it (Sec. 3.3.1) */
#define TDGL_OPEN 1      /* open / Neumann face, zero normal current (Sec. 3.3.2)          */

#define TDGL_MAX_ITER 256   /* upper bound for tdgl_params.max_iter    */
#define TDGL_MAX_CYCLES 64  /* upper bound for tdgl_params.mu_max_cycles */

/* Parameters of one instance.  The mesh of Sec. 3: nodes x = i hx,
 * y = j hy, z = k hz; system size L = n h on periodic axes and (n-1) h on
 * open axes. */
typedef struct tdgl_params {
    int nx, ny, nz;       /* nodes per axis, >= 1; nx*ny*nz < 2^31          */
    double hx, hy, hz;    /* mesh spacing (xi_0), > 0                        */
    int bc[3];            /* TDGL_PERIODIC or TDGL_OPEN for x, y, z          */
    double g;             /* anisotropy (Sec. 2.1): z terms carry 1/g^2      */
    double u;             /* relaxation constant u of Eq. GL_dimensionless   */
    double dt;            /* time step; the CN step uses ht = dt / u         */
    double tol;           /* stop when max_m |r_m|^2 < tol (Eq. convergence) */
    int max_iter;         /* Jacobi sweep cap per step (1..TDGL_MAX_ITER)    */
    int driven;           /* 1: solve K and mu~ (Sec. 2.2); 0: K = mu~ = 0    */
    double mu_tol;        /* Poisson stop: max_m |Delta mu~ - f|_m below      */
    double mu_rtol;       /*   max(mu_tol, mu_rtol * that residual at the start of the step's solve) */
    int mu_max_cycles;    /* multigrid cycle cap per step (1..TDGL_MAX_CYCLES) */
    int strict;           /* 1: tdgl_step returns TDGL_ENOCONV on a capped solve */
    int tile_cz;          /* z planes per stencil work-group; 0 = library default */
    int tile_rows;        /* y rows per stencil thread: 0 (default 2), 1, 2 or 4;
                             every instance of a context must agree
                             (tdgl_autotune may change both tile fields) */
    int poisson;          /* 0: direct spectral solve where the box allows it
                             (periodic x and y, open z, sizes with factors 2,3,5),
                             multigrid otherwise; 1: always multigrid */
    int reserved0;        /* must be zero */
    double noise_T;       /* Langevin term of Eq. b (Sec. 3.1.2, noise terms):
                             reduced temperature T-bar >= 0, 0 = off.  Every
                             node and step draws zeta = zeta_1 + i zeta_2,
                             both uniform on [-zeta_max, zeta_max] with
                             zeta_max^2 = 3 T-bar u / (2 dt hx hy hz); b gains
                             ht zeta.  The draws come from Philox4x32-10
                             (Salmon et al., SC'11) with counter (m, n mod
                             2^32, n / 2^32, 0) for node m = i + nx (j + ny k)
                             and step counter n (the scalars' n before the
                             step), key (seed mod 2^32, seed / 2^32); output
                             words r0, r1 map to (2 (r >> 8) - (2^24 - 1))
                             2^-24, exact in FP32.  A step therefore depends
                             only on the state, the seed and n.            */
    unsigned long long noise_seed; /* key of the noise generator            */
    int reserved[2];      /* must be zero */
} tdgl_params;

/* Per-call statistics of tdgl_step (filled only when a pointer is given;
 * that makes the call synchronising). */
typedef struct tdgl_step_stats {
    int steps;              /* steps advanced                                  */
    int sweeps_min, sweeps_max;
    long long sweeps_sum;   /* Jacobi sweeps over all steps                    */
    int capped_steps;       /* steps whose Jacobi solve hit max_iter           */
    float last_res2;        /* max |r|^2 of the last sweep's input iterate     */
    int mu_cycles_sum;      /* multigrid cycles over all steps                 */
    int mu_capped_steps;    /* steps whose Poisson solve hit mu_max_cycles      */
    float mu_last_res;      /* last Poisson residual max-norm                  */
    long long sweep_passes; /* Jacobi-kernel passes that did a full pass over
                               the grid: sweeps - 1 per step (the first
                               iterate comes from the assemble pass), or,
                               with two-sweep passes, sweeps / 2 when the
                               pairs start at the second iterate and
                               (sweeps + 1) / 2 when one single sweep comes
                               first; launches that exit at once and
                               corrective sweeps excluded */
    int single_first_steps; /* steps whose two-sweep solve began with one
                               single sweep, so that the pairs end on even
                               iterates (chosen when the recent sweep
                               counts are mostly even)               */
} tdgl_step_stats;

/* Scalars that, with psi~ and mu~, make up the full state (exact resume). */
typedef struct tdgl_scalars {
    double K;        /* current phase of Eq. psi_transformation              */
    double t;        /* simulated time                                       */
    double V_sum;    /* sum of E_x over the steps in the voltage window      */
    long long n;     /* steps taken                                          */
    long long n_avg; /* steps in the voltage window                          */
    double E_last;   /* E_x of the last step                                 */
    double J_av_last;/* J_av of the last step (Sec. 3.1.1)                   */
} tdgl_scalars;

/* Observables, reduced in double precision on the device. */
typedef struct tdgl_obs {
    double F;        /* GL free energy of the current psi~ (see tdgl_observables) */
    double E_last;   /* E_x = J_ext - J_av of the last step                  */
    double E_mean;   /* V_sum / n_avg: time-averaged electric field          */
    double V_mean;   /* Lx * E_mean: time-averaged voltage across the sample */
    double J_av;     /* J_av of the last step                                */
    double K;        /* current phase                                        */
    double res2_last;/* last Jacobi max |r|^2                                */
    double mu_mean_w;/* weighted mean of mu~ as stored (the solver subtracts it) */
    double psi2_mean;/* mean |psi~|^2                                        */
    long long n, n_avg;
} tdgl_obs;

typedef struct tdgl_ctx tdgl_ctx;

/* Thread-local description of the last failure on this thread. */
const char *tdgl_last_error(void);

/* Validates `n` parameter sets and returns the workspace size in bytes a
 * context holding them needs.  Host only; touches no device.  Rejects an
 * open x axis together with driven = 1 (a current along x needs periodic x,
 * Sec. 3.3.2). */
tdgl_status tdgl_plan(int n, const tdgl_params *params, size_t *ws_bytes);

/* Creates a context with `n` instances on the current device, carving all
 * device state out of `ws` (ws_bytes >= tdgl_plan's result, 256-byte
 * aligned).  `stream` is a hipStream_t (NULL: the default stream).  Every
 * instance starts with psi~ = 1, mu~ = 0, K = 0, eps = 1, B = 0, J = 0.
 * Synchronising (uploads small coefficient tables). */
tdgl_status tdgl_create(int n, const tdgl_params *params, void *ws, size_t ws_bytes,
                        void *stream, tdgl_ctx **out);

/* Destroys the context (the workspace stays the caller's).  Synchronising. */
tdgl_status tdgl_destroy(tdgl_ctx *ctx);

/* Number of instances in the context. */
tdgl_status tdgl_size(const tdgl_ctx *ctx, int *n);

/* Host-only helper: the field rounded to whole flux quanta through the
 * periodic cross sections (Sec. 3.3.1, "Implications for the magnetic
 * field"): Bz = 2 pi n_z / (Lx Ly) if x and y are periodic, Bx =
 * 2 pi n_x / (Ly Lz) if y and z are periodic; other components unchanged. */
tdgl_status tdgl_quantize_field(const tdgl_params *p, double Bx, double Bz,
                                double *Bx_eff, double *Bz_eff);

/* Sets the uniform field in the xz plane (Eq. B_xz) and rebuilds the link
 * tables (Eq. link_variables, Sec. 3.3.1 phase jump).  quantize = 1 rounds
 * as tdgl_quantize_field and reports the result; quantize = 0 requires the
 * field to be quantised already (relative error 1e-9), else TDGL_EINVAL. */
tdgl_status tdgl_set_field(tdgl_ctx *ctx, int inst, double Bx, double Bz, int quantize,
                           double *Bx_eff, double *Bz_eff);

/* Rounding for a field in the yz plane (Eq. B_yz): Bz = 2 pi n_z / (Lx Ly)
 * if x and y are periodic, By = 2 pi n_y / (Lx Lz) if x and z are (Sec.
 * 3.3.1, the flux through each periodic cross section is a whole number of
 * quanta); a field component across an open axis is unchanged. */
tdgl_status tdgl_quantize_field_yz(const tdgl_params *p, double By, double Bz,
                                   double *By_eff, double *Bz_eff);

/* Sets a uniform field in the yz plane, B = (0, By, Bz) (Eq. B_yz), and
 * rebuilds the link tables.  The current stays along x.  The vector
 * potential is A = (-y Bz + z By, 0, 0): every link variable but the x link
 * is 1, the x link of node (i, j, k) is exp(i hx (K + Bz j hy - By k hz)),
 * and the periodic y seam carries psi_{i,-1,k} = exp(i xbar_i Ly Bz)
 * psi_{i,ny-1,k}, xbar_i = i hx - Lx/2.  This is the paper's field in
 * another gauge: psi~ here relates to psi~ in the gauge of Eq. A_yz (x
 * quasi-periodic, Sec. 3.3.1) by psi_paper = exp(i (j hy Bz - k hz By)
 * xbar_i) psi, and every gauge-invariant quantity (|psi|^2, currents, mu~,
 * E, F) is the same.  With By != 0 on a periodic z axis the z wrap carries
 * a phase too: psi_{i,j,-1} = exp(-i xbar_i Lz By) psi_{i,j,nz-1}; such a
 * context runs single sweeps only (TDGL_EINVAL if its tiling is fused:
 * set fused = 0 first; the autotuner then skips two-sweep candidates and
 * tdgl_set_tiling refuses them).  A context holding a yz-plane field has no
 * persistent solve (that tiling is switched off and refused).  tdgl_set_field returns the
 * instance to the xz plane.  quantize as for tdgl_set_field. */
tdgl_status tdgl_set_field_yz(tdgl_ctx *ctx, int inst, double By, double Bz, int quantize,
                              double *By_eff, double *Bz_eff);

/* Sets the applied current density J_x,ext (Eq. J_external).  Requires a
 * driven instance unless J_ext == 0. */
tdgl_status tdgl_set_current(tdgl_ctx *ctx, int inst, double J_ext);

/* Copies eps (float[N], Eq. epsilon on the grid nodes, Sec. 3.4 (i)). */
tdgl_status tdgl_set_eps(tdgl_ctx *ctx, int inst, const float *eps);

/* Inclusion generator (Sec. 3.4): candidate spheres (centres double[3*nc]
 * as x,y,z triples in xi_0; diameters double[nc]) are added in order until
 * the covered node fraction reaches `target`; nodes inside an added sphere
 * (any periodic image; open axes clipped; |r_m - c|^2 <= (d/2)^2 evaluated
 * in double precision without fused multiply-add) get eps_in, all others
 * eps_out.  Reports the number of spheres used and the covered fraction.
 * Synchronising.  Uses the instance's b/M array (rebuilt by every step) as
 * scratch. */
tdgl_status tdgl_gen_inclusions(tdgl_ctx *ctx, int inst, const double *centres,
                                const double *diameters, int nc, double target,
                                float eps_in, float eps_out, int *n_used, double *fraction);

/* Inclusion generator for general convex candidates (Sec. 3.4; the
 * ellipsoids and tilted columns of Fig. 2d/e): as tdgl_gen_inclusions, with
 * candidate s given by 16 doubles of `shapes` (device memory, double[16*nc]):
 *     c[3] | Q_xx Q_yy Q_zz Q_xy Q_xz Q_yz | n[3] | hlen | ext[3].
 * A node image u (integer coordinates, d = u h - c) is inside iff
 *     q = (((Qxx dx) dx + (Qyy dy) dy) + (Qzz dz) dz)
 *         + 2 (((Qxy dx) dy + (Qxz dx) dz) + (Qyz dy) dz) <= 1
 * and, when hlen >= 0, |(nx dx + ny dy) + nz dz| <= hlen, all in double
 * precision without fused multiply-add.  A sphere of radius r is Q = I/r^2,
 * an ellipsoid Q = R diag(a^-2, b^-2, c^-2) R^T, a column of radius rho
 * along the unit vector n Q = (I - n n^T)/rho^2 with hlen its half length.
 * ext: half-widths of an axis-aligned box around c that holds the shape;
 * only images in that box (one node margin) are tested, clipped on open
 * axes and kept within one period of the centre on periodic ones.  A
 * candidate with a non-finite entry or a negative ext covers nothing.
 * Synchronising; uses the b/M array (rebuilt by every step) as scratch. */
tdgl_status tdgl_gen_shapes(tdgl_ctx *ctx, int inst, const double *shapes, int nc, double target,
                            float eps_in, float eps_out, int *n_used, double *fraction);

/* Insulating inclusions (Sec. 3.4, item (ii): no-current boundary
 * conditions across the internal edges that bound them).  mask: device
 * memory, unsigned char[N], nonzero = insulating node.  Reading of the paper
 * (which gives no discretisation): every edge between a superconducting and
 * an insulating node is cut out of the covariant Laplacian and psi is 0 on
 * insulating nodes, so no SUPERcurrent crosses an insulator surface; the
 * Poisson equation for mu~ stays on the full grid, so the normal current
 * -grad mu~ is not blocked.  With psi = 0 there, cutting an edge changes
 * only the diagonal of its superconducting end, by c_a = 1/h_a^2
 * (1/(g h_z)^2 along z, 2 c_a for the doubled inner neighbour of an open
 * face node), which is what raising eps by c_a does; so this call rewrites
 * the instance's eps in place (eps += the cut shares, added in float in
 * the order x-, x+, y-, y+, z-, z+; eps = -2^50 on insulating nodes, which
 * keeps psi there below 1e-14 of the neighbours') and zeroes psi on the
 * insulating nodes.  Call it once after eps is final (tdgl_set_eps or a
 * generator); a second call before eps is set or generated again would add
 * the shares twice and returns TDGL_ESTATE.  Synchronising. */
tdgl_status tdgl_set_insulators(tdgl_ctx *ctx, int inst, const unsigned char *mask);

/* Tessellation pattern (Sec. 3.4; the Voronoi polycrystal of Fig. 2c):
 * every node takes values[s] (float[ns], device memory) of its nearest seed
 * s (seeds: double[3*ns] xyz positions, device memory).  The per-axis
 * separation of node x = i h from seed c is |x - c| on an open axis and
 * min(|d|, |d - L|, |d + L|), d = x - c, on a periodic axis of length
 * L = n h (the nearest image for seeds inside the box); an axis whose bit
 * (1 x, 2 y, 4 z) is not in `axes` contributes 0, e.g. axes = 3 for
 * columnar crystallites.  metric 0: Euclidean, (dx^2 + dy^2) + dz^2;
 * 1: absolute, (dx + dy) + dz; 2: maximum, max(max(dx, dy), dz); double
 * precision without fused multiply-add.  Equal distances go to the lowest
 * seed index; seeds with a non-finite coordinate are skipped; ns = 0 leaves
 * eps as it is.  Combine with other patterns through tdgl_get_eps /
 * tdgl_set_eps.  Cost O(N ns).  Synchronising.  TDGL_EINVAL for ns < 0,
 * null arrays, metric outside 0..2 or axes outside 1..7. */
tdgl_status tdgl_gen_voronoi(tdgl_ctx *ctx, int inst, const double *seeds, const float *values, int ns,
                             int metric, int axes);

/* Copies the instance's eps (float[N]) out, e.g. after tdgl_gen_inclusions. */
tdgl_status tdgl_get_eps(tdgl_ctx *ctx, int inst, float *eps);

/* psi~ in/out: complex64[N].  mu~ in/out: float[N] (weighted mean removed
 * on output). */
tdgl_status tdgl_set_psi(tdgl_ctx *ctx, int inst, const void *psi);
tdgl_status tdgl_get_psi(tdgl_ctx *ctx, int inst, void *psi);
tdgl_status tdgl_set_mu(tdgl_ctx *ctx, int inst, const float *mu);
tdgl_status tdgl_get_mu(tdgl_ctx *ctx, int inst, float *mu);

/* Scalars for exact resume.  Synchronising. */
tdgl_status tdgl_get_scalars(tdgl_ctx *ctx, int inst, tdgl_scalars *s);
tdgl_status tdgl_set_scalars(tdgl_ctx *ctx, int inst, const tdgl_scalars *s);

/* Starts a new voltage-averaging window (V_sum = n_avg = 0). */
tdgl_status tdgl_voltage_window_reset(tdgl_ctx *ctx, int inst);

/*
 * Advances every instance by nsteps implicit time steps.  One step
 * (Sec. 3.1, 3.2 and the kernel sequence of Sec. 4.1):
 *   1. assemble b and diag(M) of Eq. GL_linearized / Eq. b from psi^-,
 *      eps, mu~ and the links at K (|psi|^2 lagged, Eq. GL_numCN);
 *   2. Jacobi iterations of Eq. final from psi^(0) = psi^- until the input
 *      residual of a sweep satisfies Eq. convergence (max|r|^2 < tol) or
 *      max_iter; that sweep's output is the new psi~;
 *   3. driven only: J_av (Sec. 3.1.1), E_x = J_ext - J_av, K += dt E_x,
 *      voltage sum, phase rewind K -> K - (2 pi/hx) floor(K hx / 2 pi)
 *      (Sec. 2.2);
 *   4. driven only: Poisson equation of Sec. 3.2 for mu~ with the links at
 *      the new K, weighted mean of mu~ fixed to zero.  With x and y
 *      periodic and params.poisson = 0 (the default) it is solved directly:
 *      real FFT along x, FFT along y, one tridiagonal system along z per
 *      (kx, ky) by Thomas' algorithm in FP64, inverse FFTs.  Otherwise by
 *      multigrid V-cycles whose smoother is the pseudo-time relaxation of
 *      Sec. 3.2 (damped Jacobi) until max|Delta mu~ - f| < max(mu_tol,
 *      mu_rtol * its value before the first cycle).
 * Enqueues work; the host learns when a Jacobi solve has converged by
 * reading convergence words that the sweep kernels store into pinned,
 * mapped host memory (it spins on them; no device-to-host copies), and
 * queues one or two speculative sweep launches ahead.  stats may be NULL.
 * With strict = 1, returns TDGL_ENOCONV after the first step whose Jacobi
 * solve hit max_iter.
 */
tdgl_status tdgl_step(tdgl_ctx *ctx, int nsteps, tdgl_step_stats *stats);

/* Observables of one instance: F is the discrete GL free energy
 *   hx hy hz [ sum_m w_m (-eps_m |psi_m|^2 + |psi_m|^4 / 2)
 *              + sum_edges w_e |U_e psi_{m+a} - psi_m|^2 / (g_a^2 h_a^2) ]
 * (w: 1/2 per open face containing the node or edge), whose derivative by
 * psi*_m is -w_m hx hy hz times the right side of Eq. GL_dimensionless.
 * Synchronising. */
tdgl_status tdgl_observables(tdgl_ctx *ctx, int inst, tdgl_obs *obs);

/* Advances every instance by nsteps steps exactly as tdgl_step does, as
 * replays of one captured HIP graph per step: the step is issued as a fixed
 * sequence -- the assemble kernel, budget - 1 Jacobi sweep launches (a sweep
 * whose instance has already met the tolerance exits at once), the current,
 * K and Poisson right side, and the Poisson solve with every multigrid cycle
 * launched (converged or capped instances skip the rest) -- so no step waits
 * on the host.  A solve that needs more than `budget` sweeps (1 <= budget <=
 * the largest max_iter) stops there and counts as capped; with budget >= the
 * sweeps a solve needs, results are bit-identical to tdgl_step.  The graph is
 * captured on a private stream on the first call (and again after the
 * budget or the tiling changes) and launched on the context's stream.
 * stats (nullable; makes the call synchronising) come from counters kept on
 * the device.  Not available while per-kernel profiling is active
 * (TDGL_ESTATE). */
tdgl_status tdgl_step_graph(tdgl_ctx *ctx, int nsteps, int budget, tdgl_step_stats *stats);

/* Solves the Poisson equation of Sec. 3.2, Delta_h mu = f (7-point stencil,
 * plain wrap on periodic axes, Neumann reflection on open faces), for a
 * given right side with the instance's solver (spectral or multigrid, as
 * for a step) and returns mu with zero weighted mean.  f and mu are
 * float[N] device arrays; the weighted mean of f is projected out first.
 * The context must hold exactly one driven instance.  Overwrites the
 * instance's stored mu~ (the next step starts from this solution). */
tdgl_status tdgl_poisson_solve(tdgl_ctx *ctx, const float *f, float *mu);

/* Stencil tiling: work-groups of 64 x 4*rows grid columns marching through
 * z runs of `chunk` planes. */
typedef struct tdgl_tiling {
    int rows;        /* rows of the tile per thread: 1, 2 or 4               */
    int chunk;       /* z planes per work-group (instance 0 for tdgl_autotune) */
    int streaming;   /* 1: non-temporal hints on the read-once streams of the
                        sweep and assemble passes (default: on when the
                        context's sweep arrays exceed 256 MB)               */
    int fused;       /* 1: Jacobi sweeps run two per pass over HBM (the
                        second iterate on the tile from the first on the tile
                        and its one-node ring); results are bit-identical */
    int persistent;  /* 1: each Jacobi solve is one cooperative launch that
                        loops over the sweeps with grid-wide barriers (no
                        host round trip per sweep; single sweeps only; step
                        statistics then come from device counters and a
                        strict failure is reported at the end of the call).
                        tdgl_autotune picks it only when its timed sweeps,
                        barriers included, beat separate launches by 10 %. */
    double sweep_us; /* measured time of one Jacobi sweep of the whole context
                        (tdgl_autotune; 0 from tdgl_get_tiling)             */
    int chunk2;      /* z planes per work-group of the two-sweep passes'
                        super-tile kernel (fused = 1); 0: chunk.  The stencil
                        passes (assemble, Poisson right side, single sweeps)
                        keep chunk                                          */
    int rhs_rows;    /* rows per thread of the Poisson right-side pass: 0 =
                        rows, or 4 (64 x 16 tiles, z runs chosen as for
                        chunk); the result does not depend on it           */
    int super_rows;  /* rows of the two-sweep passes' super-tiles (64 wide):
                        16 or 32 (32 needs rows 2 or 4); 0: 32 for rows 2
                        and 4, 16 for rows 1.  Taller tiles re-read fewer
                        halo rows, shorter ones fit more work-groups per CU;
                        the result does not depend on it                  */
} tdgl_tiling;

/* Picks the stencil tiling of the context by timing one Jacobi sweep for
 * each candidate (rows in {1, 2, 4} x chunk in {heuristic, 4, 8, 16, 32,
 * 64, 128, 256} up to the deepest instance's z x streaming hints off/on x
 * one or two sweeps per pass; the two-sweep candidates vary chunk2 and the
 * super-tile height (super_rows 16 or 32) and keep
 * the stencil chunk of the fastest single sweep with the same rows and
 * hints) on the context's stream and keeping the fastest per iteration;
 * then 16 sweeps of
 * that tiling in one persistent launch are timed, and persistent solves are
 * chosen when they are at least 10 % faster per sweep.  The timing sweeps
 * read the current psi~ and b/M, (ht/2)/M arrays and write only the spare
 * psi~ buffer, so the solver state is unchanged.  psi~, mu~ and the step
 * statistics of later steps are the same bits for every tiling (the node
 * arithmetic is written contraction-proof); only F, a sum of per-tile FP64
 * partials, depends on the tiling through its summation order.
 * The choice is cached in the process per context shape (every instance's
 * grid, boundary kinds and driven flag) and, when cache_path is not NULL,
 * in that text file (read first, appended after a search).  No device
 * allocation.  chosen may be NULL.  Synchronising. */
tdgl_status tdgl_autotune(tdgl_ctx *ctx, const char *cache_path, tdgl_tiling *chosen);

/* Sets the tiling of every instance without timing (rows in {1, 2, 4};
 * chunk 0 = heuristic, else z planes per work-group; streaming, fused and
 * persistent 0 or 1, not fused and persistent together; sweep_us ignored).
 * No allocation; synchronises the stream.  tdgl_step_graph always uses
 * separate sweep launches. */
tdgl_status tdgl_set_tiling(tdgl_ctx *ctx, const tdgl_tiling *t);

/* Current tiling of instance inst (rows are shared by the context). */
tdgl_status tdgl_get_tiling(const tdgl_ctx *ctx, int inst, tdgl_tiling *out);

/* Bytes of the caller-owned workspace tdgl_voltage_grad needs for nsteps
 * steps with a checkpoint every ckpt_every steps: ceil(nsteps/ckpt_every)
 * checkpoints and one segment of ckpt_every+1 states of psi~ (complex64) and
 * mu~ (float) plus a few node arrays.  Host only. */
tdgl_status tdgl_adjoint_plan(const tdgl_ctx *ctx, int nsteps, int ckpt_every, size_t *bytes);

/* Advances the context's single driven instance by nsteps steps, exactly as
 * tdgl_step(ctx, nsteps) would, and returns the time-averaged electric field
 *     Vbar = (1/W) sum_{n = window_begin}^{nsteps-1} E_n,
 *     E_n = J_ext - J_av (Sec. 3.1.1, Eq. K_ODE),  W = nsteps - window_begin,
 * (steps counted from 0 within this call) together with its gradient
 * d Vbar / d eps_m at every node (float[N], device memory, overwritten).  The
 * gradient is that of the implicit step itself -- Crank-Nicolson system,
 * J_av, K update and Poisson solve differentiated exactly (implicit-function
 * adjoint, Sec. 3.1-3.2), the phase rewind having derivative one -- so it
 * matches finite differences when the solves are converged tightly (small
 * tol and mu_tol).  Reverse sweep over the steps; the states of each segment
 * of ckpt_every steps but the last are recomputed from a checkpoint (the
 * last segment's states are kept from the forward run, so ckpt_every >=
 * nsteps recomputes nothing: the whole trajectory sits in the workspace,
 * 12 bytes per node and step).  ws/ws_bytes: the
 * workspace of tdgl_adjoint_plan (256-byte aligned).  The field may lie in
 * the xz or the yz plane (the gradient and Vbar are gauge invariant).  The
 * context ends in the state after nsteps steps.  Synchronising. */
tdgl_status tdgl_voltage_grad(tdgl_ctx *ctx, int nsteps, int window_begin, int ckpt_every, void *ws,
                              size_t ws_bytes, double *vbar, float *grad_eps);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as tdgl_voltage_grad, same arguments and results (bit for
 * bit), with the adjoint buffers in a fixed 64 MiB device array of the
 * library instead of a caller workspace.  The request must fit it:
 * tdgl_adjoint_plan(ctx, nsteps, ckpt_every) <= 67108864 bytes, else
 * TDGL_EWS and nothing runs.  Allocates nothing (no hipMalloc, hipFree or
 * allocating library call); the context itself is created beforehand as
 * usual.  Each device keeps its own array until the process ends, and it
 * holds the last call's contents (every buffer the computation reads first
 * is cleared or written by the call itself).  Calls that overlap on one
 * device share the array and race: serialise them.  Synchronising. */
tdgl_status tdgl_voltage_grad_noalloc(tdgl_ctx *ctx, int nsteps, int window_begin, int ckpt_every,
                                      double *vbar, float *grad_eps);

/* Kernel classes of the per-kernel profile (the time profile of one step,
 * kernel by kernel, as in the paper's performance section, Sec. 4.3). */
#define TDGL_K_ASSEMBLE 0   /* assemble b, M_mm fused with the first Jacobi iteration */
#define TDGL_K_SWEEP 1      /* one Jacobi iteration (all later sweeps)              */
#define TDGL_K_CURRENT 2    /* J_av partial sums and the K update                   */
#define TDGL_K_RHS 3        /* Poisson right side and its weighted mean              */
#define TDGL_K_MG_FINE 4    /* Poisson solve on the full grid (FFT passes, or multigrid finest level) */
#define TDGL_K_MG_COARSE 5  /* multigrid work on coarser levels (incl. transfers)   */
#define TDGL_K_OTHER 6      /* solve bookkeeping and the mu~ mean                   */
#define TDGL_K_COUNT 7

typedef struct tdgl_prof {
    long long launches[TDGL_K_COUNT]; /* launches per class                          */
    double ms[TDGL_K_COUNT];          /* summed device time per class (HIP events)  */
} tdgl_prof;

/* Starts timing the kernel classes whose bit is set in `mask` (bit c for
 * class c): every launch of such a kernel inside tdgl_step is bracketed by
 * two HIP events on the context's stream.  Resets the accumulators. */
tdgl_status tdgl_profile_start(tdgl_ctx *ctx, unsigned mask);

/* Stops timing and returns the per-class launch counts and summed event
 * times since tdgl_profile_start.  Synchronising. */
tdgl_status tdgl_profile_stop(tdgl_ctx *ctx, tdgl_prof *out);

#ifdef __cplusplus
}
#endif
#endif /* TDGL_H */
