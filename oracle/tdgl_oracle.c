/*
 * tdgl_oracle.c -- plain FP64 reference for the implicit TDGL time step of
 * Sadovskyy, Koshelev, Phillips, Karpeyev, Glatz, "Stable large-scale solver
 * for Ginzburg-Landau equations for superconductors" (arXiv:1409.8340).
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark load this library.
 * It shares no source with the HIP path.
 *
 * Everything is double precision, written as plain loops in the order the
 * paper states the formulas; there is no tiling, fusion or reordering.
 * OpenMP only splits the outermost (z) loop; every reduction is done per
 * z-plane into an array and summed serially so results do not depend on the
 * thread count.
 *
 * Grid and indexing (Sec. 3, "Discretization"): nodes (i,j,k),
 * m = i + nx*(j + ny*k), x fastest.
 *
 * Link variables (Sec. 3.1, Eq. link_variables) are passed per edge:
 * lx[m] is the link on the edge m -> m+x, ly[m] on m -> m+y, lz[m] on
 * m -> m+z.  Wrap edges of periodic axes are included (the quasi-periodic
 * phase jump of Sec. 3.3.1 is carried by the wrap-edge link).  Entries on the
 * last layer of an open axis are never read.  The caller builds these arrays
 * (oracle.py does so from the Landau gauge of Sec. 2.3); any other gauge
 * can be passed, which is how gauge covariance is tested.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct {
    int nx, ny, nz;
    int open_x, open_y, open_z; /* 1: open (Neumann, Sec. 3.3.2), 0: periodic */
    double hx, hy, hz;
    double g;                   /* anisotropy, Sec. 2.1: z terms carry 1/g^2 */
} orc_grid;

static long idx(const orc_grid *G, int i, int j, int k)
{
    return (long)i + (long)G->nx * ((long)j + (long)G->ny * (long)k);
}

static double coef(const orc_grid *G, int axis)
{
    if (axis == 0) return 1.0 / (G->hx * G->hx);
    if (axis == 1) return 1.0 / (G->hy * G->hy);
    return 1.0 / (G->g * G->g * G->hz * G->hz);
}

/* Position of node m along one axis and that axis' size / boundary kind. */
static void axis_info(const orc_grid *G, int axis, int i, int j, int k,
                      int *pos, int *n, int *open, long *stride)
{
    if (axis == 0) { *pos = i; *n = G->nx; *open = G->open_x; *stride = 1; }
    else if (axis == 1) { *pos = j; *n = G->ny; *open = G->open_y; *stride = G->nx; }
    else { *pos = k; *n = G->nz; *open = G->open_z; *stride = (long)G->nx * G->ny; }
}

/*
 * Neighbour part of the covariant Laplacian along one axis at node m:
 *   U_m psi_{m+a} + conj(U_{m-a}) psi_{m-a}
 * (Eq. LaplUV_xz).  At an open face the ghost node is eliminated with the
 * Neumann rule of Sec. 3.3.2 (U* psi_{-1} = U psi_1), which doubles the inner
 * neighbour.  An open axis with a single node has no neighbours.
 */
static cplx axis_neighbours(const orc_grid *G, const cplx *link, const cplx *psi,
                            int axis, int i, int j, int k)
{
    int pos, n, open;
    long s;
    axis_info(G, axis, i, j, k, &pos, &n, &open, &s);
    long m = idx(G, i, j, k);
    if (open) {
        if (n == 1) return 0.0;
        if (pos == 0) return 2.0 * link[m] * psi[m + s];
        if (pos == n - 1) return 2.0 * conj(link[m - s]) * psi[m - s];
        return link[m] * psi[m + s] + conj(link[m - s]) * psi[m - s];
    }
    long mf = (pos == n - 1) ? m - (long)(n - 1) * s : m + s;  /* forward, wrapped */
    long mb = (pos == 0) ? m + (long)(n - 1) * s : m - s;      /* backward, wrapped */
    return link[m] * psi[mf] + conj(link[mb]) * psi[mb];
}

/* Sum over axes of coef_a * axis_neighbours: the off-diagonal part of the
 * discrete covariant Laplacian, so that L psi = NS(psi) - 2 S psi with
 * S = 1/hx^2 + 1/hy^2 + 1/(g^2 hz^2). */
void orc_neighbour_sum(const orc_grid *G, const cplx *lx, const cplx *ly,
                       const cplx *lz, const cplx *psi, cplx *out)
{
    const cplx *L[3] = {lx, ly, lz};
#pragma omp parallel for schedule(static)
    for (int k = 0; k < G->nz; ++k)
        for (int j = 0; j < G->ny; ++j)
            for (int i = 0; i < G->nx; ++i) {
                cplx acc = 0.0;
                for (int a = 0; a < 3; ++a)
                    acc += coef(G, a) * axis_neighbours(G, L[a], psi, a, i, j, k);
                out[idx(G, i, j, k)] = acc;
            }
}

/* S = sum of 1/h_a^2 over the axes that have neighbours (an open axis with
 * a single node contributes no second difference at all). */
static double diag_sum(const orc_grid *G)
{
    double s = 0.0;
    if (!(G->open_x && G->nx == 1)) s += coef(G, 0);
    if (!(G->open_y && G->ny == 1)) s += coef(G, 1);
    if (!(G->open_z && G->nz == 1)) s += coef(G, 2);
    return s;
}

/* Discrete covariant Laplacian (Eq. LaplUV_xz with the boundary forms of
 * Sec. 3.3). */
void orc_laplacian(const orc_grid *G, const cplx *lx, const cplx *ly,
                   const cplx *lz, const cplx *psi, cplx *out)
{
    orc_neighbour_sum(G, lx, ly, lz, psi, out);
    long N = (long)G->nx * G->ny * G->nz;
    double S2 = 2.0 * diag_sum(G);
    for (long m = 0; m < N; ++m) out[m] -= S2 * psi[m];
}

/*
 * Crank-Nicolson system of Sec. 3.1 (Eq. GL_numCN with |psi|^2 lagged,
 * Eq. GL_linearized, Eq. b), noise term zero:
 *   b_m    = psi_m^- + (ht/2) [ (eps_m - i u mu_m) psi_m^- - |psi_m^-|^2 psi_m^-
 *                               + (L psi^-)_m ]
 *   M_mm   = 1 + (ht/2) [ |psi_m^-|^2 + 2 S + i u mu_m - eps_m ]
 *   M_m,m' = -(ht/2) * (link / h_a^2) for the neighbours of m.
 * mu may be NULL (no scalar potential).
 */
void orc_assemble(const orc_grid *G, const cplx *lx, const cplx *ly, const cplx *lz,
                  const cplx *psi_prev, const double *eps, const double *mu,
                  double u, double ht, cplx *b, cplx *diag)
{
    long N = (long)G->nx * G->ny * G->nz;
    cplx *lap = malloc(sizeof(cplx) * (size_t)N);
    orc_laplacian(G, lx, ly, lz, psi_prev, lap);
    double S2 = 2.0 * diag_sum(G);
    for (long m = 0; m < N; ++m) {
        double mum = mu ? mu[m] : 0.0;
        cplx p = psi_prev[m];
        double a2 = creal(p) * creal(p) + cimag(p) * cimag(p);
        b[m] = p + 0.5 * ht * ((eps[m] - I * u * mum) * p - a2 * p + lap[m]);
        diag[m] = 1.0 + 0.5 * ht * (a2 + S2 + I * u * mum - eps[m]);
    }
    free(lap);
}

/* y = M psi for the matrix above. */
void orc_apply_M(const orc_grid *G, const cplx *lx, const cplx *ly, const cplx *lz,
                 const cplx *diag, double ht, const cplx *psi, cplx *out)
{
    long N = (long)G->nx * G->ny * G->nz;
    orc_neighbour_sum(G, lx, ly, lz, psi, out);
    for (long m = 0; m < N; ++m) out[m] = diag[m] * psi[m] - 0.5 * ht * out[m];
}

/*
 * One Jacobi iteration (Eq. final):
 *   psi_out_m = ( b_m - sum_{m' != m} M_mm' psi_in_m' ) / M_mm.
 * Returns max_m |r_m|^2 for the residual r = b - M psi_in of the input
 * iterate (Eq. convergence), evaluated through the identity
 * r = M_mm (psi_out - psi_in).
 */
double orc_jacobi_sweep(const orc_grid *G, const cplx *lx, const cplx *ly,
                        const cplx *lz, const cplx *b, const cplx *diag, double ht,
                        const cplx *psi_in, cplx *psi_out)
{
    long N = (long)G->nx * G->ny * G->nz;
    orc_neighbour_sum(G, lx, ly, lz, psi_in, psi_out);
    double rmax = 0.0;
    for (long m = 0; m < N; ++m) {
        cplx nxt = (b[m] + 0.5 * ht * psi_out[m]) / diag[m];
        cplx r = diag[m] * (nxt - psi_in[m]);
        double r2 = creal(r) * creal(r) + cimag(r) * cimag(r);
        if (r2 > rmax || isnan(r2)) rmax = r2; /* a NaN, once seen, stays */
        psi_out[m] = nxt;
    }
    return rmax;
}

/* Direct evaluation of max |b - M psi|^2 (used to check the identity above). */
double orc_residual_max2(const orc_grid *G, const cplx *lx, const cplx *ly,
                         const cplx *lz, const cplx *b, const cplx *diag, double ht,
                         const cplx *psi)
{
    long N = (long)G->nx * G->ny * G->nz;
    cplx *mp = malloc(sizeof(cplx) * (size_t)N);
    orc_apply_M(G, lx, ly, lz, diag, ht, psi, mp);
    double rmax = 0.0;
    for (long m = 0; m < N; ++m) {
        cplx r = b[m] - mp[m];
        double r2 = creal(r) * creal(r) + cimag(r) * cimag(r);
        if (r2 > rmax || isnan(r2)) rmax = r2;
    }
    free(mp);
    return rmax;
}

/*
 * Average supercurrent along x (Sec. 3.1.1):
 *   J_av = 1/(2 N hx) sum_m Im[ psi_m^* ( U psi_{i+1} - U^* psi_{i-1} ) ]
 * with the x links lx; open x uses the Neumann ghost (the term then vanishes
 * on the faces).  Partial sums per z-plane, summed serially.
 */
double orc_jav(const orc_grid *G, const cplx *lx, const cplx *psi)
{
    double *part = calloc((size_t)G->nz, sizeof(double));
    long sx = 1;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < G->nz; ++k) {
        double acc = 0.0;
        for (int j = 0; j < G->ny; ++j)
            for (int i = 0; i < G->nx; ++i) {
                long m = idx(G, i, j, k);
                cplx fwd, bwd;
                if (G->open_x) {
                    if (G->nx == 1) continue;
                    if (i == 0) { fwd = lx[m] * psi[m + sx]; bwd = fwd; }
                    else if (i == G->nx - 1) { bwd = conj(lx[m - sx]) * psi[m - sx]; fwd = bwd; }
                    else { fwd = lx[m] * psi[m + sx]; bwd = conj(lx[m - sx]) * psi[m - sx]; }
                } else {
                    long mf = (i == G->nx - 1) ? m - (G->nx - 1) : m + 1;
                    long mb = (i == 0) ? m + (G->nx - 1) : m - 1;
                    fwd = lx[m] * psi[mf];
                    bwd = conj(lx[mb]) * psi[mb];
                }
                acc += cimag(conj(psi[m]) * (fwd - bwd));
            }
        part[k] = acc;
    }
    double s = 0.0;
    for (int k = 0; k < G->nz; ++k) s += part[k];
    free(part);
    long N = (long)G->nx * G->ny * G->nz;
    return s / (2.0 * (double)N * G->hx);
}

/*
 * Right-hand side of the discrete Poisson equation (Sec. 3.2):
 *   f_m = sum_a (1/h_a^2) Im[ psi_m^* ( U psi_{m+a} + U^* psi_{m-a} ) ]
 * (1/(g^2 hz^2) on z), with the same open-face ghosts as the Laplacian.
 */
void orc_poisson_rhs(const orc_grid *G, const cplx *lx, const cplx *ly,
                     const cplx *lz, const cplx *psi, double *f)
{
    const cplx *L[3] = {lx, ly, lz};
#pragma omp parallel for schedule(static)
    for (int k = 0; k < G->nz; ++k)
        for (int j = 0; j < G->ny; ++j)
            for (int i = 0; i < G->nx; ++i) {
                long m = idx(G, i, j, k);
                double acc = 0.0;
                for (int a = 0; a < 3; ++a)
                    acc += coef(G, a) * cimag(conj(psi[m]) *
                                              axis_neighbours(G, L[a], psi, a, i, j, k));
                f[m] = acc;
            }
}

/*
 * Discrete Laplacian of a real scalar (left side of the Poisson equation,
 * Sec. 3.2): plain wrap on periodic axes (mu has no phase jump,
 * Sec. 3.3.1), Neumann reflection mu_{-1} = mu_1 on open faces.
 */
void orc_poisson_apply(const orc_grid *G, const double *mu, double *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < G->nz; ++k)
        for (int j = 0; j < G->ny; ++j)
            for (int i = 0; i < G->nx; ++i) {
                long m = idx(G, i, j, k);
                double acc = 0.0;
                for (int a = 0; a < 3; ++a) {
                    int pos, n, open;
                    long s;
                    axis_info(G, a, i, j, k, &pos, &n, &open, &s);
                    double fw, bw;
                    if (open) {
                        if (n == 1) continue;
                        if (pos == 0) { fw = mu[m + s]; bw = fw; }
                        else if (pos == n - 1) { bw = mu[m - s]; fw = bw; }
                        else { fw = mu[m + s]; bw = mu[m - s]; }
                    } else {
                        fw = mu[(pos == n - 1) ? m - (long)(n - 1) * s : m + s];
                        bw = mu[(pos == 0) ? m + (long)(n - 1) * s : m - s];
                    }
                    acc += coef(G, a) * (fw + bw - 2.0 * mu[m]);
                }
                out[m] = acc;
            }
}

/* Trapezoid weight of a node: 1/2 per open face the node lies on. */
static double node_weight(const orc_grid *G, int i, int j, int k)
{
    double w = 1.0;
    if (G->open_x && G->nx > 1 && (i == 0 || i == G->nx - 1)) w *= 0.5;
    if (G->open_y && G->ny > 1 && (j == 0 || j == G->ny - 1)) w *= 0.5;
    if (G->open_z && G->nz > 1 && (k == 0 || k == G->nz - 1)) w *= 0.5;
    return w;
}

void orc_node_weights(const orc_grid *G, double *w)
{
    for (int k = 0; k < G->nz; ++k)
        for (int j = 0; j < G->ny; ++j)
            for (int i = 0; i < G->nx; ++i) w[idx(G, i, j, k)] = node_weight(G, i, j, k);
}

/*
 * Discrete GL free energy whose derivative reproduces the right-hand side of
 * Eq. GL_dimensionless (without noise and scalar potential):
 *   F = hx hy hz [ sum_m w_m ( -eps_m |psi_m|^2 + |psi_m|^4 / 2 )
 *                 + sum_edges w_e |U_e psi_{m+a} - psi_m|^2 / (g_a^2 h_a^2) ]
 * so that dF/dpsi_m^* = -w_m hx hy hz (eps psi - |psi|^2 psi + L psi)_m.
 * w_m: node weight; w_e: product of 1/2 over the open faces that contain the
 * whole edge.  Sums per z-plane, summed serially.
 */
double orc_free_energy(const orc_grid *G, const cplx *lx, const cplx *ly,
                       const cplx *lz, const double *eps, const cplx *psi)
{
    const cplx *L[3] = {lx, ly, lz};
    double *part = calloc((size_t)G->nz, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int k = 0; k < G->nz; ++k) {
        double acc = 0.0;
        for (int j = 0; j < G->ny; ++j)
            for (int i = 0; i < G->nx; ++i) {
                long m = idx(G, i, j, k);
                double a2 = creal(psi[m]) * creal(psi[m]) + cimag(psi[m]) * cimag(psi[m]);
                acc += node_weight(G, i, j, k) * (-eps[m] * a2 + 0.5 * a2 * a2);
                for (int a = 0; a < 3; ++a) {
                    int pos, n, open;
                    long s;
                    axis_info(G, a, i, j, k, &pos, &n, &open, &s);
                    if (pos == n - 1 && open) continue;  /* no edge beyond an open face */
                    long mf = (pos == n - 1) ? m - (long)(n - 1) * s : m + s;
                    /* edge weight: 1/2 per open face (of another axis) containing it */
                    double we = 1.0;
                    for (int b = 0; b < 3; ++b) {
                        if (b == a) continue;
                        int pb, nb, ob;
                        long sb;
                        axis_info(G, b, i, j, k, &pb, &nb, &ob, &sb);
                        if (ob && nb > 1 && (pb == 0 || pb == nb - 1)) we *= 0.5;
                    }
                    cplx d = L[a][m] * psi[mf] - psi[m];
                    acc += we * coef(G, a) * (creal(d) * creal(d) + cimag(d) * cimag(d));
                }
            }
        part[k] = acc;
    }
    double s = 0.0;
    for (int k = 0; k < G->nz; ++k) s += part[k];
    free(part);
    return s * G->hx * G->hy * G->hz;
}

/* Weighted sum  sum_m w_m x_m  (serial, per-plane partials). */
double orc_weighted_sum(const orc_grid *G, const double *x)
{
    double s = 0.0;
    for (int k = 0; k < G->nz; ++k) {
        double acc = 0.0;
        for (int j = 0; j < G->ny; ++j)
            for (int i = 0; i < G->nx; ++i) acc += node_weight(G, i, j, k) * x[idx(G, i, j, k)];
        s += acc;
    }
    return s;
}

/*
 * Insulating inclusions (Sec. 3.4, item (ii)): no-current (open) boundary
 * conditions across the internal edges that bound an insulating region.
 *
 * reading: every edge with an insulating end (mask != 0) is taken out of the
 * covariant Laplacian -- row m of a superconducting node keeps
 *     sum over its remaining edges e of  w_e c_a (U_e psi_n - psi_m),
 * where c_a is the axis coefficient and w_e = 2 for the single inner edge of
 * an open outer face node (Sec. 3.3.2), else 1 -- and psi is 0 on insulating
 * nodes, whose rows are not part of the system.
 *
 * This routine returns the two parts of that operator at every node:
 *     out[m]  = sum_e w_e c_a U_e psi_n      (the remaining neighbours)
 *     dsum[m] = sum_e w_e c_a                (so L_cut psi = out - dsum psi)
 * both 0 on insulating nodes.  Links as for orc_neighbour_sum; U on the edge
 * m -> m-a is conj of the link stored at m-a.
 */
void orc_cut_neighbour_sum(const orc_grid *G, const cplx *lx, const cplx *ly,
                           const cplx *lz, const unsigned char *mask, const cplx *psi,
                           cplx *out, double *dsum)
{
    const cplx *L[3] = {lx, ly, lz};
#pragma omp parallel for schedule(static)
    for (int k = 0; k < G->nz; ++k)
        for (int j = 0; j < G->ny; ++j)
            for (int i = 0; i < G->nx; ++i) {
                long m = idx(G, i, j, k);
                cplx acc = 0.0;
                double dacc = 0.0;
                if (!mask[m]) {
                    for (int a = 0; a < 3; ++a) {
                        int pos, n, open;
                        long s;
                        axis_info(G, a, i, j, k, &pos, &n, &open, &s);
                        if (open && n == 1) continue;
                        double w = (open && (pos == 0 || pos == n - 1)) ? 2.0 : 1.0;
                        for (int d = -1; d <= 1; d += 2) {
                            int t = pos + d;
                            if (open && (t < 0 || t >= n)) continue;
                            long nb;
                            if (t < 0) nb = m + (long)(n - 1) * s;        /* periodic wrap */
                            else if (t >= n) nb = m - (long)(n - 1) * s;
                            else nb = m + d * s;
                            if (mask[nb]) continue;                        /* cut edge */
                            cplx U = (d == 1) ? L[a][m] : conj(L[a][nb]);
                            acc += w * coef(G, a) * U * psi[nb];
                            dacc += w * coef(G, a);
                        }
                    }
                }
                out[m] = acc;
                if (dsum) dsum[m] = dacc;
            }
}

/* Thread count of the loops above (OpenMP over z), for timing the oracle at
 * a chosen number of host threads. */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }
