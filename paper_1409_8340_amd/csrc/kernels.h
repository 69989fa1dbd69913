// kernels.h -- declarations of the libtdgl kernels (defined in k_*.hip).
#pragma once
#include "tdgl_dev.h"

namespace tdgl {

enum { MODE_FIRST = 0, MODE_SWEEP = 1, MODE_RHS = 2, MODE_ENERGY = 3, MODE_NS = 4, MODE_FIRSTN = 5 };
// MODE_FIRSTN: MODE_FIRST with the Langevin term (a separate instantiation,
// so that the noiseless assemble carries none of the generator's registers).
constexpr bool is_first_mode(int m) { return m == MODE_FIRST || m == MODE_FIRSTN; }
constexpr int JAV_CPT = 16;     // least cells per thread of the flat reductions (a multiple of 8)
constexpr int JAV_CPT_MAX = 64; // most cells per thread, taken while 2048 or more work-groups remain
constexpr int CO_THREADS = 1024;
constexpr int FIN_THREADS = 256;  // threads per instance of the solve finalizers

template <int R, bool NT, bool YZ>
__global__ void k_sweep2(const Inst *insts, const int *prefix, int ninst, int l, unsigned long long *pub,
                         unsigned seq);
template <bool YZ>
__global__ void k_seam_ring(const Inst *insts, const int *prefix, int ninst, int l);
template <int R, bool NT, bool YZ, int TY>
__global__ void k_sweep2i(const Inst *insts, const int *prefix, int ninst, int l, unsigned long long *pub,
                          unsigned seq);
template <int R, bool NT>
__global__ void k_jacobi_persist(const Inst *insts, const int *prefix, int ninst, int l0, int lcap, int ntiles);
template <int MODE, int R, bool NT, bool YZ>
__global__ void k_stencil(const Inst *insts, const int *prefix, int ninst, int l, const float2 *ext_in,
                          float2 *ext_out, unsigned long long *pub, unsigned seq);

__global__ void k_links(const Inst *insts, int which, const double *Kp);
__global__ void k_solve_finalize(const Inst *insts, int ninst, int count_step, int nl, int fused,
                                 unsigned long long *pub, unsigned seq);
__global__ void k_acc_reset(const Inst *insts, int ninst);
__global__ void k_jav_partial(const Inst *insts, const int *prefix, int ninst);
__global__ void k_kupdate(const Inst *insts, const int *nparts);
__global__ void k_reduce_to_state(const Inst *insts, const int *nparts, int field, int driven_only);
__global__ void k_psi2_partial(const Inst *insts, const int *prefix, int ninst);
__global__ void k_fill_c(float2 *p, long n, float re, float im);
__global__ void k_fill_f(float *p, long n, float v);
__global__ void k_fill_u(unsigned *p, long n, unsigned v);
__global__ void k_psi_io(const Inst *insts, int inst, float2 *ext, int to_ext);
__global__ void k_mu_io(const Inst *insts, int inst, float *ext, int to_ext);
__global__ void k_state_set(const Inst *insts, int inst, int field, double v);

__global__ void k_mg_smooth(const Inst *insts, const int *prefix, int ninst, int lv, int isrc,
                            int idst, int cyc, float omega);
__global__ void k_mg_residual(const Inst *insts, const int *prefix, int ninst, int lv, int isrc,
                              int cyc);
__global__ void k_mg_restrict(const Inst *insts, const int *prefix, int ninst, int lv, int cyc,
                              float omega);
__global__ void k_mg_prolong(const Inst *insts, const int *prefix, int ninst, int lv, int ifine,
                             int cyc);
__global__ void k_mg_coarsest(const Inst *insts, int ninst, int cyc);
__global__ void k_mg_finalize(const Inst *insts, int ninst, int count_step);
__global__ void k_mu_mean_partial(const Inst *insts, const int *prefix, int ninst, int which);

template <bool P2, int XC>
__global__ void k_fft_x(const Inst *insts, const int *prefix, int ninst, int dir, const float *in_ext,
                        float *out_ext);
template <bool P2>
__global__ void k_fft_y(const Inst *insts, const int *prefix, int ninst, int dir);
template <int RMAX>
__global__ void k_fft_zsolve(const Inst *insts, const int *prefix, int ninst);
__global__ void k_fft_tables(const Inst *insts, int inst);
__host__ __device__ int fft_x_pairs(int nx);
__host__ __device__ int fft_y_stride(int ny);
struct FftYPlan {
    int G;       // whole planes per tile (ntk = 1)
    int ntk;     // tiles per plane (G = 1)
    int TK;      // columns per tile: G P, or about P / ntk
    int blocks;  // tiles of the instance
};
__host__ __device__ FftYPlan fft_y_plan(int nx, int ny, int nz);
__host__ __device__ int fft_pitch(int nx);
__host__ __device__ size_t fft_z_lds(int nz);
constexpr int FFT_ZTK = 16;     // kx columns per work-group of the z solve
constexpr int FFT_ZMAX = 256;   // largest nz of the spectral path
constexpr int FFT_ZSERIAL = 16; // up to this nz one lane solves a whole z system (no wavefront scan)
constexpr int FFT_MAXN = 8192;  // points per work-group of the x and y passes
constexpr int FFT_XY_THREADS = 1024;  // threads per work-group of the y passes
constexpr int FFT_X_THREADS = 256;    // threads per work-group of the x passes
constexpr int FFT_X_PTS = 1024;       // complex points per work-group of the x passes (target)

__global__ void k_adj_save(const Inst *insts, float2 *dpsi, float *dmu, double *dK, int raw);
__global__ void k_adj_load(const Inst *insts, const float2 *spsi, const float *smu, const double *sK);
__global__ void k_adj_logE(const Inst *insts, double *Elog, int n);
__global__ void k_adj_vbar(const double *Elog, int wb, int nsteps, double *vbar);
__global__ void k_adj_zero(AdjState *adj);
__global__ void k_adj_prep_f(const Inst *insts, const float *mubar);
__global__ void k_adj_g(const Inst *insts, const float2 *psin, float2 *g);
__global__ void k_adj_facc(const Inst *insts, float2 *psibar, const float2 *ns_psi, const float2 *ns_g);
__global__ void k_adj_edge_f(const Inst *insts, const float2 *psin);
__global__ void k_adj_jterm(const Inst *insts, float2 *psibar, const float2 *psin, const AdjState *adj);
__global__ void k_adj_maxabs(const Inst *insts, const float2 *psibar);
__global__ void k_adj_assemble(const Inst *insts, const float2 *psibar, const float2 *psim, const float *mum,
                               const float2 *lamW, const float2 *lamW_old, int extrap, const AdjState *adj);
__global__ void k_adj_scale_nu(const Inst *insts, const AdjState *adj, float2 *tmp);
__global__ void k_adj_sources(const Inst *insts, float2 *psibar, float *mubar, float *epsbar, const float2 *psim,
                              const float2 *psin, const float *mum, const float2 *ns_l, const AdjState *adj);
__global__ void k_adj_edge_s(const Inst *insts, const float2 *psim, const float2 *psin, const AdjState *adj);
__global__ void k_adj_reduce(const Inst *insts, int nparts, int which, double ew, AdjState *adj);

__global__ void k_incl_first(const Inst *insts, int inst, const double *centres, const double *diam,
                             int nc, unsigned *first);
__global__ void k_voronoi(const Inst *insts, int inst, const double *seeds, const float *values, int ns,
                          int metric, int axes);
__global__ void k_insulate(const Inst *insts, int inst, const unsigned char *mask);
__global__ void k_incl_first_q(const Inst *insts, int inst, const double *shapes, int nc, unsigned *first);
__global__ void k_incl_count(const unsigned *first, long N, int nc, unsigned *cnt);
__global__ void k_incl_scan(const Inst *insts, int inst, const unsigned *cnt, int nc, double target);
__global__ void k_incl_write(const Inst *insts, int inst, const unsigned *first, float eps_in,
                             float eps_out);

}  // namespace tdgl
