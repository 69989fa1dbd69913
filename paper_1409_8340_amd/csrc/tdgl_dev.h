// tdgl_dev.h -- device-side data structures and helpers of libtdgl (gfx950).
//
// One "instance" is one independent TDGL system.  Its device descriptor
// (Inst) carries sizes, coefficients and pointers into the caller's
// workspace; kernels receive the array of descriptors of a context and map
// their work-groups onto instances through a prefix table, so a single
// launch advances every instance of a batch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdgl {

constexpr int kMaxIter = 256;    // Jacobi sweeps per step (cap)
constexpr int kMaxCycles = 64;   // multigrid cycles per step (cap)
constexpr int kMaxLevels = 16;   // multigrid levels
constexpr int NSLOT = 32;        // atomic slots per convergence row

// Tile of the 2.5D stencil kernels: 64 x-columns (one wavefront wide) by
// 4R y-rows; 256 threads, each owning R consecutive rows of one column, march
// through a chunk of z planes.  R = 2 or 4 (chosen per context).
constexpr int TX = 64;
constexpr int WG = 256;
constexpr int LDX = TX + 2;            // LDS plane pitch (float2 units)

// Tile of the multigrid kernels: 64 x 4 columns, z chunk.
constexpr int MTX = 64;
constexpr int MTY = 4;

// Scalar state of one instance, kept in device memory so that a whole step
// runs without host round trips.  FP64 for everything that accumulates.
struct DevState {
    double K;         // current phase (Sec. 2.2)
    double t;         // simulated time
    double V_sum;     // sum of E over the voltage window
    double E_last;    // last E_x
    double J_last;    // last J_av
    double n;         // steps taken
    double n_avg;     // steps in window
    double f_mean;    // weighted mean of the last Poisson right side
    double mu_mean;   // weighted mean of mu as stored after the last solve
    double F;         // free energy (observables)
    double psi2;      // mean |psi|^2 (observables)
    double Jext;      // applied current
    double Bx, Bz;    // field (quantised)
    int cur;          // index of the psi buffer holding the current state
    int sweeps;       // Jacobi sweeps of the last step
    int capped;       // last solve hit the cap
    int mu_cycles;    // multigrid cycles of the last step
    int mu_capped;
    int in_window;    // accumulate E into V_sum
    int n_used;       // inclusion generator: spheres used
    float last_res2;  // max |r|^2 tested by the last sweep of the last solve
    double frac;      // inclusion generator: covered fraction
    float mu_last_res;// Poisson residual max-norm at the end of the last solve
    int pad2;
    int fix;          // two-sweep mode: the result needs the corrective sweep
    int pad3;
    // step statistics accumulated on the device (graph-replayed steps)
    double acc_sweeps, acc_capped, acc_mu_cycles, acc_mu_capped, acc_passes;
    int acc_sw_min, acc_sw_max;
    double By;        // y component of a yz-plane field (quantised)
    int yz;           // 1: the field lies in the yz plane (Eq. B_yz)
    int pad4;
};

// Scalars of the adjoint sweep over one step (device resident).
struct AdjState {
    double Kbar;   // adjoint of K, accumulated backwards through the steps
    double Jbar;   // adjoint of J_av of the current step
    double scale;  // normalisation of the adjoint Crank-Nicolson system
    double pad;
};

struct MGLevel {
    int nx, ny, nz, N;
    int per[3];
    const float *am[3], *ap[3];   // FV coefficients to the -/+ neighbour, per axis index
    const float *vol[3];          // control volume factors per axis index
    float *mu[2];                 // ping-pong iterates (level 0: mu[0] is the solution)
    float *rhs;                   // right side (level 0: f)
    float *r;                     // residual
    // transfer to the next coarser level (unused on the coarsest)
    const int *pk[3];             // prolongation: per fine index two coarse indices
    const float *pw[3];           //   and their weights
    const int *rk[3];             // restriction: per coarse index three fine indices
    const float *rw[3];           //   and their weights (volume-weighted)
    double vsum;                  // sum of control volumes
    int tiles_x, tiles_y, tiles_z, chunk;
};

struct Inst {
    int nx, ny, nz, N;
    int per[3];          // 1: periodic axis, 0: open
    int driven;
    float cx, cy, cz;    // 1/hx^2, 1/hy^2, 1/(g^2 hz^2); 0 on an open one-node axis
    float S2;            // 2 (cx + cy + cz)
    float ht2;           // ht / 2 with ht = dt / u
    float u;
    float tol;           // Jacobi stop threshold on max |r|^2
    float zeta_max;      // Langevin amplitude (0: no noise)
    unsigned seed0, seed1;  // key of the noise generator
    float mu_tol;
    double hx, hy, hz, dt;
    double w_sum;        // sum of node weights (1/2 per open face)
    float2 *psi[2];
    float2 *bh;          // b / M_mm
    float2 *dh;          // (ht/2) / M_mm
    float *eps;
    float *mu;           // == lev[0].mu[0]
    float *f;            // == lev[0].rhs
    float2 *ux;          // x links per y index: exp(i hx (K + Bz ybar_j))
    float2 *uz;          // z links per y index: exp(-i hz Bx ybar_j)
    float2 *P;           // y wrap phase per (i,k): exp(i (i hx Ly Bz - k hz Ly Bx))
    float2 *wz;          // x-link factor per z plane: exp(-i hx By k hz) (yz field), else 1
    float2 *zs;          // z-seam phase per x of a yz field on a periodic z axis: psi_{i,j,-1} =
                         // zs[i] psi_{i,j,nz-1}, zs[i] = exp(-i xbar_i Lz By); else 1
    DevState *st;
    // Convergence words.  Work-groups reduce their maxima with atomics into
    // one of NSLOT slots (chosen by block index) placed in separate cache
    // lines, so that thousands of groups do not serialise on one address;
    // readers take the max over the slots.  Word (row l, slot s) of this
    // instance is res[(l * NSLOT + s) * rstride]; the instances of a context
    // are interleaved (rstride >= instance count) so one copy polls a batch.
    unsigned *res;       // row l: max |r|^2 of the input iterate of sweep l (float bits)
    unsigned *mures;     // row c: Poisson residual max-norm at the top of cycle c
    int rstride;
    float mu_rtol;       // Poisson stop relative to the residual at the top of cycle 0
    int max_iter, mu_max_cycles;
    double *part;        // per-work-group partial sums
    int part_cap;
    int tiles_x, tiles_y, tiles_z, chunk;   // stencil tiling (chunk: z planes per tile)
    int chunk2, tiles_z2;                   // z planes per work-group of the two-sweep super-tile kernel
    int tys;                                // rows of its super-tiles (16 or 32)
    int tiles_y4, chunk4, tiles_z4;         // 64 x 16 tiling of the Poisson right side with four rows per thread
    int rows;                               // rows per thread R (tile 64 x 4R)
    // two-sweep passes: (x, y) tiles that are not interior (tile_interior2),
    // as txi + tiles_x tyi in increasing order, and the z planes per
    // work-group of their kernel
    int *btile;
    int nbt, bchunk;
    int seam2;           // super-tiles start at y = 0 and cover the quasi-periodic y seam
    float2 *sring;       // seam2: Jacobi updates of rows ny-1 and 0, [plane][2][x], made per two-sweep pass
    // two-sweep super-tiles: copies of b/M and (ht/2)/M of the nodes beside
    // each 64-column tile column c (x = 64c - 1 below edge_r, x = 64c + 64
    // from edge_r), laid out [c][z][y][2], so that a super-tile reads the 16
    // rows of one side as one run instead of a line per row (null when the
    // tiling has no two-sweep passes or the offsets do not fit 32 bits);
    // edge_ob, edge_od: edge relative to bh and to dh, in complex values
    float2 *edge;
    unsigned edge_r, edge_ob, edge_od;
                         // (periodic y, ny a multiple of the super-tile height); else they start one tile row in
    int nlev;
    MGLevel lev[kMaxLevels];
    // direct spectral Poisson solve (periodic x and y, open z)
    int fft;             // 1: the Poisson equation is solved by FFT, 0: by multigrid
    int nxrad, nyrad;    // FFT radix plans along x and y
    int xrad[16], yrad[16];
    float2 *spec;        // half spectrum, nz * ny rows of pitch sp >= nx/2 + 1
    int sp;              // row pitch of spec (complex elements)
    int fxg;             // row-pair groups per work-group of the x passes (their loads overlap the transforms)
    int fcpt;            // cells per thread of the flat reductions (J_av, |psi|^2)
    float2 *twx, *twy;   // twiddles exp(-2 pi i k / n) along x and y
    double *zip;         // Thomas pivots of the z systems, ny * (nx/2 + 1) columns of nz
};

// ---------------------------------------------------------------------------
// helpers
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // conj(a) * b
    return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float s, float2 a) { return make_float2(s * a.x, s * a.y); }
__device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ float2 cdiv(float2 a, float2 b) {
    float d = 1.0f / (b.x * b.x + b.y * b.y);
    return make_float2((a.x * b.x + a.y * b.y) * d, (a.y * b.x - a.x * b.y) * d);
}

// Work-groups are dispatched round-robin over the 8 XCDs (blockIdx % 8).
// Remap so that each XCD receives a contiguous range of logical tiles: tiles
// that share halos then share that XCD's L2.
// The plain-load two-sweep kernel works on 64 x TYS super-tiles: M =
// TYS / 4R wavefront groups of the 64 x 4R tile, so WG * M threads.  TYS is
// a tiling choice, 16 or 32 rows (32 needs R >= 2: R = 2 then takes 1024
// threads, R = 4 512); by default 32 for R = 2 and 4, 16 for R = 1 (1024
// threads).  The taller the tile, the smaller the share of its two-node y
// halo and of its ring rows, which the neighbouring super-tiles read again;
// the shorter, the more groups per CU.
__host__ __device__ constexpr int tys_default(int rows) { return rows == 1 ? 16 : 32; }
constexpr int TYS_MIN = 16;  // the smallest super-tile height (every other one is a multiple of it)
__host__ __device__ constexpr int sweep2i_mult(int rows, int tys) { return tys / (4 * rows); }
// Super-tile rows start one 64 x 4R tile row into the grid (y0 = 4R + TYS j,
// j < sweep2i_rows), so that a quasi-periodic y seam leaves only the first
// and the last tile row to the general kernel -- unless the instance is
// periodic in y with ny a multiple of TYS (seam2): then they start at
// y0 = TYS j and the super-tiles on the seam apply its phase themselves.
__host__ __device__ inline int sweep2i_rows(int ny, int rows, int tys, bool seam) {
    if (seam) return ny / tys;
    const int r = ny - 4 * rows;
    return r > 0 ? (r + tys - 1) / tys : 0;
}
__host__ __device__ inline int sweep2i_y0(int j, int rows, int tys, bool seam) {
    return (seam ? 0 : 4 * rows) + tys * j;
}
__host__ __device__ inline bool seam2_ok(bool yper, int ny, int tys) { return yper && ny % tys == 0; }

// A tile every node of which, with its two-node halo, is a real node or a
// plain periodic image in x: full in x, and its halo inside the grid in y
// and (unless x is periodic) in x -- no quasi-periodic phase, no open-face
// ghost, no node outside the grid.  Such tiles take the plain-load
// two-sweep kernel.
// seam: the y halo may cross the periodic y seam (seam2 instances).
__host__ __device__ inline bool tile_interior2(int x0, int y0, int tyv, int nx, int ny, bool xper,
                                               bool seam = false) {
    const bool xin = xper ? (x0 + TX <= nx) : (x0 >= 2 && x0 + TX + 2 <= nx);
    return xin && (seam ? y0 + tyv <= ny : (y0 >= 2 && y0 + tyv + 2 <= ny));
}

// Buffer of the input psi^(l) of the two-sweep pass l, relative to cur:
// pairs from odd l follow psi^(1) (in cur ^ 1), pairs from even l follow one
// single sweep's psi^(2) (in cur); either way consecutive pairs alternate.
__host__ __device__ inline int pair_src(int l) { return ((l + 2 - (l & 1)) >> 1) & 1; }

// Full passes over the grid after the assemble kernel for a solve of s
// sweeps (k_solve_finalize's schedules; the corrective sweep not counted).
__host__ __device__ inline int pass_count(int fused, int s) {
    if (fused == 0) return s - 1;
    if (fused == 1) return s / 2;
    return s == 1 ? 0 : (s + 1) / 2;
}

// Slots (complex-value index of the b/M copy; (ht/2)/M follows it) of the
// side copies of node (x, y, z), -1 where it is not beside a tile column:
// x = 64c - 1 is the left side of column c, x = 64c + 64 its right side
// (across the periodic x wrap where there is one).
__device__ __forceinline__ void edge_slots(const Inst &I, int x, int y, int z, int &el, int &er) {
    const int nx = I.nx;
    const bool xper = I.per[0] != 0;
    int cl = -1, cr = -1;
    if (((x + 1) & 63) == 0 && x + 1 < nx) cl = (x + 1) >> 6;
    else if (xper && x == nx - 1) cl = 0;
    if ((x & 63) == 0 && x >= 64) cr = (x >> 6) - 1;
    else if (xper && x == 0 && (nx & 63) == 0) cr = I.tiles_x - 1;
    const unsigned zy = (unsigned)z * (unsigned)I.ny + (unsigned)y, cz = (unsigned)I.nz * (unsigned)I.ny;
    el = cl >= 0 ? (int)(2u * ((unsigned)cl * cz + zy)) : -1;
    er = cr >= 0 ? (int)(I.edge_r + 2u * ((unsigned)cr * cz + zy)) : -1;
}

__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, l = b >> 3;
    return x * q + (x < r ? x : r) + l;
}

// Instance owning logical block `b` of a batched launch (prefix has ninst+1
// entries; instance i owns [prefix[i], prefix[i+1])).
__device__ __forceinline__ int find_inst(const int *__restrict__ prefix, int ninst, int b) {
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Convergence rows: slot word for an atomic update and the row maximum.
__device__ __forceinline__ unsigned *row_slot(unsigned *base, int rstride, int row, int block) {
    return base + ((size_t)row * NSLOT + (block & (NSLOT - 1))) * rstride;
}
// The words are read with device-scope atomic loads: in a persistent
// kernel they were written by other work-groups' atomics since this
// work-group last looked, and no cached copy may answer.  The whole
// wavefront reads a row at once: lane s loads slot s mod NSLOT, a butterfly
// over each half-wave combines them, and every lane returns the row
// maximum.  All 64 lanes must be active.
__device__ __forceinline__ float row_max_wave(const unsigned *base, int rstride, int row) {
    static_assert(NSLOT == 32, "one slot per lane of a half-wave");
    const int s = (int)(threadIdx.x & (NSLOT - 1));
    unsigned m = __hip_atomic_load(base + ((size_t)row * NSLOT + s) * rstride, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int o = NSLOT / 2; o >= 1; o >>= 1) {
        const unsigned v = (unsigned)__shfl_xor((int)m, o, 64);
        m = v > m ? v : m;
    }
    return __uint_as_float(m);
}

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds, each
// two 32 x 32 -> 64-bit products of counter words with fixed multipliers,
// the high halves mixed with the other two words and the key, the key
// advanced by two Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(unsigned c[4], unsigned k0, unsigned k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const unsigned lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const unsigned lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const unsigned n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}
// 2 zeta_m of step n (the Langevin term of Eq. b enters as (ht/2) 2 zeta):
// the first two words of Philox4x32-10 at counter (m, n lo, n hi, 0) under
// the instance's key, each mapped to (2 (r >> 8) - (2^24 - 1)) 2^-24, an
// exact FP32 value in (-1, 1), times 2 zeta_max (the doubling is exact).
__device__ __forceinline__ float2 langevin2(const Inst &I, unsigned m, unsigned long long n) {
    unsigned c[4] = {m, (unsigned)n, (unsigned)(n >> 32), 0u};
    philox4x32_10(c, I.seed0, I.seed1);
    const float s = 2.f * I.zeta_max;
    const float a = (float)(2 * (int)(c[0] >> 8) - 16777215) * 0x1p-24f;
    const float b = (float)(2 * (int)(c[1] >> 8) - 16777215) * 0x1p-24f;
    return make_float2(s * a, s * b);
}

// Convergence value v of one (row, instance) handed to the host: one
// 64-bit system-scope store into pinned host memory, the high word the
// solve's sequence number so that the host tells this solve's value from an
// older one without clearing the buffer.
__device__ __forceinline__ void publish(unsigned long long *w, unsigned seq, float v) {
    const unsigned long long x = ((unsigned long long)seq << 32) | (unsigned long long)__float_as_uint(v);
    __hip_atomic_store(w, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Node weight: 1/2 per open face the node lies on (trapezoid rule).
__device__ __forceinline__ float node_w(const Inst &I, int x, int y, int k) {
    float w = 1.f;
    if (!I.per[0] && I.nx > 1 && (x == 0 || x == I.nx - 1)) w *= 0.5f;
    if (!I.per[1] && I.ny > 1 && (y == 0 || y == I.ny - 1)) w *= 0.5f;
    if (!I.per[2] && I.nz > 1 && (k == 0 || k == I.nz - 1)) w *= 0.5f;
    return w;
}

// Max-reduction of non-negative floats over a work-group into one word
// (float bits compare as unsigned for non-negative values; a NaN's bits
// exceed +inf's, so a NaN wins and is never taken for convergence).
template <int NT>
__device__ __forceinline__ void wg_max_to(unsigned *dst, float v, float *lds_scratch) {
    unsigned u = __float_as_uint(v);
    for (int o = 32; o > 0; o >>= 1) {
        unsigned w = __shfl_xor(u, o, 64);
        u = (w > u) ? w : u;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) lds_scratch[wv] = __uint_as_float(u);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned m = 0;
        for (int i = 0; i < NT / 64; ++i) {
            unsigned w = __float_as_uint(lds_scratch[i]);
            m = (w > m) ? w : m;
        }
        atomicMax(dst, m);
    }
}

// Sum of doubles over a work-group; thread 0 returns the total.
template <int NT>
__device__ __forceinline__ double wg_sum(double v, double *lds_scratch) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds_scratch[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i) s += lds_scratch[i];
    return s;
}

}  // namespace tdgl
