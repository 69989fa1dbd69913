// k_fft.hip -- direct spectral solve of the scalar-potential Poisson equation
// on gfx950 for a periodic x, periodic y, open z box.
//
// The 7-point operator of Sec. 3.2 separates: discrete Fourier modes
// diagonalise its x and y parts (periodic wrap), leaving for every
// (kx, ky) a real tridiagonal system along z (Neumann reflection at the
// open faces):
//     c_z mu_{k-1} - (lam_xy + 2 c_z) mu_k + c_z mu_{k+1} = f^_k,
// with the inner neighbour doubled on the two face rows and
//     lam_xy = c_x (2 - 2 cos(2 pi kx / nx)) + c_y (2 - 2 cos(2 pi ky / ny)).
// Steps: real-to-complex FFT along x (two rows per complex transform), FFT
// along y, the z systems by Thomas' algorithm with precomputed pivots in
// double precision (its two sweeps evaluated as prefix scans of affine maps
// across a wavefront), inverse FFT along y, complex-to-real inverse along x.  The (0, 0) system
// is singular (the constant mode); its right side is projected onto the
// range (zero weighted mean) and its solution shifted to zero weighted mean,
// which fixes sum_m w_m mu_m = 0 for the whole grid.
//
// The FFTs are Stockham auto-sort transforms in LDS: each pass reads all of
// a thread's butterfly inputs into registers, synchronises, and writes the
// outputs to their sorted positions, so a single LDS buffer suffices.
#include "kernels.h"
#include "stencil.h"

namespace tdgl {

namespace {

// In-register DFT of size R (sign -1 forward, +1 inverse).
template <int R>
__device__ __forceinline__ void dft(float2 *v, float sign);

template <>
__device__ __forceinline__ void dft<2>(float2 *v, float) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <>
__device__ __forceinline__ void dft<3>(float2 *v, float sign) {
    const float c1 = -0.5f, s1 = sign * 0.86602540378443864676f;
    const float2 a = v[0], b = v[1], c = v[2];
    const float2 t = cadd(b, c), d = csub(b, c);
    v[0] = cadd(a, t);
    const float2 m = make_float2(a.x + c1 * t.x, a.y + c1 * t.y);
    // i * s1 * d
    const float2 j = make_float2(-s1 * d.y, s1 * d.x);
    v[1] = cadd(m, j);
    v[2] = csub(m, j);
}

template <>
__device__ __forceinline__ void dft<4>(float2 *v, float sign) {
    const float2 a = v[0], b = v[1], c = v[2], d = v[3];
    const float2 s0 = cadd(a, c), s1 = csub(a, c), s2 = cadd(b, d), s3 = csub(b, d);
    // i * sign * s3
    const float2 j = make_float2(-sign * s3.y, sign * s3.x);
    v[0] = cadd(s0, s2);
    v[2] = csub(s0, s2);
    v[1] = cadd(s1, j);
    v[3] = csub(s1, j);
}

template <>
__device__ __forceinline__ void dft<5>(float2 *v, float sign) {
    const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
    const float s1 = sign * 0.95105651629515357212f, s2 = sign * 0.58778525229247312917f;
    const float2 a = v[0];
    const float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    const float2 d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
    v[0] = make_float2(a.x + t1.x + t2.x, a.y + t1.y + t2.y);
    const float2 m1 = make_float2(a.x + c1 * t1.x + c2 * t2.x, a.y + c1 * t1.y + c2 * t2.y);
    const float2 m2 = make_float2(a.x + c2 * t1.x + c1 * t2.x, a.y + c2 * t1.y + c1 * t2.y);
    // i * (s1 d1 + s2 d2) and i * (s2 d1 - s1 d2)
    const float2 e1 = make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y);
    const float2 e2 = make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y);
    const float2 j1 = make_float2(-e1.y, e1.x), j2 = make_float2(-e2.y, e2.x);
    v[1] = cadd(m1, j1);
    v[4] = csub(m1, j1);
    v[2] = cadd(m2, j2);
    v[3] = csub(m2, j2);
}

constexpr int FFT_THREADS = FFT_XY_THREADS;  // threads of the y passes
constexpr int ZS_THREADS = 256;              // threads of the z solve (4 wavefronts)
constexpr int FFT_MAXPTS = FFT_MAXN;  // points per work-group of the y passes (all sequences)


// q = floor(t / d) for 0 <= t < 2^20 and 1 <= d <= 2^13, from a float
// reciprocal: (t + 1/2) / d stays at least 1/(2d) away from an integer,
// far more than the rounding of the product.
__device__ __forceinline__ int fdiv(int t, float inv_d) { return (int)(((float)t + 0.5f) * inv_d); }

// One Stockham pass of radix R over `nseq` sequences of length n stored in
// LDS at buf[s * sstride + e] (element e), by NT threads; MAXC bounds the
// points n * nseq.  Ns = product of the radices of the previous passes.
// tw[k] = exp(-2 pi i k / n) (conjugated for the inverse transform,
// sign = +1).
template <int R, int NT, int MAXC>
__device__ __forceinline__ void fft_pass(float2 *buf, int n, int Ns, int nseq, int sstride, const float2 *tw,
                                         float sign) {
    constexpr int MAXBF = (MAXC / R + NT - 1) / NT;
    const int nb = n / R;
    const int total = nb * nseq;
    const float inv_nb = 1.0f / (float)nb, inv_ns = 1.0f / (float)Ns;
    const int tstep = n / (Ns * R);
    float2 v[MAXBF][R];
    int dst[MAXBF];
#pragma unroll
    for (int i = 0; i < MAXBF; ++i) {
        const int t = threadIdx.x + i * NT;
        if (t < total) {
            const int s = fdiv(t, inv_nb), j = t - s * nb;
            const int jq = fdiv(j, inv_ns), jm = j - jq * Ns;
            const float2 *row = buf + s * sstride;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float2 a = row[j + r * nb];
                if (r == 0 || jm == 0) {
                    v[i][r] = a;
                } else {
                    float2 w = tw[jm * r * tstep];
                    w.y *= -sign;
                    v[i][r] = cmul(a, w);
                }
            }
            dft<R>(v[i], sign);
            dst[i] = s * sstride + jq * Ns * R + jm;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXBF; ++i) {
        const int t = threadIdx.x + i * NT;
        if (t < total) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[dst[i] + r * Ns] = v[i][r];
        }
    }
    __syncthreads();
}

// Full transform of nseq sequences in LDS (natural order in and out).
// P2: the length is a power of two (radices 4 and 2 only), which keeps the
// kernels small enough for two 1024-thread work-groups per CU.
template <bool P2, int NT, int MAXC>
__device__ __forceinline__ void fft_lds(float2 *buf, int n, const int *rad, int nrad, int nseq, int sstride,
                                        const float2 *tw, float sign) {
    int Ns = 1;
    for (int p = 0; p < nrad; ++p) {
        const int R = rad[p];
        if (R == 4) fft_pass<4, NT, MAXC>(buf, n, Ns, nseq, sstride, tw, sign);
        else if (P2 || R == 2) fft_pass<2, NT, MAXC>(buf, n, Ns, nseq, sstride, tw, sign);
        else if (R == 3) fft_pass<3, NT, MAXC>(buf, n, Ns, nseq, sstride, tw, sign);
        else fft_pass<5, NT, MAXC>(buf, n, Ns, nseq, sstride, tw, sign);
        Ns *= R;
    }
}

// Coefficients of row k of the z system of column (kx, ky):
//   a_k mu_{k-1} + b_k mu_k + c_k mu_{k+1} = d_k.
// Face rows carry the doubled inner neighbour (Neumann reflection); the
// singular (0, 0) column has row 0 replaced by mu_0 = 0.
__device__ __forceinline__ void zrow(int k, int nz, double cz, bool singular, double &a, double &c) {
    if (nz == 1 || (singular && k == 0)) { a = 0.0; c = 0.0; return; }
    a = (k == 0) ? 0.0 : (k == nz - 1 ? 2.0 * cz : cz);
    c = (k == nz - 1) ? 0.0 : (k == 0 ? 2.0 * cz : cz);
}

}  // namespace

// Row pairs per work-group of the x passes: about FFT_X_PTS complex points
// (one pair of 1024-point rows), at least one pair.
__host__ __device__ int fft_x_pairs(int nx) {
    int p = FFT_X_PTS / nx;
    return p < 1 ? 1 : (p > 32 ? 32 : p);
}
// Tiles of the y passes over an instance's columns (z, kx), P = nx/2 + 1
// per plane: a work-group holds at most FFT_MAXPTS points (and 1024
// columns).  Where a whole plane's P columns fit, a tile is G whole planes
// (as many as fit); otherwise each plane is cut into ntk tiles of about
// equal width.  Tiles start on a plane or at kx = j TK within one, so their
// rows start on the same 128-byte lines for every plane.
__host__ __device__ FftYPlan fft_y_plan(int nx, int ny, int nz) {
    const int P = nx / 2 + 1;
    int t = FFT_MAXPTS / ny;
    t = t < 1 ? 1 : (t > 1024 ? 1024 : t);
    FftYPlan q;
    if (t >= P) {
        q.G = t / P < nz ? t / P : nz;
        q.ntk = 1;
        q.TK = q.G * P;
    } else {
        q.G = 1;
        q.ntk = (P + t - 1) / t;
        q.TK = (P + q.ntk - 1) / q.ntk;
    }
    q.blocks = ((nz + q.G - 1) / q.G) * q.ntk;
    return q;
}
// LDS stride of the y passes' columns (complex elements).
__host__ __device__ int fft_y_stride(int ny) { return ny + 1; }
// Row pitch (complex elements) of the half spectrum: nx/2 + 1 rounded up to
// 16 elements, so that every row starts on a 128-byte line.
__host__ __device__ int fft_pitch(int nx) { return (nx / 2 + 1 + 15) & ~15; }

// Forward real-to-complex FFT along x of `in` (real rows of length nx) into
// spec (nx/2+1 bins per row), fft_x_pairs(nx) row pairs per work-group of
// FFT_X_THREADS threads; XC bounds the complex points per group (FFT_X_PTS,
// or 4 FFT_X_PTS for longer rows), which sizes the butterfly registers.
// The twiddles are staged in LDS after the data (dynamic LDS: (pairs + 1)
// nx complex values).  Two real rows a, b travel as one complex row
// a + i b; their spectra are separated with the conjugate symmetry
//   A_k = (Z_k + conj Z_{n-k}) / 2,  B_k = (Z_k - conj Z_{n-k}) / (2 i).
// Also the inverse (complex-to-real) along x: dir = +1 reads spec, writes
// `out`.
template <bool P2, int XC>
__global__ __launch_bounds__(FFT_X_THREADS) void k_fft_x(const Inst *__restrict__ insts,
                                                       const int *__restrict__ prefix, int ninst,
                                                       int dir, const float *in_ext, float *out_ext) {
    extern __shared__ float2 sm[];
    const int ii = find_inst(prefix, ninst, blockIdx.x);
    const Inst &I = insts[ii];
    const int nx = I.nx, P = nx / 2 + 1, sp = I.sp;
    const int rows = I.ny * I.nz;
    const int pairs = fft_x_pairs(nx);
    float2 *stw = sm + pairs * nx;
    // loads are issued XB per thread at a time (twiddles, then the rows)
    // before any of them is stored to LDS
    constexpr int XB = 4;
    for (int t0 = threadIdx.x; t0 < nx; t0 += XB * FFT_X_THREADS) {
        float2 v[XB];
#pragma unroll
        for (int c = 0; c < XB; ++c) {
            const int t = t0 + c * FFT_X_THREADS;
            v[c] = t < nx ? ld2((const gf2 *)I.twx, t) : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int c = 0; c < XB; ++c) {
            const int t = t0 + c * FFT_X_THREADS;
            if (t < nx) stw[t] = v[c];
        }
    }
    const gf1 *in = (const gf1 *)(in_ext ? in_ext : I.f);
    gf1 *out = (gf1 *)(out_ext ? out_ext : I.mu);
    gf2 *spec = (gf2 *)I.spec;
    const float inv_nx = 1.0f / (float)nx, inv_p = 1.0f / (float)P;
    // a work-group takes I.fxg consecutive groups of `pairs` row pairs; the
    // loads of the next group are issued before the current one is
    // transformed, so they are in flight while the group works in LDS (PF;
    // for rows longer than FFT_X_PTS the held points would cost too many
    // registers, and each group loads its own).  Sequence s (pair) of a
    // group holds rows row0 + 2 s (real part) and row0 + 2 s + 1; every
    // thread holds ML of a group's points.
    constexpr bool PF = XC <= FFT_X_PTS;
    constexpr int ML = PF ? XC / FFT_X_THREADS : 4;  // points held (PF), or loaded per batch
    const int tot = pairs * nx;
    const int g0 = (blockIdx.x - prefix[ii]) * I.fxg;
    if (dir < 0) {
        float a[ML], b[ML];
        auto load = [&](int row0, int t0) {
#pragma unroll
            for (int c = 0; c < ML; ++c) {
                const int t = t0 + c * FFT_X_THREADS;
                const int s = fdiv(t, inv_nx), e = t - s * nx;
                const int ra = row0 + 2 * s, rb = ra + 1;
                a[c] = (t < tot && ra < rows) ? in[(size_t)ra * nx + e] : 0.f;
                b[c] = (t < tot && rb < rows) ? in[(size_t)rb * nx + e] : 0.f;
            }
        };
        auto stage = [&](int t0) {
#pragma unroll
            for (int c = 0; c < ML; ++c) {
                const int t = t0 + c * FFT_X_THREADS;
                if (t < tot) sm[t] = make_float2(a[c], b[c]);
            }
        };
        if (PF) load(g0 * 2 * pairs, threadIdx.x);
        for (int g = 0; g < I.fxg; ++g) {
            const int row0 = (g0 + g) * 2 * pairs;
            if (row0 >= rows) break;
            if (PF) {
                stage(threadIdx.x);
            } else {
                for (int t0 = threadIdx.x; t0 < tot; t0 += ML * FFT_X_THREADS) {
                    load(row0, t0);
                    stage(t0);
                }
            }
            __syncthreads();
            if (PF && g + 1 < I.fxg) load(row0 + 2 * pairs, threadIdx.x);
            fft_lds<P2, FFT_X_THREADS, XC>(sm, nx, I.xrad, I.nxrad, pairs, nx, stw, -1.f);
            for (int t = threadIdx.x; t < pairs * P; t += FFT_X_THREADS) {
                const int s = fdiv(t, inv_p), k = t - s * P;
                const float2 z = sm[s * nx + k];
                const float2 zc = sm[s * nx + (k == 0 ? 0 : nx - k)];
                // A = (z + conj zc)/2, B = (z - conj zc)/(2i)
                const float2 A = make_float2(0.5f * (z.x + zc.x), 0.5f * (z.y - zc.y));
                const float2 B = make_float2(0.5f * (z.y + zc.y), -0.5f * (z.x - zc.x));
                const int ra = row0 + 2 * s, rb = ra + 1;
                if (ra < rows) st2(spec, (unsigned)ra * sp + k, A);
                if (rb < rows) st2(spec, (unsigned)rb * sp + k, B);
            }
            __syncthreads();
        }
    } else {
        float2 A[ML], B[ML];
        auto load = [&](int row0, int t0) {
#pragma unroll
            for (int c = 0; c < ML; ++c) {
                const int t = t0 + c * FFT_X_THREADS;
                const int s = fdiv(t, inv_nx), k = t - s * nx;
                const int ra = row0 + 2 * s, rb = ra + 1;
                const int kk = k < P ? k : nx - k;
                A[c] = (t < tot && ra < rows) ? ld2(spec, (unsigned)ra * sp + kk) : make_float2(0.f, 0.f);
                B[c] = (t < tot && rb < rows) ? ld2(spec, (unsigned)rb * sp + kk) : make_float2(0.f, 0.f);
            }
        };
        auto stage = [&](int t0) {
#pragma unroll
            for (int c = 0; c < ML; ++c) {
                const int t = t0 + c * FFT_X_THREADS;
                if (t >= tot) continue;
                const int k = t - fdiv(t, inv_nx) * nx;
                float2 a = A[c], b = B[c];
                if (k >= P) { a.y = -a.y; b.y = -b.y; }
                // W = A + i B
                sm[t] = make_float2(a.x - b.y, a.y + b.x);
            }
        };
        if (PF) load(g0 * 2 * pairs, threadIdx.x);
        for (int g = 0; g < I.fxg; ++g) {
            const int row0 = (g0 + g) * 2 * pairs;
            if (row0 >= rows) break;
            if (PF) {
                stage(threadIdx.x);
            } else {
                for (int t0 = threadIdx.x; t0 < tot; t0 += ML * FFT_X_THREADS) {
                    load(row0, t0);
                    stage(t0);
                }
            }
            __syncthreads();
            if (PF && g + 1 < I.fxg) load(row0 + 2 * pairs, threadIdx.x);
            fft_lds<P2, FFT_X_THREADS, XC>(sm, nx, I.xrad, I.nxrad, pairs, nx, stw, +1.f);
            for (int t = threadIdx.x; t < pairs * nx; t += FFT_X_THREADS) {
                const int s = fdiv(t, inv_nx), e = t - s * nx;
                const int ra = row0 + 2 * s, rb = ra + 1;
                const float2 w = sm[t];
                if (ra < rows) out[(size_t)ra * nx + e] = w.x;
                if (rb < rows) out[(size_t)rb * nx + e] = w.y;
            }
            __syncthreads();
        }
    }
}

// FFT along y of the half spectrum, forward (dir = -1) or inverse (+1):
// a work-group takes one tile of fft_y_plan -- TK consecutive kx of one
// plane on tall grids, G whole planes on short ones -- all y.  Consecutive
// tiles share 128-byte lines, so neighbouring logical tiles run on one XCD.
template <bool P2>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_y(const Inst *__restrict__ insts,
                                                       const int *__restrict__ prefix, int ninst,
                                                       int dir) {
    extern __shared__ float2 sm[];
    const int ii = find_inst(prefix, ninst, blockIdx.x);
    const Inst &I = insts[ii];
    const int nx = I.nx, ny = I.ny, nz = I.nz, P = nx / 2 + 1, sp = I.sp;
    const FftYPlan pl = fft_y_plan(nx, ny, nz);
    const int TK = pl.TK;
    const int nblk = prefix[ii + 1] - prefix[ii];
    const int lb = xcd_remap(blockIdx.x - prefix[ii], nblk);
    const int zt = lb / pl.ntk, j = lb - zt * pl.ntk;
    // the tile starts at kx = r0 of plane z0; column c is kx = r0 + c of
    // that plane (per-plane tiles) or kx = c - q P of plane z0 + q, q =
    // floor(c / P) (whole planes, r0 = 0); offsets within a tile fit 32 bits
    const int z0 = zt * pl.G, r0 = j * TK;
    const bool whole = pl.ntk == 1;
    const int tk = whole ? min(pl.G, nz - z0) * P : min(TK, P - r0);
    const unsigned zs = (unsigned)ny * (unsigned)sp;
    const gf2 *__restrict__ specr = (const gf2 *)(I.spec + (size_t)z0 * zs);
    gf2 *__restrict__ specw = (gf2 *)(I.spec + (size_t)z0 * zs);
    const float inv_tk = 1.0f / (float)TK, inv_p = 1.0f / (float)P;
    auto col = [&](int c) -> unsigned {
        if (!whole) return (unsigned)(r0 + c);
        const int q = fdiv(c, inv_p);
        return (unsigned)q * zs + (unsigned)(c - q * P);
    };
    // columns sit ss = ny + 1 apart in LDS: the staging loop writes (and the
    // final loop reads) TK columns per y with consecutive lanes, which a
    // power-of-two stride would put on one bank
    const int ss = fft_y_stride(ny);
    float2 *stw = sm + TK * ss;
    for (int t = threadIdx.x; t < ny; t += FFT_THREADS) stw[t] = ld2((const gf2 *)I.twy, t);
    // loads are issued YB per thread at a time before any of them is
    // stored to LDS
    constexpr int YB = 8;
    const int tot = ny * TK;
    for (int t0 = threadIdx.x; t0 < tot; t0 += YB * FFT_THREADS) {
        float2 v[YB];
#pragma unroll
        for (int q = 0; q < YB; ++q) {
            const int t = t0 + q * FFT_THREADS;
            const int y = fdiv(t, inv_tk), c = t - y * TK;
            v[q] = (t < tot && c < tk) ? ld2(specr, col(c) + (unsigned)(y * sp)) : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int q = 0; q < YB; ++q) {
            const int t = t0 + q * FFT_THREADS;
            const int y = fdiv(t, inv_tk), c = t - y * TK;
            if (t < tot) sm[c * ss + y] = v[q];
        }
    }
    __syncthreads();
    fft_lds<P2, FFT_THREADS, FFT_MAXPTS>(sm, ny, I.yrad, I.nyrad, TK, ss, stw, (float)dir);
    for (int t = threadIdx.x; t < ny * TK; t += FFT_THREADS) {
        const int y = fdiv(t, inv_tk), c = t - y * TK;
        if (c < tk) st2(specw, col(c) + (unsigned)(y * sp), sm[c * ss + y]);
    }
}

// Set-up of the spectral solver of instance `inst`: twiddle tables
// exp(-2 pi i k / n) for x and y (FP64 arguments, rounded once to FP32), and
// for every z system its Thomas pivots ip_k = 1 / (b_k - a_k c'_{k-1}),
// c'_k = c_k ip_k, in FP64, stored column by column at ((ky P + kx) nz + k).
// The operator does not change between steps, so this runs once.
__global__ void k_fft_tables(const Inst *__restrict__ insts, int inst) {
    const Inst &I = insts[inst];
    const int nx = I.nx, ny = I.ny, nz = I.nz, P = nx / 2 + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nx) {
        double s, c;
        sincospi(-2.0 * (double)t / (double)nx, &s, &c);
        I.twx[t] = make_float2((float)c, (float)s);
    }
    if (t < ny) {
        double s, c;
        sincospi(-2.0 * (double)t / (double)ny, &s, &c);
        I.twy[t] = make_float2((float)c, (float)s);
    }
    if (t < ny * P) {
        const int ky = t / P, kx = t - ky * P;
        const double cz = I.cz, cx = I.cx, cy = I.cy;
        const double lam = cx * (2.0 - 2.0 * cospi(2.0 * kx / (double)nx)) +
                           cy * (2.0 - 2.0 * cospi(2.0 * ky / (double)ny));
        const bool singular = (kx == 0 && ky == 0);
        double cprev = 0.0;
        double *ip = I.zip + (size_t)t * nz;
        for (int k = 0; k < nz; ++k) {
            double a, c;
            zrow(k, nz, cz, singular, a, c);
            double b = (nz == 1) ? -lam : -(lam + 2.0 * cz);
            if (singular && k == 0) b = 1.0;
            const double p = 1.0 / (b - a * cprev);
            ip[k] = p;
            cprev = c * p;
        }
    }
}

template __global__ void k_fft_x<false, FFT_X_PTS>(const Inst *, const int *, int, int, const float *, float *);
template __global__ void k_fft_x<true, FFT_X_PTS>(const Inst *, const int *, int, int, const float *, float *);
template __global__ void k_fft_x<false, 4 * FFT_X_PTS>(const Inst *, const int *, int, int, const float *, float *);
template __global__ void k_fft_x<true, 4 * FFT_X_PTS>(const Inst *, const int *, int, int, const float *, float *);
template __global__ void k_fft_y<false>(const Inst *, const int *, int, int);
template __global__ void k_fft_y<true>(const Inst *, const int *, int, int);

// The z systems, one per (kx, ky), in double precision.  A work-group loads
// a tile of ZTK consecutive kx at one ky and all z (coalesced rows); each
// wavefront then solves the columns of the tile, one or two at a time.
// With the pivots of the set-up, Thomas' two sweeps are first-order linear
// recurrences,
//   y_k = -a_k ip_k y_{k-1} + ip_k d_k,   mu_k = -c_k ip_k mu_{k+1} + y_k,
// i.e. compositions of affine maps, which a segment of L lanes evaluates as
// a prefix scan (lane l owns rows l RPL .. l RPL + RPL - 1): compose the
// lane's maps, scan the lane maps across the segment with shuffles, then
// replay the rows from the lane's incoming value.  The result is scaled by
// 1/(nx ny) (the two inverse FFTs are unnormalised).
constexpr int ZTK = FFT_ZTK;
constexpr int ZPAD = ZTK + 1;  // LDS row stride (float2): spreads the column reads over banks
__host__ __device__ size_t fft_z_lds(int nz) { return (size_t)nz * ZPAD * sizeof(float2); }

// Thin boxes (nz <= FFT_ZSERIAL, e.g. a film of one plane): the cost of the
// scan is per system, not per row, so here one lane takes one (kx, ky)
// system, with consecutive lanes on consecutive kx (coalesced rows), and runs
// Thomas' two sweeps with the stored pivots in registers.
__device__ __forceinline__ void zsolve_lane(const Inst &I, int lb) {
    const int nx = I.nx, ny = I.ny, nz = I.nz, P = nx / 2 + 1;
    const int col = lb * ZS_THREADS + threadIdx.x;
    if (col >= ny * P) return;
    const int ky = col / P, kx = col - ky * P;
    const size_t zstride = (size_t)ny * I.sp;
    float2 *spec = I.spec + (size_t)ky * I.sp + kx;
    const double *ipc = I.zip + (size_t)col * nz;
    const double cz = I.cz;
    const double scale = 1.0 / ((double)nx * (double)ny);
    const bool singular = (kx == 0 && ky == 0);
    double yr[FFT_ZSERIAL], yi[FFT_ZSERIAL];
#pragma unroll
    for (int k = 0; k < FFT_ZSERIAL; ++k) {
        const float2 v = k < nz ? spec[(size_t)k * zstride] : make_float2(0.f, 0.f);
        yr[k] = v.x;
        yi[k] = v.y;
    }
    // weighted mean over z (1/2 on the two end rows of an open axis)
    auto wmean = [&](double &mr, double &mi) {
        double sr = 0.0, si = 0.0, sw = 0.0;
#pragma unroll
        for (int k = 0; k < FFT_ZSERIAL; ++k)
            if (k < nz) {
                const double wk = (nz > 1 && (k == 0 || k == nz - 1)) ? 0.5 : 1.0;
                sr += wk * yr[k];
                si += wk * yi[k];
                sw += wk;
            }
        mr = sr / sw;
        mi = si / sw;
    };
    if (singular) {
        // project the right side onto the range and pin row 0
        double mr, mi;
        wmean(mr, mi);
#pragma unroll
        for (int k = 0; k < FFT_ZSERIAL; ++k) {
            yr[k] -= mr;
            yi[k] -= mi;
        }
        yr[0] = 0.0;
        yi[0] = 0.0;
    }
    double ur = 0.0, ui = 0.0;
#pragma unroll
    for (int k = 0; k < FFT_ZSERIAL; ++k)
        if (k < nz) {
            double a, cc;
            zrow(k, nz, cz, singular, a, cc);
            const double ip = ipc[k];
            const double Ak = -a * ip, s = ip * scale;
            ur = Ak * ur + s * yr[k];
            ui = Ak * ui + s * yi[k];
            yr[k] = ur;
            yi[k] = ui;
        }
    double xr = 0.0, xi = 0.0;
#pragma unroll
    for (int k = FFT_ZSERIAL - 1; k >= 0; --k)
        if (k < nz) {
            double a, cc;
            zrow(k, nz, cz, singular, a, cc);
            const double Ck = -cc * ipc[k];
            xr = Ck * xr + yr[k];
            xi = Ck * xi + yi[k];
            yr[k] = xr;
            yi[k] = xi;
        }
    if (singular) {
        // shift the constant mode to zero weighted mean
        double mr, mi;
        wmean(mr, mi);
#pragma unroll
        for (int k = 0; k < FFT_ZSERIAL; ++k) {
            yr[k] -= mr;
            yi[k] -= mi;
        }
    }
#pragma unroll
    for (int k = 0; k < FFT_ZSERIAL; ++k)
        if (k < nz) spec[(size_t)k * zstride] = make_float2((float)yr[k], (float)yi[k]);
}

// RMAX: z rows per lane of the scan for every instance of the launch (2 up
// to nz = 64, else 4): fewer registers, more work-groups per CU for the
// shallow boxes.  Columns of up to 32 RMAX rows are scanned on 32-lane
// segments (two columns per wavefront), deeper ones on the whole
// wavefront.
template <int RMAX>
__global__ __launch_bounds__(ZS_THREADS) void k_fft_zsolve(const Inst *__restrict__ insts,
                                                            const int *__restrict__ prefix,
                                                            int ninst) {
    extern __shared__ float2 tile[];
    const int ii = find_inst(prefix, ninst, blockIdx.x);
    const Inst &I = insts[ii];
    if (I.nz <= FFT_ZSERIAL) {
        zsolve_lane(I, blockIdx.x - prefix[ii]);
        return;
    }
    const int nx = I.nx, ny = I.ny, nz = I.nz, P = nx / 2 + 1, sp = I.sp;
    const int ntk = (P + ZTK - 1) / ZTK;
    const int lb = blockIdx.x - prefix[ii];
    const int ky = lb / ntk, kx0 = (lb - ky * ntk) * ZTK;
    const int tk = min(ZTK, P - kx0);
    const unsigned zstride = (unsigned)ny * (unsigned)sp;
    gf2 *spec = (gf2 *)(I.spec + (size_t)ky * sp + kx0);
    // loads are issued ZB per thread at a time before any of them is
    // stored to LDS
    constexpr int ZB = 8;
    const int tot = nz * ZTK;
    for (int t0 = threadIdx.x; t0 < tot; t0 += ZB * ZS_THREADS) {
        float2 v[ZB];
#pragma unroll
        for (int q = 0; q < ZB; ++q) {
            const int t = t0 + q * ZS_THREADS;
            const int k = t / ZTK, c = t - k * ZTK;
            v[q] = (t < tot && c < tk) ? ld2(spec, (unsigned)k * zstride + c) : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int q = 0; q < ZB; ++q) {
            const int t = t0 + q * ZS_THREADS;
            const int k = t / ZTK, c = t - k * ZTK;
            if (t < tot) tile[k * ZPAD + c] = v[q];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double cz = I.cz;
    const double scale = 1.0 / ((double)nx * (double)ny);
    static_assert(RMAX * 64 <= FFT_ZMAX, "scan rows per lane");
    // the scan runs on segments of L lanes, 64 / L columns per wavefront at
    // a time: the scan's cost is per column, so columns of up to 32 RMAX
    // rows take 32-lane segments (with nz <= 32 the same maps are composed
    // in the same order as on 64 lanes, whose upper half would only hold
    // identity maps)
    const int L = nz <= 32 * RMAX ? 32 : 64;
    const int S = 64 / L;
    const int sl = lane & (L - 1), sg = lane / L;
    const int rpl = (nz + L - 1) / L;
    const int k0 = sl * rpl;
    // pivots of the wavefront's next column are loaded while the current
    // one is solved
    double ipn[RMAX];
    auto load_piv = [&](int c, double *dst) {
        const gd1 *ipc = (const gd1 *)(I.zip + ((size_t)ky * P + kx0 + c) * nz);
#pragma unroll
        for (int q = 0; q < RMAX; ++q) {
            const int k = k0 + q;
            dst[q] = (c < tk && q < rpl && k < nz) ? ipc[k] : 0.0;
        }
    };
    load_piv(w * S + sg, ipn);
    for (int c = w * S + sg; c < tk; c += 4 * S) {
        const int kx = kx0 + c;
        const bool singular = (kx == 0 && ky == 0);
        double yr[RMAX], yi[RMAX], ip[RMAX];
#pragma unroll
        for (int q = 0; q < RMAX; ++q) ip[q] = ipn[q];
        load_piv(c + 4 * S, ipn);
#pragma unroll
        for (int q = 0; q < RMAX; ++q) {
            const int k = k0 + q;
            const bool ok = q < rpl && k < nz;
            const float2 v = ok ? tile[k * ZPAD + c] : make_float2(0.f, 0.f);
            yr[q] = v.x;
            yi[q] = v.y;
        }
        // the singular column: project the right side onto the range
        // (zero weighted mean) and pin row 0
        if (singular) {
            double sr = 0.0, si = 0.0, sw = 0.0;
#pragma unroll
            for (int q = 0; q < RMAX; ++q) {
                const int k = k0 + q;
                if (q < rpl && k < nz) {
                    const double wk = (nz > 1 && (k == 0 || k == nz - 1)) ? 0.5 : 1.0;
                    sr += wk * yr[q];
                    si += wk * yi[q];
                    sw += wk;
                }
            }
            for (int o = L / 2; o > 0; o >>= 1) {
                sr += __shfl_xor(sr, o, L);
                si += __shfl_xor(si, o, L);
                sw += __shfl_xor(sw, o, L);
            }
#pragma unroll
            for (int q = 0; q < RMAX; ++q) {
                yr[q] -= sr / sw;
                yi[q] -= si / sw;
                if (k0 + q == 0) { yr[q] = 0.0; yi[q] = 0.0; }
            }
        }
        // forward sweep: lane map y_out = A y_in + B
        double A = 1.0, Br = 0.0, Bi = 0.0;
#pragma unroll
        for (int q = 0; q < RMAX; ++q) {
            const int k = k0 + q;
            if (q < rpl && k < nz) {
                double a, cc;
                zrow(k, nz, cz, singular, a, cc);
                const double Ak = -a * ip[q], s = ip[q] * scale;
                Br = Ak * Br + s * yr[q];
                Bi = Ak * Bi + s * yi[q];
                A = Ak * A;
            }
        }
        for (int o = 1; o < L; o <<= 1) {
            const double pA = __shfl_up(A, o, L), pr = __shfl_up(Br, o, L), pi = __shfl_up(Bi, o, L);
            if (sl >= o) {
                Br = A * pr + Br;
                Bi = A * pi + Bi;
                A = A * pA;
            }
        }
        double ur = __shfl_up(Br, 1, L), ui = __shfl_up(Bi, 1, L);
        if (sl == 0) { ur = 0.0; ui = 0.0; }
#pragma unroll
        for (int q = 0; q < RMAX; ++q) {
            const int k = k0 + q;
            if (q < rpl && k < nz) {
                double a, cc;
                zrow(k, nz, cz, singular, a, cc);
                const double Ak = -a * ip[q], s = ip[q] * scale;
                ur = Ak * ur + s * yr[q];
                ui = Ak * ui + s * yi[q];
                yr[q] = ur;
                yi[q] = ui;
            }
        }
        // backward sweep: lane map x_first = C x_in + D, x_in = mu of the
        // next lane's first row
        double C = 1.0, Dr = 0.0, Di = 0.0;
#pragma unroll
        for (int q = RMAX - 1; q >= 0; --q) {
            const int k = k0 + q;
            if (q < rpl && k < nz) {
                double a, cc;
                zrow(k, nz, cz, singular, a, cc);
                const double Ck = -cc * ip[q];
                Dr = Ck * Dr + yr[q];
                Di = Ck * Di + yi[q];
                C = Ck * C;
            }
        }
        for (int o = 1; o < L; o <<= 1) {
            const double nC = __shfl_down(C, o, L), nr = __shfl_down(Dr, o, L), ni = __shfl_down(Di, o, L);
            if (sl + o < L) {
                Dr = C * nr + Dr;
                Di = C * ni + Di;
                C = C * nC;
            }
        }
        double xr = __shfl_down(Dr, 1, L), xi = __shfl_down(Di, 1, L);
        if (sl == L - 1) { xr = 0.0; xi = 0.0; }
#pragma unroll
        for (int q = RMAX - 1; q >= 0; --q) {
            const int k = k0 + q;
            if (q < rpl && k < nz) {
                double a, cc;
                zrow(k, nz, cz, singular, a, cc);
                const double Ck = -cc * ip[q];
                xr = Ck * xr + yr[q];
                xi = Ck * xi + yi[q];
                yr[q] = xr;
                yi[q] = xi;
            }
        }
        if (singular) {
            // shift the constant mode to zero weighted mean
            double sr = 0.0, si = 0.0, sw = 0.0;
#pragma unroll
            for (int q = 0; q < RMAX; ++q) {
                const int k = k0 + q;
                if (q < rpl && k < nz) {
                    const double wk = (nz > 1 && (k == 0 || k == nz - 1)) ? 0.5 : 1.0;
                    sr += wk * yr[q];
                    si += wk * yi[q];
                    sw += wk;
                }
            }
            for (int o = L / 2; o > 0; o >>= 1) {
                sr += __shfl_xor(sr, o, L);
                si += __shfl_xor(si, o, L);
                sw += __shfl_xor(sw, o, L);
            }
#pragma unroll
            for (int q = 0; q < RMAX; ++q) {
                yr[q] -= sr / sw;
                yi[q] -= si / sw;
            }
        }
#pragma unroll
        for (int q = 0; q < RMAX; ++q) {
            const int k = k0 + q;
            if (q < rpl && k < nz) tile[k * ZPAD + c] = make_float2((float)yr[q], (float)yi[q]);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nz * ZTK; t += ZS_THREADS) {
        const int k = t / ZTK, c = t - k * ZTK;
        if (c < tk) st2(spec, (unsigned)k * zstride + c, tile[k * ZPAD + c]);
    }
}

template __global__ void k_fft_zsolve<2>(const Inst *, const int *, int);
template __global__ void k_fft_zsolve<4>(const Inst *, const int *, int);

}  // namespace tdgl
