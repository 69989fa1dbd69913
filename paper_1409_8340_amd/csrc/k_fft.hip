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
// along y, the z systems by parallel cyclic reduction in double precision,
// inverse FFT along y, complex-to-real inverse along x.  The (0, 0) system
// is singular (the constant mode); its right side is projected onto the
// range (zero weighted mean) and its solution shifted to zero weighted mean,
// which fixes sum_m w_m mu_m = 0 for the whole grid.
//
// The FFTs are Stockham auto-sort transforms in LDS: each pass reads all of
// a thread's butterfly inputs into registers, synchronises, and writes the
// outputs to their sorted positions, so a single LDS buffer suffices.
#include "kernels.h"

namespace tdgl {

namespace {

// exp(i pi x) for x in [-2, 2]
__device__ __forceinline__ float2 expi_pi(float x) {
    float s, c;
    sincospif(x, &s, &c);
    return make_float2(c, s);
}

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

constexpr int FFT_THREADS = 256;
constexpr int FFT_MAXPTS = FFT_MAXN;  // points per work-group (all sequences)

// One Stockham pass of radix R over `nseq` sequences of length n stored in
// LDS at buf[s * sstride + e] (element e).  Ns = product of the radices of
// the previous passes.
template <int R>
__device__ void fft_pass(float2 *buf, int n, int Ns, int nseq, int sstride, float sign) {
    constexpr int MAXBF = (FFT_MAXPTS / R + FFT_THREADS - 1) / FFT_THREADS;
    const int nb = n / R;
    const int total = nb * nseq;
    float2 v[MAXBF][R];
    int dst[MAXBF];
#pragma unroll
    for (int i = 0; i < MAXBF; ++i) {
        const int t = threadIdx.x + i * FFT_THREADS;
        if (t < total) {
            const int s = t / nb, j = t - s * nb;
            const int jm = j % Ns;
            const float x = sign * 2.0f * (float)jm / (float)(Ns * R);
            float2 *row = buf + s * sstride;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float2 a = row[j + r * nb];
                v[i][r] = (r == 0 || jm == 0) ? a : cmul(a, expi_pi(x * r));
            }
            dft<R>(v[i], sign);
            dst[i] = s * sstride + (j / Ns) * Ns * R + jm;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXBF; ++i) {
        const int t = threadIdx.x + i * FFT_THREADS;
        if (t < total) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[dst[i] + r * Ns] = v[i][r];
        }
    }
    __syncthreads();
}

// Full transform of nseq sequences in LDS (natural order in and out).
__device__ void fft_lds(float2 *buf, int n, const int *rad, int nrad, int nseq, int sstride, float sign) {
    int Ns = 1;
    for (int p = 0; p < nrad; ++p) {
        const int R = rad[p];
        if (R == 4) fft_pass<4>(buf, n, Ns, nseq, sstride, sign);
        else if (R == 2) fft_pass<2>(buf, n, Ns, nseq, sstride, sign);
        else if (R == 3) fft_pass<3>(buf, n, Ns, nseq, sstride, sign);
        else fft_pass<5>(buf, n, Ns, nseq, sstride, sign);
        Ns *= R;
    }
}

}  // namespace

// Row pairs per work-group of the x passes: 2 * pairs * nx <= FFT_MAXPTS.
__host__ __device__ int fft_x_pairs(int nx) {
    int p = FFT_MAXPTS / (2 * nx);
    return p < 1 ? 1 : (p > 32 ? 32 : p);
}
// kx columns per work-group of the y passes: TK * ny <= FFT_MAXPTS.
__host__ __device__ int fft_y_cols(int ny) {
    int t = FFT_MAXPTS / ny;
    return t < 1 ? 1 : (t > 16 ? 16 : t);
}

// Forward real-to-complex FFT along x of `in` (real rows of length nx) into
// spec (nx/2+1 bins per row).  Two real rows a, b travel as one complex row
// a + i b; their spectra are separated with the conjugate symmetry
//   A_k = (Z_k + conj Z_{n-k}) / 2,  B_k = (Z_k - conj Z_{n-k}) / (2 i).
// Also the inverse (complex-to-real) along x: dir = +1 reads spec, writes
// `out`.
__global__ __launch_bounds__(FFT_THREADS) void k_fft_x(const Inst *__restrict__ insts,
                                                       const int *__restrict__ prefix, int ninst,
                                                       int dir, const float *in_ext, float *out_ext) {
    extern __shared__ float2 sm[];
    const int ii = find_inst(prefix, ninst, blockIdx.x);
    const Inst &I = insts[ii];
    const int nx = I.nx, P = nx / 2 + 1;
    const int rows = I.ny * I.nz;
    const int pairs = fft_x_pairs(nx);
    const int row0 = (blockIdx.x - prefix[ii]) * 2 * pairs;
    const float *in = in_ext ? in_ext : I.f;
    float *out = out_ext ? out_ext : I.mu;
    float2 *spec = I.spec;
    // sequence s (pair) holds rows row0 + 2 s (real part) and row0 + 2 s + 1
    if (dir < 0) {
        for (int t = threadIdx.x; t < pairs * nx; t += FFT_THREADS) {
            const int s = t / nx, e = t - s * nx;
            const int ra = row0 + 2 * s, rb = ra + 1;
            const float a = ra < rows ? in[(size_t)ra * nx + e] : 0.f;
            const float b = rb < rows ? in[(size_t)rb * nx + e] : 0.f;
            sm[s * nx + e] = make_float2(a, b);
        }
        __syncthreads();
        fft_lds(sm, nx, I.xrad, I.nxrad, pairs, nx, -1.f);
        for (int t = threadIdx.x; t < pairs * P; t += FFT_THREADS) {
            const int s = t / P, k = t - s * P;
            const float2 z = sm[s * nx + k];
            const float2 zc = sm[s * nx + (k == 0 ? 0 : nx - k)];
            // A = (z + conj zc)/2, B = (z - conj zc)/(2i)
            const float2 A = make_float2(0.5f * (z.x + zc.x), 0.5f * (z.y - zc.y));
            const float2 B = make_float2(0.5f * (z.y + zc.y), -0.5f * (z.x - zc.x));
            const int ra = row0 + 2 * s, rb = ra + 1;
            if (ra < rows) spec[(size_t)ra * P + k] = A;
            if (rb < rows) spec[(size_t)rb * P + k] = B;
        }
    } else {
        for (int t = threadIdx.x; t < pairs * nx; t += FFT_THREADS) {
            const int s = t / nx, k = t - s * nx;
            const int ra = row0 + 2 * s, rb = ra + 1;
            const bool lo = k < P;
            const int kk = lo ? k : nx - k;
            float2 A = ra < rows ? spec[(size_t)ra * P + kk] : make_float2(0.f, 0.f);
            float2 B = rb < rows ? spec[(size_t)rb * P + kk] : make_float2(0.f, 0.f);
            if (!lo) { A.y = -A.y; B.y = -B.y; }
            // W = A + i B
            sm[s * nx + k] = make_float2(A.x - B.y, A.y + B.x);
        }
        __syncthreads();
        fft_lds(sm, nx, I.xrad, I.nxrad, pairs, nx, +1.f);
        for (int t = threadIdx.x; t < pairs * nx; t += FFT_THREADS) {
            const int s = t / nx, e = t - s * nx;
            const int ra = row0 + 2 * s, rb = ra + 1;
            const float2 w = sm[s * nx + e];
            if (ra < rows) out[(size_t)ra * nx + e] = w.x;
            if (rb < rows) out[(size_t)rb * nx + e] = w.y;
        }
    }
}

// FFT along y of the half spectrum, forward (dir = -1) or inverse (+1):
// a work-group takes TK consecutive kx at one z, all y.
__global__ __launch_bounds__(FFT_THREADS) void k_fft_y(const Inst *__restrict__ insts,
                                                       const int *__restrict__ prefix, int ninst,
                                                       int dir) {
    extern __shared__ float2 sm[];
    const int ii = find_inst(prefix, ninst, blockIdx.x);
    const Inst &I = insts[ii];
    const int nx = I.nx, ny = I.ny, P = nx / 2 + 1;
    const int TK = fft_y_cols(ny);
    const int ntk = (P + TK - 1) / TK;
    const int lb = blockIdx.x - prefix[ii];
    const int z = lb / ntk, kx0 = (lb - z * ntk) * TK;
    const int tk = min(TK, P - kx0);
    float2 *spec = I.spec + (size_t)z * ny * P;
    for (int t = threadIdx.x; t < ny * TK; t += FFT_THREADS) {
        const int y = t / TK, c = t - y * TK;
        sm[c * ny + y] = c < tk ? spec[(size_t)y * P + kx0 + c] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    fft_lds(sm, ny, I.yrad, I.nyrad, TK, ny, (float)dir);
    for (int t = threadIdx.x; t < ny * TK; t += FFT_THREADS) {
        const int y = t / TK, c = t - y * TK;
        if (c < tk) spec[(size_t)y * P + kx0 + c] = sm[c * ny + y];
    }
}

// The z systems, one per (kx, ky), by parallel cyclic reduction in double
// precision.  A work-group loads a tile of ZTK consecutive kx at one ky and
// all z; each wavefront then solves columns of the tile one at a time, its
// 64 lanes owning rows k = lane + 64 i.  The result is scaled by 1/(nx ny)
// (the two inverse FFTs are unnormalised).
constexpr int ZTK = FFT_ZTK;
constexpr int ZMAX = FFT_ZMAX;
__global__ __launch_bounds__(FFT_THREADS) void k_fft_zsolve(const Inst *__restrict__ insts,
                                                            const int *__restrict__ prefix,
                                                            int ninst) {
    __shared__ float2 tile[ZMAX * ZTK];
    __shared__ double pa[4][ZMAX], pb[4][ZMAX], pc[4][ZMAX], pdr[4][ZMAX], pdi[4][ZMAX];
    const int ii = find_inst(prefix, ninst, blockIdx.x);
    const Inst &I = insts[ii];
    const int nx = I.nx, ny = I.ny, nz = I.nz, P = nx / 2 + 1;
    const int ntk = (P + ZTK - 1) / ZTK;
    const int lb = blockIdx.x - prefix[ii];
    const int ky = lb / ntk, kx0 = (lb - ky * ntk) * ZTK;
    const int tk = min(ZTK, P - kx0);
    const size_t zstride = (size_t)ny * P;
    float2 *spec = I.spec + (size_t)ky * P + kx0;
    for (int t = threadIdx.x; t < nz * ZTK; t += FFT_THREADS) {
        const int k = t / ZTK, c = t - k * ZTK;
        tile[k * ZTK + c] = c < tk ? spec[(size_t)k * zstride + c] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double cz = I.cz, cx = I.cx, cy = I.cy;
    const double scale = 1.0 / ((double)nx * (double)ny);
    const double lam_y = cy * (2.0 - 2.0 * cospi(2.0 * ky / (double)ny));
    constexpr int RPL = ZMAX / 64;  // rows per lane
    for (int c = w; c < tk; c += 4) {
        const int kx = kx0 + c;
        const double lam = cx * (2.0 - 2.0 * cospi(2.0 * kx / (double)nx)) + lam_y;
        const bool singular = (kx == 0 && ky == 0);
        double a[RPL], b[RPL], cc[RPL], dr[RPL], di[RPL];
        // compatibility projection of the singular column
        double mr = 0.0, mi = 0.0;
        if (singular) {
            double sr = 0.0, si = 0.0, sw = 0.0;
            for (int k = lane; k < nz; k += 64) {
                const double wk = (nz > 1 && (k == 0 || k == nz - 1)) ? 0.5 : 1.0;
                const float2 v = tile[k * ZTK + c];
                sr += wk * v.x;
                si += wk * v.y;
                sw += wk;
            }
            for (int o = 32; o > 0; o >>= 1) {
                sr += __shfl_xor(sr, o, 64);
                si += __shfl_xor(si, o, 64);
                sw += __shfl_xor(sw, o, 64);
            }
            mr = sr / sw;
            mi = si / sw;
        }
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int k = lane + 64 * q;
            if (k < nz) {
                const float2 v = tile[k * ZTK + c];
                a[q] = (k == 0) ? 0.0 : (k == nz - 1 ? 2.0 * cz : cz);
                cc[q] = (k == nz - 1) ? 0.0 : (k == 0 ? 2.0 * cz : cz);
                b[q] = -(lam + 2.0 * cz);
                dr[q] = (v.x - mr) * scale;
                di[q] = (v.y - mi) * scale;
                if (nz == 1) { a[q] = 0.0; cc[q] = 0.0; b[q] = -lam; }
                if (singular && k == 0) { a[q] = 0.0; cc[q] = 0.0; b[q] = 1.0; dr[q] = 0.0; di[q] = 0.0; }
            } else {
                a[q] = 0.0; cc[q] = 0.0; b[q] = 1.0; dr[q] = 0.0; di[q] = 0.0;
            }
        }
        for (int s = 1; s < nz; s <<= 1) {
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                const int k = lane + 64 * q;
                if (k < nz) { pa[w][k] = a[q]; pb[w][k] = b[q]; pc[w][k] = cc[q]; pdr[w][k] = dr[q]; pdi[w][k] = di[q]; }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                const int k = lane + 64 * q;
                if (k < nz) {
                    double na = 0.0, nc = 0.0, nb = b[q], ndr = dr[q], ndi = di[q];
                    if (k - s >= 0) {
                        const double al = -a[q] / pb[w][k - s];
                        na = al * pa[w][k - s];
                        nb += al * pc[w][k - s];
                        ndr += al * pdr[w][k - s];
                        ndi += al * pdi[w][k - s];
                    }
                    if (k + s < nz) {
                        const double ga = -cc[q] / pb[w][k + s];
                        nc = ga * pc[w][k + s];
                        nb += ga * pa[w][k + s];
                        ndr += ga * pdr[w][k + s];
                        ndi += ga * pdi[w][k + s];
                    }
                    a[q] = na; cc[q] = nc; b[q] = nb; dr[q] = ndr; di[q] = ndi;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        double xr[RPL], xi[RPL];
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            xr[q] = dr[q] / b[q];
            xi[q] = di[q] / b[q];
        }
        if (singular) {
            // shift the constant mode to zero weighted mean
            double sr = 0.0, si = 0.0, sw = 0.0;
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                const int k = lane + 64 * q;
                if (k < nz) {
                    const double wk = (nz > 1 && (k == 0 || k == nz - 1)) ? 0.5 : 1.0;
                    sr += wk * xr[q];
                    si += wk * xi[q];
                    sw += wk;
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                sr += __shfl_xor(sr, o, 64);
                si += __shfl_xor(si, o, 64);
                sw += __shfl_xor(sw, o, 64);
            }
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                xr[q] -= sr / sw;
                xi[q] -= si / sw;
            }
        }
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int k = lane + 64 * q;
            if (k < nz) tile[k * ZTK + c] = make_float2((float)xr[q], (float)xi[q]);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nz * ZTK; t += FFT_THREADS) {
        const int k = t / ZTK, c = t - k * ZTK;
        if (c < tk) spec[(size_t)k * zstride + c] = tile[k * ZTK + c];
    }
}

}  // namespace tdgl
