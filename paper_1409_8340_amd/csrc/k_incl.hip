// k_incl.hip -- inclusion generator of Sec. 3.4 on the GPU.
//
// Candidate spheres are added in order until the covered node fraction
// reaches the target.  Instead of adding them one by one, every node records
// the index of the FIRST candidate that covers it (atomicMin); the covered
// count after s spheres is then the number of nodes whose first index is
// below s, a prefix sum over a per-candidate histogram.  The smallest s whose
// count reaches the target is the sequential answer, found in one pass.
#include "kernels.h"

namespace tdgl {

// Largest reach |c| + r (in node spacings) of a candidate's box: 2^50.
constexpr double kInclReach = 1125899906842624.0;

// One work-group per candidate sphere: visit the integer bounding box of
// the sphere (one node margin), test each node image exactly and record the
// smallest covering index.  The membership test
//     ((dx*dx + dy*dy) + dz*dz) <= (d/2)*(d/2),  dx = u*hx - cx,
// is evaluated in double precision with contraction into fused multiply-add
// disabled, so it is bit-reproducible.  u is the unwrapped integer node
// coordinate; periodic axes wrap it onto the grid, open axes clip.
__global__ __launch_bounds__(256) void k_incl_first(const Inst *__restrict__ insts, int inst,
                                                    const double *__restrict__ centres,
                                                    const double *__restrict__ diam, int nc,
                                                    unsigned *__restrict__ first) {
#pragma clang fp contract(off)
    const Inst &I = insts[inst];
    const int s = blockIdx.x;
    if (s >= nc) return;
    const double h[3] = {I.hx, I.hy, I.hz};
    const int n[3] = {I.nx, I.ny, I.nz};
    const double r = 0.5 * diam[s];
    const double r2 = r * r;
    // non-finite or negative input: the sphere covers nothing
    if (!(r >= 0.0) || !(r < 1e30)) return;
    long lo[3], cnt[3];
    for (int a = 0; a < 3; ++a) {
        const double c = centres[3 * s + a];
        // a box reaching beyond 2^50 node spacings (or non-finite) covers
        // nothing; below that bound every box end is an exact integer
        if (!(fabs(c) + r <= kInclReach * h[a])) return;
        long l0 = (long)floor((c - r) / h[a]) - 1;
        long h0 = (long)ceil((c + r) / h[a]) + 1;
        if (!I.per[a]) {
            if (l0 < 0) l0 = 0;
            if (h0 > n[a] - 1) h0 = n[a] - 1;
        } else {
            // one period around the centre holds the nearest image of every
            // node, and a node is inside iff its nearest image is
            const long cc = (long)floor(c / h[a]);
            if (l0 < cc - n[a] - 1) l0 = cc - n[a] - 1;
            if (h0 > cc + n[a] + 1) h0 = cc + n[a] + 1;
        }
        lo[a] = l0;
        cnt[a] = h0 - l0 + 1;
        if (cnt[a] <= 0) return;
    }
    const double cx = centres[3 * s], cy = centres[3 * s + 1], cz = centres[3 * s + 2];
    const long tot = cnt[0] * cnt[1] * cnt[2];
    for (long t = threadIdx.x; t < tot; t += blockDim.x) {
        const long ux = lo[0] + t % cnt[0];
        const long uy = lo[1] + (t / cnt[0]) % cnt[1];
        const long uz = lo[2] + t / (cnt[0] * cnt[1]);
        const double dx = (double)ux * h[0] - cx;
        const double dy = (double)uy * h[1] - cy;
        const double dz = (double)uz * h[2] - cz;
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        if (d2 <= r2) {
            const long ix = ((ux % n[0]) + n[0]) % n[0];
            const long iy = ((uy % n[1]) + n[1]) % n[1];
            const long iz = ((uz % n[2]) + n[2]) % n[2];
            atomicMin(&first[(iz * n[1] + iy) * n[0] + ix], (unsigned)s);
        }
    }
}

// The same for general convex candidates (ellipsoids, columns): shape s is
// 16 doubles,
//     c[3] | Q_xx Q_yy Q_zz Q_xy Q_xz Q_yz | n[3] | hlen | ext[3],
// and a node image is inside iff, with d = u h - c,
//     q = (((Qxx dx) dx + (Qyy dy) dy) + (Qzz dz) dz)
//         + 2 (((Qxy dx) dy + (Qxz dx) dz) + (Qyz dy) dz)  <=  1
// and, when hlen >= 0, |(nx dx + ny dy) + nz dz| <= hlen; double precision,
// no contraction.  The images tested are those of the box c +- ext (one node
// margin), clipped on open axes and held within one period of the centre on
// periodic ones.
__global__ __launch_bounds__(256) void k_incl_first_q(const Inst *__restrict__ insts, int inst,
                                                      const double *__restrict__ shapes, int nc,
                                                      unsigned *__restrict__ first) {
#pragma clang fp contract(off)
    const Inst &I = insts[inst];
    const int s = blockIdx.x;
    if (s >= nc) return;
    const double *sh = shapes + 16 * (size_t)s;
    const double h[3] = {I.hx, I.hy, I.hz};
    const int n[3] = {I.nx, I.ny, I.nz};
    for (int k = 0; k < 16; ++k)
        if (!(fabs(sh[k]) < 1e30)) return;  // non-finite input: the shape covers nothing
    long lo[3], cnt[3];
    for (int a = 0; a < 3; ++a) {
        const double c = sh[a], e = sh[13 + a];
        if (!(e >= 0.0) || !(fabs(c) + e <= kInclReach * h[a])) return;
        long l0 = (long)floor((c - e) / h[a]) - 1;
        long h0 = (long)ceil((c + e) / h[a]) + 1;
        if (!I.per[a]) {
            if (l0 < 0) l0 = 0;
            if (h0 > n[a] - 1) h0 = n[a] - 1;
        } else {
            const long cc = (long)floor(c / h[a]);
            if (l0 < cc - n[a] - 1) l0 = cc - n[a] - 1;
            if (h0 > cc + n[a] + 1) h0 = cc + n[a] + 1;
        }
        lo[a] = l0;
        cnt[a] = h0 - l0 + 1;
        if (cnt[a] <= 0) return;
    }
    const double cx = sh[0], cy = sh[1], cz = sh[2];
    const double qxx = sh[3], qyy = sh[4], qzz = sh[5], qxy = sh[6], qxz = sh[7], qyz = sh[8];
    const double ax = sh[9], ay = sh[10], az = sh[11], hlen = sh[12];
    const long tot = cnt[0] * cnt[1] * cnt[2];
    for (long t = threadIdx.x; t < tot; t += blockDim.x) {
        const long ux = lo[0] + t % cnt[0];
        const long uy = lo[1] + (t / cnt[0]) % cnt[1];
        const long uz = lo[2] + t / (cnt[0] * cnt[1]);
        const double dx = (double)ux * h[0] - cx;
        const double dy = (double)uy * h[1] - cy;
        const double dz = (double)uz * h[2] - cz;
        const double q = (((qxx * dx) * dx + (qyy * dy) * dy) + (qzz * dz) * dz) +
                         2.0 * (((qxy * dx) * dy + (qxz * dx) * dz) + (qyz * dy) * dz);
        bool in = q <= 1.0;
        if (in && hlen >= 0.0) in = fabs((ax * dx + ay * dy) + az * dz) <= hlen;
        if (in) {
            const long ix = ((ux % n[0]) + n[0]) % n[0];
            const long iy = ((uy % n[1]) + n[1]) % n[1];
            const long iz = ((uz % n[2]) + n[2]) % n[2];
            atomicMin(&first[(iz * n[1] + iy) * n[0] + ix], (unsigned)s);
        }
    }
}

// Histogram of first covering indices.
__global__ void k_incl_count(const unsigned *__restrict__ first, long N, int nc,
                             unsigned *__restrict__ cnt) {
    for (long m = blockIdx.x * (long)blockDim.x + threadIdx.x; m < N; m += (long)gridDim.x * blockDim.x) {
        const unsigned f = first[m];
        if (f < (unsigned)nc) atomicAdd(&cnt[f], 1u);
    }
}

// Smallest s with sum_{t <= s} cnt[t] >= need; one work-group of 1024.
// Writes the sphere count (s + 1) and the covered fraction into the state.
__global__ __launch_bounds__(1024) void k_incl_scan(const Inst *__restrict__ insts, int inst,
                                                    const unsigned *__restrict__ cnt, int nc,
                                                    double target) {
    __shared__ unsigned long long tsum[1024];
    __shared__ int found;
    const Inst &I = insts[inst];
    const double need = target * (double)I.N;
    const int per = (nc + 1023) / 1024;
    const int b0 = threadIdx.x * per, b1 = min(b0 + per, nc);
    unsigned long long s = 0;
    for (int t = b0; t < b1; ++t) s += cnt[t];
    tsum[threadIdx.x] = s;
    if (threadIdx.x == 0) found = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        // sequential exclusive scan over the 1024 thread sums
        unsigned long long acc = 0;
        for (int i = 0; i < 1024; ++i) {
            const unsigned long long v = tsum[i];
            tsum[i] = acc;
            acc += v;
        }
    }
    __syncthreads();
    DevState *st = I.st;
    if (need <= 0.0) {
        if (threadIdx.x == 0) { st->n_used = 0; st->frac = 0.0; }
        return;
    }
    unsigned long long acc = tsum[threadIdx.x];
    for (int t = b0; t < b1; ++t) {
        const unsigned long long next = acc + cnt[t];
        if ((double)acc < need && (double)next >= need) {
            // exactly one thread sees the crossing
            st->n_used = t + 1;
            st->frac = (double)next / (double)I.N;
            found = 1;
        }
        acc = next;
    }
    __syncthreads();
    if (threadIdx.x == 1023 && !found) {
        st->n_used = nc;
        st->frac = (double)acc / (double)I.N;
    }
}

__global__ void k_incl_write(const Inst *__restrict__ insts, int inst,
                             const unsigned *__restrict__ first, float eps_in, float eps_out) {
    const Inst &I = insts[inst];
    const unsigned used = (unsigned)I.st->n_used;
    for (long m = blockIdx.x * (long)blockDim.x + threadIdx.x; m < I.N; m += (long)gridDim.x * blockDim.x)
        I.eps[m] = first[m] < used ? eps_in : eps_out;
}

// Insulating inclusions (Sec. 3.4, item (ii)): no current across the edges
// between a superconducting node and an insulating one.  With psi = 0 held
// on the insulating nodes, cutting those edges out of the covariant
// Laplacian leaves the neighbour sum of every superconducting node as it
// is and only removes the edge's share of the diagonal, c_a = 1/h_a^2
// (1/(g h_z)^2 on z; 2 c_a for the doubled inner neighbour of an open face
// node).  That is the same as raising eps at the node by the cut shares, so
// the stencil passes need no mask: this kernel adds the shares to eps
// (float, in the order x-, x+, y-, y+, z-, z+), and gives insulating nodes
// eps = -2^50, whose diagonal keeps psi there at |psi| < 1e-14 once it
// starts at zero, and zeroes psi on them.
__global__ void k_insulate(const Inst *__restrict__ insts, int inst, const unsigned char *__restrict__ mask) {
    const Inst &I = insts[inst];
    const int nx = I.nx, ny = I.ny, nz = I.nz;
    float2 *psi = I.psi[I.st->cur];
    const float c[3] = {I.cx, I.cy, I.cz};
    const int n[3] = {nx, ny, nz};
    const long str[3] = {1, nx, (long)nx * ny};
    for (long m = blockIdx.x * (long)blockDim.x + threadIdx.x; m < I.N; m += (long)gridDim.x * blockDim.x) {
        if (mask[m]) {
            I.eps[m] = -1125899906842624.0f;
            psi[m] = make_float2(0.f, 0.f);
            continue;
        }
        const int q[3] = {(int)(m % nx), (int)((m / nx) % ny), (int)(m / ((long)nx * ny))};
        float e = I.eps[m];
        for (int a = 0; a < 3; ++a) {
            if (c[a] == 0.f) continue;  // one-node open axis: no edges
            for (int d = -1; d <= 1; d += 2) {
                const int t = q[a] + d;
                long nb;
                float share = c[a];
                if (t >= 0 && t < n[a]) {
                    nb = m + d * str[a];
                    // open face node: its single inner neighbour counts twice
                    if (!I.per[a] && (q[a] == 0 || q[a] == n[a] - 1)) share = 2.f * c[a];
                } else if (I.per[a]) {
                    nb = m + (t < 0 ? (long)(n[a] - 1) : -(long)(n[a] - 1)) * str[a];
                } else {
                    continue;
                }
                if (mask[nb]) e += share;
            }
        }
        I.eps[m] = e;
    }
}

}  // namespace tdgl
