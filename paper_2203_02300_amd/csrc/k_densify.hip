// k_densify.hip -- depth densification by quadratic optimisation (Sec. 6,
// Eq. 13-20), solved with Jacobi-preconditioned conjugate gradients.
//
// The normal equations of Eq. 20 at pixel p (q over the 4-neighbours):
//   (lambda_d w_sparse + lambda_s2 w_stable + sum_q c_pq) D(p) - sum_q c_pq D(q)
//     = lambda_d w_sparse D_sparse + lambda_s2 w_stable D_pre,
//   c_pq = 2 lambda_s w_pq  (the double sum of Eq. 20 visits each pair twice)
// with w_pq of Eq. 16-17.  The operator is a 5-point stencil with per-edge
// coefficients c_right (p, p + x) and c_down (p, p + y), 0 off the grid.
//
// Solver state is FP64 (x, r, p; z = r / diag is formed on the fly).  One
// iteration is two launches:
//   dir:    beta = rz_new / rz_old; p' = z + beta p; q = A p'; block sums of p'.q
//   update: alpha = rz_new / (p'.q); x += alpha p'; r -= alpha q; block sums
//           of r.z and r.r
// Every block forms alpha and beta itself from the previous launch's block
// sums, added in one fixed order, so every block gets the same bits and the
// whole solve is deterministic without grid-wide synchronisation.  When
// r.r <= tol^2 b.b the update launch sets a flag and every later launch
// returns at once (no pixel is touched).
#include "dco_internal.h"

namespace {

constexpr int kDzThreads = 256;
constexpr int kDzPix = 4;  // pixels per thread: a block covers 1024 consecutive pixels

constexpr int kDzWaves = kDzThreads / 64;

// Block sums of N values per thread, in one fixed order: an xor-butterfly
// across each wavefront (every lane ends with the same bits: each step adds
// the same two values in either order), then the wavefront totals in a fixed
// tree.  Every thread returns the N sums.  Two barriers whatever N is.
template <int N>
__device__ inline void block_sums(double (&v)[N], double* red /* N x kDzWaves */) {
#pragma unroll
    for (int j = 0; j < N; ++j)
        for (int o = 32; o > 0; o >>= 1) v[j] += __shfl_xor(v[j], o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int j = 0; j < N; ++j) red[j * kDzWaves + w] = v[j];
    }
    __syncthreads();
    static_assert(kDzWaves == 4, "fixed tree of four wavefront totals");
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const double* t = red + j * kDzWaves;
        v[j] = (t[0] + t[1]) + (t[2] + t[3]);
    }
    __syncthreads();  // red may be reused
}

// Sums of N arrays of n block partials, the same bits in every block: thread
// t adds entries t, t + 256, ... in turn, then block_sums.
template <int N>
__device__ inline void partial_sums(const double* const (&part)[N], int n, double (&out)[N],
                                    double* red) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double s = 0.0;
        for (int i = threadIdx.x; i < n; i += kDzThreads) s += part[j][i];
        out[j] = s;
    }
    block_sums<N>(out, red);
}

// Coefficients, right-hand side and the initial state x = 0, r = b, p = 0,
// block sums of r.z, r.r and b.b.  Eq. 16: w_pq = 0 when exactly one of p, q
// is on the depth contour, else max(1 - min(s_p, s_q), 0) with s = Mfuse MI.
__global__ __launch_bounds__(kDzThreads) void k_dz_setup(
    const float* __restrict__ Ds, const float* __restrict__ Dpre,
    const uint8_t* __restrict__ Bdp, const float* __restrict__ Mfuse,
    const float* __restrict__ MI, int W, int H, double lam_d, double lam_s, double lam_s2,
    double* __restrict__ cr, double* __restrict__ cd, double* __restrict__ diag_out,
    double* __restrict__ invdiag, double* __restrict__ x, double* __restrict__ r,
    double* __restrict__ p0, double* __restrict__ p1, double* __restrict__ rz_part,
    double* __restrict__ rr_part, double* __restrict__ bb_part, double* __restrict__ rz_init,
    int* __restrict__ flags) {
    __shared__ double red[2 * kDzWaves];
    const int P = W * H;
    double rz = 0.0, rr = 0.0;
    for (int k = 0; k < kDzPix; ++k) {
        const int i = (blockIdx.x * kDzPix + k) * kDzThreads + threadIdx.x;
        if (i >= P) break;
        const int y = i / W, xx = i - y * W;
        const double s = (double)Mfuse[i] * (double)MI[i];
        const int b = Bdp[i] != 0;
        auto w = [&](int j) {
            const int bj = Bdp[j] != 0;
            if (b + bj == 1) return 0.0;
            const double sj = (double)Mfuse[j] * (double)MI[j];
            return fmax(1.0 - fmin(s, sj), 0.0);
        };
        const double c_r = xx + 1 < W ? 2.0 * lam_s * w(i + 1) : 0.0;
        const double c_d = y + 1 < H ? 2.0 * lam_s * w(i + W) : 0.0;
        const double c_l = xx > 0 ? 2.0 * lam_s * w(i - 1) : 0.0;
        const double c_u = y > 0 ? 2.0 * lam_s * w(i - W) : 0.0;
        const double ds = Ds[i], dp = Dpre ? (double)Dpre[i] : 0.0;
        const double wsp = ds > 0.0 ? 1.0 : 0.0, wst = dp > 0.0 ? 1.0 : 0.0;
        const double diag = lam_d * wsp + lam_s2 * wst + c_r + c_d + c_l + c_u;
        const double bi = lam_d * wsp * ds + lam_s2 * wst * dp;
        const double id = diag > 0.0 ? 1.0 / diag : 0.0;
        cr[i] = c_r;
        cd[i] = c_d;
        diag_out[i] = diag;
        invdiag[i] = id;
        x[i] = 0.0;
        r[i] = bi;
        p0[i] = 0.0;
        p1[i] = 0.0;
        rz += bi * bi * id;
        rr += bi * bi;
    }
    double sums[2] = {rz, rr};
    block_sums<2>(sums, red);
    if (threadIdx.x == 0) {
        rz_part[blockIdx.x] = sums[0];
        rr_part[blockIdx.x] = sums[1];
        bb_part[blockIdx.x] = sums[1];
        rz_init[blockIdx.x] = 1.0;  // any nonzero "old" r.z: p starts at 0
    }
    if (blockIdx.x == 0 && threadIdx.x < 2) flags[threadIdx.x] = 0;
}

struct DzState {
    const double* cr;
    const double* cd;
    const double* diag;
    const double* invdiag;
    double* x;
    double* r;
    double* q;
    const double* bb_part;
    int* flags;  // [0] converged, [1] iterations done
    int W, H, nblk;
    double tol2;
};

// The convergence flag as one value for the whole block.
__device__ inline bool solve_done(const int* flags) {
    __shared__ int done;
    if (threadIdx.x == 0) done = *(const volatile int*)&flags[0];
    __syncthreads();
    return done != 0;
}

// p_out = r / diag + beta p_in (4-neighbours recomputed from r and p_in);
// q = A p_out; block sums of p_out . q.
__global__ __launch_bounds__(kDzThreads) void k_dz_dir(DzState s, const double* __restrict__ rz_new,
                                                       const double* __restrict__ rz_old,
                                                       const double* __restrict__ p_in,
                                                       double* __restrict__ p_out,
                                                       double* __restrict__ pq_part) {
    __shared__ double red[2 * kDzWaves];
    if (solve_done(s.flags)) return;
    const double* const parts[2] = {rz_new, rz_old};
    double rz[2];
    partial_sums<2>(parts, s.nblk, rz, red);
    const double beta = rz[0] / rz[1];
    const int W = s.W, P = W * s.H;
    double pq = 0.0;
    for (int k = 0; k < kDzPix; ++k) {
        const int i = (blockIdx.x * kDzPix + k) * kDzThreads + threadIdx.x;
        if (i >= P) break;
        const int y = i / W, xx = i - y * W;
        auto pn = [&](int j) { return s.r[j] * s.invdiag[j] + beta * p_in[j]; };
        const double pc = pn(i);
        double off = 0.0;  // sum over the 4-neighbours of c_pq p(q), in a fixed order
        if (xx + 1 < W) off += s.cr[i] * pn(i + 1);
        if (xx > 0) off += s.cr[i - 1] * pn(i - 1);
        if (y + 1 < s.H) off += s.cd[i] * pn(i + W);
        if (y > 0) off += s.cd[i - W] * pn(i - W);
        const double qi = s.diag[i] * pc - off;
        p_out[i] = pc;
        s.q[i] = qi;
        pq += pc * qi;
    }
    double sum[1] = {pq};
    block_sums<1>(sum, red);
    if (threadIdx.x == 0) pq_part[blockIdx.x] = sum[0];
}

// alpha = rz / pq; x += alpha p; r -= alpha q; block sums of r.z and r.r of
// the new residual.  Convergence (r.r <= tol^2 b.b, from the previous
// update's sums) stops the solve before any pixel changes.
__global__ __launch_bounds__(kDzThreads) void k_dz_update(DzState s,
                                                          const double* __restrict__ rz_in,
                                                          const double* __restrict__ rr_in,
                                                          const double* __restrict__ pq_part,
                                                          const double* __restrict__ p,
                                                          double* __restrict__ rz_out,
                                                          double* __restrict__ rr_out) {
    __shared__ double red[4 * kDzWaves];
    if (solve_done(s.flags)) return;
    const double* const parts[4] = {rr_in, s.bb_part, pq_part, rz_in};
    double sums[4];
    partial_sums<4>(parts, s.nblk, sums, red);
    const double rr = sums[0], bb = sums[1], pq = sums[2];
    if (rr <= s.tol2 * bb) {  // converged before this step: the same decision in every block
        if (blockIdx.x == 0 && threadIdx.x == 0) s.flags[0] = 1;
        return;
    }
    const double alpha = pq > 0.0 ? sums[3] / pq : 0.0;
    const int P = s.W * s.H;
    double rz = 0.0, rrn = 0.0;
    for (int k = 0; k < kDzPix; ++k) {
        const int i = (blockIdx.x * kDzPix + k) * kDzThreads + threadIdx.x;
        if (i >= P) break;
        s.x[i] += alpha * p[i];
        const double ri = s.r[i] - alpha * s.q[i];
        s.r[i] = ri;
        rz += ri * ri * s.invdiag[i];
        rrn += ri * ri;
    }
    double out[2] = {rz, rrn};
    block_sums<2>(out, red);
    if (threadIdx.x == 0) {
        rz_out[blockIdx.x] = out[0];
        rr_out[blockIdx.x] = out[1];
        if (blockIdx.x == 0) s.flags[1] += 1;
    }
}

__global__ __launch_bounds__(kDzThreads) void k_dz_out(const double* __restrict__ x, int P,
                                                       float* __restrict__ D) {
    const int i = blockIdx.x * kDzThreads + threadIdx.x;
    if (i < P) D[i] = (float)x[i];
}

}  // namespace

int densify_blocks(int W, int H) {
    return (W * H + kDzThreads * kDzPix - 1) / (kDzThreads * kDzPix);
}

hipError_t launch_densify_setup(const DensifyBufs& b, const float* Ds, const float* Dpre,
                                const uint8_t* Bdp, const float* Mfuse, const float* MI, int W,
                                int H, double lam_d, double lam_s, double lam_s2, hipStream_t st) {
    const int nb = densify_blocks(W, H);
    hipLaunchKernelGGL(k_dz_setup, dim3(nb), dim3(kDzThreads), 0, st, Ds, Dpre, Bdp, Mfuse, MI, W,
                       H, lam_d, lam_s, lam_s2, b.cr, b.cd, b.diag, b.invdiag, b.x, b.r, b.p[0],
                       b.p[1], b.rz[1], b.rr[1], b.bb, b.rz[0], b.flags);
    return hipGetLastError();
}

// Iterations [0, n) of one launch sequence; n even, so parities repeat.
hipError_t launch_densify_iters(const DensifyBufs& b, int W, int H, double tol, int n,
                                hipStream_t st) {
    const int nb = densify_blocks(W, H);
    DzState s{b.cr, b.cd, b.diag, b.invdiag, b.x, b.r, b.q, b.bb, b.flags, W, H, nb, tol * tol};
    for (int it = 0; it < n; ++it) {
        const int a = it & 1;  // rz[1 - a] is the newest r.z, rz[a] the one before
        hipLaunchKernelGGL(k_dz_dir, dim3(nb), dim3(kDzThreads), 0, st, s, b.rz[1 - a], b.rz[a],
                           b.p[a], b.p[1 - a], b.pq);
        hipLaunchKernelGGL(k_dz_update, dim3(nb), dim3(kDzThreads), 0, st, s, b.rz[1 - a],
                           b.rr[1 - a], b.pq, b.p[1 - a], b.rz[a], b.rr[a]);
    }
    return hipGetLastError();
}

hipError_t launch_densify_out(const DensifyBufs& b, int W, int H, float* D, hipStream_t st) {
    const int P = W * H;
    hipLaunchKernelGGL(k_dz_out, dim3((P + kDzThreads - 1) / kDzThreads), dim3(kDzThreads), 0, st,
                       b.x, P, D);
    return hipGetLastError();
}
