// Spar-IBP: fixed-support Wasserstein barycenters by iterative Bregman
// projections on sparse sketches (the paper's barycenter section: eq. (rwb),
// Alg. IBP, eq. (pois-k), Alg. Spar-IBP).
//
// The sketches are built by the Spar-Sink sampling kernels (mask, transpose,
// scan, fill) with the probability factors below.  The iteration runs two
// launches per step on the concatenated CSR / CSC of all measures:
//   k_ibp_cols  v_k = b_k / (K~_k^T u_k)                   (line = (k, j))
//   k_ibp_rows  g_k = K~_k v_k;  q = prod_k g_k^(w_k);  u_k = q / g_k
//                                                          (line = i, all k)
// Sixteen lanes share a line; every line's sum is a fixed xor tree over the
// lanes' partial sums, accumulated in FP64 (FP32 stored values are widened).
// The stop test |q^t - q^(t-1)|_1 is reduced by block 0 of the next column
// launch from the row launch's block partials (fixed order), so no launch
// waits on another block of its own grid; see IbpArgs for the protocol.
#include "common.hpp"
#include "internal.hpp"

namespace ss {

namespace {

constexpr int kLinesPerBlock = 16;   // 16 lanes per line, 256 threads

inline unsigned grid_lines(int64_t lines, int cap) {
    int64_t g = (lines + kLinesPerBlock - 1) / kLinesPerBlock;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

// ------------------------------------------------------------------ sketches
// Alg. Spar-IBP: p_ij = sqrt(b_j) / (n sum_j sqrt(b_j)) for every row, so
// s p* = min(1, c sqrt(b_j) + s g / n^2) with c = (1 - g) s / (n sum_j sqrt(b_j))
// (shrinkage weight g, Sec. 4).  The row factor holds c for every row and the
// column factor sqrt(b_j), so the Spar-Sink mask and fill kernels apply as is.
__global__ void k_ibp_sqrt(const double* __restrict__ b, int64_t n, double* __restrict__ rb) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) rb[j] = sqrt(b[j]);
}

__global__ void k_ibp_rowfac(double* __restrict__ rf, int64_t n, double s, double w,
                             const double* __restrict__ sum_rb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double c = s / ((double)n * sum_rb[0]);
    if (i < n) rf[i] = c * w;
}

hipError_t launch_ibp_prep(const double* b, int64_t n, double s, double shrink_w, double* row_fac,
                           double* col_fac, double* scratch, double* stats, hipStream_t st) {
    const unsigned g = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_ibp_sqrt, dim3(g), dim3(kBlock), 0, st, b, n, col_fac);
    hipError_t e = launch_tree_sum(col_fac, n, scratch, stats + ST_SB, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ibp_rowfac, dim3(g), dim3(kBlock), 0, st, row_fac, n, s, shrink_w,
                       stats + ST_SB);
    return hipGetLastError();
}

// Number of zero counts (empty lines) added into *out.
__global__ __launch_bounds__(256) void k_ibp_empty(const int32_t* __restrict__ cnt, int64_t n,
                                                   unsigned long long* __restrict__ out) {
    __shared__ double sh[16];
    double c = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        c += cnt[i] == 0 ? 1.0 : 0.0;
    c = block_sum(c, sh);
    if (threadIdx.x == 0 && c > 0.0) atomicAdd(out, (unsigned long long)c);
}

hipError_t launch_ibp_empty(const int32_t* cnt, int64_t n, unsigned long long* out,
                            hipStream_t st) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(k_ibp_empty, dim3((unsigned)g), dim3(kBlock), 0, st, cnt, n, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ loop
// u_k = 1 for every measure, q^0 = 1/n.
__global__ void k_ibp_init(double* __restrict__ u, int64_t nu, double* __restrict__ q0, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nu) u[i] = 1.0;
    if (i < n) q0[i] = 1.0 / (double)n;
}

hipError_t launch_ibp_init(double* u, int64_t nu, double* q0, int64_t n, hipStream_t st) {
    const int64_t t = nu > n ? nu : n;
    hipLaunchKernelGGL(k_ibp_init, dim3((unsigned)((t + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       u, nu, q0, n);
    return hipGetLastError();
}

// Dot product of one CSR/CSC line (entries [lo, hi) + base) with the
// gathered vector x: the 16 lanes of a group stride the entries, four
// independent loads per lane in flight, four partial sums per lane added in a
// fixed order, then the xor tree over the lanes; every lane returns the total.
template <typename V>
__device__ __forceinline__ double line_dot(const V* __restrict__ val, const int32_t* __restrict__ idx,
                                           int64_t base, int64_t lo, int64_t hi,
                                           const double* __restrict__ x, int lane16) {
    const V* __restrict__ pv = val + base;
    const int32_t* __restrict__ pi = idx + base;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t e = lo + lane16;
    for (; e + 48 < hi; e += 64) {
        const int32_t i0 = pi[e], i1 = pi[e + 16], i2 = pi[e + 32], i3 = pi[e + 48];
        const V v0 = pv[e], v1 = pv[e + 16], v2 = pv[e + 32], v3 = pv[e + 48];
        a0 += (double)v0 * x[i0];
        a1 += (double)v1 * x[i1];
        a2 += (double)v2 * x[i2];
        a3 += (double)v3 * x[i3];
    }
    for (; e < hi; e += 16) a0 += (double)pv[e] * x[pi[e]];
    return group_sum<16>((a0 + a1) + (a2 + a3));
}

// Block 0 of a column launch closes the previous step: err(t-1) from the row
// launch's partials in a fixed order, the stop decision, the history entry.
__device__ __forceinline__ void ibp_close(const IbpArgs& A, int t, double* sh) {
    IterState* S = A.st;
    if (t >= 2) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < A.nb_rows; b += blockDim.x) acc += A.partials[b];
        const double err = block_sum(acc, sh);
        if (threadIdx.x == 0) {
            if (A.err_hist) A.err_hist[t - 2] = err;
            if (err <= A.tol || t - 1 >= A.max_iter) {
                S->err_final = err;
                S->stop_iter = t - 1;
            }
        }
    }
    if (threadIdx.x == 0) S->cnt_v = t;
}

// v_k = b_k / (K~_k^T u_k) for every (k, j); 0 where the product is 0.
template <typename V>
__global__ __launch_bounds__(256) void k_ibp_cols(IbpArgs A) {
    __shared__ double sh[16];
    __shared__ int ctl[2];
    // the state is read once per block so every wave takes the same branch
    if (threadIdx.x == 0) {
        ctl[0] = A.st->stop_iter != 0 || A.st->nonfinite != 0;
        ctl[1] = A.st->cnt_u + 1;   // cnt_u: the last row half-step that ran
    }
    __syncthreads();
    if (ctl[0]) return;
    const int t = ctl[1];
    if (blockIdx.x == 0) ibp_close(A, t, sh);
    if (t > A.max_iter) return;
    const V* __restrict__ val = (const V*)A.val_t;
    double* __restrict__ vout = A.v[t & 1];
    const int grp = threadIdx.x >> 4, l16 = threadIdx.x & 15;
    const int64_t n = A.n, lines = (int64_t)A.count * n;
    for (int64_t L = (int64_t)blockIdx.x * kLinesPerBlock + grp; L < lines;
         L += (int64_t)gridDim.x * kLinesPerBlock) {
        const int64_t k = L / n, j = L - k * n;
        const int64_t* cp = A.col_ptr + k * (n + 1);
        const double den = line_dot<V>(val, A.row_idx, k * A.cap, cp[j], cp[j + 1], A.u + k * n,
                                       l16);
        if (l16 == 0) vout[L] = den > 0.0 ? A.b[L] / den : 0.0;
    }
}

// g_k = K~_k v_k for every measure of row i, q_i = prod_k g_k^(w_k) (as
// exp(sum_k w_k log g_k); 0 if a factor with positive weight is 0), then
// u_k = q_i / g_k (0 where g_k = 0); block partials of |q^t - q^(t-1)|.
template <typename V>
__global__ __launch_bounds__(256) void k_ibp_rows(IbpArgs A) {
    __shared__ double sh[16];
    __shared__ int ctl[2];
    IterState* S = A.st;
    if (threadIdx.x == 0) {
        ctl[0] = S->stop_iter != 0 || S->nonfinite != 0;
        ctl[1] = S->cnt_v;   // the step whose column half-step just ran
    }
    __syncthreads();
    if (ctl[0]) return;
    const int t = ctl[1];
    if (t > A.max_iter) return;
    const V* __restrict__ val = (const V*)A.val;
    const double* __restrict__ v = A.v[t & 1];
    const double* __restrict__ qold = A.q[(t - 1) & 1];
    double* __restrict__ qnew = A.q[t & 1];
    const int grp = threadIdx.x >> 4, l16 = threadIdx.x & 15;
    const int64_t n = A.n;
    const int count = A.count;
    double part = 0.0;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kLinesPerBlock + grp; i < n;
         i += (int64_t)gridDim.x * kLinesPerBlock) {
        // lane l keeps g_k for k = l, l + 16, l + 32, l + 48
        double mine0 = 0.0, mine1 = 0.0, mine2 = 0.0, mine3 = 0.0;
        double lq = 0.0;
        bool zero = false;
        for (int k = 0; k < count; ++k) {
            const int64_t* rp = A.row_ptr + (int64_t)k * (n + 1);
            const double g = line_dot<V>(val, A.col_idx, (int64_t)k * A.cap, rp[i], rp[i + 1],
                                         v + (int64_t)k * n, l16);
            const double wk = A.w[k];
            if (wk > 0.0) {
                if (g > 0.0)
                    lq += wk * log(g);
                else
                    zero = true;
            }
            const bool own = (k & 15) == l16;
            const int r = k >> 4;
            mine0 = (own && r == 0) ? g : mine0;
            mine1 = (own && r == 1) ? g : mine1;
            mine2 = (own && r == 2) ? g : mine2;
            mine3 = (own && r == 3) ? g : mine3;
        }
        const double qi = zero ? 0.0 : exp(lq);
        bad = bad || !isfinite(qi);
        for (int r = 0; r < 4; ++r) {
            const int k = 16 * r + l16;
            if (k >= count) break;
            const double g = r == 0 ? mine0 : r == 1 ? mine1 : r == 2 ? mine2 : mine3;
            A.u[(int64_t)k * n + i] = g > 0.0 ? qi / g : 0.0;
        }
        if (l16 == 0) {
            qnew[i] = qi;
            part += fabs(qi - qold[i]);
        }
    }
    if (bad) S->nonfinite = 1;
    part = block_sum(part, sh);
    if (threadIdx.x == 0) A.partials[blockIdx.x] = part;
    if (blockIdx.x == 0 && threadIdx.x == 0) S->cnt_u = t;
}

int ibp_row_blocks(int64_t n) { return (int)grid_lines(n, kMaxLoopBlocks); }

hipError_t launch_ibp_iteration(int precision, const IbpArgs& A, hipStream_t st) {
    const unsigned gc = grid_lines((int64_t)A.count * A.n, 8 * kMaxLoopBlocks);
    const unsigned gr = (unsigned)A.nb_rows;
    if (precision == P_F64) {
        hipLaunchKernelGGL(k_ibp_cols<double>, dim3(gc), dim3(256), 0, st, A);
        hipLaunchKernelGGL(k_ibp_rows<double>, dim3(gr), dim3(256), 0, st, A);
    } else {
        hipLaunchKernelGGL(k_ibp_cols<float>, dim3(gc), dim3(256), 0, st, A);
        hipLaunchKernelGGL(k_ibp_rows<float>, dim3(gr), dim3(256), 0, st, A);
    }
    return hipGetLastError();
}

}  // namespace ss
