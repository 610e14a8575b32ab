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
// gathered vector x.  The line's entries are read as aligned quads (16-byte
// loads of four indices and of four FP32 values, two 16-byte loads of FP64
// values): the 16 lanes of a group take quads l, l + 16, ..., two at a time,
// and lanes 0..2 take the at most three entries before the first aligned
// quad and after the last one.  Per lane the products are added in a fixed
// order, then the xor tree over the lanes; every lane returns the total.
template <typename V>
__device__ __forceinline__ void quad_load(const V* p, double* out);
template <>
__device__ __forceinline__ void quad_load<float>(const float* p, double* out) {
    const float4 q = *(const float4*)p;
    out[0] = q.x;
    out[1] = q.y;
    out[2] = q.z;
    out[3] = q.w;
}
template <>
__device__ __forceinline__ void quad_load<double>(const double* p, double* out) {
    const double2 a = *(const double2*)p, b = *(const double2*)(p + 2);
    out[0] = a.x;
    out[1] = a.y;
    out[2] = b.x;
    out[3] = b.y;
}

template <typename V>
__device__ __forceinline__ double line_dot(const V* __restrict__ val, const int32_t* __restrict__ idx,
                                           int64_t base, int64_t lo, int64_t hi,
                                           const double* __restrict__ x, int lane16) {
    // absolute entry indices; the arrays start 256-byte aligned, so an entry
    // index divisible by 4 starts an aligned quad
    const int64_t E0 = base + lo, E1 = base + hi;
    int64_t A = (E0 + 3) & ~(int64_t)3;
    if (A > E1) A = E1;
    int64_t B = E1 & ~(int64_t)3;
    if (B < A) B = A;
    double a0 = 0.0, a1 = 0.0, ht = 0.0;
    if (E0 + lane16 < A) ht += (double)val[E0 + lane16] * x[idx[E0 + lane16]];
    if (B + lane16 < E1) ht += (double)val[B + lane16] * x[idx[B + lane16]];
    const int64_t nq = (B - A) / 4;
    for (int64_t q = lane16; q < nq; q += 32) {
        const int64_t e = A + 4 * q;
        const bool two = q + 16 < nq;
        const int4 ia = *(const int4*)(idx + e);
        const int4 ib = two ? *(const int4*)(idx + e + 64) : make_int4(0, 0, 0, 0);
        double va[4], vb[4];
        quad_load<V>(val + e, va);
        if (two) {
            quad_load<V>(val + e + 64, vb);
        } else {
            vb[0] = vb[1] = vb[2] = vb[3] = 0.0;
        }
        a0 += ((va[0] * x[ia.x] + va[1] * x[ia.y]) + (va[2] * x[ia.z] + va[3] * x[ia.w]));
        a1 += ((vb[0] * x[ib.x] + vb[1] * x[ib.y]) + (vb[2] * x[ib.z] + vb[3] * x[ib.w]));
    }
    return group_sum<16>((a0 + a1) + ht);
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

// ------------------------------------------------------------------ LDS-staged step
// Where a measure's vector (n FP64 values) fits in LDS, a block stages the
// vector its lines gather, so the random reads come from LDS instead of each
// pulling a cache line from L2: a column block takes a contiguous range of one
// measure's columns and stages u_k; a row block takes a contiguous range of
// rows and stages v_k for each measure in turn, keeping the rows' products
// g_k in LDS until q and u are formed.  Every line's sum, and every row's
// combination, runs in the same order as above, so the iterates are the same
// bit for bit; only the residual's block partials are grouped differently.
constexpr int kIbpLdsThreads = 1024;
constexpr int kIbpLdsLines = kIbpLdsThreads / 16;  // lines a round
constexpr int64_t kIbpLdsBlocks = 256;              // about one block per compute unit
constexpr size_t kIbpLdsMax = 159 * 1024;  // dynamic LDS; the rest holds the static part

static int64_t ibp_row_grid(int64_t n) {
    const int64_t r = (n + kIbpLdsLines - 1) / kIbpLdsLines;
    return r < kIbpLdsBlocks ? r : kIbpLdsBlocks;
}
static int64_t ibp_rows_per_block(int64_t n) {
    const int64_t g = ibp_row_grid(n);
    return (n + g - 1) / g;
}
static size_t ibp_row_lds(int64_t n, int count) {
    return ((size_t)n + (size_t)count * (size_t)ibp_rows_per_block(n)) * 8;
}
static bool ibp_lds_fits(int64_t n, int count) { return ibp_row_lds(n, count) <= kIbpLdsMax; }
static int64_t ibp_col_blocks_per_measure(int64_t n, int count) {
    int64_t b = (kIbpLdsBlocks + count - 1) / count;
    return b < n ? b : n;
}

// Copies src[0, n) into the LDS vector xs: each thread issues its (up to)
// kIbpStage loads before storing any, so a 16384-entry vector takes one
// round of load latency instead of one per element.
constexpr int kIbpStage = 16;

__device__ __forceinline__ void ibp_stage(double* xs, const double* __restrict__ src, int64_t n) {
    for (int64_t e0 = threadIdx.x; e0 < n; e0 += (int64_t)blockDim.x * kIbpStage) {
        double t[kIbpStage];
#pragma unroll
        for (int q = 0; q < kIbpStage; ++q) {
            const int64_t e = e0 + (int64_t)q * blockDim.x;
            t[q] = e < n ? src[e] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kIbpStage; ++q) {
            const int64_t e = e0 + (int64_t)q * blockDim.x;
            if (e < n) xs[e] = t[q];
        }
    }
}

template <typename V>
__global__ __launch_bounds__(kIbpLdsThreads) void k_ibp_cols_lds(IbpArgs A, int64_t bpm) {
    extern __shared__ double xs[];  // u_k
    __shared__ double sh[16];
    __shared__ int ctl[2];
    if (threadIdx.x == 0) {
        ctl[0] = A.st->stop_iter != 0 || A.st->nonfinite != 0;
        ctl[1] = A.st->cnt_u + 1;
    }
    __syncthreads();
    if (ctl[0]) return;
    const int t = ctl[1];
    if (blockIdx.x == 0) ibp_close(A, t, sh);
    if (t > A.max_iter) return;
    const int64_t n = A.n;
    const int64_t k = blockIdx.x / bpm, jb = blockIdx.x % bpm;
    const int64_t per = (n + bpm - 1) / bpm;
    const int64_t j0 = jb * per, j1 = j0 + per < n ? j0 + per : n;
    ibp_stage(xs, A.u + k * n, n);
    __syncthreads();
    const V* __restrict__ val = (const V*)A.val_t;
    double* __restrict__ vout = A.v[t & 1];
    const int grp = threadIdx.x >> 4, l16 = threadIdx.x & 15;
    const int64_t* cp = A.col_ptr + k * (n + 1);
    for (int64_t j = j0 + grp; j < j1; j += kIbpLdsLines) {
        const double den = line_dot<V>(val, A.row_idx, k * A.cap, cp[j], cp[j + 1], xs, l16);
        if (l16 == 0) vout[k * n + j] = den > 0.0 ? A.b[k * n + j] / den : 0.0;
    }
}

template <typename V>
__global__ __launch_bounds__(kIbpLdsThreads) void k_ibp_rows_lds(IbpArgs A, int64_t rpb) {
    extern __shared__ double dyn[];  // v_k, then g_k of the block's rows (count x rpb)
    __shared__ double sh[16];
    __shared__ int ctl[2];
    IterState* S = A.st;
    if (threadIdx.x == 0) {
        ctl[0] = S->stop_iter != 0 || S->nonfinite != 0;
        ctl[1] = S->cnt_v;
    }
    __syncthreads();
    if (ctl[0]) return;
    const int t = ctl[1];
    if (t > A.max_iter) return;
    const int64_t n = A.n;
    const int count = A.count;
    double* xs = dyn;
    double* gk = dyn + n;
    const V* __restrict__ val = (const V*)A.val;
    const double* __restrict__ v = A.v[t & 1];
    const double* __restrict__ qold = A.q[(t - 1) & 1];
    double* __restrict__ qnew = A.q[t & 1];
    const int grp = threadIdx.x >> 4, l16 = threadIdx.x & 15;
    const int64_t i0 = (int64_t)blockIdx.x * rpb, i1 = i0 + rpb < n ? i0 + rpb : n;
    for (int k = 0; k < count; ++k) {
        __syncthreads();  // the previous measure's vector is read
        ibp_stage(xs, v + (int64_t)k * n, n);
        __syncthreads();
        const int64_t* rp = A.row_ptr + (int64_t)k * (n + 1);
        for (int64_t i = i0 + grp; i < i1; i += kIbpLdsLines) {
            const double g = line_dot<V>(val, A.col_idx, (int64_t)k * A.cap, rp[i], rp[i + 1], xs,
                                         l16);
            if (l16 == 0) gk[(int64_t)k * rpb + (i - i0)] = g;
        }
    }
    __syncthreads();
    double part = 0.0;
    bool bad = false;
    for (int64_t i = i0 + grp; i < i1; i += kIbpLdsLines) {
        const int64_t r = i - i0;
        double lq = 0.0;
        bool zero = false;
        for (int k = 0; k < count; ++k) {
            const double g = gk[(int64_t)k * rpb + r];
            const double wk = A.w[k];
            if (wk > 0.0) {
                if (g > 0.0)
                    lq += wk * log(g);
                else
                    zero = true;
            }
        }
        const double qi = zero ? 0.0 : exp(lq);
        bad = bad || !isfinite(qi);
        for (int k = l16; k < count; k += 16) {
            const double g = gk[(int64_t)k * rpb + r];
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

hipError_t ibp_lds_init() {
    static hipError_t status = [] {
        const void* fns[] = {(const void*)&k_ibp_cols_lds<double>, (const void*)&k_ibp_cols_lds<float>,
                             (const void*)&k_ibp_rows_lds<double>, (const void*)&k_ibp_rows_lds<float>};
        for (const void* f : fns) {
            const hipError_t e =
                hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kIbpLdsMax);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }();
    return status;
}

int ibp_row_blocks(int64_t n, int count) {
    return ibp_lds_fits(n, count) ? (int)ibp_row_grid(n) : (int)grid_lines(n, kMaxLoopBlocks);
}

hipError_t launch_ibp_iteration(int precision, const IbpArgs& A, hipStream_t st) {
    if (ibp_lds_fits(A.n, A.count)) {
        const int64_t bpm = ibp_col_blocks_per_measure(A.n, A.count);
        const int64_t rpb = ibp_rows_per_block(A.n);
        const dim3 gc((unsigned)(bpm * A.count)), gr((unsigned)A.nb_rows);
        const size_t lc = (size_t)A.n * 8, lr = ibp_row_lds(A.n, A.count);
        if (precision == P_F64) {
            hipLaunchKernelGGL(k_ibp_cols_lds<double>, gc, dim3(kIbpLdsThreads), lc, st, A, bpm);
            hipLaunchKernelGGL(k_ibp_rows_lds<double>, gr, dim3(kIbpLdsThreads), lr, st, A, rpb);
        } else {
            hipLaunchKernelGGL(k_ibp_cols_lds<float>, gc, dim3(kIbpLdsThreads), lc, st, A, bpm);
            hipLaunchKernelGGL(k_ibp_rows_lds<float>, gr, dim3(kIbpLdsThreads), lr, st, A, rpb);
        }
        return hipGetLastError();
    }
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
