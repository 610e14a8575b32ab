// Batches of independent OT problems: the Sinkhorn loop (Alg. 1) of every
// problem inside one persistent launch, and the estimate (Alg. 3) per problem.
//
// Every side of a batched problem has at most 4096 points, so a problem's
// scalings (u, its next value, v) fit in LDS and one block can run the whole
// loop of a problem with block barriers only: no grid synchronisation, no
// per-iteration launches.  Blocks take problems from a device queue in
// decreasing size order (longest first), so uneven sizes balance over the
// persistent grid.  Each line (row of the CSR for u, column of the CSC for v)
// is reduced by a group of L lanes; the sparse entries stream from HBM with
// 16-bit local indices, the gathered scaling comes from LDS.
//
// A warm start (init_log_u / init_log_v) is judged against the plain start
// u = v = 1 in the problem's first u-update: the same pass forms K~v0 and K~1,
// so it yields both candidates for u^1 and the L1 row marginal error of both
// starting points, sum |u0_i (K~v0)_i - a_i| and sum |(K~1)_i - a_i| (over
// rows with entries).  The start is kept only when it is finite, its u^1 is
// finite and its error is no larger than the plain start's; otherwise the
// problem continues from the plain start's u^1, so its iterates are exactly
// those of a solve without a warm start.
//
// The stop test is the one of the single-problem solver: err(t) is the L1
// marginal error of the iterate (u^t, v^t) on K~ -- the column part is formed
// in the v-update of iteration t, the row part in the u-update of iteration
// t + 1 -- and the solver returns the first iterate with err(t) <= tol.  All
// sums have a fixed order for a given schedule.
#include <math.h>

#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace ss {

template <int PREC>
struct BTypes {
    typedef typename std::conditional<PREC == P_F64, double, float>::type V;  // value, scaling
};

// One half-step of problem-local lines 0..nl: w = sum_k val_k x[idx_k],
// y_new = marg / w (0 on an empty line or w <= 0).  Returns this thread's
// share of the residual: ROLE 0 |y_prev w - marg| (iterate t - 1, t >= 2),
// ROLE 1 |y_new w - marg| (iterate t).
// A lane's entries of a line are k0 + lane, k0 + lane + L, ... and are added
// in that order; kBUnroll of them are loaded at once (a line of the batched
// workloads, about 8 ln n entries, takes one pass), and the next line's
// offsets are loaded while the current line streams, so a line costs about
// one memory round trip instead of one per entry.
constexpr int kBUnroll = 16;

template <int ROLE, int PREC, int L>
__device__ __forceinline__ double b_half(const int64_t* __restrict__ ptr,
                                         const uint16_t* __restrict__ idx,
                                         const typename BTypes<PREC>::V* __restrict__ val,
                                         int64_t nl, const typename BTypes<PREC>::V* xin,
                                         const typename BTypes<PREC>::V* yprev,
                                         typename BTypes<PREC>::V* yout,
                                         const double* __restrict__ marg, int t, int* bad) {
    typedef typename BTypes<PREC>::V V;
    const int lane = threadIdx.x % L;
    const int g = threadIdx.x / L, ng = blockDim.x / L;
    double res = 0.0;
    int64_t k0 = 0, k1 = 0;
    if (g < nl) {
        k0 = ptr[g];
        k1 = ptr[g + 1];
    }
    for (int64_t r = g; r < nl; r += ng) {
        int64_t n0 = 0, n1 = 0;
        if (r + ng < nl) {
            n0 = ptr[r + ng];
            n1 = ptr[r + ng + 1];
        }
        V acc = 0;
        for (int64_t kb = k0 + lane; kb < k1; kb += kBUnroll * L) {
            V ve[kBUnroll];
            uint16_t ie[kBUnroll];
#pragma unroll
            for (int e = 0; e < kBUnroll; ++e) {
                const int64_t k = kb + (int64_t)e * L;
                ve[e] = k < k1 ? val[k] : (V)0;
                ie[e] = k < k1 ? idx[k] : (uint16_t)0;
            }
#pragma unroll
            for (int e = 0; e < kBUnroll; ++e)
                if (kb + (int64_t)e * L < k1) acc = fma(ve[e], xin[ie[e]], acc);
        }
        acc = group_sum<L>(acc);
        if (lane == 0) {
            const double w = (double)acc;
            const double m = marg[r];
            const bool ne = k1 > k0;
            const double yn = (ne && w > 0.0) ? m / w : 0.0;
            const V ys = (V)yn;
            yout[r] = ys;
            if (!isfinite((double)ys)) *bad = 1;
            if (ne) {
                if (ROLE == 0) {
                    if (t >= 2) res += fabs((double)yprev[r] * w - m);
                } else {
                    res += fabs((double)ys * w - m);
                }
            }
        }
        k0 = n0;
        k1 = n1;
    }
    return res;
}

// The first u-update of a warm-started problem: one pass over the rows forms
// w = K~ v0 and w1 = K~ 1 (the plain start's product, added in the same order
// as the fma of b_half with a gathered 1, so the plain u^1 is bit-identical to
// a cold solve's).  Writes the warm u^1 to uw and the plain u^1 over u0 (row r
// is read and written by the same lane only).  Returns this thread's shares of
// sum |u0_r w_r - a_r| and sum |w1_r - a_r| over rows with entries; *badw and
// *badp flag a non-finite warm or plain u^1.
template <int PREC, int L>
__device__ __forceinline__ void b_first_judged(const int64_t* __restrict__ ptr,
                                               const uint16_t* __restrict__ idx,
                                               const typename BTypes<PREC>::V* __restrict__ val,
                                               int64_t nl, const typename BTypes<PREC>::V* v0,
                                               typename BTypes<PREC>::V* u0,
                                               typename BTypes<PREC>::V* uw,
                                               const double* __restrict__ marg, double* rw,
                                               double* rp, int* badw, int* badp) {
    typedef typename BTypes<PREC>::V V;
    const int lane = threadIdx.x % L;
    const int g = threadIdx.x / L, ng = blockDim.x / L;
    double sw = 0.0, sp = 0.0;
    for (int64_t r = g; r < nl; r += ng) {
        const int64_t k0 = ptr[r], k1 = ptr[r + 1];
        V acc = 0, acc1 = 0;
        for (int64_t k = k0 + lane; k < k1; k += L) {
            const V e = val[k];
            acc = fma(e, v0[idx[k]], acc);
            acc1 = fma(e, (V)1, acc1);
        }
        acc = group_sum<L>(acc);
        acc1 = group_sum<L>(acc1);
        if (lane == 0) {
            const double w = (double)acc, w1 = (double)acc1;
            const double m = marg[r];
            const bool ne = k1 > k0;
            const V yw = (V)((ne && w > 0.0) ? m / w : 0.0);
            const V yp = (V)((ne && w1 > 0.0) ? m / w1 : 0.0);
            const double ur = (double)u0[r];
            uw[r] = yw;
            u0[r] = yp;
            if (!isfinite((double)yw)) *badw = 1;
            if (!isfinite((double)yp)) *badp = 1;
            if (ne) {
                sw += fabs(ur * w - m);
                sp += fabs(w1 - m);
            }
        }
    }
    *rw = sw;
    *rp = sp;
}

template <int PREC, int L>
__global__ __launch_bounds__(1024) void k_b_iterate(BIterArgs A) {
    typedef typename BTypes<PREC>::V V;
    extern __shared__ __align__(16) unsigned char dsm[];
    V* ua = (V*)dsm;
    V* ub = ua + A.nmax;
    V* vv = ub + A.nmax;
    __shared__ int s_q;
    __shared__ double sh[32];
    // a sketch larger than its arrays was not stored: nothing to iterate
    if (A.row_ptr[A.rows] > A.cap || A.col_ptr[A.cols] > A.cap) return;
    const V* val = (const V*)A.val;
    const V* val_t = (const V*)A.val_t;
    for (;;) {
        if (threadIdx.x == 0) s_q = atomicAdd(A.queue, 1);
        __syncthreads();
        const int q = s_q;
        __syncthreads();
        if (q >= A.count) break;
        const int k = A.order[q];
        const BProb P = A.prob[k];
        // a start with a NaN or +inf log-scaling (or one whose exponential
        // overflows) is not used
        int bad_init = 0;
        for (int64_t i = threadIdx.x; i < P.n; i += blockDim.x) {
            const double l = A.init_log_u ? A.init_log_u[P.xo + i] : 0.0;
            const V e = (V)exp(l);
            if (isnan(l) || !isfinite((double)e)) bad_init = 1;
            ua[i] = e;
        }
        for (int64_t j = threadIdx.x; j < P.m; j += blockDim.x) {
            const double l = A.init_log_v ? A.init_log_v[P.yo + j] : 0.0;
            const V e = (V)exp(l);
            if (isnan(l) || !isfinite((double)e)) bad_init = 1;
            vv[j] = e;
        }
        const bool warm = A.init_log_u || A.init_log_v;
        bad_init = __syncthreads_or(bad_init);
        V* u = ua;
        V* un = ub;
        double res_col = 0.0, err = INFINITY;
        int iters = 0, status = SS_NOT_CONVERGED, kept = warm ? 1 : -1;
        for (int t = 1;; ++t) {
            int bad = 0;
            double r;
            if (warm && t == 1) {
                double rw, rp;
                int badw = 0, badp = 0;
                b_first_judged<PREC, L>(A.row_ptr + P.xo, A.col_idx, val, P.n, vv, ua, ub,
                                        A.a_eff + P.xo, &rw, &rp, &badw, &badp);
                block_sum2(rw, rp, sh);
                badw = __syncthreads_or(badw);
                badp = __syncthreads_or(badp);
                // !(rw <= rp) also holds when rw is NaN
                kept = (bad_init || badw || !(rw <= rp)) ? 0 : 1;
                bad = kept ? badw : badp;
                // the kept u^1 is the one the swap below makes current
                if (!kept) {
                    u = ub;
                    un = ua;
                }
                r = 0.0;
            } else {
                r = b_half<0, PREC, L>(A.row_ptr + P.xo, A.col_idx, val, P.n, vv, u, un,
                                       A.a_eff + P.xo, t, &bad);
                r = block_sum(r, sh);
            }
            if (__syncthreads_or(bad)) {
                status = SS_E_NONFINITE;
                iters = t - 1;
                break;
            }
            if (t >= 2) {
                err = r + res_col;
                if (err <= A.tol) {
                    status = SS_OK;
                    iters = t - 1;
                    break;
                }
            }
            if (t == A.max_iter + 1) {
                iters = A.max_iter;
                break;
            }
            V* tmp = u;
            u = un;
            un = tmp;
            double c = b_half<1, PREC, L>(A.col_ptr + P.yo, A.row_idx, val_t, P.m, u, vv, vv,
                                          A.b_eff + P.yo, t, &bad);
            res_col = block_sum(c, sh);
            if (__syncthreads_or(bad)) {
                status = SS_E_NONFINITE;
                iters = t;
                break;
            }
        }
        // the returned iterate: u (the value before the last u-update) and v
        for (int64_t i = threadIdx.x; i < P.n; i += blockDim.x) {
            ((V*)A.u)[P.xo + i] = u[i];
            if (A.u_out) A.u_out[P.xo + i] = (double)u[i];
        }
        for (int64_t j = threadIdx.x; j < P.m; j += blockDim.x) {
            ((V*)A.v)[P.yo + j] = vv[j];
            if (A.v_out) A.v_out[P.yo + j] = (double)vv[j];
        }
        if (threadIdx.x == 0) {
            A.stat[k].iters = iters;
            A.stat[k].err = err;
            A.stat[k].status = status;
            A.stat[k].warm = kept;
        }
        __syncthreads();
    }
}

size_t batch_iter_lds(int precision, int nmax, int mmax) {
    return (size_t)(2 * nmax + mmax) * (precision == P_F64 ? 8 : 4);
}

template <int PREC, int L>
static const void* iter_fn() {
    return (const void*)&k_b_iterate<PREC, L>;
}

static const void* iter_kernel(int precision, int lanes) {
    if (precision == P_F64) {
        switch (lanes) {
            case 4: return iter_fn<P_F64, 4>();
            case 8: return iter_fn<P_F64, 8>();
            case 16: return iter_fn<P_F64, 16>();
            default: return iter_fn<P_F64, 32>();
        }
    }
    switch (lanes) {
        case 4: return iter_fn<P_F32, 4>();
        case 8: return iter_fn<P_F32, 8>();
        case 16: return iter_fn<P_F32, 16>();
        default: return iter_fn<P_F32, 32>();
    }
}

// Largest dynamic LDS any batch needs: u, u', v of 4096 FP64 each.
constexpr size_t kBatchLdsMax = 3 * kBatchMaxSide * 8;

hipError_t batch_init() {
    static hipError_t status = [] {
        hipError_t e = hipSuccess;
        for (int prec : {P_F64, P_F32})
            for (int lanes : {4, 8, 16, 32}) {
                const hipError_t r = hipFuncSetAttribute(iter_kernel(prec, lanes),
                                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                                         (int)kBatchLdsMax);
                if (r != hipSuccess) e = r;
            }
        return e;
    }();
    return status;
}

int batch_iter_grid(int precision, int lanes, int block, int nmax, int mmax) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, iter_kernel(precision, lanes), block,
                                                     batch_iter_lds(precision, nmax, mmax)) != hipSuccess)
        return 0;
    return cus * (per > 0 ? per : 1);
}

hipError_t launch_batch_iterate(int precision, int lanes, int block, int grid, const BIterArgs& a,
                                hipStream_t st) {
    const size_t lds = batch_iter_lds(precision, a.nmax, a.mmax);
    const dim3 g((unsigned)grid), b((unsigned)block);
#define SS_BITER(P, L) hipLaunchKernelGGL((k_b_iterate<P, L>), g, b, lds, st, a)
    if (precision == P_F64) {
        switch (lanes) {
            case 4: SS_BITER(P_F64, 4); break;
            case 8: SS_BITER(P_F64, 8); break;
            case 16: SS_BITER(P_F64, 16); break;
            default: SS_BITER(P_F64, 32); break;
        }
    } else {
        switch (lanes) {
            case 4: SS_BITER(P_F32, 4); break;
            case 8: SS_BITER(P_F32, 8); break;
            case 16: SS_BITER(P_F32, 16); break;
            default: SS_BITER(P_F32, 32); break;
        }
    }
#undef SS_BITER
    return hipGetLastError();
}

// ------------------------------------------------------------------ estimate
// One block per problem, 16 lanes per row: sum T~ C, sum T~ (log T~ - 1) and
// sum T~ (log u + log v - 1) over the kept entries (Alg. 3; 0 log 0 = 0).
// With log T~ = log u + log v + log K~ the second is the third plus
// sum T~ log K~, so an entry takes one logarithm (the specified one); log v
// is formed once per column.
constexpr int kBObjLanes = 16;
constexpr int kBObjUnroll = 4;  // entries a lane loads before using any

// Block (k, b) of kBObjSplit per problem sums rows b, b + kBObjSplit, ... of
// problem k (in groups of blockDim / kBObjLanes rows) into its partials.  The
// problem's v and log v are staged in LDS (the entries gather them at random
// columns).
template <int PREC, int D>
__global__ __launch_bounds__(256) void k_b_objective(BObjArgs A) {
    typedef typename BTypes<PREC>::V V;
    __shared__ double sh[16];
    __shared__ V vs[SS_BATCH_MAX_SIDE];
    __shared__ double lvs[SS_BATCH_MAX_SIDE];
    if (A.row_ptr[A.rows] > A.cap || A.col_ptr[A.cols] > A.cap) return;
    const int k = blockIdx.x / kBObjSplit, blk = blockIdx.x % kBObjSplit;
    const BProb P = A.prob[k];
    for (int64_t j = threadIdx.x; j < P.m; j += blockDim.x) {
        const V v = ((const V*)A.v)[P.yo + j];
        vs[j] = v;
        lvs[j] = log_spec((double)v);
    }
    __syncthreads();
    const int sub = threadIdx.x % kBObjLanes;
    const double inv_cmax = A.stat[k].inv_cmax;
    const V* __restrict__ u = (const V*)A.u + P.xo;
    const V* __restrict__ val = (const V*)A.val;
    const uint16_t* __restrict__ cidx = A.col_idx;
    const double* __restrict__ x = A.x + P.xo * A.d;
    const double* __restrict__ y = A.y + P.yo * A.d;
    constexpr int RPB = 256 / kBObjLanes;  // rows in flight per block
    double s_tc = 0.0, s_lk = 0.0, s_sp = 0.0;
    for (int64_t r = (int64_t)blk * RPB + threadIdx.x / kBObjLanes; r < P.n;
         r += (int64_t)kBObjSplit * RPB) {
        const int64_t k0 = A.row_ptr[P.xo + r], k1 = A.row_ptr[P.xo + r + 1];
        const double ur = (double)u[r];
        const double lu = log_spec(ur);
        for (int64_t e0 = k0 + sub; e0 < k1; e0 += kBObjUnroll * kBObjLanes) {
            int o[kBObjUnroll];
            V kv[kBObjUnroll];
#pragma unroll
            for (int q = 0; q < kBObjUnroll; ++q) {
                const int64_t e = e0 + q * kBObjLanes;
                const bool in = e < k1;
                o[q] = in ? (int)cidx[e] : 0;
                kv[q] = in ? val[e] : (V)0;
            }
#pragma unroll
            for (int q = 0; q < kBObjUnroll; ++q) {
                const double vo = (double)vs[o[q]];
                const double t = ur * (double)kv[q] * vo;
                if (t > 0.0) {
                    const double c = sqdist<D>(x + r * A.d, y + o[q] * A.d, A.d) * inv_cmax;
                    s_tc += t * c;
                    s_lk += t * log_spec((double)kv[q]);
                    s_sp += t * ((lu + lvs[o[q]]) - 1.0);
                }
            }
        }
    }
    s_tc = block_sum(s_tc, sh);
    s_lk = block_sum(s_lk, sh);
    s_sp = block_sum(s_sp, sh);
    if (threadIdx.x == 0) {
        double* pt = A.part + ((int64_t)k * kBObjSplit + blk) * 3;
        pt[0] = s_tc;
        pt[1] = s_sp + s_lk;
        pt[2] = s_sp;
    }
}

// Per problem: the partials of its blocks in block order.
__global__ void k_b_obj_final(BObjArgs A, int count) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    if (A.row_ptr[A.rows] > A.cap || A.col_ptr[A.cols] > A.cap) return;
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < kBObjSplit; ++b)
        for (int q = 0; q < 3; ++q) s[q] += A.part[((int64_t)k * kBObjSplit + b) * 3 + q];
    A.stat[k].transport = s[0];
    A.stat[k].negent = s[1];
    A.stat[k].sparseobj = s[2];
}

template <int PREC, int D>
static void run_b_obj(int count, const BObjArgs& a, hipStream_t st) {
    hipLaunchKernelGGL((k_b_objective<PREC, D>), dim3((unsigned)(count * kBObjSplit)), dim3(256), 0,
                       st, a);
    hipLaunchKernelGGL(k_b_obj_final, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, a,
                       count);
}

template <int D>
static void run_b_obj_d(int precision, int count, const BObjArgs& a, hipStream_t st) {
    if (precision == P_F64)
        run_b_obj<P_F64, D>(count, a, st);
    else
        run_b_obj<P_F32, D>(count, a, st);
}

hipError_t launch_batch_objective(int precision, int count, const BObjArgs& a, hipStream_t st) {
    switch (a.d) {
        case 2: run_b_obj_d<2>(precision, count, a, st); break;
        case 3: run_b_obj_d<3>(precision, count, a, st); break;
        case 10: run_b_obj_d<10>(precision, count, a, st); break;
        default: run_b_obj_d<0>(precision, count, a, st); break;
    }
    return hipGetLastError();
}

__global__ void k_b_log_scaling(int precision, const void* __restrict__ y,
                                double* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = precision == P_F64 ? ((const double*)y)[i] : (double)((const float*)y)[i];
    out[i] = log(v);
}

hipError_t launch_batch_log_scaling(int precision, const void* y, double* out, int64_t n,
                                    hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_b_log_scaling, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       precision, y, out, n);
    return hipGetLastError();
}

}  // namespace ss
