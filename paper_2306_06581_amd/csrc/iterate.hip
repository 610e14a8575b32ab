// Sinkhorn scaling loop on the sparse sketch (Alg. 1 / Alg. 2 applied to K~).
//
// One kernel serves both half-steps: for every line r of a sparse matrix M
// (the CSR of K~ for the u-update, the CSC for the v-update) it forms
// w_r = sum_k M_rk x_k, writes the new scaling y_r = marg_r / w_r (OT) or
// (marg_r / w_r)^theta (UOT, theta = lam/(lam+eps)), and adds its residual
// term.  A group of LPR lanes owns a line; the matrix entries stream once from
// HBM, the gathered vector stays in L2.  The residual is reduced per block in
// a fixed tree and the last block (ticketed) sums the block partials in index
// order, so the stop test is deterministic.
//
// Log-domain variant (appendix, proof of Thm. 3): the matrix stores
// l_rk = log K~_rk in FP32, the vectors hold FP64 potentials f = log u,
// g = log v, and w_r becomes a stabilised streaming log-sum-exp.
#include <math.h>

#include "common.hpp"
#include "internal.hpp"
#include "scaling.hpp"

namespace ss {

template <int PREC, int LPR, bool UOT>
__global__ __launch_bounds__(256) void k_iterate(IterArgs A) {
    typedef typename Scal<PREC>::V V;
    typedef typename Scal<PREC>::Y Y;
    IterState* st = A.st;
    const int marginal = A.stop_rule == 0;
    const int t = iteration_begin(st, A.role, marginal, A.max_iter);
    if (t == 0) return;

    const int tid = threadIdx.x;
    const int sub = tid % LPR;
    const int64_t line = (int64_t)blockIdx.x * (kBlock / LPR) + tid / LPR;
    const V* __restrict__ val = (const V*)A.val;
    const int32_t* __restrict__ idx = A.idx;
    const Y* __restrict__ xin = (const Y*)A.xin;

    int64_t k0 = 0, k1 = 0;
    if (line < A.nlines) {
        k0 = A.ptr[line];
        k1 = A.ptr[line + 1];
    }
    double w;
    if constexpr (PREC != P_LOG) {
        V acc = 0;
        for (int64_t k = k0 + sub; k < k1; k += LPR) {
            const V v = __builtin_nontemporal_load(&val[k]);
            const int32_t c = __builtin_nontemporal_load(&idx[k]);
            acc = fma(v, xin[c], acc);
        }
        w = (double)group_sum<LPR>(acc);
    } else {
        // streaming log-sum-exp: running max mx and sum s of exp(z - mx)
        double mx = -INFINITY;
        float s = 0.0f;
        for (int64_t k = k0 + sub; k < k1; k += LPR) {
            const float l = __builtin_nontemporal_load(&val[k]);
            const int32_t c = __builtin_nontemporal_load(&idx[k]);
            const double z = (double)l + xin[c];
            if (z > mx) {
                s = s * __expf((float)(mx - z)) + 1.0f;
                mx = z;
            } else {
                s += __expf((float)(z - mx));
            }
        }
        const double M = group_max<LPR>(mx);
        float part = (mx == -INFINITY) ? 0.0f : s * __expf((float)(mx - M));
        part = group_sum<LPR>(part);
        w = (M == -INFINITY || !(part > 0.0f)) ? -INFINITY : M + log((double)part);
    }
    double res = 0.0;
    if (sub == 0 && line < A.nlines)
        res = line_update<PREC, UOT>(A.role, marginal, t, k1 > k0, A.marg[line], A.theta, A.yprev,
                                     A.yout, line, w, st);
    iteration_end(res, st, A.partials, A.role, marginal, t, A.max_iter, A.tol, A.err_hist);
}

int iterate_blocks(int lanes, int64_t nlines) {
    const int64_t per = kBlock / lanes;
    return (int)((nlines + per - 1) / per);
}

template <int PREC, int LPR>
static void run_iter(const IterArgs& a, hipStream_t st) {
    const int nb = iterate_blocks(LPR, a.nlines);
    if (a.theta != 1.0)
        hipLaunchKernelGGL((k_iterate<PREC, LPR, true>), dim3(nb), dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL((k_iterate<PREC, LPR, false>), dim3(nb), dim3(kBlock), 0, st, a);
}

template <int PREC>
static void run_iter_p(int lanes, const IterArgs& a, hipStream_t st) {
    switch (lanes) {
        case 4: run_iter<PREC, 4>(a, st); break;
        case 8: run_iter<PREC, 8>(a, st); break;
        case 16: run_iter<PREC, 16>(a, st); break;
        case 32: run_iter<PREC, 32>(a, st); break;
        default: run_iter<PREC, 64>(a, st); break;
    }
}

hipError_t launch_iterate(int precision, int lanes, const IterArgs& a, hipStream_t st) {
    if (precision == P_F64)
        run_iter_p<P_F64>(lanes, a, st);
    else if (precision == P_F32)
        run_iter_p<P_F32>(lanes, a, st);
    else
        run_iter_p<P_LOG>(lanes, a, st);
    return hipGetLastError();
}

// u^0 / v^0: ones (or exp of the warm start); potentials 0 (or the warm start).
__global__ void k_init_scaling(int precision, void* y, const double* init_log, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double l = init_log ? init_log[i] : 0.0;
    if (precision == P_F64) ((double*)y)[i] = init_log ? exp(l) : 1.0;
    if (precision == P_F32) ((float*)y)[i] = init_log ? (float)exp(l) : 1.0f;
    if (precision == P_LOG) ((double*)y)[i] = l;
}

hipError_t launch_init_scaling(int precision, void* y, const double* init_log, int64_t n,
                               hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_scaling, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       precision, y, init_log, n);
    return hipGetLastError();
}

__global__ void k_export_scaling(int precision, const void* y, double* out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (precision == P_F64) out[i] = ((const double*)y)[i];
    if (precision == P_F32) out[i] = (double)((const float*)y)[i];
    if (precision == P_LOG) out[i] = exp(((const double*)y)[i]);
}

hipError_t launch_export_scaling(int precision, const void* y, double* out, int64_t n,
                                 hipStream_t st) {
    if (n <= 0 || out == nullptr) return hipSuccess;
    hipLaunchKernelGGL(k_export_scaling, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       precision, y, out, n);
    return hipGetLastError();
}

}  // namespace ss
