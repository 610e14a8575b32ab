// Per-line scaling update and the ticketed end-of-iteration logic shared by the
// sparse (iterate.hip) and dense (dense.hip) Sinkhorn loops.
#pragma once

#include <math.h>

#include "common.hpp"
#include "internal.hpp"

namespace ss {

template <int PREC>
struct Scal;
template <>
struct Scal<P_F64> {
    typedef double V;  // stored matrix value / accumulator
    typedef double Y;  // stored scaling or potential
};
template <>
struct Scal<P_F32> {
    typedef float V;
    typedef float Y;
};
template <>
struct Scal<P_LOG> {
    typedef float V;
    typedef double Y;
};

// Common entry test of an iteration kernel; returns the iteration number t or
// 0 if the kernel has nothing to do (stopped, non-finite, or past max_iter).
__device__ __forceinline__ int iteration_begin(const IterState* st, int role, int marginal,
                                               int max_iter) {
    const int t = st->iter + 1;
    if (st->stop_iter != 0 || st->nonfinite != 0) return 0;
    const int tmax = max_iter + ((role == 0 && marginal) ? 1 : 0);
    return t > tmax ? 0 : t;
}

// New scaling of one line and its residual term.
//  linear (PREC F64/F32): `w` = (M x)_r;   log (PREC LOG): `w` = log-sum-exp.
//  role 0 (u-update): marginal residual of the previous iterate
//                     |u_prev^(1/th) w - a| (valid for t >= 2);
//  role 1 (v-update): marginal residual of the new iterate |v^(1/th) w - b|.
//  delta rule: |y_new - y_prev| in the linear scale.
template <int PREC, bool UOT>
__device__ __forceinline__ double line_update(int role, int marginal, int t, bool nonempty,
                                              double m, double theta, const void* yprev, void* yout,
                                              int64_t line, double w, IterState* st) {
    typedef typename Scal<PREC>::Y Y;
    double res = 0.0;
    if (PREC != P_LOG) {
        const double yp = (double)((const Y*)yprev)[line];
        double yn = 0.0;
        if (nonempty && w > 0.0) {
            const double q = m / w;
            yn = UOT ? pow(q, theta) : q;
        }
        const Y ys = (Y)yn;
        ((Y*)yout)[line] = ys;
        if (!isfinite((double)ys)) st->nonfinite = 1;
        if (nonempty) {
            if (marginal) {
                const double yr = role == 0 ? yp : (double)ys;
                const double yq = UOT ? pow(yr, 1.0 / theta) : yr;
                if (role == 1 || t >= 2) res = fabs(yq * w - m);
            } else {
                res = fabs((double)ys - yp);
            }
        }
    } else {
        const double fp = ((const double*)yprev)[line];
        double fn = -INFINITY;
        if (nonempty && w != -INFINITY) fn = theta * (log(m) - w);
        ((double*)yout)[line] = fn;
        if (isnan(fn) || fn == INFINITY) st->nonfinite = 1;
        if (nonempty) {
            if (marginal) {
                const double fr = role == 0 ? fp : fn;
                if (role == 1 || t >= 2) res = fabs(exp(fr / theta + w) - m);
            } else {
                res = fabs(exp(fn) - exp(fp));
            }
        }
    }
    return res;
}

// Block reduction of the residual, then the last block of the launch closes
// the iteration: role 0 completes err(t-1) (marginal rule) and may stop; role
// 1 records the column residual (marginal) or err(t) (delta) and bumps iter.
__device__ __forceinline__ void iteration_end(double res, IterState* st, double* partials, int role,
                                              int marginal, int t, int max_iter, double tol,
                                              double* err_hist) {
    __shared__ double sh[4];
    __shared__ int is_last;
    const int tid = threadIdx.x;
    const double bsum = block_sum256(res, sh);
    if (tid == 0) {
        partials[blockIdx.x] = bsum;
        __threadfence();
        const unsigned tk = atomicAdd(&st->ticket[role], 1u);
        is_last = (tk == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    double v = 0.0;
    for (unsigned b = tid; b < gridDim.x; b += kBlock) v += load_agent(&partials[b]);
    const double total = block_sum256(v, sh);
    if (tid != 0) return;
    st->ticket[role] = 0;
    if (role == 0) {
        if (marginal) {
            if (t >= 2) {
                const double err = total + st->err_col;
                if (err_hist) err_hist[t - 2] = err;
                if (err <= tol || t - 1 >= max_iter) {
                    st->err_final = err;
                    st->stop_iter = t - 1;
                }
            }
        } else {
            st->err_row = total;
        }
    } else {
        if (marginal) {
            st->err_col = total;
        } else {
            const double err = st->err_row + total;
            if (err_hist) err_hist[t - 1] = err;
            if (err <= tol || t >= max_iter) {
                st->err_final = err;
                st->stop_iter = t;
            }
        }
        st->iter = t;
    }
}

}  // namespace ss
