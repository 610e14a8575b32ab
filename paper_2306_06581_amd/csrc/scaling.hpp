// Per-line scaling update and the end-of-iteration logic shared by the
// sparse (iterate.hip) and dense (dense.hip) Sinkhorn loops.
//
// Iteration t is two launches, the u-update (role 0) and the v-update
// (role 1).  No launch waits on another block of itself: every block writes
// one residual partial, and block 0 of the NEXT launch reduces those partials
// in index order (kernel boundaries order the two) and takes the stop
// decision.  So there are no atomics and no device-wide fences in the loop.
// The iteration number travels in two counters (cnt_u read by u-launches,
// written by v-launches' block 0; cnt_v the other way round), so no launch
// reads a word that its own block 0 writes.
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
    typedef double G;  // gathered copy of the other side's scaling
};
template <>
struct Scal<P_F32> {
    typedef float V;
    typedef float Y;
    typedef float G;
};
// Log domain: potentials are kept in FP64; the sparse product gathers an FP32
// copy (absolute error |f| 2^-24, the same order as the FP32 log-kernel
// entries it is added to).
template <>
struct Scal<P_LOG> {
    typedef float V;
    typedef double Y;
    typedef float G;
};

// Sum of nb partials in a fixed order (all threads of the block call it).
__device__ __forceinline__ double reduce_partials(const double* p, int nb, double* sh) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) v += p[b];
    return block_sum(v, sh);
}

// Entry of an iteration launch.  Block 0 closes the previous launch:
//  u-launch of iteration t (t >= 2) reduces the v-launch partials of t-1:
//     marginal rule: the column residual of iterate t-1 -> err_col;
//     delta rule:    err(t-1) = |du| + |dv| -> history, stop test.
//  v-launch of iteration t reduces the u-launch partials of t:
//     marginal rule: err(t-1) = row residual + err_col -> history, stop test;
//     delta rule:    |du| of iteration t -> err_row.
// Returns t if this launch updates scalings, 0 if it has nothing (more) to do.
__device__ __forceinline__ int loop_enter(IterState* st, int role, int marginal, int max_iter,
                                          double tol, const double* prev, int prev_nb,
                                          double* err_hist) {
    __shared__ double sh[16];
    // The flags may change while this launch runs (block 0 below, or a block
    // that meets a non-finite value), so one thread reads them and the block
    // takes a single decision: no divergent exit before a barrier.
    __shared__ int s_t;
    if (threadIdx.x == 0) {
        const int tt = role == 0 ? st->cnt_u + 1 : st->cnt_v;
        const bool go = st->stop_iter == 0 && st->nonfinite == 0 && tt <= max_iter + 1;
        s_t = go ? tt : 0;
    }
    __syncthreads();
    const int t = s_t;
    if (t == 0) return 0;
    if (blockIdx.x == 0) {
        const bool close = role == 1 || t >= 2;
        const double total = close ? reduce_partials(prev, prev_nb, sh) : 0.0;
        if (threadIdx.x == 0) {
            bool decide = false;
            double err = 0.0;
            if (role == 0) {
                if (t >= 2) {
                    if (marginal) {
                        st->err_col = total;
                    } else {
                        err = st->err_row + total;
                        decide = true;
                    }
                }
                st->cnt_v = t;
            } else {
                if (marginal) {
                    if (t >= 2) {
                        err = total + st->err_col;
                        decide = true;
                    }
                } else {
                    st->err_row = total;
                }
                st->cnt_u = t;
            }
            if (decide) {
                if (err_hist) err_hist[t - 2] = err;
                if (err <= tol || t - 1 >= max_iter) {
                    st->err_final = err;
                    st->stop_iter = t - 1;
                }
            }
        }
    }
    // u-launch t = max_iter + 1 still forms the row residual of iterate
    // max_iter (marginal rule); everything else past max_iter only closes.
    if (role == 0) return (t <= max_iter || (marginal && t == max_iter + 1)) ? t : 0;
    return t <= max_iter ? t : 0;
}

// Same test as loop_enter without the closing work (for launches that only
// produce inputs of the launch that closes, e.g. the dense partial sums).
__device__ __forceinline__ int loop_peek(const IterState* st, int role, int marginal, int max_iter) {
    __shared__ int s_t;
    if (threadIdx.x == 0) {
        const int t = role == 0 ? st->cnt_u + 1 : st->cnt_v;
        int go = st->stop_iter == 0 && st->nonfinite == 0 && t <= max_iter + 1;
        if (go) go = role == 0 ? (t <= max_iter || (marginal && t == max_iter + 1)) : t <= max_iter;
        s_t = go ? t : 0;
    }
    __syncthreads();
    return s_t;
}

// New scaling of one line and its residual term.
//  linear (PREC F64/F32): `w` = (M x)_r;   log (PREC LOG): `w` = log-sum-exp.
//  role 0 (u-update): marginal residual of the previous iterate
//                     |u_prev^(1/th) w - a| (valid for t >= 2);
//  role 1 (v-update): marginal residual of the new iterate |v^(1/th) w - b|.
//  delta rule: |y_new - y_prev| in the linear scale.
// `yp` is the previous value (scaling, or potential in the log domain).
// Not inlined: its FP64 transcendental code would otherwise pin constants in
// registers across the callers' streaming loops.
template <int PREC, bool UOT>
// `yg` (log domain, may be NULL) receives the FP32 gathered copy.
__device__ __attribute__((noinline)) double line_update(int role, int marginal, int t, bool nonempty,
                                              double m, double theta, double yp, void* yout,
                                              float* yg, int64_t line, double w, IterState* st) {
    typedef typename Scal<PREC>::Y Y;
    double res = 0.0;
    if (PREC != P_LOG) {
        double yn = 0.0;
        if (nonempty && w > 0.0) {
            const double q = m / w;
            yn = UOT ? exp(theta * log(q)) : q;
        }
        const Y ys = (Y)yn;
        ((Y*)yout)[line] = ys;
        if (!isfinite((double)ys)) st->nonfinite = 1;
        if (nonempty) {
            if (marginal) {
                const double yr = role == 0 ? yp : (double)ys;
                const double yq = UOT ? (yr > 0.0 ? exp(log(yr) / theta) : 0.0) : yr;
                if (role == 1 || t >= 2) res = fabs(yq * w - m);
            } else {
                res = fabs((double)ys - yp);
            }
        }
    } else {
        const double fp = yp;
        double fn = -INFINITY;
        if (nonempty && w != -INFINITY) fn = theta * (log(m) - w);
        ((double*)yout)[line] = fn;
        if (yg) yg[line] = (float)fn;
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

}  // namespace ss
