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
// The closing reads nothing this launch writes and writes nothing this launch
// reads (the other blocks only test the stop flag, and a launch that runs
// after the stop writes buffers the result does not come from), so block 0
// may close at any point of its work.
//
// loop_start returns the iteration number t, 0 if the loop has stopped (then
// nothing is left to close).  `s_t` is LDS scratch of the caller.
__device__ __forceinline__ int loop_start(const IterState* st, int role, int max_iter, int* s_t) {
    // The flags may change while this launch runs (block 0's closing, or a
    // block that meets a non-finite value), so one thread reads them and the
    // block takes a single decision: no divergent exit before a barrier.
    if (threadIdx.x == 0) {
        const int tt = role == 0 ? st->cnt_u + 1 : st->cnt_v;
        const bool go = st->stop_iter == 0 && st->nonfinite == 0 && tt <= max_iter + 1;
        *s_t = go ? tt : 0;
    }
    __syncthreads();
    return *s_t;
}

// Whether launch t updates scalings (else it only closes): u-launch
// t = max_iter + 1 still forms the row residual of iterate max_iter (marginal
// rule); everything else past max_iter only closes.
__device__ __forceinline__ bool loop_updates(int role, int marginal, int max_iter, int t) {
    if (role == 0) return t <= max_iter || (marginal && t == max_iter + 1);
    return t <= max_iter;
}

// Block 0's closing decision for launch t >= 1 from the sum of the previous
// launch's partials (thread 0 of block 0 calls it).
__device__ __forceinline__ void loop_decide(IterState* st, int role, int marginal, int max_iter,
                                            double tol, double* err_hist, int t, double total) {
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
        st->err_last = err;
        if (err_hist) err_hist[t - 2] = err;
        if (err <= tol || t - 1 >= max_iter) {
            st->err_final = err;
            st->stop_iter = t - 1;
        }
    }
}

// Whether launch t sums the previous launch's partials (the first u-launch
// has none).
__device__ __forceinline__ bool loop_closes(int role, int t) { return role == 1 || t >= 2; }

// Block 0's closing work for launch t >= 1 (every thread of block 0 calls it;
// `sh`: 16 doubles of LDS).
__device__ __forceinline__ void loop_close(IterState* st, int role, int marginal, int max_iter,
                                           double tol, const double* prev, int prev_nb,
                                           double* err_hist, int t, double* sh) {
    const double total = loop_closes(role, t) ? reduce_partials(prev, prev_nb, sh) : 0.0;
    if (threadIdx.x == 0) loop_decide(st, role, marginal, max_iter, tol, err_hist, t, total);
}

// Start and closing together; returns t if this launch updates scalings, 0
// if it has nothing (more) to do.  `sh` (16 doubles) and `s_t`: LDS scratch.
__device__ __forceinline__ int loop_enter(IterState* st, int role, int marginal, int max_iter,
                                          double tol, const double* prev, int prev_nb,
                                          double* err_hist, double* sh, int* s_t) {
    const int t = loop_start(st, role, max_iter, s_t);
    if (t == 0) return 0;
    if (blockIdx.x == 0) loop_close(st, role, marginal, max_iter, tol, prev, prev_nb, err_hist, t, sh);
    return loop_updates(role, marginal, max_iter, t) ? t : 0;
}

// The same with static LDS scratch.
__device__ __forceinline__ int loop_enter(IterState* st, int role, int marginal, int max_iter,
                                          double tol, const double* prev, int prev_nb,
                                          double* err_hist) {
    __shared__ double sh[16];
    __shared__ int s_t;
    return loop_enter(st, role, marginal, max_iter, tol, prev, prev_nb, err_hist, sh, &s_t);
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
// `yp` is the previous value (scaling, or potential in the log domain);
// `lm` = log(m) (used in the log domain).  The new value is returned already
// rounded to the stored type Y.
// Not inlined: its FP64 transcendental code would otherwise pin constants in
// registers across the callers' streaming loops.  It touches no memory: a
// called function waits for all of its memory operations before returning,
// so the caller stores the result (line_store) and the stores overlap.
struct LineNew {
    double y;
    double res;
};

template <int PREC, bool UOT>
__device__ __attribute__((noinline)) LineNew line_new(int role, int marginal, int t, bool nonempty,
                                                      double m, double lm, double theta, double yp,
                                                      double w) {
    typedef typename Scal<PREC>::Y Y;
    double res = 0.0;
    double y;
    if (PREC != P_LOG) {
        double yn = 0.0;
        if (nonempty && w > 0.0) {
            const double q = m / w;
            yn = UOT ? exp(theta * log(q)) : q;
        }
        y = (double)(Y)yn;
        if (nonempty) {
            if (marginal) {
                const double yr = role == 0 ? yp : y;
                const double yq = UOT ? (yr > 0.0 ? exp(log(yr) / theta) : 0.0) : yr;
                if (role == 1 || t >= 2) res = fabs(yq * w - m);
            } else {
                res = fabs(y - yp);
            }
        }
    } else {
        const double fp = yp;
        double fn = -INFINITY;
        if (nonempty && w != -INFINITY) fn = theta * (lm - w);
        y = fn;
        if (nonempty) {
            if (marginal) {
                const double fr = role == 0 ? fp : fn;
                if (role == 1 || t >= 2) res = fabs(exp(fr / theta + w) - m);
            } else {
                res = fabs(exp(fn) - exp(fp));
            }
        }
    }
    return {y, res};
}

// Stores the new value of a line and flags a non-finite one.  `yg` (log
// domain, may be NULL) receives the FP32 gathered copy in base-2 units,
// f log2(e), the form the sparse product adds to its base-2 entries.
template <int PREC>
__device__ __forceinline__ void line_store(void* yout, float* yg, int64_t line, double y,
                                           IterState* st) {
    typedef typename Scal<PREC>::Y Y;
    ((Y*)yout)[line] = (Y)y;
    if (PREC != P_LOG) {
        if (!isfinite(y)) st->nonfinite = 1;
    } else {
        if (yg) yg[line] = (float)(y * kLog2e);
        if (isnan(y) || y == INFINITY) st->nonfinite = 1;
    }
}

}  // namespace ss
