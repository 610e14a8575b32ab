// Estimate of Alg. 3 / Alg. 4 on the returned iterate, in FP64:
//   <T~, C> - eps H(T~)  (+ lam KL(T~ 1 | a) + lam KL(T~' 1 | b) for UOT),
// with T~_ij = u_i K~_ij v_j over the kept entries, C recomputed from the
// coordinates, 0 log 0 = 0 (Sec. 2 notation).  Rows pass: transport term,
// entropy term, sparse-problem term sum T~ (log u_i + log v_j - 1) and the
// row KL; columns pass: the column KL.  Per-block partials are summed in
// index order by a one-block reduction launch (deterministic, no atomics).
#include <math.h>

#include "common.hpp"
#include "internal.hpp"

namespace ss {

constexpr int kObjLanes = 16;

template <int PREC>
__device__ __forceinline__ double scal_log(const void* p, int64_t i) {
    if (PREC == P_LOG) return ((const double*)p)[i];
    if (PREC == P_F64) return log(((const double*)p)[i]);
    return log((double)((const float*)p)[i]);
}

template <int PREC>
__device__ __forceinline__ double scal_lin(const void* p, int64_t i) {
    if (PREC == P_LOG) return exp(((const double*)p)[i]);
    if (PREC == P_F64) return ((const double*)p)[i];
    return (double)((const float*)p)[i];
}

// T~ entry from the line scaling, the stored value and the other scaling.
template <int PREC>
__device__ __forceinline__ double plan_entry(double yl_lin, double yl_log, const void* val, int64_t k,
                                             const void* zs, int64_t o) {
    if (PREC == P_LOG) return exp(yl_log + (double)((const float*)val)[k] + ((const double*)zs)[o]);
    if (PREC == P_F64) return yl_lin * ((const double*)val)[k] * ((const double*)zs)[o];
    return yl_lin * (double)((const float*)val)[k] * (double)((const float*)zs)[o];
}

template <int PREC, int D>
__global__ __launch_bounds__(256) void k_objective(ObjArgs A) {
    __shared__ double sh[4];
    const int tid = threadIdx.x, sub = tid % kObjLanes;
    const int64_t line = (int64_t)blockIdx.x * (kBlock / kObjLanes) + tid / kObjLanes;
    double s_tc = 0.0, s_ent = 0.0, s_sp = 0.0, s_line = 0.0;
    if (line < A.nlines) {
        const int64_t k0 = A.ptr[line], k1 = A.ptr[line + 1];
        const double yl = scal_lin<PREC>(A.ys, line);
        const double ylog = scal_log<PREC>(A.ys, line);
        const double* xl = A.x + line * A.d;
        for (int64_t k = k0 + sub; k < k1; k += kObjLanes) {
            const int64_t o = A.idx[k];
            const double t = plan_entry<PREC>(yl, ylog, A.val, k, A.zs, o);
            s_line += t;
            if (A.role == 0 && t > 0.0) {
                const double c = cost_value(sqdist<D>(xl, A.y + o * A.d, A.d), A.cost, A.inv_cmax,
                                            A.wfr_w);
                s_tc += t * c;
                const double lt = log(t);
                s_ent += t * (lt - 1.0);
                s_sp += t * ((ylog + scal_log<PREC>(A.zs, o)) - 1.0);
            }
        }
    }
    s_tc = group_sum<kObjLanes>(s_tc);
    s_ent = group_sum<kObjLanes>(s_ent);
    s_sp = group_sum<kObjLanes>(s_sp);
    s_line = group_sum<kObjLanes>(s_line);
    double kl = 0.0;
    if (sub == 0 && line < A.nlines && A.uot) {
        const double m = A.marg[line];
        kl = (s_line > 0.0 ? s_line * log(s_line / m) : 0.0) - s_line + m;
    }
    if (sub != 0) s_tc = s_ent = s_sp = s_line = 0.0;
    double q[5] = {s_tc, s_ent, s_sp, kl, s_line};
    double tot[5];
#pragma unroll
    for (int r = 0; r < 5; ++r) tot[r] = block_sum256(q[r], sh);
    const unsigned nb = gridDim.x;
    if (tid == 0) {
#pragma unroll
        for (int r = 0; r < 5; ++r) A.partials[(int64_t)r * nb + blockIdx.x] = tot[r];
    }
}

// One block: stats[slot[q]] = fixed-order sum of src[q][0..len[q]).
__global__ __launch_bounds__(256) void k_reduce_stats(ReduceSpec r, double* stats) {
    __shared__ double sh[4];
    for (int q = 0; q < r.nq; ++q) {
        double v = 0.0;
        for (int64_t b = threadIdx.x; b < r.len[q]; b += kBlock) v += r.src[q][b];
        const double tot = block_sum256(v, sh);
        if (threadIdx.x == 0) stats[r.slot[q]] = tot;
    }
}

hipError_t launch_reduce_stats(const ReduceSpec& r, double* stats, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_stats, dim3(1), dim3(kBlock), 0, st, r, stats);
    return hipGetLastError();
}

template <int PREC, int D>
static void run_obj(const ObjArgs& a, hipStream_t st) {
    const int nb = (int)((a.nlines + (kBlock / kObjLanes) - 1) / (kBlock / kObjLanes));
    hipLaunchKernelGGL((k_objective<PREC, D>), dim3(nb), dim3(kBlock), 0, st, a);
    ReduceSpec r;
    r.nq = 0;
    const int rows[5] = {ST_TRANSPORT, ST_NEGENT, ST_SPARSEOBJ, ST_KL_A, ST_ROWSUM};
    const int cols[5] = {-1, -1, -1, ST_KL_B, ST_COLSUM};
    for (int q = 0; q < 5; ++q) {
        const int slot = a.role == 0 ? rows[q] : cols[q];
        if (slot < 0) continue;
        r.src[r.nq] = a.partials + (int64_t)q * nb;
        r.len[r.nq] = nb;
        r.slot[r.nq] = slot;
        ++r.nq;
    }
    (void)launch_reduce_stats(r, a.stats, st);
}

template <int D>
static void run_obj_d(int precision, const ObjArgs& a, hipStream_t st) {
    if (precision == P_F64)
        run_obj<P_F64, D>(a, st);
    else if (precision == P_F32)
        run_obj<P_F32, D>(a, st);
    else
        run_obj<P_LOG, D>(a, st);
}

// Envelope gradient of the sparse problem's value (the divergence of the
// generative-modelling section): 16 lanes per line stride its entries, T~ as
// in the estimate, a fixed xor tree per coordinate, then one read-modify-write
// of the line's d outputs (lines are disjoint, launches on one stream).  With
// the Euclidean cost an entry's term is weighted by 1 / |x_i - y_j| (0 where
// the points coincide).
template <int PREC, int D>
__global__ __launch_bounds__(256) void k_plan_grad(GradArgs A) {
    const int tid = threadIdx.x, sub = tid % kObjLanes;
    const int64_t line = (int64_t)blockIdx.x * (kBlock / kObjLanes) + tid / kObjLanes;
    if (line >= A.nlines) return;   // the whole 16-lane group leaves together
    const int64_t k0 = A.ptr[line], k1 = A.ptr[line + 1];
    const double yl = scal_lin<PREC>(A.ys, line);
    const double ylog = scal_log<PREC>(A.ys, line);
    const int d = D > 0 ? D : A.d;
    const double* xl = A.xl + line * d;
    if constexpr (D > 0) {
        double acc[D];
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = 0.0;
        for (int64_t e = k0 + sub; e < k1; e += kObjLanes) {
            const int64_t o = A.idx[e];
            double t = plan_entry<PREC>(yl, ylog, A.val, e, A.zs, o);
            double df[D];
#pragma unroll
            for (int k = 0; k < D; ++k) df[k] = xl[k] - A.xo[o * D + k];
            if (A.euclid) {
                double q = df[0] * df[0];
#pragma unroll
                for (int k = 1; k < D; ++k) q = q + df[k] * df[k];
                t = q > 0.0 ? t / sqrt(q) : 0.0;
            }
#pragma unroll
            for (int k = 0; k < D; ++k) acc[k] += t * df[k];
        }
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double g = group_sum<kObjLanes>(acc[k]);
            if (sub == 0) A.out[line * D + k] += A.coef * g;
        }
    } else {
        for (int k = 0; k < d; ++k) {
            double acc = 0.0;
            for (int64_t e = k0 + sub; e < k1; e += kObjLanes) {
                const int64_t o = A.idx[e];
                double t = plan_entry<PREC>(yl, ylog, A.val, e, A.zs, o);
                if (A.euclid) {
                    double q = 0.0;
                    for (int kk = 0; kk < d; ++kk) {
                        const double u = xl[kk] - A.xo[o * d + kk];
                        q = q + u * u;
                    }
                    t = q > 0.0 ? t / sqrt(q) : 0.0;
                }
                acc += t * (xl[k] - A.xo[o * d + k]);
            }
            const double g = group_sum<kObjLanes>(acc);
            if (sub == 0) A.out[line * d + k] += A.coef * g;
        }
    }
}

template <int D>
static void run_grad_d(int precision, const GradArgs& a, hipStream_t st) {
    const int nb = (int)((a.nlines + (kBlock / kObjLanes) - 1) / (kBlock / kObjLanes));
    if (precision == P_F64)
        hipLaunchKernelGGL((k_plan_grad<P_F64, D>), dim3(nb), dim3(kBlock), 0, st, a);
    else if (precision == P_F32)
        hipLaunchKernelGGL((k_plan_grad<P_F32, D>), dim3(nb), dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL((k_plan_grad<P_LOG, D>), dim3(nb), dim3(kBlock), 0, st, a);
}

hipError_t launch_plan_grad(int precision, const GradArgs& a, hipStream_t st) {
    if (a.nlines <= 0) return hipSuccess;
    switch (a.d) {
        case 2: run_grad_d<2>(precision, a, st); break;
        case 3: run_grad_d<3>(precision, a, st); break;
        case 10: run_grad_d<10>(precision, a, st); break;
        default: run_grad_d<0>(precision, a, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_objective(int precision, const ObjArgs& a, hipStream_t st) {
    if (a.nlines <= 0) return hipSuccess;
    switch (a.d) {
        case 2: run_obj_d<2>(precision, a, st); break;
        case 3: run_obj_d<3>(precision, a, st); break;
        case 10: run_obj_d<10>(precision, a, st); break;
        default: run_obj_d<0>(precision, a, st); break;
    }
    return hipGetLastError();
}

}  // namespace ss
