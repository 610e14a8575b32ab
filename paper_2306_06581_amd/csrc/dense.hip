// Dense Sinkhorn baseline (Alg. 1 / Alg. 2 on the full kernel) with
// K_ij = exp(-C_ij/eps) recomputed from the coordinates in every half-step;
// K is never stored.  Each half-step is two launches:
//   k_dense_partial: block = 256 lines x one column segment; the other side's
//                    coordinates and scaling are staged through LDS in tiles
//                    of 256 and every thread keeps R lines in registers.
//   k_dense_finish:  one thread per line sums its segment partials in order,
//                    applies the scaling update and the residual, and the
//                    next launch's block 0 closes the iteration.
// FP32 mode: FP32 coordinates (converted on load), one v_exp_f32 per entry.
// LOG mode: stabilised streaming log-sum-exp, FP64 potentials, FP32 exp.
// FP64 mode: everything FP64 (small problems, parity).
#include <math.h>

#include "common.hpp"
#include "internal.hpp"
#include "scaling.hpp"

namespace ss {

constexpr int kDenseTile = 256;

template <int PREC>
struct DenseT;
template <>
struct DenseT<P_F64> {
    typedef double C;  // coordinate / distance type
    static constexpr int R = 1;
};
template <>
struct DenseT<P_F32> {
    typedef float C;
    static constexpr int R = 2;
};
template <>
struct DenseT<P_LOG> {
    typedef float C;
    static constexpr int R = 2;
};

struct DensePartial {
    DenseArgs a;
    int nseg;
    int64_t seg_len;
    int64_t row_tiles;
    void* part;      // [nseg][nl]: float sums (F32), double sums (F64), double max (LOG)
    float* part_s;   // [nseg][nl]: LOG sums
};

template <int PREC, int D, bool WFR>
__global__ __launch_bounds__(256) void k_dense_partial(DensePartial P) {
    typedef typename DenseT<PREC>::C Cf;
    constexpr int R = DenseT<PREC>::R;
    constexpr int DD = D > 0 ? D : 16;
    const DenseArgs& A = P.a;
    if (loop_peek(A.st, A.role, A.stop_rule == 0, A.max_iter) == 0) return;
    __shared__ Cf ys[kDenseTile * DD];
    __shared__ double vs[kDenseTile];
    const int d = D > 0 ? D : A.d;
    const int tid = threadIdx.x;
    const int64_t rt = blockIdx.x % P.row_tiles, seg = blockIdx.x / P.row_tiles;
    const int64_t j0 = seg * P.seg_len;
    const int64_t j1 = (j0 + P.seg_len < A.no) ? j0 + P.seg_len : A.no;

    Cf xr[R][DD];
    int64_t lines[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        lines[r] = rt * (kBlock * R) + r * kBlock + tid;
        const int64_t li = lines[r] < A.nl ? lines[r] : 0;
#pragma unroll
        for (int k = 0; k < DD; ++k) xr[r][k] = (k < d) ? (Cf)A.xl[li * d + k] : (Cf)0;
    }
    double acc64[R];
    float acc32[R];
    double mx[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        acc64[r] = 0.0;
        acc32[r] = 0.0f;
        mx[r] = -INFINITY;
    }
    const double scale = A.scale;                       // inv_cmax / eps
    const float scale2 = (float)(A.scale * 1.4426950408889634);  // times log2(e)
    // WFR: log2 K = (2/eps) log2 cos(sqrt(c) w), K = 0 from sqrt(c) w = pi/2 on
    const float wf = (float)A.wfr_w;
    const float two_eps = (float)(2.0 / A.eps);
    const float two_eps_ln = (float)(2.0 / A.eps * 0.6931471805599453);

    for (int64_t jt = j0; jt < j1; jt += kDenseTile) {
        __syncthreads();
        const int64_t j = jt + tid;
        if (j < j1) {
#pragma unroll
            for (int k = 0; k < DD; ++k) ys[tid * DD + k] = (k < d) ? (Cf)A.xo[j * d + k] : (Cf)0;
            if (PREC == P_F64) vs[tid] = ((const double*)A.xin)[j];
            if (PREC == P_F32) vs[tid] = (double)((const float*)A.xin)[j];
            if (PREC == P_LOG) vs[tid] = ((const double*)A.xin)[j];
        }
        __syncthreads();
        const int cnt = (int)((j1 - jt) < kDenseTile ? (j1 - jt) : kDenseTile);
        for (int jj = 0; jj < cnt; ++jj) {
            const double vj = vs[jj];
            const float vjf = (float)vj;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                Cf c = 0;
                if (D > 0) {
#pragma unroll
                    for (int k = 0; k < DD; ++k) {
                        const Cf t = xr[r][k] - ys[jj * DD + k];
                        c = c + t * t;
                    }
                } else {
                    for (int k = 0; k < d; ++k) {
                        const Cf t = xr[r][k] - ys[jj * DD + k];
                        c = c + t * t;
                    }
                }
                if (PREC == P_F64) {
                    const double C = WFR ? cost_value((double)c, kCostWfr, 1.0, A.wfr_w)
                                         : (double)c * A.inv_cmax;
                    acc64[r] = acc64[r] + exp(-(C / A.eps)) * vj;
                } else if (PREC == P_F32) {
                    if (WFR) {
                        const float z = __fsqrt_rn((float)c) * wf;
                        const float k2 = z < (float)kHalfPi
                                             ? two_eps * __log2f(__cosf(z)) : -INFINITY;
                        acc32[r] = fmaf(__builtin_amdgcn_exp2f(k2), vjf, acc32[r]);
                    } else {
                        acc32[r] = fmaf(__builtin_amdgcn_exp2f(-(float)c * scale2), vjf, acc32[r]);
                    }
                } else {
                    if (WFR) {
                        const float zc = __fsqrt_rn((float)c) * wf;
                        if (!(zc < (float)kHalfPi)) continue;   // K = 0: no term
                        const double lk = (double)(two_eps_ln * __log2f(__cosf(zc)));
                        const double z = vj + lk;
                        const double dz = z - mx[r];
                        const float e = __expf(-(float)fabs(dz));
                        if (dz > 0.0) {
                            acc32[r] = acc32[r] * e + 1.0f;
                            mx[r] = z;
                        } else {
                            acc32[r] += e;
                        }
                        continue;
                    }
                    const double z = vj - (double)c * scale;
                    const double dz = z - mx[r];
                    const float e = __expf(-(float)fabs(dz));
                    if (dz > 0.0) {
                        acc32[r] = acc32[r] * e + 1.0f;
                        mx[r] = z;
                    } else {
                        acc32[r] += e;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (lines[r] >= A.nl) continue;
        const int64_t o = seg * A.nl + lines[r];
        if (PREC == P_F64) ((double*)P.part)[o] = acc64[r];
        if (PREC == P_F32) ((float*)P.part)[o] = acc32[r];
        if (PREC == P_LOG) {
            ((double*)P.part)[o] = mx[r];
            P.part_s[o] = acc32[r];
        }
    }
}

template <int PREC, bool UOT>
__global__ __launch_bounds__(256) void k_dense_finish(DensePartial P) {
    __shared__ double sh[4];
    const DenseArgs& A = P.a;
    const int marginal = A.stop_rule == 0;
    const int t = loop_enter(A.st, A.role, marginal, A.max_iter, A.tol, A.prev_partials,
                             A.prev_nblocks, A.err_hist);
    if (t == 0) return;
    const int64_t line = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double res = 0.0;
    if (line < A.nl) {
        double w;
        if (PREC == P_F64) {
            w = 0.0;
            for (int s = 0; s < P.nseg; ++s) w += ((const double*)P.part)[s * A.nl + line];
        } else if (PREC == P_F32) {
            float wf = 0.0f;
            for (int s = 0; s < P.nseg; ++s) wf += ((const float*)P.part)[s * A.nl + line];
            w = (double)wf;
        } else {
            double M = -INFINITY;
            for (int s = 0; s < P.nseg; ++s) M = fmax(M, ((const double*)P.part)[s * A.nl + line]);
            float S = 0.0f;
            for (int s = 0; s < P.nseg; ++s) {
                const double ms = ((const double*)P.part)[s * A.nl + line];
                if (ms != -INFINITY) S += P.part_s[s * A.nl + line] * __expf((float)(ms - M));
            }
            w = (M == -INFINITY || !(S > 0.0f)) ? -INFINITY : M + log((double)S);
        }
        const double yp = PREC == P_F32 ? (double)((const float*)A.yprev)[line]
                                        : ((const double*)A.yprev)[line];
        const double mg = A.marg[line];
        const LineNew o = line_new<PREC, UOT>(A.role, marginal, t, A.no > 0, mg,
                                              PREC == P_LOG ? log(mg) : 0.0, A.theta, yp, w);
        line_store<PREC>(A.yout, nullptr, line, o.y, A.st);
        res = o.res;
    }
    const double bsum = block_sum256(res, sh);
    if (threadIdx.x == 0) A.partials[blockIdx.x] = bsum;
}

int dense_blocks(int64_t nlines) { return (int)((nlines + kBlock - 1) / kBlock); }

static void dense_shape(int R, int64_t nl, int64_t no, int64_t* row_tiles, int* nseg,
                        int64_t* seg_len) {
    *row_tiles = (nl + kBlock * R - 1) / (kBlock * R);
    const int64_t col_tiles = (no + kDenseTile - 1) / kDenseTile;
    int64_t s = (2048 + *row_tiles - 1) / *row_tiles;
    if (s > col_tiles) s = col_tiles;
    if (s > 64) s = 64;
    if (s < 1) s = 1;
    *seg_len = ((col_tiles + s - 1) / s) * kDenseTile;
    *nseg = (int)((no + *seg_len - 1) / *seg_len);
    if (*nseg < 1) *nseg = 1;
}

// Scratch needed by one half-step (bytes), for workspace sizing.
size_t dense_partial_bytes(int64_t nl, int64_t no) {
    int64_t rt;
    int ns;
    int64_t sl;
    dense_shape(1, nl, no, &rt, &ns, &sl);
    int ns2;
    dense_shape(2, nl, no, &rt, &ns2, &sl);
    if (ns2 > ns) ns = ns2;
    return (size_t)ns * (size_t)nl * (8 + 4);
}

template <int PREC, int D>
static void run_dense(const DenseArgs& a, void* part, hipStream_t st) {
    DensePartial P;
    P.a = a;
    dense_shape(DenseT<PREC>::R, a.nl, a.no, &P.row_tiles, &P.nseg, &P.seg_len);
    P.part = part;
    P.part_s = (float*)((char*)part + (size_t)P.nseg * a.nl * 8);
    if (a.cost == kCostWfr)
        hipLaunchKernelGGL((k_dense_partial<PREC, D, true>), dim3((unsigned)(P.row_tiles * P.nseg)),
                           dim3(kBlock), 0, st, P);
    else
        hipLaunchKernelGGL((k_dense_partial<PREC, D, false>), dim3((unsigned)(P.row_tiles * P.nseg)),
                           dim3(kBlock), 0, st, P);
    if (a.theta != 1.0)
        hipLaunchKernelGGL((k_dense_finish<PREC, true>), dim3(dense_blocks(a.nl)), dim3(kBlock), 0,
                           st, P);
    else
        hipLaunchKernelGGL((k_dense_finish<PREC, false>), dim3(dense_blocks(a.nl)), dim3(kBlock), 0,
                           st, P);
}

template <int D>
static void run_dense_d(int precision, const DenseArgs& a, void* part, hipStream_t st) {
    if (precision == P_F64)
        run_dense<P_F64, D>(a, part, st);
    else if (precision == P_F32)
        run_dense<P_F32, D>(a, part, st);
    else
        run_dense<P_LOG, D>(a, part, st);
}

hipError_t launch_dense_half(int precision, const DenseArgs& a, void* part, hipStream_t st) {
    if (a.d > 16) return hipErrorInvalidValue;
    switch (a.d) {
        case 2: run_dense_d<2>(precision, a, part, st); break;
        case 3: run_dense_d<3>(precision, a, part, st); break;
        case 10: run_dense_d<10>(precision, a, part, st); break;
        default: run_dense_d<0>(precision, a, part, st); break;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ objective
// Row pass (role 0): per (row, column segment) partial sums of T C,
// T (log T - 1), T (log u + log v - 1) and T; column pass (role 1): T only.
struct DenseObj {
    DenseObjArgs a;
    int role;
    const double* xl;
    const double* xo;
    int64_t nl, no;
    const void* yl;    // line scaling
    const void* yo;    // other scaling
    int nseg;
    int64_t seg_len, row_tiles;
    double* linepart;  // [nseg][nl]
    double* bpart;     // [3][row_tiles * nseg]
};

template <int PREC>
__device__ __forceinline__ double lin_of(const void* p, int64_t i) {
    if (PREC == P_F64) return ((const double*)p)[i];
    if (PREC == P_F32) return (double)((const float*)p)[i];
    return exp(((const double*)p)[i]);
}
template <int PREC>
__device__ __forceinline__ double log_of(const void* p, int64_t i) {
    if (PREC == P_LOG) return ((const double*)p)[i];
    return log(lin_of<PREC>(p, i));
}

template <int PREC, int D>
__global__ __launch_bounds__(256) void k_dense_obj_partial(DenseObj O) {
    __shared__ double sh[4];
    const DenseObjArgs& A = O.a;
    const int d = D > 0 ? D : A.d;
    const int64_t rt = blockIdx.x % O.row_tiles, seg = blockIdx.x / O.row_tiles;
    const int64_t line = rt * kBlock + threadIdx.x;
    const int64_t j0 = seg * O.seg_len;
    const int64_t j1 = (j0 + O.seg_len < O.no) ? j0 + O.seg_len : O.no;
    double s_tc = 0.0, s_ent = 0.0, s_sp = 0.0, s_l = 0.0;
    if (line < O.nl) {
        const double* xi = O.xl + line * d;
        const double ul = lin_of<PREC>(O.yl, line);
        const double lul = log_of<PREC>(O.yl, line);
        for (int64_t j = j0; j < j1; ++j) {
            // entry (i, j) with i the row: distances always as |x_i - y_j|^2
            const double c = O.role == 0 ? sqdist<D>(xi, O.xo + j * d, d)
                                         : sqdist<D>(O.xo + j * d, xi, d);
            const double C = cost_value(c, A.cost, A.inv_cmax, A.wfr_w);
            const double lk = -(C / A.eps);
            double t;
            if (PREC == P_LOG)
                t = exp(lul + lk + log_of<PREC>(O.yo, j));
            else
                t = ul * exp(lk) * lin_of<PREC>(O.yo, j);
            s_l += t;
            if (O.role == 0 && t > 0.0) {
                s_tc += t * C;
                s_ent += t * (log(t) - 1.0);
                s_sp += t * ((lul + log_of<PREC>(O.yo, j)) - 1.0);
            }
        }
        O.linepart[seg * O.nl + line] = s_l;
    }
    const double q[3] = {s_tc, s_ent, s_sp};
    const unsigned nb = gridDim.x;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double tot = block_sum256(q[r], sh);
        if (threadIdx.x == 0) O.bpart[(int64_t)r * nb + blockIdx.x] = tot;
    }
}

__global__ __launch_bounds__(256) void k_dense_obj_finish(DenseObj O, unsigned nbpart) {
    __shared__ double sh[4];
    const DenseObjArgs& A = O.a;
    const int64_t line = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double kl = 0.0, tot_l = 0.0;
    if (line < O.nl) {
        double L = 0.0;
        for (int s = 0; s < O.nseg; ++s) L += O.linepart[s * O.nl + line];
        const double m = O.role == 0 ? A.a[line] : A.b[line];
        if (A.uot) kl = (L > 0.0 ? L * log(L / m) : 0.0) - L + m;
        tot_l = L;
    }
    const double bk = block_sum256(kl, sh);
    const double bl = block_sum256(tot_l, sh);
    if (threadIdx.x == 0) {
        A.partials[blockIdx.x] = bk;
        A.partials[gridDim.x + blockIdx.x] = bl;
    }
}

template <int PREC, int D>
static void run_dense_obj(const DenseObjArgs& a, hipStream_t st) {
    for (int role = 0; role < 2; ++role) {
        DenseObj O;
        O.a = a;
        O.role = role;
        O.xl = role == 0 ? a.x : a.y;
        O.xo = role == 0 ? a.y : a.x;
        O.nl = role == 0 ? a.n : a.m;
        O.no = role == 0 ? a.m : a.n;
        O.yl = role == 0 ? a.u : a.v;
        O.yo = role == 0 ? a.v : a.u;
        dense_shape(1, O.nl, O.no, &O.row_tiles, &O.nseg, &O.seg_len);
        O.linepart = role == 0 ? a.rowsum : a.colsum;
        O.bpart = a.partials + 2 * dense_blocks(O.nl) + 8;
        const unsigned nbp = (unsigned)(O.row_tiles * O.nseg);
        hipLaunchKernelGGL((k_dense_obj_partial<PREC, D>), dim3(nbp), dim3(kBlock), 0, st, O);
        const unsigned nbl = (unsigned)dense_blocks(O.nl);
        hipLaunchKernelGGL(k_dense_obj_finish, dim3(nbl), dim3(kBlock), 0, st, O, nbp);
        // line-level sums (KL, mass) then the per-entry sums of the partial pass
        ReduceSpec r;
        r.nq = role == 0 ? 5 : 2;
        r.src[0] = a.partials;
        r.len[0] = nbl;
        r.slot[0] = role == 0 ? ST_KL_A : ST_KL_B;
        r.src[1] = a.partials + nbl;
        r.len[1] = nbl;
        r.slot[1] = role == 0 ? ST_ROWSUM : ST_COLSUM;
        for (int q = 0; q < 3; ++q) {
            r.src[2 + q] = O.bpart + (int64_t)q * nbp;
            r.len[2 + q] = nbp;
        }
        r.slot[2] = ST_TRANSPORT;
        r.slot[3] = ST_NEGENT;
        r.slot[4] = ST_SPARSEOBJ;
        (void)launch_reduce_stats(r, a.stats, st);
    }
}

template <int D>
static void run_dense_obj_d(const DenseObjArgs& a, hipStream_t st) {
    if (a.precision == P_F64)
        run_dense_obj<P_F64, D>(a, st);
    else if (a.precision == P_F32)
        run_dense_obj<P_F32, D>(a, st);
    else
        run_dense_obj<P_LOG, D>(a, st);
}

hipError_t launch_dense_objective(const DenseObjArgs& a, hipStream_t st) {
    switch (a.d) {
        case 2: run_dense_obj_d<2>(a, st); break;
        case 3: run_dense_obj_d<3>(a, st); break;
        case 10: run_dense_obj_d<10>(a, st); break;
        default: run_dense_obj_d<0>(a, st); break;
    }
    return hipGetLastError();
}

}  // namespace ss
