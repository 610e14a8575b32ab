// Sinkhorn scaling loop on the sparse sketch (Alg. 1 / Alg. 2 applied to K~).
//
// One kernel serves both half-steps: for every line r of a sparse matrix M
// (the CSR of K~ for the u-update, the CSC for the v-update) it forms
// w_r = sum_k M_rk x_k, writes the new scaling y_r = marg_r / w_r (OT) or
// (marg_r / w_r)^theta (UOT, theta = lam/(lam+eps)), and adds its residual
// term.  The matrix entries stream once from HBM; the gathered vector is read
// through LDS (see k_iterate).  The residual is reduced per block in a fixed
// tree; block 0 of the next launch sums the block partials in index order and
// takes the stop decision, so the stop test is deterministic and the loop has
// no atomics or device-wide fences.
//
// Log-domain variant (appendix, proof of Thm. 3): the matrix stores
// l_rk = log K~_rk in FP32, the vectors hold FP64 potentials f = log u,
// g = log v, and w_r becomes a stabilised streaming log-sum-exp.
#include <math.h>

#include <type_traits>

#include "common.hpp"
#include "internal.hpp"
#include "scaling.hpp"

namespace ss {

// Sparse product with the gathered vector swept through LDS.
//
// Random 4- or 8-byte gathers from a vector of 10^4..10^6 entries miss the L1
// and each pulls a whole cache line from L2, which (not HBM) bounds a plain CSR
// product at these densities.  Here the gathered vector is read in slices of
// SLB bytes staged in LDS (coalesced 16-byte loads), and a line's entries are
// cut at the slice boundaries into segments (split points computed once per
// solve by k_split; entries are column-sorted within a line, so each segment
// is contiguous).  A block takes R consecutive lines and hands out lanes per
// (slice, line) segment, slice-major: ceil(quads / J) lanes each, so the wave's
// quad loads cover contiguous stretches of the entry arrays.  Every lane loads
// its J quads of values and indices into registers (all loads in flight at
// once), the block stages the slices its lanes need, one after the other, and
// while slice s is resident the lanes of slice-s segments add their terms.
// Per-lane partials are folded per line in (slice, lane) order through LDS;
// when the segments need more than BS lanes the block makes several passes.
// Every sum has a fixed order, so results are deterministic.
template <int PREC>
struct IterCfg {
    static constexpr int J = PREC == P_F64 ? 3 : 7;  // quads per lane per pass
    static constexpr int E = 4 * J;                  // entries per lane per pass
};

template <int BS>
struct SliceCfg {
    static constexpr int bytes = BS == 1024 ? 131072 : 32768;
};

constexpr int kMaxPairs = 2048;  // (slice, line) segments per block step
static_assert(SliceCfg<1024>::bytes / 4 <= 32768 && SliceCfg<256>::bytes / 4 <= 32768,
              "slice offsets and their sentinel must fit in 16 bits");

int slice_elems(int precision, int block) {
    const int bytes = block == 1024 ? SliceCfg<1024>::bytes : SliceCfg<256>::bytes;
    return bytes / (precision == P_F32 ? 4 : 8);
}

int iterate_slices(int precision, int block, int64_t nx) {
    const int64_t sl = slice_elems(precision, block);
    return (int)((nx + sl - 1) / sl);
}

// Lines per block step: a quarter of the threads, fewer when the lines have
// many slices (at most kMaxPairs segments per step).  0 when even one line
// has more than kMaxPairs slices: the gathered vector is too long.
int iterate_lines_per_step(int precision, int block, int64_t nx) {
    const int64_t ns = (nx + slice_elems(precision, block) - 1) / slice_elems(precision, block);
    if (ns > kMaxPairs) return 0;
    int r = block / 4;
    while (r > 1 && (int64_t)r * ns > kMaxPairs) r >>= 1;
    return r;
}

// split[line * (ns + 1) + s] = offset (from the line start) of the line's
// first entry with index >= s * SL; s = 0..ns.  Binary search per boundary.
__global__ void k_split(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                        int64_t nlines, int ns, int64_t SL, int32_t* __restrict__ split) {
    const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (line >= nlines) return;
    const int64_t k0 = ptr[line], k1 = ptr[line + 1];
    int32_t* out = split + line * (ns + 1);
    out[0] = 0;
    for (int s = 1; s < ns; ++s) {
        const int64_t bound = (int64_t)s * SL;
        int64_t lo = k0, hi = k1;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)idx[mid] < bound)
                lo = mid + 1;
            else
                hi = mid;
        }
        out[s] = (int32_t)(lo - k0);
    }
    out[ns] = (int32_t)(k1 - k0);
}

hipError_t launch_split(const int64_t* ptr, const int32_t* idx, int64_t nlines, int ns,
                        int64_t slice, int32_t* split, hipStream_t st) {
    if (nlines <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_split, dim3((unsigned)((nlines + 255) / 256)), dim3(256), 0, st, ptr, idx,
                       nlines, ns, slice, split);
    return hipGetLastError();
}

template <typename V>
__device__ __forceinline__ void load_quad(const V* p, V* out);
template <>
__device__ __forceinline__ void load_quad<float>(const float* p, float* out) {
    const float4 q = *(const float4*)p;
    out[0] = q.x;
    out[1] = q.y;
    out[2] = q.z;
    out[3] = q.w;
}
template <>
__device__ __forceinline__ void load_quad<double>(const double* p, double* out) {
    const double2 a = *(const double2*)p;
    const double2 b = *(const double2*)(p + 2);
    out[0] = a.x;
    out[1] = a.y;
    out[2] = b.x;
    out[3] = b.y;
}

// xs[0 .. SL) = x[base .. base + SL) (zero past nx), 16 bytes per load.
template <typename Y, int BS, int SL>
__device__ __forceinline__ void stage_slice(Y* xs, const Y* __restrict__ x, int64_t base,
                                            int64_t nx) {
    constexpr int K = 16 / (int)sizeof(Y);  // elements per 16-byte load
    constexpr int NV = SL / K;
#pragma unroll 4
    for (int i = threadIdx.x; i < NV; i += BS) {
        const int64_t g = base + (int64_t)i * K;
        if (g + K <= nx) {
            *(float4*)(xs + i * K) = *(const float4*)(x + g);
        } else {
#pragma unroll
            for (int u = 0; u < K; ++u) xs[i * K + u] = g + u < nx ? x[g + u] : (Y)0;
        }
    }
}

// log-sum-exp pair (m, s) meaning m + log(s): merge b into a.
__device__ __forceinline__ void lse_merge(double& m, float& s, double mb, float sb) {
    if (mb == -INFINITY) return;
    if (m == -INFINITY) {
        m = mb;
        s = sb;
        return;
    }
    if (mb > m) {
        s = s * __expf((float)(m - mb)) + sb;
        m = mb;
    } else {
        s += sb * __expf((float)(mb - m));
    }
}

// Last index p in [0, n) with a[p] <= key (a nondecreasing, a[0] <= key).
__device__ __forceinline__ int last_le(const int* a, int n, int key) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid] <= key)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <int PREC, int BS, bool UOT>
__global__ __launch_bounds__(BS) void k_iterate(IterArgs A) {
    typedef typename Scal<PREC>::V V;
    typedef typename Scal<PREC>::Y Y;
    typedef typename std::conditional<PREC == P_F32, float, double>::type T;
    constexpr int J = IterCfg<PREC>::J;
    constexpr int E = IterCfg<PREC>::E;
    constexpr int SL = SliceCfg<BS>::bytes / (int)sizeof(Y);
    constexpr int RMAX = BS / 4;
    extern __shared__ __align__(16) unsigned char dsm[];
    Y* xs = (Y*)dsm;
    __shared__ int lstart[kMaxPairs + 1];  // first lane of each (slice, line) segment
    __shared__ int64_t lbase[RMAX];        // first entry of each line of the step
    __shared__ union {
        T acc[BS];
        struct {
            double m[BS];
            float s[BS];
        } lse;
    } part;                                // per-lane partials of the current pass
    __shared__ T racc[RMAX];               // per-line accumulation over passes
    __shared__ double rm[RMAX];
    __shared__ float rs[RMAX];
    __shared__ int wsum[BS / kWave];
    __shared__ double sh[16];
    IterState* st = A.st;
    const int marginal = A.stop_rule == 0;
    const int t = loop_enter(st, A.role, marginal, A.max_iter, A.tol, A.prev_partials,
                             A.prev_nblocks, A.err_hist);
    if (t == 0) return;

    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const V* __restrict__ val = (const V*)A.val;
    const int32_t* __restrict__ idx = A.idx;
    const Y* __restrict__ xin = (const Y*)A.xin;
    const int ns = A.nslices;
    const int R = A.lines_per_step;
    const int P = ns * R;                      // segments of a step, slice-major
    const int per = (P + BS - 1) / BS;         // segments per thread for the scan
    const int64_t nrb = (A.nlines + R - 1) / R;
    double res = 0.0;
    for (int64_t rb = blockIdx.x; rb < nrb; rb += gridDim.x) {
        const int64_t r0 = rb * R;
        __syncthreads();  // LDS of the previous step is free
        if (tid < R) {
            const int64_t line = r0 + tid;
            lbase[tid] = line < A.nlines ? A.ptr[line] : 0;
            racc[tid] = 0;
            rm[tid] = -INFINITY;
            rs[tid] = 0.0f;
        }
        __syncthreads();
        // ---- lanes per segment: ceil(quads / J); thread tid scans segments
        //      [tid * per, tid * per + per) then a block-wide exclusive scan
        constexpr int KMAX = kMaxPairs / 256;  // per <= kMaxPairs / BS
        int cnt[KMAX];
        int mine = 0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int p = tid * per + k;
            int lanes = 0;
            if (k < per && p < P) {
                const int s = p / R, i = p - s * R;
                const int64_t line = r0 + i;
                if (line < A.nlines) {
                    const int32_t* sp = A.split + line * (ns + 1);
                    const int64_t k0 = lbase[i] + sp[s], k1 = lbase[i] + sp[s + 1];
                    const int64_t a0 = k0 & ~(int64_t)3;
                    const int nq = k1 > k0 ? (int)((k1 - a0 + 3) >> 2) : 0;
                    lanes = (nq + J - 1) / J;
                }
            }
            cnt[k] = lanes;
            mine += lanes;
        }
        const int incl = wave_inclusive_scan(mine);
        if (lane == kWave - 1) wsum[tid / kWave] = incl;
        __syncthreads();
        {
            int off = 0;
            for (int w = 0; w < tid / kWave; ++w) off += wsum[w];
            int run = off + incl - mine;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const int p = tid * per + k;
                if (k < per && p < P) lstart[p] = run;
                run += cnt[k];
            }
            if (tid == BS - 1) lstart[P] = run;
        }
        __syncthreads();
        const int total = lstart[P];
        const int npass = (total + BS - 1) / BS;
        for (int pass = 0; pass < npass; ++pass) {
            const int L = pass * BS + tid;
            const bool active = L < total;
            const int p = last_le(lstart, P, active ? L : total - 1);
            const int s = p / R, i = p - s * R;
            const int64_t line = r0 + i;
            // slices touched by this pass: from the first to the last lane's
            const int s_lo = last_le(lstart, P, pass * BS) / R;
            const int s_hi = last_le(lstart, P, (pass + 1) * BS < total ? (pass + 1) * BS - 1
                                                                        : total - 1) / R;
            // ---- this lane's quads of its segment
            int64_t k0 = 0, k1 = 0;
            if (active) {
                const int32_t* sp = A.split + line * (ns + 1);
                k0 = lbase[i] + sp[s];
                k1 = lbase[i] + sp[s + 1];
            }
            const int64_t a0 = k0 & ~(int64_t)3;
            const int64_t nq = k1 > k0 ? (k1 - a0 + 3) >> 2 : 0;
            const int sidx = L - lstart[p];             // lane index within the segment
            const int nl = lstart[p + 1] - lstart[p];   // lanes of the segment
            V v[E];
            // position of each entry in the lane's slice, two 16-bit halves per
            // word (SL <= 32768); SL marks a discarded entry
            uint32_t offp[E / 2];
            // Loads are never predicated: the quad index is clamped into the
            // segment (an empty range reads the quad at its offset, which lies
            // in the padded entry arrays) and entries outside [k0, k1) get the
            // offset SL, which the slice test discards.
            const uint32_t lo = (uint32_t)(k0 - a0), span = (uint32_t)(k1 - k0);
            const int64_t qmax = nq > 0 ? nq - 1 : 0;
            const int32_t sbase = s * SL;
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int64_t qd = (int64_t)sidx + (int64_t)j * nl;
                const int64_t qq = qd < qmax ? qd : qmax;
                load_quad<V>(val + a0 + 4 * qq, v + 4 * j);
                const int4 ci = *(const int4*)(idx + a0 + 4 * qq);
                const uint32_t rel = (uint32_t)(4 * qd) - lo;  // position within the segment
                const uint32_t o0 = rel + 0 < span ? (uint32_t)(ci.x - sbase) : SL;
                const uint32_t o1 = rel + 1 < span ? (uint32_t)(ci.y - sbase) : SL;
                const uint32_t o2 = rel + 2 < span ? (uint32_t)(ci.z - sbase) : SL;
                const uint32_t o3 = rel + 3 < span ? (uint32_t)(ci.w - sbase) : SL;
                offp[2 * j + 0] = o0 | (o1 << 16);
                offp[2 * j + 1] = o2 | (o3 << 16);
            }
            T acc = 0;
            double mx = -INFINITY;  // log domain: running max and sum of exp(z - mx)
            float ls = 0.0f;
            for (int sl = s_lo; sl <= s_hi; ++sl) {
                __syncthreads();  // the previous slice is no longer read
                stage_slice<Y, BS, SL>(xs, xin, (int64_t)sl * SL, A.nx);
                __syncthreads();
                if (active && s == sl) {
#pragma unroll
                    for (int g = 0; g < E; g += 4) {
                        Y xv[4];
                        bool in[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            // opaque copies keep the compiler from hoisting the
                            // tests and conversions out of the slice loop (that
                            // would hold E more registers across it)
                            uint32_t w = offp[(g + u) >> 1];
                            asm volatile("" : "+v"(w));
                            const uint32_t o = (u & 1) ? w >> 16 : w & 0xFFFFu;
                            in[u] = o < (uint32_t)SL;
                            xv[u] = xs[in[u] ? o : 0];
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if constexpr (PREC == P_LOG) {
                                // streaming log-sum-exp without branches: one
                                // exp of -|z - mx| rescales the sum or the term
                                float vf = v[g + u];
                                asm volatile("" : "+v"(vf));
                                const double z = (double)vf + xv[u];
                                const double dz = in[u] ? z - mx : -INFINITY;
                                const float e = __expf(-(float)fabs(dz));
                                const bool up = dz > 0.0;
                                ls = up ? fmaf(ls, e, 1.0f) : (in[u] ? ls + e : ls);
                                mx = up ? z : mx;
                            } else {
                                acc = fma(v[g + u], in[u] ? xv[u] : (Y)0, acc);
                            }
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
            // ---- fold the lane partials of every line, in (slice, lane) order
            if constexpr (PREC == P_LOG) {
                part.lse.m[tid] = mx;
                part.lse.s[tid] = ls;
            } else {
                part.acc[tid] = acc;
            }
            __syncthreads();
            if (tid < R) {
                T a = racc[tid];
                double m = rm[tid];
                float sum = rs[tid];
                for (int ss = 0; ss < ns; ++ss) {
                    const int q = ss * R + tid;
                    const int b = lstart[q] > pass * BS ? lstart[q] : pass * BS;
                    const int e = lstart[q + 1] < (pass + 1) * BS ? lstart[q + 1] : (pass + 1) * BS;
                    for (int l = b; l < e; ++l) {
                        if constexpr (PREC == P_LOG)
                            lse_merge(m, sum, part.lse.m[l - pass * BS], part.lse.s[l - pass * BS]);
                        else
                            a += part.acc[l - pass * BS];
                    }
                }
                racc[tid] = a;
                rm[tid] = m;
                rs[tid] = sum;
            }
            __syncthreads();
        }
        // ---- scaling update of every line of the step
        if (tid < R && r0 + tid < A.nlines) {
            const int64_t line = r0 + tid;
            const bool nonempty = A.ptr[line + 1] > lbase[tid];
            double w;
            if constexpr (PREC == P_LOG)
                w = (rm[tid] == -INFINITY || !(rs[tid] > 0.0f)) ? -INFINITY
                                                                : rm[tid] + log((double)rs[tid]);
            else
                w = (double)racc[tid];
            res += line_update<PREC, UOT>(A.role, marginal, t, nonempty, A.marg[line], A.theta,
                                          (double)((const Y*)A.yprev)[line], A.yout, line, w, st);
        }
    }
    const double bsum = block_sum(res, sh);
    if (tid == 0) A.partials[blockIdx.x] = bsum;
}

template <int PREC, int BS>
static hipError_t run_iter(const IterArgs& a, hipStream_t st) {
    const int nb = iterate_blocks(a.nlines, a.lines_per_step);
    const size_t lds = SliceCfg<BS>::bytes;
    if (a.theta != 1.0)
        hipLaunchKernelGGL((k_iterate<PREC, BS, true>), dim3(nb), dim3(BS), lds, st, a);
    else
        hipLaunchKernelGGL((k_iterate<PREC, BS, false>), dim3(nb), dim3(BS), lds, st, a);
    return hipGetLastError();
}

template <int PREC, int BS, bool UOT>
static hipError_t allow_lds() {
    return hipFuncSetAttribute((const void*)&k_iterate<PREC, BS, UOT>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, SliceCfg<BS>::bytes);
}

// Raises the dynamic LDS limit of every instantiation (once, before any
// launch or graph capture).
hipError_t iterate_init() {
    static hipError_t status = [] {
        hipError_t e = hipSuccess;
        const hipError_t r[] = {allow_lds<P_F64, 1024, false>(), allow_lds<P_F64, 1024, true>(),
                                allow_lds<P_F32, 1024, false>(), allow_lds<P_F32, 1024, true>(),
                                allow_lds<P_LOG, 1024, false>(), allow_lds<P_LOG, 1024, true>(),
                                allow_lds<P_F64, 256, false>(),  allow_lds<P_F64, 256, true>(),
                                allow_lds<P_F32, 256, false>(),  allow_lds<P_F32, 256, true>(),
                                allow_lds<P_LOG, 256, false>(),  allow_lds<P_LOG, 256, true>()};
        for (hipError_t x : r)
            if (x != hipSuccess) e = x;
        return e;
    }();
    return status;
}

// Block size: 1024 threads (256 lines, 128 KB slices) when there are enough
// lines for a block per compute unit, else 256 threads (64 lines, 32 KB).
int iterate_block_size(int64_t nlines) { return nlines >= 256 * 256 ? 1024 : 256; }

int iterate_blocks(int64_t nlines, int lines_per_step) {
    const int64_t per = lines_per_step;
    const int64_t nb = (nlines + per - 1) / per;
    return (int)(nb < kMaxLoopBlocks ? nb : kMaxLoopBlocks);
}

hipError_t launch_iterate(int precision, int block, const IterArgs& a, hipStream_t st) {
    if (precision == P_F64) return block == 1024 ? run_iter<P_F64, 1024>(a, st) : run_iter<P_F64, 256>(a, st);
    if (precision == P_F32) return block == 1024 ? run_iter<P_F32, 1024>(a, st) : run_iter<P_F32, 256>(a, st);
    return block == 1024 ? run_iter<P_LOG, 1024>(a, st) : run_iter<P_LOG, 256>(a, st);
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
