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
// SL elements copied into LDS by direct global-to-LDS loads, and each line's
// entries are cut at the slice boundaries into segments (entries are
// column-sorted within a line, so every segment is contiguous).
//
// Lane plan (built once per solve by build_plan):
//  * a segment of c entries gets ceil(c / E) lanes of E entry slots;
//  * lines are grouped into steps of consecutive lines whose lanes fit one
//    block (line weights are scanned and cut every T; the number of steps is
//    a multiple of the resident blocks, so the persistent grid is balanced);
//  * inside a step the segments are ordered slice-major, so the lanes of one
//    slice are contiguous, and the lanes are cut into passes of BS;
//  * the entries are repacked so that quad j of the lanes of one pass is
//    contiguous: a wave's load instruction reads one unbroken run of memory.
//    The column index is stored as its 16-bit offset inside the slice; empty
//    slots hold the offset SL, which no test accepts;
//  * per step the first lane of every segment (lst) and per lane its segment
//    (lseg) are stored, so the kernel needs no scan or search to start.
//
// Iteration kernel: a block takes a step, starts the copy of the first slice
// into LDS, loads every lane's E values and offsets into registers, and while
// slice s is resident the lanes of slice-s segments add their terms.  Per-lane
// partials are folded per line in (slice, lane) order through LDS, so every
// sum has a fixed order and the results are deterministic.
template <int PREC>
struct IterCfg {
    static constexpr int J = PREC == P_F64 ? 3 : 9;   // quads per lane
    static constexpr int E = 4 * J;                   // entry slots per lane
};

template <int BS>
struct SliceCfg {
    static constexpr int bytes = BS == 1024 ? 131072 : 32768;
    static constexpr int lines = BS / 2;  // most lines a step may hold
};

constexpr int kMaxPairs = 2048;  // (slice, line) segments per step
static_assert(SliceCfg<1024>::bytes / 4 <= 32768 && SliceCfg<256>::bytes / 4 <= 32768,
              "slice offsets and their sentinel must fit in 16 bits");

int entries_per_lane(int precision) {
    return precision == P_F64 ? IterCfg<P_F64>::E : IterCfg<P_F32>::E;
}

int slice_elems(int precision, int block) {
    const int bytes = block == 1024 ? SliceCfg<1024>::bytes : SliceCfg<256>::bytes;
    return bytes / (precision == P_F64 ? 8 : 4);
}

int iterate_slices(int precision, int block, int64_t nx) {
    const int64_t sl = slice_elems(precision, block);
    return (int)((nx + sl - 1) / sl);
}

// Smallest line weight: keeps the lines of a step <= BS / 2 and the segments
// of a step <= kMaxPairs (a step holds at most ceil(BS / minw) lines).
static int min_weight(int block, int ns) {
    int w = 2;
    while ((int64_t)((block + w - 1) / w) * ns > kMaxPairs) ++w;
    return w;
}

bool plan_shape(int precision, int block, int64_t nlines, int64_t nx, int64_t cap, IterPlan* p) {
    const int64_t ns = (nx + slice_elems(precision, block) - 1) / slice_elems(precision, block);
    if (ns > kMaxPairs) return false;
    p->block = block;
    p->ns = (int)ns;
    p->slice = slice_elems(precision, block);
    const int E = entries_per_lane(precision);
    // lanes = sum over segments of ceil(c / E) <= cap / E + nonempty segments
    const int64_t segs = cap < nlines * ns ? cap : nlines * ns;
    p->lanes_max = cap / E + segs + 1;
    // steps: K <= W / Tcap + resident blocks, W <= lanes + nlines * minw,
    // Tcap >= BS / 2
    const int64_t W = p->lanes_max + nlines * (int64_t)min_weight(block, (int)ns);
    p->kmax = W / (block / 2) + kMaxLoopBlocks + 2;
    return true;
}

size_t plan_value_bytes(int precision, const IterPlan& p) {
    return (size_t)p.lanes_max * entries_per_lane(precision) * (precision == P_F64 ? 8 : 4);
}

size_t plan_offset_bytes(int precision, const IterPlan& p) {
    return (size_t)p.lanes_max * entries_per_lane(precision) * 2;
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

// Lanes of every line and its step weight max(lanes, minw); largest weight.
__global__ void k_plan_lanes(const int32_t* __restrict__ split, int64_t nlines, int ns, int E,
                             int minw, int32_t* __restrict__ lanes, int32_t* __restrict__ weight,
                             PlanInfo* info) {
    const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int w = 0;
    if (line < nlines) {
        const int32_t* sp = split + line * (ns + 1);
        int l = 0;
        for (int s = 0; s < ns; ++s) l += (sp[s + 1] - sp[s] + E - 1) / E;
        lanes[line] = l;
        w = l > minw ? l : minw;
        weight[line] = w;
    }
    w = group_max<kWave>(w);
    if ((threadIdx.x & (kWave - 1)) == 0 && w > 0) atomicMax(&info->maxw, w);
}

// Step weight T and step count K (one thread).
__global__ void k_plan_setup(const int64_t* __restrict__ wptr, int64_t nlines, int block,
                             int64_t resident, int64_t kmax, PlanInfo* info) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t W = wptr[nlines];
    const int64_t maxw = info->maxw;
    int64_t tcap = block - maxw + 1;
    if (tcap < block / 2) tcap = block / 2;
    const int64_t kb = (W + tcap - 1) / tcap;
    int64_t K = (kb + resident - 1) / resident * resident;
    if (K > nlines) K = nlines;
    if (K < kb) K = kb;
    if (K > kmax) K = kmax;
    info->K = K;
    info->T = (W + K - 1) / K;
}

// rstart[k] = first line of step k, line i in step floor(wptr[i] / T).
__global__ void k_plan_bounds(const int64_t* __restrict__ wptr, int64_t nlines,
                              const PlanInfo* __restrict__ info, int32_t* __restrict__ rstart) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > nlines) return;
    const int64_t T = info->T, K = info->K;
    const int64_t prev = i > 0 ? wptr[i - 1] / T : -1;
    const int64_t cur = i < nlines ? wptr[i] / T : K;
    for (int64_t k = prev + 1; k <= cur; ++k) rstart[k] = (int32_t)i;
}

// Lane layout of a step: segment p = s * nl + i (slice-major) of line r0 + i
// gets ceil(count / E) lanes from lstart[p] on; lstart[P] = total lanes.
// Returns the total in every thread.  wsum: BS / 64 ints of LDS.
template <int BS, int E>
__device__ int step_lanes(const int32_t* __restrict__ split, int ns, int64_t r0, int nl,
                          int* lstart, int* wsum) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int P = ns * nl;
    const int per = (P + BS - 1) / BS;
    constexpr int KMAX = kMaxPairs / BS;  // per <= KMAX
    int cnt[KMAX];
    int mine = 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int p = tid * per + k;
        int lanes = 0;
        if (k < per && p < P) {
            const int s = p / nl, i = p - s * nl;
            const int32_t* sp = split + (r0 + i) * (ns + 1);
            lanes = (sp[s + 1] - sp[s] + E - 1) / E;
        }
        cnt[k] = lanes;
        mine += lanes;
    }
    const int incl = wave_inclusive_scan(mine);
    if (lane == kWave - 1) wsum[tid / kWave] = incl;
    __syncthreads();
    int run = 0;
    for (int w = 0; w < tid / kWave; ++w) run += wsum[w];
    run += incl - mine;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int p = tid * per + k;
        if (k < per && p < P) lstart[p] = run;
        run += cnt[k];
    }
    if (tid == BS - 1) lstart[P] = run;
    __syncthreads();
    return lstart[P];
}

// Last index p in [0, n) with a[p * stride] <= key (nondecreasing, a[0] <= key).
__device__ __forceinline__ int last_le(const int* a, int n, int stride, int key) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid * stride] <= key)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Packed position of slot (quad j, element 0) of lane l in pass q of a step
// whose lanes start at global lane g0, with w lanes in that pass.
__device__ __forceinline__ int64_t packed_at(int64_t g0, int q, int BS, int E, int w, int j, int l) {
    return (g0 + (int64_t)q * BS) * E + ((int64_t)j * w + l) * 4;
}

// One block per step: writes the step's lane starts, every lane's segment and
// every slot of every lane.
template <int PREC, int BS>
__global__ __launch_bounds__(BS) void k_pack(const int64_t* __restrict__ ptr,
                                             const int32_t* __restrict__ idx,
                                             const void* __restrict__ val_, IterPlan p) {
    typedef typename Scal<PREC>::V V;
    constexpr int J = IterCfg<PREC>::J;
    constexpr int E = IterCfg<PREC>::E;
    __shared__ int lstart[kMaxPairs + 1];
    __shared__ int wsum[BS / kWave];
    const int64_t k = blockIdx.x;
    if (k >= p.info->K) return;
    const V* __restrict__ val = (const V*)val_;
    V* __restrict__ pval = (V*)p.pval;
    const int64_t r0 = p.rstart[k];
    const int nl = (int)(p.rstart[k + 1] - r0);
    if (nl == 0) return;
    const int ns = p.ns;
    const int total = step_lanes<BS, E>(p.split, ns, r0, nl, lstart, wsum);
    const int64_t g0 = p.lane_ptr[r0];
    const int32_t SL = (int32_t)p.slice;
    const int P = ns * nl;
    int32_t* lst = p.lst + r0 * ns + k;
    for (int i = threadIdx.x; i <= P; i += BS) lst[i] = lstart[i];
    for (int q = 0; q * BS < total; ++q) {
        const int L = q * BS + threadIdx.x;
        const int w = total - q * BS < BS ? total - q * BS : BS;
        if (L >= total) break;
        const int seg = last_le(lstart, P, 1, L);
        p.lseg[g0 + L] = seg;
        const int s = seg / nl, i = seg - s * nl;
        const int64_t line = r0 + i;
        const int32_t* sp = p.split + line * (ns + 1);
        const int64_t e0 = ptr[line] + sp[s] + (int64_t)(L - lstart[seg]) * E;
        const int64_t e1 = ptr[line] + sp[s + 1];
        for (int j = 0; j < J; ++j) {
            const int64_t at = packed_at(g0, q, BS, E, w, j, threadIdx.x);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t e = e0 + 4 * j + u;
                pval[at + u] = e < e1 ? val[e] : (V)0;
                p.poff[at + u] = (uint16_t)(e < e1 ? idx[e] - s * SL : SL);
            }
        }
    }
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

typedef __attribute__((address_space(3))) void* lds_ptr;

// Starts the copy of x[base .. base + SL) into xs (direct global-to-LDS loads,
// 16 bytes per lane, 1 KB per wave instruction; the wave-uniform LDS address
// goes to M0 and lane l lands 16 l bytes after it).  Elements past nx are not
// copied: no entry refers to them.  The caller waits (s_waitcnt + barrier)
// before reading xs.
template <typename G, int BS, int SL>
__device__ __forceinline__ void stage_issue(G* xs, const G* __restrict__ x, int64_t base,
                                            int64_t nx) {
    constexpr int K = 16 / (int)sizeof(G);        // elements per lane load
    constexpr int NCH = SL / (kWave * K);         // wave chunks per slice
    const int w = threadIdx.x / kWave, l = threadIdx.x & (kWave - 1);
#pragma unroll 1
    for (int c = w; c < NCH; c += BS / kWave) {
        const int64_t g = base + (int64_t)c * kWave * K + (int64_t)l * K;
        if (g + K <= nx) {
            __builtin_amdgcn_global_load_lds((const void*)(x + g), (lds_ptr)(xs + c * kWave * K), 16,
                                             0, 0);
        } else {
#pragma unroll
            for (int u = 0; u < K; ++u)
                if (g + u < nx) xs[c * kWave * K + l * K + u] = x[g + u];
        }
    }
}

__device__ __forceinline__ void stage_wait() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
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

template <int PREC, int BS, bool UOT>
__global__ __launch_bounds__(BS) void k_iterate(IterArgs A) {
    typedef typename Scal<PREC>::V V;
    typedef typename Scal<PREC>::Y Y;
    typedef typename Scal<PREC>::G G;
    typedef typename std::conditional<PREC == P_F64, double, float>::type T;  // lane partial
    constexpr int J = IterCfg<PREC>::J;
    constexpr int E = IterCfg<PREC>::E;
    constexpr int SL = SliceCfg<BS>::bytes / (int)sizeof(G);
    constexpr int RMAX = SliceCfg<BS>::lines;
    extern __shared__ __align__(16) unsigned char dsm[];
    G* xs = (G*)dsm;
    __shared__ __align__(16) int lstart[kMaxPairs + 4];  // first lane of each segment
    __shared__ union {
        T acc[BS];
        struct {
            float m[BS];
            float s[BS];
        } lse;
    } part;                                // per-lane partials of the current pass
    __shared__ union {
        double acc[RMAX];
        struct {
            double m[RMAX];
            float s[RMAX];
        } lse;
    } line_acc;                            // per-line accumulation over passes
    __shared__ double sh[16];
    IterState* st = A.st;
    const int marginal = A.stop_rule == 0;
    const int t = loop_enter(st, A.role, marginal, A.max_iter, A.tol, A.prev_partials,
                             A.prev_nblocks, A.err_hist);
    if (t == 0) return;

    const int tid = threadIdx.x;
    const V* __restrict__ pval = (const V*)A.pval;
    const uint16_t* __restrict__ poff = A.poff;
    const G* __restrict__ xin = (const G*)A.xin;
    const int ns = A.nslices;
    const int64_t K = A.info->K;
    double res = 0.0;
    for (int64_t k = blockIdx.x; k < K; k += gridDim.x) {
        __syncthreads();  // LDS of the previous step is free
        // speculatively start copying slice 0: every step needs it unless its
        // lines have no entry there
        stage_issue<G, BS, SL>(xs, xin, 0, A.nx);
        int cur = 0;
        const int64_t r0 = A.rstart[k];
        const int nl = (int)(A.rstart[k + 1] - r0);
        const int P = ns * nl;
        const int64_t g0 = A.lane_ptr[r0];
        const int total = (int)(A.lane_ptr[r0 + nl] - g0);
        // lane starts of the step's segments -> LDS (direct loads, 4 bytes a lane)
        {
            const int32_t* lst = A.lst + r0 * ns + k;
            for (int c = tid & ~(kWave - 1); c <= P; c += BS)
                if (c + (tid & (kWave - 1)) <= P)
                    __builtin_amdgcn_global_load_lds((const void*)(lst + c + (tid & (kWave - 1))),
                                                     (lds_ptr)(lstart + c), 4, 0, 0);
        }
        // inputs of the line updates
        int64_t pn0 = 0, pn1 = 0;
        double mg = 0.0, yp = 0.0;
        if (tid < nl) {
            const int64_t line = r0 + tid;
            pn0 = A.ptr[line];
            pn1 = A.ptr[line + 1];
            mg = A.marg[line];
            yp = (double)((const Y*)A.yprev)[line];
            if constexpr (PREC == P_LOG) {
                line_acc.lse.m[tid] = -INFINITY;
                line_acc.lse.s[tid] = 0.0f;
            } else {
                line_acc.acc[tid] = 0.0;
            }
        }
        for (int q = 0; q * BS < total; ++q) {
            const int L = q * BS + tid;
            const int w = total - q * BS < BS ? total - q * BS : BS;
            const bool active = L < total;
            const int lc = active ? tid : w - 1;  // lanes past the end re-read the last lane
            // ---- this lane's slots: values and 16-bit slice offsets
            V v[E];
            uint32_t offp[E / 2];  // two offsets per word
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int64_t at = packed_at(g0, q, BS, E, w, j, lc);
                load_quad<V>(pval + at, v + 4 * j);
                const uint2 o = *(const uint2*)(poff + at);
                offp[2 * j + 0] = o.x;
                offp[2 * j + 1] = o.y;
            }
            const int seg = A.lseg[g0 + q * BS + lc];
            stage_wait();  // slice `cur`, the lane starts and the loads above
            const int s = seg / nl;
            // slices touched by this pass: those of its first and last lanes
            const int s_lo = last_le(lstart, ns, nl, q * BS);
            const int s_hi = last_le(lstart, ns, nl, q * BS + w - 1);
            T acc = 0;
            float mx = -INFINITY;  // log domain: running max and sum of exp(z - mx)
            float ls = 0.0f;
            for (int sl = s_lo; sl <= s_hi; ++sl) {
                if (sl != cur) {
                    __syncthreads();  // the previous slice is no longer read
                    stage_issue<G, BS, SL>(xs, xin, (int64_t)sl * SL, A.nx);
                    stage_wait();
                    cur = sl;
                }
                if (active && s == sl) {
#pragma unroll
                    for (int g = 0; g < E; g += 4) {
                        G xv[4];
                        bool in[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            // opaque copies keep the compiler from hoisting the
                            // tests out of the slice loop (that would hold E
                            // more registers across it)
                            uint32_t wd = offp[(g + u) >> 1];
                            asm volatile("" : "+v"(wd));
                            const uint32_t o = (u & 1) ? wd >> 16 : wd & 0xFFFFu;
                            in[u] = o < (uint32_t)SL;
                            xv[u] = xs[in[u] ? o : 0];
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if constexpr (PREC == P_LOG) {
                                // streaming log-sum-exp without branches: one
                                // exp of -|z - mx| rescales the sum or the term;
                                // a NaN difference (both -inf) adds nothing
                                const float z = v[g + u] + xv[u];
                                const float dz = in[u] ? z - mx : -INFINITY;
                                const float e = __expf(-fabsf(dz));
                                const bool up = dz > 0.0f;
                                ls = up ? fmaf(ls, e, 1.0f) : (dz > -INFINITY ? ls + e : ls);
                                mx = up ? z : mx;
                            } else {
                                acc = fma(v[g + u], in[u] ? xv[u] : (G)0, acc);
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
            if (tid < nl) {
                double a = 0.0, m = -INFINITY;
                float sum = 0.0f;
                if constexpr (PREC == P_LOG) {
                    m = line_acc.lse.m[tid];
                    sum = line_acc.lse.s[tid];
                } else {
                    a = line_acc.acc[tid];
                }
                for (int ss = 0; ss < ns; ++ss) {
                    const int pp = ss * nl + tid;
                    const int b = lstart[pp] > q * BS ? lstart[pp] : q * BS;
                    const int e = lstart[pp + 1] < q * BS + w ? lstart[pp + 1] : q * BS + w;
                    for (int l = b; l < e; ++l) {
                        if constexpr (PREC == P_LOG)
                            lse_merge(m, sum, (double)part.lse.m[l - q * BS], part.lse.s[l - q * BS]);
                        else
                            a += (double)part.acc[l - q * BS];
                    }
                }
                if constexpr (PREC == P_LOG) {
                    line_acc.lse.m[tid] = m;
                    line_acc.lse.s[tid] = sum;
                } else {
                    line_acc.acc[tid] = a;
                }
            }
        }
        if (total == 0) stage_wait();  // no pass waited for the speculative copy
        // ---- scaling update of every line of the step
        if (tid < nl) {
            const int64_t line = r0 + tid;
            double w;
            if constexpr (PREC == P_LOG) {
                const double m = line_acc.lse.m[tid];
                const float sum = line_acc.lse.s[tid];
                w = (m == -INFINITY || !(sum > 0.0f)) ? -INFINITY : m + log((double)sum);
            } else {
                w = line_acc.acc[tid];
            }
            res += line_update<PREC, UOT>(A.role, marginal, t, pn1 > pn0, mg, A.theta, yp, A.yout,
                                          A.yg, line, w, st);
        }
    }
    const double bsum = block_sum(res, sh);
    if (tid == 0) A.partials[blockIdx.x] = bsum;
}

template <int PREC, int BS>
static hipError_t run_iter(const IterArgs& a, int grid, hipStream_t st) {
    const size_t lds = SliceCfg<BS>::bytes;
    if (a.theta != 1.0)
        hipLaunchKernelGGL((k_iterate<PREC, BS, true>), dim3(grid), dim3(BS), lds, st, a);
    else
        hipLaunchKernelGGL((k_iterate<PREC, BS, false>), dim3(grid), dim3(BS), lds, st, a);
    return hipGetLastError();
}

template <int PREC, int BS, bool UOT>
static hipError_t allow_lds() {
    return hipFuncSetAttribute((const void*)&k_iterate<PREC, BS, UOT>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, SliceCfg<BS>::bytes);
}

// Resident blocks of k_iterate<PREC, BS> on the current device.
template <int PREC, int BS>
static int resident_blocks() {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)&k_iterate<PREC, BS, true>,
                                                     BS, SliceCfg<BS>::bytes) != hipSuccess)
        return 0;
    const int r = cus * (per > 0 ? per : 1);
    return r < kMaxLoopBlocks ? r : kMaxLoopBlocks;
}

static int g_resident[3][2];

// Raises the dynamic LDS limit of every instantiation and records how many
// blocks of each stay resident (once, before any launch or graph capture).
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
        g_resident[P_F64][0] = resident_blocks<P_F64, 256>();
        g_resident[P_F64][1] = resident_blocks<P_F64, 1024>();
        g_resident[P_F32][0] = resident_blocks<P_F32, 256>();
        g_resident[P_F32][1] = resident_blocks<P_F32, 1024>();
        g_resident[P_LOG][0] = resident_blocks<P_LOG, 256>();
        g_resident[P_LOG][1] = resident_blocks<P_LOG, 1024>();
        for (auto& row : g_resident)
            for (int x : row)
                if (x <= 0 && e == hipSuccess) e = hipErrorInvalidDeviceFunction;
        return e;
    }();
    return status;
}

// Block size: 1024 threads (128 KB slices) when there are enough lines for a
// block per compute unit, else 256 threads (32 KB slices).
int iterate_block_size(int64_t nlines) { return nlines >= 256 * 256 ? 1024 : 256; }

template <int PREC, int BS>
static void launch_pack(const IterPlan& p, const int64_t* ptr, const int32_t* idx, const void* val,
                        hipStream_t st) {
    hipLaunchKernelGGL((k_pack<PREC, BS>), dim3((unsigned)p.kmax), dim3(BS), 0, st, ptr, idx, val, p);
}

hipError_t build_plan(int precision, const IterPlan& p, const int64_t* ptr, const int32_t* idx,
                      const void* val, int64_t nlines, hipStream_t st) {
    if (nlines <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((nlines + 255) / 256);
    hipLaunchKernelGGL(k_split, dim3(nb), dim3(256), 0, st, ptr, idx, nlines, p.ns, p.slice,
                       p.split);
    hipError_t e = launch_fill_u32((uint32_t*)p.info, sizeof(PlanInfo) / 4, 0u, st);
    if (e != hipSuccess) return e;
    const int E = entries_per_lane(precision);
    hipLaunchKernelGGL(k_plan_lanes, dim3(nb), dim3(256), 0, st, p.split, nlines, p.ns, E,
                       min_weight(p.block, p.ns), p.lanes, p.weight, p.info);
    e = launch_scan(p.lanes, nlines, p.lane_ptr, p.scan, st);
    if (e == hipSuccess) e = launch_scan(p.weight, nlines, p.wptr, p.scan, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_plan_setup, dim3(1), dim3(64), 0, st, p.wptr, nlines, p.block,
                       (int64_t)p.grid, p.kmax, p.info);
    hipLaunchKernelGGL(k_plan_bounds, dim3((unsigned)((nlines + 1 + 255) / 256)), dim3(256), 0, st,
                       p.wptr, nlines, p.info, p.rstart);
    if (precision == P_F64)
        p.block == 1024 ? launch_pack<P_F64, 1024>(p, ptr, idx, val, st)
                        : launch_pack<P_F64, 256>(p, ptr, idx, val, st);
    else
        p.block == 1024 ? launch_pack<P_F32, 1024>(p, ptr, idx, val, st)
                        : launch_pack<P_F32, 256>(p, ptr, idx, val, st);
    return hipGetLastError();
}

int iterate_grid(int precision, int block) {
    return g_resident[precision][block == 1024 ? 1 : 0];
}

hipError_t launch_iterate(int precision, int block, int grid, const IterArgs& a, hipStream_t st) {
    if (precision == P_F64)
        return block == 1024 ? run_iter<P_F64, 1024>(a, grid, st) : run_iter<P_F64, 256>(a, grid, st);
    if (precision == P_F32)
        return block == 1024 ? run_iter<P_F32, 1024>(a, grid, st) : run_iter<P_F32, 256>(a, grid, st);
    return block == 1024 ? run_iter<P_LOG, 1024>(a, grid, st) : run_iter<P_LOG, 256>(a, grid, st);
}

// u^0 / v^0: ones (or exp of the warm start); potentials 0 (or the warm start).
__global__ void k_init_scaling(int precision, void* y, float* yg, const double* init_log,
                               int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double l = init_log ? init_log[i] : 0.0;
    if (precision == P_F64) ((double*)y)[i] = init_log ? exp(l) : 1.0;
    if (precision == P_F32) ((float*)y)[i] = init_log ? (float)exp(l) : 1.0f;
    if (precision == P_LOG) {
        ((double*)y)[i] = l;
        if (yg) yg[i] = (float)l;
    }
}

hipError_t launch_init_scaling(int precision, void* y, float* yg, const double* init_log,
                               int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_scaling, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       precision, y, yg, init_log, n);
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
