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
// g = log v, and w_r becomes a stabilised log-sum-exp.
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
// SL elements copied into LDS by direct global-to-LDS loads, two slice buffers
// deep, and each line's entries are cut at the slice boundaries into segments
// (entries are column-sorted within a line, so every segment is contiguous).
//
// Lane plan (built once per solve by build_plan):
//  * a segment of c entries takes ceil(c / 4) quads;
//  * lines are grouped into steps of consecutive lines (line weights, in
//    quads, are scanned and cut every T; the number of steps is a multiple of
//    the resident blocks, so the persistent grid is balanced);
//  * inside a step the segments are laid out slice-major, one after another,
//    in lanes of J quads; a lane holds at most two segments (the tail of one
//    and the head of the next, both of one slice), so a segment that would be
//    the third of a lane starts the next lane instead;
//  * lanes are cut into passes of BS and the entries are repacked so that
//    quad j of the lanes of one pass is contiguous: a wave's load instruction
//    reads one unbroken run of memory.  The column index is stored as its
//    byte offset inside the slice; an empty slot holds offset 0 and the
//    neutral value (0, or -inf in the log domain), so the product needs no
//    test per entry;
//  * per lane the plan stores its slice and the quad where its second segment
//    starts, per segment its first and last quad, so the kernel needs no scan
//    or search.
//
// Iteration kernel: a block takes a step, starts the copies of its first two
// slices, loads every lane's E values and offsets into registers, and while
// slice s is resident the lanes of slice s add their terms into one
// accumulator per segment, while slice s + 1 is copied into the other buffer.
// Lane partials are folded per line in (slice, lane) order through LDS, so
// every sum has a fixed order and the results are deterministic.
//
// Log domain: entries are stored as l log2(e) and the gathered potentials as
// g log2(e), so a lane computes its base-2 log-sum-exp in two passes (maximum,
// then sum of exp2 of the differences).
template <int PREC>
struct IterCfg {
    static constexpr int J = PREC == P_F64 ? 3 : 7;   // quads per lane
    static constexpr int E = 4 * J;                   // entry slots per lane
};

template <int BS>
struct SliceCfg {
    static constexpr int buf = BS == 1024 ? 65536 : 16384;  // bytes of one slice buffer
    static constexpr int data = buf;                        // bytes of gathered data
    static constexpr int lines = BS / 2;                    // most lines a step may hold
    // dynamic LDS: two slice buffers, segment quad ranges, line accumulators,
    // reduction scratch
    static constexpr int lds = 2 * buf + 2 * 2048 * 4 + lines * 8 + 512;
};

constexpr int kMaxPairs = 2048;  // (slice, line) segments per step
constexpr int kPassesMax = 8;    // passes per step under the multi-pass policy
static_assert(SliceCfg<1024>::buf <= 65536, "byte offsets must fit in 16 bits");
static_assert(SliceCfg<1024>::lds <= 160 * 1024 && 3 * SliceCfg<256>::lds <= 160 * 1024,
              "LDS budget");

int entries_per_lane(int precision) {
    return precision == P_F64 ? IterCfg<P_F64>::E : IterCfg<P_F32>::E;
}

static int quads_per_lane(int precision) { return entries_per_lane(precision) / 4; }

int slice_elems(int precision, int block) {
    const int bytes = block == 1024 ? SliceCfg<1024>::data : SliceCfg<256>::data;
    return bytes / (precision == P_F64 ? 8 : 4);
}

int iterate_slices(int precision, int block, int64_t nx) {
    const int64_t sl = slice_elems(precision, block);
    return (int)((nx + sl - 1) / sl);
}

// Largest step weight the planner aims for (quads): 15/16 of a full pass.
__host__ __device__ static int64_t step_quads(int block, int J) { return (int64_t)block * J * 15 / 16; }

// Smallest line weight (quads): keeps the lines of a step <= BS / 2 and the
// segments of a step <= kMaxPairs (a step holds at most ceil(T / minw) lines,
// T <= step_quads).
static int min_weight(int block, int ns, int J) {
    const int64_t tq = step_quads(block, J);
    int w = 2 * J;
    while (((tq + w - 1) / w + 1) * ns > kMaxPairs || (tq + w - 1) / w + 1 > block / 2) ++w;
    return w;
}

bool plan_shape(int precision, int block, int64_t nlines, int64_t nx, int64_t cap, IterPlan* p) {
    const int64_t ns = (nx + slice_elems(precision, block) - 1) / slice_elems(precision, block);
    if (ns > kMaxPairs / 2) return false;
    p->block = block;
    p->ns = (int)ns;
    p->slice = slice_elems(precision, block);
    const int J = quads_per_lane(precision);
    // nonempty segments; lanes <= quads / J + padding / J + one partial lane
    // per (step, slice), with quads <= cap / 4 + segs and padding < J a segment
    const int64_t segs = cap < nlines * ns ? cap : nlines * ns;
    p->lanes_max = cap / (4 * J) + 2 * segs + 1;
    // steps: K <= W / Tmin + resident blocks, W <= quads + nlines * minw,
    // Tmin >= block * J / 4
    const int64_t W = cap / 4 + segs + nlines * (int64_t)min_weight(block, (int)ns, J);
    p->kmax = W / ((int64_t)block * J / 4) + kMaxLoopBlocks + 2;
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

// Quads of every line; their total and the total of the line weights under
// the single-pass policy's floor minw1 (atomic adds of integers: exact).
__global__ void k_plan_quads(const int32_t* __restrict__ split, int64_t nlines, int ns, int minw1,
                             int32_t* __restrict__ quads, PlanInfo* info) {
    const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t q = 0, w = 0;
    if (line < nlines) {
        const int32_t* sp = split + line * (ns + 1);
        for (int s = 0; s < ns; ++s) q += (sp[s + 1] - sp[s] + 3) / 4;
        quads[line] = (int32_t)q;
        w = q > minw1 ? q : minw1;
    }
    q = group_sum<kWave>(q);
    w = group_sum<kWave>(w);
    if ((threadIdx.x & (kWave - 1)) == 0 && w > 0) {
        atomicAdd((unsigned long long*)&info->Q, (unsigned long long)q);
        atomicAdd((unsigned long long*)&info->W1, (unsigned long long)w);
    }
}

// Step policy (one thread).  Each pass of a step first copies the slices its
// lanes read, so a launch copies about ns + passes - 1 slices per step.
//  * single-pass: step weight at most 15/16 of a pass (tcap1), line weights
//    floored at minw1 (a step then holds few enough lines and segments for
//    the LDS tables); kept whenever it needs no more steps than there are
//    resident blocks (one step, one pass per block);
//  * multi-pass: otherwise, kmin = S * resident steps of up to kPassesMax
//    passes, S the fewest with S * resident * L >= 3/2 nlines (L = most lines
//    a step may hold, less one), and the floor minw = ceil((Q + kmin) /
//    (kmin L - nlines)): a step of weight T <= (Q + nlines minw) / kmin + 1
//    then holds at most T / minw + 1 <= L + 1 lines.  Taken when it needs
//    fewer steps than the single-pass policy.
__global__ void k_plan_policy(int64_t nlines, int block, int J, int ns, int minw1,
                              int64_t resident, int64_t kmax, PlanInfo* info) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t tcap1 = step_quads(block, J) - (int64_t)ns * J;
    if (tcap1 < (int64_t)block * J / 4) tcap1 = (int64_t)block * J / 4;
    const int64_t k1 = (((info->W1 + tcap1 - 1) / tcap1) + resident - 1) / resident * resident;
    info->minw = minw1;
    info->tcap = tcap1;
    info->kmin = 0;
    if (k1 <= resident) return;
    const int64_t Q = info->Q;
    int64_t L = block / 2 < kMaxPairs / ns ? block / 2 : kMaxPairs / ns;
    L -= 1;
    int64_t tmax = (int64_t)kPassesMax * step_quads(block, J) - (int64_t)ns * J;
    int64_t S = (Q + resident * tmax - 1) / (resident * tmax);
    if (S < 1) S = 1;
    while (2 * S * resident * L < 3 * nlines) ++S;
    const int64_t kmin = S * resident;
    // the line bound needs K >= kmin, which the clamps of k_plan_setup to
    // nlines and kmax could break
    if (kmin >= k1 || L < 1 || kmin > nlines || kmin > kmax) return;
    int64_t w = (Q + kmin + kmin * L - nlines - 1) / (kmin * L - nlines);
    if (w < 2 * J) w = 2 * J;
    if (w > tmax) w = tmax;
    info->minw = (int32_t)w;
    info->tcap = tmax;
    info->kmin = kmin;
}

// Step weight of every line, max(quads, minw) under the chosen floor.
__global__ void k_plan_weights(const int32_t* __restrict__ quads, int64_t nlines,
                               const PlanInfo* __restrict__ info, int32_t* __restrict__ weight) {
    const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (line >= nlines) return;
    const int32_t q = quads[line], w = info->minw;
    weight[line] = q > w ? q : w;
}

// Step weight T and step count K (one thread).  The single-pass cap leaves
// 1/16 of a pass of `block` lanes, plus one partial lane per slice, for the
// last line of a step (which may run past T) and the layout's padding; line
// weights are floored, so a step's quads are usually well below its weight.
// A step that still overflows takes another pass.
__global__ void k_plan_setup(const int64_t* __restrict__ wptr, int64_t nlines, int64_t resident,
                             int64_t kmax, PlanInfo* info) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t W = wptr[nlines];
    const int64_t tcap = info->tcap;
    const int64_t kb = (W + tcap - 1) / tcap;
    int64_t K = kb > info->kmin ? kb : info->kmin;
    K = (K + resident - 1) / resident * resident;
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

// One block per step: the packed quad range [qs, qe) of every segment
// p = s * nl + i (line r0 + i, slice s) and the step's lane count.  Segments
// of one slice follow each other; a slice starts on a new lane; a segment
// starts on the next lane when the lane it would start in already holds two
// segments.  A thread lays out one slice (from quad 0), a block scan over the
// slices' lane counts gives each slice its first lane, and the ranges are
// shifted there.
__global__ __launch_bounds__(256) void k_layout(const int32_t* __restrict__ split, int ns, int J,
                                                const int32_t* __restrict__ rstart,
                                                const PlanInfo* __restrict__ info, int64_t kmax,
                                                int32_t* __restrict__ qs, int32_t* __restrict__ qe,
                                                int32_t* __restrict__ steplanes) {
    __shared__ int nq[kMaxPairs];   // quads of each segment, then its start in its slice
    __shared__ int qe_l[kMaxPairs];  // end of each segment in its slice
    __shared__ int sl_lanes[kMaxPairs / 2 + 1];  // per slice: lanes, then first lane
    __shared__ int wsum[256 / kWave];
    const int64_t k = blockIdx.x;
    if (k >= kmax) return;
    if (k >= info->K) {
        if (threadIdx.x == 0) steplanes[k] = 0;
        return;
    }
    const int64_t r0 = rstart[k];
    const int nl = (int)(rstart[k + 1] - r0);
    const int P = ns * nl;
    const int tid = threadIdx.x;
    for (int p = tid; p < P; p += blockDim.x) {
        const int s = p / nl, i = p - s * nl;
        const int32_t* sp = split + (r0 + i) * (ns + 1);
        nq[p] = (sp[s + 1] - sp[s] + 3) / 4;
    }
    __syncthreads();
    for (int s = tid; s < ns; s += blockDim.x) {
        int pos = 0;
        int prev = 0;  // start of the last segment placed in this slice
        for (int i = 0; i < nl; ++i) {
            const int p = s * nl + i;
            const int n = nq[p];
            if (n > 0) {
                const int lane0 = pos / J;
                // the lane at pos already holds a segment that started inside it
                // and the one before: start on the next lane
                if (pos != lane0 * J && prev > lane0 * J) pos = (lane0 + 1) * J;
                prev = pos;
            }
            nq[p] = pos;
            pos += n;
            qe_l[p] = pos;
        }
        sl_lanes[s] = (pos + J - 1) / J;
    }
    __syncthreads();
    // exclusive scan of the slices' lane counts (ns <= kMaxPairs / 2)
    const int per = (ns + 255) / 256;
    int mine = 0;
    for (int u = 0; u < per; ++u) {
        const int s = tid * per + u;
        if (s < ns) mine += sl_lanes[s];
    }
    const int incl = wave_inclusive_scan(mine);
    if ((tid & (kWave - 1)) == kWave - 1) wsum[tid / kWave] = incl;
    __syncthreads();
    int run = incl - mine;
    for (int w = 0; w < tid / kWave; ++w) run += wsum[w];
    const int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();  // every thread has read its slices' counts
    for (int u = 0; u < per; ++u) {
        const int s = tid * per + u;
        if (s < ns) {
            const int c = sl_lanes[s];
            sl_lanes[s] = run;
            run += c;
        }
    }
    __syncthreads();
    int32_t* qs_k = qs + r0 * ns;
    int32_t* qe_k = qe + r0 * ns;
    for (int p = tid; p < P; p += blockDim.x) {
        const int shift = sl_lanes[p / nl] * J;
        qs_k[p] = nq[p] + shift;
        qe_k[p] = qe_l[p] + shift;
    }
    if (tid == 0) steplanes[k] = total;
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

// One block per step: every lane's metadata and every slot of every lane.
// The nonempty segments of the step are compacted (their quad starts are
// strictly increasing), and each lane finds the segment holding its quad 0
// and the one starting inside it by binary search.
template <int PREC, int BS>
__global__ __launch_bounds__(256) void k_pack(const int64_t* __restrict__ ptr,
                                              const int32_t* __restrict__ idx,
                                              const void* __restrict__ val_, IterPlan p) {
    typedef typename Scal<PREC>::V V;
    typedef typename Scal<PREC>::G G;
    constexpr int J = IterCfg<PREC>::J;
    constexpr int E = IterCfg<PREC>::E;
    constexpr int PER = kMaxPairs / 256;
    __shared__ int cqs[kMaxPairs];  // quad starts of the nonempty segments
    __shared__ int cseg[kMaxPairs];  // their segment numbers
    __shared__ int wsum[256 / kWave];
    const int64_t k = blockIdx.x;
    if (k >= p.info->K) return;
    const V* __restrict__ val = (const V*)val_;
    V* __restrict__ pval = (V*)p.pval;
    uint16_t* __restrict__ poff = p.poff;
    const int64_t r0 = p.rstart[k];
    const int nl = (int)(p.rstart[k + 1] - r0);
    const int ns = p.ns;
    const int P = ns * nl;
    const int64_t g0 = p.stepoff[k];
    const int total = (int)(p.stepoff[k + 1] - g0);
    if (total == 0) return;
    const int32_t* qs = p.qs + r0 * ns;
    const int32_t* qe = p.qe + r0 * ns;
    // compaction: thread t owns segments [t * PER, t * PER + PER)
    const int tid = threadIdx.x;
    int mine = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int s = tid * PER + u;
        mine += (s < P && qe[s] > qs[s]) ? 1 : 0;
    }
    const int incl = wave_inclusive_scan(mine);
    if ((tid & (kWave - 1)) == kWave - 1) wsum[tid / kWave] = incl;
    __syncthreads();
    int at = incl - mine;
    for (int w = 0; w < tid / kWave; ++w) at += wsum[w];
    const int nc = wsum[0] + wsum[1] + wsum[2] + wsum[3];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int s = tid * PER + u;
        if (s < P && qe[s] > qs[s]) {
            cqs[at] = qs[s];
            cseg[at] = s;
            ++at;
        }
    }
    __syncthreads();
    const int64_t SL = p.slice;
    for (int L = tid; L < total; L += 256) {
        const int Q0 = L * J;
        const int a = last_le(cqs, nc, 1, Q0);
        int bq = J, b = a;
        if (a + 1 < nc && cqs[a + 1] < Q0 + J) {
            b = a + 1;
            bq = cqs[b] - Q0;
        }
        const int sa = cseg[a];
        const int s = sa / nl;
        p.lmeta[g0 + L] = (s << 8) | bq;
        const int q = L / BS, l = L - q * BS;
        const int w = total - q * BS < BS ? total - q * BS : BS;
        // the lane's two segments' entry ranges, then every load of its J
        // quads before any store (the stores cannot alias the loads)
        int64_t e0[J], ee[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int c = j < bq ? a : b;
            const int seg = cseg[c];
            const int64_t line = r0 + (seg - (seg / nl) * nl);
            const int32_t* sp = p.split + line * (ns + 1);
            const int64_t base = ptr[line];
            ee[j] = base + sp[s + 1];
            e0[j] = base + sp[s] + (int64_t)(Q0 + j - cqs[c]) * 4;
        }
        V x[E];
        uint16_t o[E];
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t e = e0[j] + u;
                const bool ok = e < ee[j];
                // empty slot: neutral value, offset 0
                if constexpr (PREC == P_LOG)
                    x[4 * j + u] = ok ? (V)((double)val[e] * kLog2e) : (V)-INFINITY;
                else
                    x[4 * j + u] = ok ? val[e] : (V)0;
                o[4 * j + u] = (uint16_t)(ok ? (idx[e] - s * SL) * (int64_t)sizeof(G) : 0);
            }
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int64_t pa = packed_at(g0, q, BS, E, w, j, l);  // a quad: 4-aligned
#pragma unroll
            for (int u = 0; u < 4; ++u) pval[pa + u] = x[4 * j + u];
            uint2 ow;
            ow.x = (uint32_t)o[4 * j] | ((uint32_t)o[4 * j + 1] << 16);
            ow.y = (uint32_t)o[4 * j + 2] | ((uint32_t)o[4 * j + 3] << 16);
            *(uint2*)(poff + pa) = ow;
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

// Element at LDS byte address `a`.
template <typename G>
__device__ __forceinline__ G lds_at(uint32_t a) {
    return *(const __attribute__((address_space(3))) G*)(size_t)a;
}

// Starts the copy of slice elements [base, base + SL) of x into the slice
// buffer at `buf` with direct global-to-LDS loads: 16 bytes a lane, 1 KB a
// wave instruction (the wave-uniform LDS address goes to M0, lane l lands
// 16 l bytes after it), and the same number of instructions in every wave.
// Lanes past the end of x read its last 16-byte group; no entry refers to
// the words they fill.  The caller waits (stage_wait) before reading the
// buffer.
template <typename G, int BS>
__device__ __forceinline__ void stage_issue(unsigned char* buf, const G* __restrict__ x,
                                            int64_t base, int64_t gmax) {
    constexpr int DATA = SliceCfg<BS>::data;
    constexpr int NCH = DATA / 1024;  // wave chunks per slice
    constexpr int NW = BS / kWave;
    static_assert(DATA % 1024 == 0 && NCH % NW == 0, "every wave issues the same number of chunks");
    const int w = threadIdx.x / kWave, l = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int i = 0; i < NCH / NW; ++i) {
        const int c = w + i * NW;
        const int byte = c * 1024 + l * 16;
        int64_t g = base + byte / (int)sizeof(G);
        if (g > gmax) g = gmax;
        __builtin_amdgcn_global_load_lds((const void*)(x + g), (lds_ptr)(buf + c * 1024), 16, 0, 0);
    }
}

__device__ __forceinline__ void stage_wait() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// Waits until at most N vector memory operations of this wave are in flight
// and its LDS and scalar memory operations are done (s_waitcnt with vmcnt = N,
// lgkmcnt = 0; gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4,
// lgkmcnt 11:8).  Vector loads complete in issue order, so this waits for all
// but the last N.
template <int N>
__device__ __forceinline__ void wait_vmcnt_lgkm0() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4));
}

// LDS byte address of slot u of a quad inside slice buffer `hsel` (0 or 1):
// 16-bit byte offsets, two to a word.  k_iterate has no static LDS, so its
// buffers start at LDS address 0 and buffer 1 at BUF.  With 64 KB buffers one
// instruction forms the address: the buffer bit goes above the offset (v_perm
// for the low half, v_alignbit for the high half); both read the
// slice-dependent bit, so the decode cannot be hoisted out of the slice loop.
template <int BS>
__device__ __forceinline__ uint32_t slot_addr(uint32_t wd, int u, uint32_t hsel) {
    constexpr uint32_t BUF = SliceCfg<BS>::buf;
    if constexpr (BUF == 65536u) {
        // perm selector: bytes 0, 1 of wd, byte 0 of hsel, then a zero byte
        return (u & 1) ? __builtin_amdgcn_alignbit(hsel, wd, 16)
                       : __builtin_amdgcn_perm(hsel, wd, 0x0C040100u);
    } else {
        const uint32_t o = (u & 1) ? (wd >> 16) : (wd & 0xFFFFu);
        return o | (hsel * BUF);
    }
}

// Natural log of a base-2 pair (m, s), (m + log2 s) ln 2; -inf when empty.
// The sum holds the term of the maximum, so s >= 1 and its FP32 base-2 log
// (v_log_f32) is accurate to a few 1e-7 absolute, below the rounding of m.
__device__ __forceinline__ double lse2_value(float m, float s) {
    return (m == -INFINITY || !(s > 0.0f))
               ? -INFINITY
               : ((double)m + (double)__builtin_amdgcn_logf(s)) * kLn2;
}

template <int PREC, int BS, bool UOT>
__global__ __launch_bounds__(BS) void k_iterate(IterArgs A) {
    typedef typename Scal<PREC>::V V;
    typedef typename Scal<PREC>::Y Y;
    typedef typename Scal<PREC>::G G;
    typedef typename std::conditional<PREC == P_F64, double, float>::type T;  // lane partial
    constexpr int J = IterCfg<PREC>::J;
    constexpr int E = IterCfg<PREC>::E;
    constexpr int BUF = SliceCfg<BS>::buf;
    constexpr int DATA = SliceCfg<BS>::data;
    constexpr int SL = DATA / (int)sizeof(G);
    constexpr int RMAX = SliceCfg<BS>::lines;
    constexpr int KG = 16 / (int)sizeof(G);
    // All LDS is dynamic, so the slice buffers start at its base:
    //   [0, 2 BUF)       two slice buffers; after the products buffer 0
    //                    holds the lane partials
    //   qs, qe           packed quad ranges of the step's segments
    //   line accumulators, reduction scratch
    extern __shared__ __align__(16) unsigned char dsm[];
    int* const qs_l = (int*)(dsm + 2 * BUF);
    int* const qe_l = qs_l + kMaxPairs;
    double* const lacc = (double*)(qe_l + kMaxPairs);  // linear: FP64 sum per line
    float* const lm = (float*)lacc;                    // log: base-2 (max, sum) per line
    float* const ls = lm + RMAX;
    double* const sh = lacc + RMAX;  // 32 doubles
    int* const s_t = (int*)(sh + 32);
    T* const partA = (T*)dsm;  // [BS] first-segment partials (linear) / maxima (log)
    T* const partB = partA + BS;
    float* const psA = (float*)(partB + BS);  // log: sums
    float* const psB = psA + BS;

    IterState* st = A.st;
    const int marginal = A.stop_rule == 0;
    const int t = loop_start(st, A.role, A.max_iter, s_t);
    if (t == 0) return;
    if (!loop_updates(A.role, marginal, A.max_iter, t)) {
        if (blockIdx.x == 0)
            loop_close(st, A.role, marginal, A.max_iter, A.tol, A.prev_partials, A.prev_nblocks,
                       A.err_hist, t, sh);
        return;
    }
    // Block 0 closes the previous launch: it loads the partials now, while
    // nothing else is in flight, and sums them with its own residual at the
    // end, so the closing adds no latency of its own.
    constexpr int PF = (kMaxLoopBlocks + BS - 1) / BS;
    double pf[PF];
    const bool closes = blockIdx.x == 0 && loop_closes(A.role, t);
#pragma unroll
    for (int i = 0; i < PF; ++i) {
        const int bi = threadIdx.x + i * BS;
        pf[i] = closes && bi < A.prev_nblocks ? A.prev_partials[bi] : 0.0;
    }
    // Summed inside the step loop, after waits for all loads (a sum after the
    // loop would make the compiler wait for the line updates' stores); block
    // 0 always has a step, other blocks load nothing.
    double prev = 0.0;
    // the last line update of this thread is stored after the block's sums
    // (the compiler would otherwise wait for the stores before them)
    int64_t pend_line = -1;
    double pend_y = 0.0;

    const int tid = threadIdx.x;
    // the slot addresses assume the dynamic LDS starts at address 0
    if ((uint32_t)(size_t)(lds_ptr)dsm != 0u) {
        if (tid == 0) st->nonfinite = 1;
        return;
    }
    const V* __restrict__ pval = (const V*)A.pval;
    const uint16_t* __restrict__ poff = A.poff;
    const G* __restrict__ xin = (const G*)A.xin;
    const int ns = A.nslices;
    const int64_t K = A.info->K;
    const int64_t gmax = (A.nx - 1) / KG * KG;
    double res = 0.0;
    for (int64_t k = blockIdx.x; k < K; k += gridDim.x) {
        __syncthreads();  // LDS of the previous step is free
        const int64_t r0 = A.rstart[k];
        const int nl = (int)(A.rstart[k + 1] - r0);
        const int P = ns * nl;
        const int64_t g0 = A.stepoff[k];
        const int total = (int)(A.stepoff[k + 1] - g0);
        // quad ranges of the step's segments -> LDS (direct loads, 4 bytes a lane)
        {
            const int32_t* q0 = A.qs + r0 * ns;
            const int32_t* q1 = A.qe + r0 * ns;
            const int l = tid & (kWave - 1);
            for (int c = tid & ~(kWave - 1); c < P; c += BS)
                if (c + l < P) {
                    __builtin_amdgcn_global_load_lds((const void*)(q0 + c + l), (lds_ptr)(qs_l + c), 4, 0, 0);
                    __builtin_amdgcn_global_load_lds((const void*)(q1 + c + l), (lds_ptr)(qe_l + c), 4, 0, 0);
                }
        }
        // inputs of the line updates
        int64_t pn0 = 0, pn1 = 0;
        double mg = 0.0, lmg = 0.0, yp = 0.0;
        if (tid < nl) {
            const int64_t line = r0 + tid;
            pn0 = A.ptr[line];
            pn1 = A.ptr[line + 1];
            mg = A.marg[line];
            if constexpr (PREC == P_LOG) lmg = A.lmarg[line];
            yp = (double)((const Y*)A.yprev)[line];
            if constexpr (PREC == P_LOG) {
                lm[tid] = -INFINITY;
                ls[tid] = 0.0f;
            } else {
                lacc[tid] = 0.0;
            }
        }
        for (int q = 0; q * BS < total; ++q) {
            const int w = total - q * BS < BS ? total - q * BS : BS;
            const bool active = tid < w;
            const int lc = active ? tid : w - 1;  // lanes past the end re-read the last lane
            const int64_t lb = g0 + (int64_t)q * BS;
            const int s_lo = A.lmeta[lb] >> 8;
            const int s_hi = A.lmeta[lb + w - 1] >> 8;
            if (q > 0) __syncthreads();  // the previous pass's fold has read buffer 0
            // ---- this lane's metadata, the copies of the pass's first two
            // slices, then the lane's slots: values and 16-bit byte offsets.
            // The memory clobbers keep the slot loads behind the copies, so
            // that waiting for all but the last 2J vector memory operations of
            // a wave waits for its copies only.
            const int meta = A.lmeta[lb + lc];
            stage_issue<G, BS>(dsm + (s_lo & 1) * BUF, xin, (int64_t)s_lo * SL, gmax);
            if (s_hi > s_lo)
                stage_issue<G, BS>(dsm + ((s_lo + 1) & 1) * BUF, xin, (int64_t)(s_lo + 1) * SL, gmax);
            asm volatile("" ::: "memory");
            V v[E];
            uint32_t offp[E / 2];  // two offsets per word
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int64_t at = lb * E + ((int64_t)j * w + lc) * 4;
                load_quad<V>(pval + at, v + 4 * j);
                const uint2 o = *(const uint2*)(poff + at);
                offp[2 * j + 0] = o.x;
                offp[2 * j + 1] = o.y;
            }
            // the first two slices and the quad ranges are in; the lanes of the
            // first pair start while the rest of the slots stream in.  A bare
            // barrier: the fence of __syncthreads would wait for every load.
            wait_vmcnt_lgkm0<2 * J>();
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            const int s = meta >> 8;
            T rA = 0, rB = 0;           // linear: sums; log: base-2 maxima
            float sA = 0.0f, sB = 0.0f;  // log: sums of exp2(z - max)
            if constexpr (PREC == P_LOG) {
                rA = -INFINITY;
                rB = -INFINITY;
            }
            // Slices sl and sl + 1 are resident together and the lanes of both
            // work; the first pair is peeled so that its lanes start as their
            // own loads arrive (inside a loop the compiler waits for all loads).
            auto work = [&](int sl) __attribute__((always_inline)) {
                if (active && (s == sl || s == sl + 1)) {
                    // the buffer of slice s, written through sl so that the address
                    // decode stays inside the slice loop
                    const uint32_t hsel = (uint32_t)(sl & 1) ^ (uint32_t)(s - sl);
                    int b = meta & 0xFF;  // quad where the second segment starts (J: none)
                    asm volatile("" : "+v"(b));  // one register, compared with inline constants
                    if constexpr (PREC == P_LOG) {
                        // pass 1: z = l + g (base 2) and the maximum of each segment
                        float m = -INFINITY, mA = -INFINITY;
#pragma unroll
                        for (int j = 0; j < J; ++j) {
                            if (j == b) {
                                mA = m;
                                m = -INFINITY;
                            }
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const uint32_t wd = offp[2 * j + (u >> 1)];
                                v[4 * j + u] += lds_at<float>(slot_addr<BS>(wd, u, hsel));
                            }
                            m = fmaxf(m, fmaxf(fmaxf(v[4 * j], v[4 * j + 1]),
                                               fmaxf(v[4 * j + 2], v[4 * j + 3])));
                            // two quads of LDS reads in flight at a time bound the
                            // registers the scheduler holds for them
                            if (j & 1) __builtin_amdgcn_sched_barrier(0);
                        }
                        // selects, not branches: a branch on b turns the pair into
                        // an indexed private array
                        const bool one = b >= J;  // a single segment
                        const float mB = one ? -INFINITY : m;
                        mA = one ? m : mA;
                        // pass 2: sums of exp2(z - max); empty slots hold z = -inf,
                        // and an empty segment sums exp2(-inf) = 0 against a shift of 0
                        const float cA = mA == -INFINITY ? 0.0f : mA;
                        const float cB = mB == -INFINITY ? 0.0f : mB;
                        float sum = 0.0f;
#pragma unroll
                        for (int j = 0; j < J; ++j) {
                            if (j == b) {
                                sA = sum;
                                sum = 0.0f;
                            }
                            const float c = j < b ? cA : cB;
                            sum += (__builtin_amdgcn_exp2f(v[4 * j] - c) +
                                    __builtin_amdgcn_exp2f(v[4 * j + 1] - c)) +
                                   (__builtin_amdgcn_exp2f(v[4 * j + 2] - c) +
                                    __builtin_amdgcn_exp2f(v[4 * j + 3] - c));
                        }
                        sB = one ? 0.0f : sum;
                        sA = one ? sum : sA;
                        rA = mA;
                        rB = mB;
                    } else {
                        T acc = 0, accA = 0;
#pragma unroll
                        for (int j = 0; j < J; ++j) {
                            if (j == b) {
                                accA = acc;
                                acc = 0;
                            }
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const uint32_t wd = offp[2 * j + (u >> 1)];
                                acc = fma(v[4 * j + u], (T)lds_at<G>(slot_addr<BS>(wd, u, hsel)), acc);
                            }
                            if (j & 1) __builtin_amdgcn_sched_barrier(0);
                        }
                        const bool one = b >= J;  // a single segment (selects, see above)
                        rA = one ? acc : accA;
                        rB = one ? (T)0 : acc;
                    }
                }
            };
            work(s_lo);
            for (int sl = s_lo + 2; sl <= s_hi; sl += 2) {
                __syncthreads();  // every wave is done with slices sl - 2, sl - 1
                stage_issue<G, BS>(dsm + (sl & 1) * BUF, xin, (int64_t)sl * SL, gmax);
                if (sl + 1 <= s_hi)
                    stage_issue<G, BS>(dsm + ((sl + 1) & 1) * BUF, xin, (int64_t)(sl + 1) * SL, gmax);
                stage_wait();
                work(sl);
            }
            __syncthreads();  // every slice read: buffer 0 takes the partials
            prev = 0.0;
#pragma unroll
            for (int i = 0; i < PF; ++i) prev += pf[i];
            if (active) {
                partA[tid] = rA;
                partB[tid] = rB;
                if constexpr (PREC == P_LOG) {
                    psA[tid] = sA;
                    psB[tid] = sB;
                }
            }
            __syncthreads();
            // ---- fold, in (slice, lane) order.  First every segment merges its
            // lanes of this pass (one thread a segment, results in buffer 1),
            // then every line merges its segments into its running total.
            float* const segm = (float*)(dsm + BUF);  // log: base-2 (max, sum) per segment
            float* const segs = segm + kMaxPairs;
            double* const sega = (double*)(dsm + BUF);  // linear: sum per segment
            for (int pp = tid; pp < P; pp += BS) {
                const int a0 = qs_l[pp], a1 = qe_l[pp];
                int lo = 1, hi = 0;  // lanes of the segment inside this pass
                if (a1 > a0) {
                    const int L0 = a0 / J, L1 = (a1 - 1) / J;
                    lo = L0 > q * BS ? L0 : q * BS;
                    hi = L1 < q * BS + w - 1 ? L1 : q * BS + w - 1;
                }
                // the segment's first lane holds it in its second slot when it
                // starts inside that lane
                const int Lsecond = a0 % J != 0 ? a0 / J : -1;
                if constexpr (PREC == P_LOG) {
                    float M = -INFINITY;
                    for (int L = lo; L <= hi; ++L) {
                        const int x = L - q * BS;
                        M = fmaxf(M, L == Lsecond ? partB[x] : partA[x]);
                    }
                    float S = 0.0f;
                    if (M != -INFINITY)
                        for (int L = lo; L <= hi; ++L) {
                            const int x = L - q * BS;
                            const bool sec = L == Lsecond;
                            S += (sec ? psB[x] : psA[x]) * __builtin_amdgcn_exp2f((sec ? partB[x] : partA[x]) - M);
                        }
                    segm[pp] = M;
                    segs[pp] = S;
                } else {
                    double a = 0.0;
                    for (int L = lo; L <= hi; ++L) {
                        const int x = L - q * BS;
                        a += (double)(L == Lsecond ? partB[x] : partA[x]);
                    }
                    sega[pp] = a;
                }
            }
            __syncthreads();
            if (tid < nl) {
                if constexpr (PREC == P_LOG) {
                    float M = lm[tid];
                    for (int ss = 0; ss < ns; ++ss) M = fmaxf(M, segm[ss * nl + tid]);
                    if (M != -INFINITY) {
                        float S = ls[tid] * __builtin_amdgcn_exp2f(lm[tid] - M);
                        for (int ss = 0; ss < ns; ++ss)
                            S += segs[ss * nl + tid] * __builtin_amdgcn_exp2f(segm[ss * nl + tid] - M);
                        lm[tid] = M;
                        ls[tid] = S;
                    }
                } else {
                    double a = lacc[tid];
                    for (int ss = 0; ss < ns; ++ss) a += sega[ss * nl + tid];
                    lacc[tid] = a;
                }
            }
        }
        if (total == 0) {
            stage_wait();  // no pass waited for the quad-range copies
            prev = 0.0;
#pragma unroll
            for (int i = 0; i < PF; ++i) prev += pf[i];
        }
        // ---- scaling update of every line of the step
        if (tid < nl) {
            const int64_t line = r0 + tid;
            double w;
            if constexpr (PREC == P_LOG) {
                w = lse2_value(lm[tid], ls[tid]);
            } else {
                w = lacc[tid];
            }
            const LineNew o = line_new<PREC, UOT>(A.role, marginal, t, pn1 > pn0, mg, lmg, A.theta,
                                                  yp, w);
            if (pend_line >= 0) line_store<PREC>(A.yout, A.yg, pend_line, pend_y, st);
            pend_line = line;
            pend_y = o.y;
            res += o.res;
        }
    }
    block_sum2(res, prev, sh);
    if (pend_line >= 0) line_store<PREC>(A.yout, A.yg, pend_line, pend_y, st);
    if (tid == 0) {
        A.partials[blockIdx.x] = res;
        if (blockIdx.x == 0)
            loop_decide(st, A.role, marginal, A.max_iter, A.tol, A.err_hist, t, prev);
    }
}

template <int PREC, int BS>
static hipError_t run_iter(const IterArgs& a, int grid, hipStream_t st) {
    const size_t lds = SliceCfg<BS>::lds;
    if (a.theta != 1.0)
        hipLaunchKernelGGL((k_iterate<PREC, BS, true>), dim3(grid), dim3(BS), lds, st, a);
    else
        hipLaunchKernelGGL((k_iterate<PREC, BS, false>), dim3(grid), dim3(BS), lds, st, a);
    return hipGetLastError();
}

template <int PREC, int BS, bool UOT>
static hipError_t allow_lds() {
    return hipFuncSetAttribute((const void*)&k_iterate<PREC, BS, UOT>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, SliceCfg<BS>::lds);
}

// Resident blocks of k_iterate<PREC, BS> on the current device.
template <int PREC, int BS>
static int resident_blocks() {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)&k_iterate<PREC, BS, true>,
                                                     BS, SliceCfg<BS>::lds) != hipSuccess)
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

// Block size: 1024 threads (64 KB slice buffers) when there are enough lines
// for a block per compute unit, else 256 threads (16 KB slice buffers).
int iterate_block_size(int64_t nlines) { return nlines >= 256 * 256 ? 1024 : 256; }

template <int PREC, int BS>
static void launch_pack(const IterPlan& p, const int64_t* ptr, const int32_t* idx, const void* val,
                        hipStream_t st) {
    hipLaunchKernelGGL((k_pack<PREC, BS>), dim3((unsigned)p.kmax), dim3(256), 0, st, ptr, idx, val, p);
}

template <int PREC>
static void launch_pack_prec(const IterPlan& p, const int64_t* ptr, const int32_t* idx,
                             const void* val, hipStream_t st) {
    if (p.block == 1024)
        launch_pack<PREC, 1024>(p, ptr, idx, val, st);
    else
        launch_pack<PREC, 256>(p, ptr, idx, val, st);
}

hipError_t build_plan(int precision, const IterPlan& p, const int64_t* ptr, const int32_t* idx,
                      const void* val, int64_t nlines, hipStream_t st) {
    if (nlines <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((nlines + 255) / 256);
    const int J = quads_per_lane(precision);
    hipLaunchKernelGGL(k_split, dim3(nb), dim3(256), 0, st, ptr, idx, nlines, p.ns, p.slice,
                       p.split);
    hipError_t e = launch_fill_u32((uint32_t*)p.info, sizeof(PlanInfo) / 4, 0u, st);
    if (e != hipSuccess) return e;
    const int minw1 = min_weight(p.block, p.ns, J);
    hipLaunchKernelGGL(k_plan_quads, dim3(nb), dim3(256), 0, st, p.split, nlines, p.ns, minw1,
                       p.quads, p.info);
    hipLaunchKernelGGL(k_plan_policy, dim3(1), dim3(64), 0, st, nlines, p.block, J, p.ns, minw1,
                       (int64_t)p.grid, p.kmax, p.info);
    hipLaunchKernelGGL(k_plan_weights, dim3(nb), dim3(256), 0, st, p.quads, nlines, p.info,
                       p.weight);
    e = launch_scan(p.weight, nlines, p.wptr, p.scan, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_plan_setup, dim3(1), dim3(64), 0, st, p.wptr, nlines, (int64_t)p.grid,
                       p.kmax, p.info);
    hipLaunchKernelGGL(k_plan_bounds, dim3((unsigned)((nlines + 1 + 255) / 256)), dim3(256), 0, st,
                       p.wptr, nlines, p.info, p.rstart);
    hipLaunchKernelGGL(k_layout, dim3((unsigned)p.kmax), dim3(256), 0, st, p.split, p.ns, J,
                       p.rstart, p.info, p.kmax, p.qs, p.qe, p.steplanes);
    e = launch_scan(p.steplanes, p.kmax, p.stepoff, p.scan, st);
    if (e != hipSuccess) return e;
    if (precision == P_F64)
        launch_pack_prec<P_F64>(p, ptr, idx, val, st);
    else if (precision == P_F32)
        launch_pack_prec<P_F32>(p, ptr, idx, val, st);
    else
        launch_pack_prec<P_LOG>(p, ptr, idx, val, st);
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

__global__ void k_log_vec(const double* __restrict__ in, double* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = log(in[i]);
}

hipError_t launch_log_vec(const double* in, double* out, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_log_vec, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
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
        if (yg) yg[i] = (float)(l * kLog2e);  // base-2 gathered copy
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
