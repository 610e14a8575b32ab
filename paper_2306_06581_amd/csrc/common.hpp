// Device-side helpers shared by the Spar-Sink kernels (gfx950, wave64).
#pragma once

#include "elemfn.hpp"
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ss {

constexpr int kWave = 64;
constexpr double kLog2e = 1.4426950408889634;  // log2(e)
constexpr double kLn2 = 0.6931471805599453;     // ln(2)
constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw, SC 2011).  Each round
// multiplies counter words 0 and 2 by the two Philox multipliers, keeps the
// 64-bit products, and mixes the high halves with words 1/3 and the key; the
// key is bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct Words4 {
    uint32_t w[4];
};

__device__ __forceinline__ Words4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                           uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        // three-input exclusive or in one instruction (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Words4 out;
    out.w[0] = c0;
    out.w[1] = c1;
    out.w[2] = c2;
    out.w[3] = c3;
    return out;
}

// Hash layout of the Poisson mask.  Column j of row i in problem k uses the
// counters (q, i, k, w) with q = (j >> 9) * 64 + (j & 63) and slot
// s = (j >> 6) & 7.  A 48-bit word holds, as its high 16 bits, half s & 1
// (low half first) of output word s >> 1 of the w = 0 call, and as its low
// 32 bits output word s & 3 of the w = 1 + (s >> 2) call; U = bits * 2^-48.
// A wave therefore covers 512 consecutive columns with one call per lane and
// eight ballots.
//
// keep(i, j) = [U < P].  U lies in [h, h + 2^-16 - 2^-48] with h = hi * 2^-16,
// so the 16-bit half alone decides unless P falls inside that interval, which
// happens with probability 2^-16 per entry; only then is the low word drawn.
__device__ __forceinline__ uint32_t coarse_half(const Words4& w, int slot) {
    const int t = slot >> 1;
    const uint32_t x = t == 0 ? w.w[0] : t == 1 ? w.w[1] : t == 2 ? w.w[2] : w.w[3];
    return (slot & 1) ? (x >> 16) : (x & 0xFFFFu);
}

__device__ __forceinline__ bool keep_decision(uint32_t hi, double P, uint32_t q, uint32_t i,
                                              uint32_t k, uint32_t k0, uint32_t k1, int slot) {
    const double h = (double)hi * 0x1p-16;
    if (h >= P) return false;
    if (h + (0x1p-16 - 0x1p-48) < P) return true;
    const Words4 lo = philox10(q, i, k, 1u + (uint32_t)(slot >> 2), k0, k1);
    // a select, not an index: `slot` may be a run-time value
    const int s4 = slot & 3;
    const uint32_t lw = s4 == 0 ? lo.w[0] : s4 == 1 ? lo.w[1] : s4 == 2 ? lo.w[2] : lo.w[3];
    const uint64_t bits = ((uint64_t)hi << 32) | (uint64_t)lw;
    const double U = (double)bits * 0x1p-48;
    return U < P;
}

// Squared Euclidean distance accumulated in coordinate order, each product and
// sum rounded separately (the library is built with FP contraction off).
template <int D>
__device__ __forceinline__ double sqdist(const double* __restrict__ xi, const double* __restrict__ yj,
                                         int d) {
    const int dd = D > 0 ? D : d;
    double t = xi[0] - yj[0];
    double acc = t * t;
#pragma unroll
    for (int k = 1; k < (D > 0 ? D : 1); ++k) {
        const double u = xi[k] - yj[k];
        acc = acc + u * u;
    }
    if (D == 0) {
        for (int k = 1; k < dd; ++k) {
            const double u = xi[k] - yj[k];
            acc = acc + u * u;
        }
    }
    return acc;
}

// C_ij from the squared Euclidean distance c.  Squared Euclidean costs:
// c * scale (scale = 1 / cmax or 1).  Wasserstein-Fisher-Rao (UOT background
// section): C = -log cos_+^2(d / (2 eta)) with d = sqrt(c), evaluated as
// -2 log cos(z), z = sqrt(c) * w, w = 1 / (2 eta), and +inf (K = 0) where
// z >= pi/2.
constexpr int kCostWfr = 2;
constexpr int kCostEuclid = 3;
constexpr double kHalfPi = 1.5707963267948966;

__device__ __forceinline__ double cost_value(double c, int kind, double scale, double w) {
    if (kind == kCostEuclid) return sqrt(c);
    if (kind != kCostWfr) return c * scale;
    const double z = sqrt(c) * w;
    return z >= kHalfPi ? INFINITY : -2.0 * log(cos(z));
}

// cost_value with the specified logarithm and cosine (elemfn.hpp): the form
// used where the cost decides a sampled entry or its stored value.
__device__ __forceinline__ double cost_spec(double c, int kind, double scale, double w) {
    if (kind == kCostEuclid) return sqrt(c);  // correctly rounded
    if (kind != kCostWfr) return c * scale;
    const double z = sqrt(c) * w;
    return z >= kHalfPi ? INFINITY : -2.0 * log_spec(cos_spec(z));
}

// Logarithm and exponential by small tables, for sums that need about 1e-15
// relative, not bit-exactness (the WFR normaliser); the
// tables cost about half the instructions of the table-free specified
// functions.  Per block, in LDS:
//  * log c, c = 2^e m, m in [1, 2): with j the top 7 bits of m's fraction,
//    c_j = 1 + (j + 1/2)/128, ti[j] = 1/c_j rounded and tl[j] = -log ti[j],
//    log c = e ln 2 + tl[j] + log(1 + r), r = m ti[j] - 1 (one fused
//    operation), |r| < 2^-8, log(1 + r) to r^7 (remainder below 1e-20);
//  * e^x = 2^(N/64) e^r, N = rint(64 x / ln 2), r = x - N ln2/64 (the split
//    ln 2 of the specified exponential), |r| <= ln2/128, e^r - 1 to r^6
//    (remainder below 1e-19), 2^(N/64) = 2^(N >> 6) te[N & 63],
//    te[j] = 2^(j/64).
// The tables come from the specified functions (1-3 ulp), so a term is
// within a few 1e-16 relative (a multiple of the logarithm multiplies its error).
struct TabLog {
    double te[64], ti[128], tl[128];
};

__device__ __forceinline__ void tab_log_init(TabLog& T) {
    for (int j = threadIdx.x; j < 64 + 128; j += blockDim.x) {
        if (j < 64) {
            T.te[j] = exp_spec((double)j * (spec::kLn2Hi / 64.0) + (double)j * (spec::kLn2Lo / 64.0));
        } else {
            const int q = j - 64;
            const double inv = 1.0 / (1.0 + ((double)q + 0.5) / 128.0);
            T.ti[q] = inv;
            T.tl[q] = -log_spec(inv);
        }
    }
}

// log c for a normal c > 0.
__device__ __forceinline__ double tab_log(double c, const TabLog& T) {
    const long long b = __double_as_longlong(c);
    const int e = (int)((b >> 52) & 0x7FF) - 1023;
    const int j = (int)((b >> 45) & 127);
    const double m = __longlong_as_double((b & 0x000FFFFFFFFFFFFFLL) | 0x3FF0000000000000LL);
    const double r = fma(m, T.ti[j], -1.0);
    double p = 1.0 / 7;
    p = fma(p, r, -1.0 / 6);
    p = fma(p, r, 1.0 / 5);
    p = fma(p, r, -0.25);
    p = fma(p, r, 1.0 / 3);
    p = fma(p, r, -0.5);
    p = fma(p, r, 1.0);
    const double ed = (double)e;
    return ed * spec::kLn2Hi + (T.tl[j] + (ed * spec::kLn2Lo + r * p));
}

// e^x for -740 <= x <= 0.
__device__ __forceinline__ double tab_exp(double x, const TabLog& T) {
    const double N = rint(x * (64.0 * spec::kLog2e));
    const double r = (x - N * (spec::kLn2Hi / 64.0)) - N * (spec::kLn2Lo / 64.0);
    double p = 1.0 / 720;
    p = fma(p, r, 1.0 / 120);
    p = fma(p, r, 1.0 / 24);
    p = fma(p, r, 1.0 / 6);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    const int n = (int)N;
    const double t = T.te[n & 63];
    return ldexp(fma(t, r * p, t), n >> 6);  // n >> 6 = floor(n / 64)
}

// ---------------------------------------------------------------------------
// Wave and block reductions.  xor-butterflies give every lane the same value
// (IEEE addition is commutative), so the results are deterministic.
// ---------------------------------------------------------------------------
template <int WIDTH, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int off = WIDTH / 2; off >= 1; off >>= 1) v = v + __shfl_xor(v, off, WIDTH);
    return v;
}

template <int WIDTH, typename T>
__device__ __forceinline__ T group_max(T v) {
#pragma unroll
    for (int off = WIDTH / 2; off >= 1; off >>= 1) {
        const T o = __shfl_xor(v, off, WIDTH);
        v = o > v ? o : v;
    }
    return v;
}

// Sum over a 256-thread block in a fixed tree; result valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double* sh) {
    v = group_sum<kWave>(v);
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return r;
}

// Sum over a block of any size (up to 16 waves) in a fixed tree; result valid
// in every thread.  sh: at least 16 doubles of LDS.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = group_sum<kWave>(v);
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < nw; ++w) r += sh[w];
    return r;
}

// Block barrier that orders LDS only: waits for this wave's LDS (and scalar
// memory) operations, not for its global stores (s_waitcnt lgkmcnt(0) with
// vmcnt and expcnt at their maxima, then s_barrier; the empty asm statements
// keep the compiler from moving memory operations across it).
__device__ __forceinline__ void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Two sums over a block in one pass, each in the tree of block_sum; results
// valid in every thread.  sh: at least 32 doubles of LDS.  The barriers order
// LDS only, so global stores still in flight do not delay the sums.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
    a = group_sum<kWave>(a);
    b = group_sum<kWave>(b);
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    lds_barrier();
    if (lane == 0) {
        sh[wv] = a;
        sh[16 + wv] = b;
    }
    lds_barrier();
    a = 0.0;
    b = 0.0;
    for (int w = 0; w < nw; ++w) {
        a += sh[w];
        b += sh[16 + w];
    }
}

__device__ __forceinline__ int block_max_int(int v, int* sh) {
    v = group_max<kWave>(v);
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    int r = sh[0];
    for (int w = 1; w < nw; ++w) r = sh[w] > r ? sh[w] : r;
    return r;
}

// Inclusive prefix sum of an int over the wave.
__device__ __forceinline__ int wave_inclusive_scan(int v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int o = __shfl_up(v, off, kWave);
        if (lane >= off) v += o;
    }
    return v;
}

// Relaxed agent-scope load, used where a block reads values other blocks of
// the same launch wrote (last-block reductions).
__device__ __forceinline__ double load_agent(const double* p) {
    const unsigned long long bits =
        __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)bits);
}

__device__ __forceinline__ void store_agent(double* p, double v) {
    __hip_atomic_store((unsigned long long*)p, (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace ss
