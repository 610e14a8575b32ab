// Sampling stage of Spar-Sink (step 1 of Alg. 3 / Alg. 4):
//   probabilities  eq. (pij-ot) / eq. (pij-uot)
//   Poisson mask   eq. (pois), drawn with a counter-based hash
//   K~ = K / p*    as CSR (from the mask) and CSC (from its bit transpose).
#include <math.h>

#include "common.hpp"
#include "internal.hpp"

namespace ss {

// ------------------------------------------------------------------ basics
__global__ void k_fill_f64(double* p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static inline unsigned grid_for(int64_t n, int block = kBlock) {
    return (unsigned)((n + block - 1) / block);
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}

// Flags a negative or non-finite mass, or a non-finite coordinate.
__global__ void k_validate(const double* a, int64_t n, const double* x, int64_t nx, double* stats) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (i < n) {
        const double v = a[i];
        bad |= !(v >= 0.0) || !isfinite(v);
    }
    if (i < nx) bad |= !isfinite(x[i]);
    if (bad) stats[ST_BAD_INPUT] = 1.0;
}

hipError_t launch_validate(const double* a, int64_t n, const double* x, int64_t nx, double* stats,
                           hipStream_t st) {
    const int64_t t = n > nx ? n : nx;
    if (t <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_validate, dim3(grid_for(t)), dim3(kBlock), 0, st, a, n, x, nx, stats);
    return hipGetLastError();
}

// ------------------------------------------------------------------ tree sum
// Sum of 1024 consecutive elements (zero padded) as a perfect binary tree of
// adjacent pairs.  Chained over levels this is the tree sum of the whole
// zero-padded power-of-two vector, independent of the launch shape.
__global__ __launch_bounds__(256) void k_tree_sum(const double* __restrict__ in, int64_t n,
                                                  double* __restrict__ out) {
    __shared__ double sh[256];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * 1024 + (int64_t)tid * 4;
    double e[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) e[k] = (base + k < n) ? in[base + k] : 0.0;
    sh[tid] = (e[0] + e[1]) + (e[2] + e[3]);
    __syncthreads();
    for (int s = 1; s < 256; s <<= 1) {
        if ((tid & (2 * s - 1)) == 0) sh[tid] = sh[tid] + sh[tid + s];
        __syncthreads();
    }
    if (tid == 0) out[blockIdx.x] = sh[0];
}

// scratch: at least 2 * ceil(n / 1024) doubles.
hipError_t launch_tree_sum(const double* in, int64_t n, double* scratch, double* out,
                           hipStream_t st) {
    if (n <= 1024) {
        hipLaunchKernelGGL(k_tree_sum, dim3(1), dim3(256), 0, st, in, n, out);
        return hipGetLastError();
    }
    int64_t len = (n + 1023) / 1024;
    double* cur = scratch;
    double* other = scratch + len;
    hipLaunchKernelGGL(k_tree_sum, dim3((unsigned)len), dim3(256), 0, st, in, n, cur);
    while (len > 1024) {
        const int64_t nb = (len + 1023) / 1024;
        hipLaunchKernelGGL(k_tree_sum, dim3((unsigned)nb), dim3(256), 0, st, cur, len, other);
        double* t = cur;
        cur = other;
        other = t;
        len = nb;
    }
    hipLaunchKernelGGL(k_tree_sum, dim3(1), dim3(256), 0, st, cur, len, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ cost scale
constexpr int kCostTileCols = 2048;

// max_ij c_ij; non-negative doubles order like their bit patterns.
template <int D>
__global__ __launch_bounds__(256) void k_cmax(const double* __restrict__ x, const double* __restrict__ y,
                                              int64_t n, int64_t m, int d, int64_t ncol_tiles,
                                              double* stats) {
    const int64_t rt = blockIdx.x / ncol_tiles, ct = blockIdx.x % ncol_tiles;
    const int64_t i = rt * 256 + threadIdx.x;
    const int64_t j0 = ct * kCostTileCols;
    const int64_t j1 = (j0 + kCostTileCols < m) ? j0 + kCostTileCols : m;
    double mx = 0.0;
    if (i < n) {
        double xi[D > 0 ? D : 1];
        const double* xp = x + i * d;
        if (D > 0) {
#pragma unroll
            for (int k = 0; k < (D > 0 ? D : 1); ++k) xi[k] = xp[k];
        }
        for (int64_t j = j0; j < j1; ++j) {
            const double c = sqdist<D>(D > 0 ? xi : xp, y + j * d, d);
            mx = c > mx ? c : mx;
        }
    }
    mx = group_max<kWave>(mx);
    if ((threadIdx.x & (kWave - 1)) == 0)
        atomicMax((unsigned long long*)&stats[ST_CMAX], (unsigned long long)__double_as_longlong(mx));
}

#define SS_DISPATCH_D(d, KERNEL, ...)                         \
    do {                                                      \
        switch (d) {                                          \
            case 2: KERNEL<2>(__VA_ARGS__); break;            \
            case 3: KERNEL<3>(__VA_ARGS__); break;            \
            case 10: KERNEL<10>(__VA_ARGS__); break;          \
            default: KERNEL<0>(__VA_ARGS__); break;           \
        }                                                     \
    } while (0)

template <int D>
static void run_cmax(const double* x, const double* y, int64_t n, int64_t m, int d, double* stats,
                     hipStream_t st) {
    const int64_t nct = (m + kCostTileCols - 1) / kCostTileCols;
    const int64_t nrt = (n + 255) / 256;
    hipLaunchKernelGGL(k_cmax<D>, dim3((unsigned)(nct * nrt)), dim3(256), 0, st, x, y, n, m, d, nct,
                       stats);
}

hipError_t launch_cmax(const double* x, const double* y, int64_t n, int64_t m, int d,
                       double* stats, hipStream_t st) {
    SS_DISPATCH_D(d, run_cmax, x, y, n, m, d, stats, st);
    return hipGetLastError();
}

// ------------------------------------------------------------------ OT prep
__global__ void k_sqrt2(const double* a, const double* b, int64_t n, int64_t m, double* ra,
                        double* rb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ra[i] = sqrt(a[i]);
    if (i < m) rb[i] = sqrt(b[i]);
}

// alpha_i = kappa sqrt(a_i), kappa = s / (S_a S_b)   (eq. (pij-ot) times s).
__global__ void k_alpha(double* ra, int64_t n, double s, const double* stats) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double kappa = s / (stats[ST_SA] * stats[ST_SB]);
    if (i < n) ra[i] = kappa * ra[i];
}

hipError_t launch_ot_prep(const double* a, const double* b, int64_t n, int64_t m, double s,
                          double* ra, double* rb, double* scratch, double* stats,
                          hipStream_t st) {
    const int64_t t = n > m ? n : m;
    hipLaunchKernelGGL(k_sqrt2, dim3(grid_for(t)), dim3(kBlock), 0, st, a, b, n, m, ra, rb);
    hipError_t e = launch_tree_sum(ra, n, scratch, stats + ST_SA, st);
    if (e != hipSuccess) return e;
    e = launch_tree_sum(rb, m, scratch, stats + ST_SB, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_alpha, dim3(grid_for(n)), dim3(kBlock), 0, st, ra, n, s, stats);
    return hipGetLastError();
}

// ------------------------------------------------------------------ UOT prep
// la_i = th_u log a_i, lb_j = th_u log b_j (th_u = lam/(2lam+eps)); ea_i = exp(la_i).
__global__ void k_uot_logs(const double* a, const double* b, int64_t n, int64_t m, double thu,
                           double* la, double* lb, double* ea) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double l = thu * log(a[i]);
        la[i] = l;
        ea[i] = exp(l);
    }
    if (i < m) lb[i] = thu * log(b[i]);
}

hipError_t launch_uot_prep(const double* a, const double* b, int64_t n, int64_t m, double lam,
                           double eps, double* la, double* lb, double* ea, hipStream_t st) {
    const double thu = lam / (2.0 * lam + eps);
    const int64_t t = n > m ? n : m;
    hipLaunchKernelGGL(k_uot_logs, dim3(grid_for(t)), dim3(kBlock), 0, st, a, b, n, m, thu, la, lb,
                       ea);
    return hipGetLastError();
}

// q_ij = exp((la_i + lb_j) - (c_ij inv_cmax) inv_tau): eq. (pij-uot) numerator.
template <int D>
__device__ __forceinline__ double uot_q(const ProbParams& pp, const double* xi, int64_t i,
                                        int64_t j) {
    const double c = sqdist<D>(xi, pp.y + j * pp.d, pp.d);
    const double C = c * pp.inv_cmax;
    return exp((pp.row_fac[i] + pp.col_fac[j]) - C * pp.inv_tau);
}

// Z = sum_ij q_ij: per-thread sums over a column tile in column order, a fixed
// block tree, then the tree sum of the block partials.
template <int D>
__global__ __launch_bounds__(256) void k_uot_z(ProbParams pp, int64_t n, int64_t m, int64_t ncol_tiles,
                                               double* partials) {
    __shared__ double sh[4];
    const int64_t rt = blockIdx.x / ncol_tiles, ct = blockIdx.x % ncol_tiles;
    const int64_t i = rt * 256 + threadIdx.x;
    const int64_t j0 = ct * kCostTileCols;
    const int64_t j1 = (j0 + kCostTileCols < m) ? j0 + kCostTileCols : m;
    double acc = 0.0;
    if (i < n) {
        const double* xp = pp.x + i * pp.d;
        double xi[D > 0 ? D : 1];
        if (D > 0) {
#pragma unroll
            for (int k = 0; k < (D > 0 ? D : 1); ++k) xi[k] = xp[k];
        }
        const double la = pp.row_fac[i];
        for (int64_t j = j0; j < j1; ++j) {
            const double c = sqdist<D>(D > 0 ? xi : xp, pp.y + j * pp.d, pp.d);
            const double C = c * pp.inv_cmax;
            acc = acc + exp((la + pp.col_fac[j]) - C * pp.inv_tau);
        }
    }
    const double tot = block_sum256(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

template <int D>
static void run_uot_z(const ProbParams& pp, int64_t n, int64_t m, double* partials, int64_t nct,
                      int64_t nrt, hipStream_t st) {
    hipLaunchKernelGGL(k_uot_z<D>, dim3((unsigned)(nct * nrt)), dim3(256), 0, st, pp, n, m, nct,
                       partials);
}

hipError_t launch_uot_z(const ProbParams& pp, int64_t n, int64_t m, double* partials,
                        double* scratch, double* stats, hipStream_t st) {
    const int64_t nct = (m + kCostTileCols - 1) / kCostTileCols;
    const int64_t nrt = (n + 255) / 256;
    SS_DISPATCH_D(pp.d, run_uot_z, pp, n, m, partials, nct, nrt, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_tree_sum(partials, nct * nrt, scratch, stats + ST_Z, st);
}

// Column factor of a rigorous upper bound on p*: for every (i, j),
// p*_ij <= ea_i * fb_j with fb_j = (s/Z) exp(lb_j) (1 + 2^-30); the margin
// covers the rounding of the sum, exponential and products (all < 1e-12).
__global__ void k_uot_bounds(const double* lb, int64_t m, double s, const double* stats,
                             double* fb) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const double kappa = s / stats[ST_Z];
    fb[j] = kappa * exp(lb[j]) * (1.0 + 0x1p-30);
}

hipError_t launch_uot_bounds(const double* lb, int64_t m, double s, const double* stats,
                             double* fb, hipStream_t st) {
    hipLaunchKernelGGL(k_uot_bounds, dim3(grid_for(m)), dim3(kBlock), 0, st, lb, m, s, stats, fb);
    return hipGetLastError();
}

// ------------------------------------------------------------------ mask
// Block tile: 16 rows x 64 mask words (4096 columns).  Wave w owns hash
// groups 4w..4w+3 of the tile (one Philox call per lane per group and row)
// and keeps its 16 column factors in registers while it walks the 16 rows.
constexpr int kMaskRows = 16;

template <bool UOT, int D>
__global__ __launch_bounds__(256) void k_mask(ProbParams pp, int64_t n, int64_t m, int64_t W,
                                              int64_t ncol_tiles, uint64_t* __restrict__ mask,
                                              int32_t* __restrict__ row_cnt,
                                              const double* __restrict__ stats) {
    __shared__ uint64_t tile[kMaskRows][64];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    const int64_t rt = blockIdx.x / ncol_tiles, ct = blockIdx.x % ncol_tiles;
    const int64_t row0 = rt * kMaskRows;
    const double kappa = UOT ? pp.s / stats[ST_Z] : 0.0;

    double cf[16];
#pragma unroll
    for (int gg = 0; gg < 4; ++gg) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int64_t g = ct * 16 + wv * 4 + gg;
            const int64_t j = 256 * g + 64 * s + lane;
            cf[gg * 4 + s] = (j < m) ? (UOT ? pp.col_bnd[j] : pp.col_fac[j]) : 0.0;
        }
    }
    for (int r = 0; r < kMaskRows; ++r) {
        const int64_t i = row0 + r;
        if (i >= n) break;
        const double rowf = UOT ? pp.row_bnd[i] : pp.row_fac[i];
        uint64_t mine = 0;
#pragma unroll
        for (int gg = 0; gg < 4; ++gg) {
            const int64_t g = ct * 16 + wv * 4 + gg;
            if (4 * g >= W) continue;
            const uint32_t q = (uint32_t)(g * 64 + lane);
            const Words4 h = philox10(q, (uint32_t)i, pp.problem_index, 0u, pp.k0, pp.k1);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int64_t j = 256 * g + 64 * s + lane;
                bool keep = false;
                if (j < m) {
                    const double P = rowf * cf[gg * 4 + s];
                    if (!UOT) {
                        keep = keep_decision(h.w[s], P, q, (uint32_t)i, pp.problem_index, pp.k0,
                                             pp.k1, s);
                    } else if ((double)h.w[s] * 0x1p-32 < P) {
                        // P is an upper bound; only candidates pay for the exact p*.
                        const double q_ij = uot_q<D>(pp, pp.x + i * pp.d, i, j);
                        const double pst = fmin(1.0, kappa * q_ij);
                        keep = keep_decision(h.w[s], pst, q, (uint32_t)i, pp.problem_index, pp.k0,
                                             pp.k1, s);
                    }
                }
                const uint64_t word = __ballot(keep);
                if (lane == gg * 4 + s) mine = word;
            }
        }
        if (lane < 16) tile[r][wv * 16 + lane] = mine;
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < kMaskRows / 4; ++rr) {
        const int r = wv + 4 * rr;
        const int64_t i = row0 + r;
        if (i >= n) continue;
        const int64_t widx = ct * 64 + lane;
        const uint64_t w = tile[r][lane];
        if (widx < W) mask[i * W + widx] = w;
        int c = (widx < W) ? __popcll(w) : 0;
        c = group_sum<kWave>(c);
        if (lane == 0 && c) atomicAdd(&row_cnt[i], c);
    }
}

template <bool UOT, int D>
static void run_mask(const ProbParams& pp, int64_t n, int64_t m, uint64_t* mask, int32_t* row_cnt,
                     const double* stats, hipStream_t st) {
    const int64_t W = (m + 63) / 64;
    const int64_t nct = (W + 63) / 64;
    const int64_t nrt = (n + kMaskRows - 1) / kMaskRows;
    hipLaunchKernelGGL((k_mask<UOT, D>), dim3((unsigned)(nct * nrt)), dim3(256), 0, st, pp, n, m, W,
                       nct, mask, row_cnt, stats);
}

template <int D>
static void run_mask_d(const ProbParams& pp, int64_t n, int64_t m, uint64_t* mask,
                       int32_t* row_cnt, const double* stats, hipStream_t st) {
    if (pp.uot)
        run_mask<true, D>(pp, n, m, mask, row_cnt, stats, st);
    else
        run_mask<false, 2>(pp, n, m, mask, row_cnt, stats, st);  // OT never reads coordinates
}

hipError_t launch_mask(const ProbParams& pp, int64_t n, int64_t m, uint64_t* mask,
                       int32_t* row_cnt, const double* stats, hipStream_t st) {
    SS_DISPATCH_D(pp.d, run_mask_d, pp, n, m, mask, row_cnt, stats, st);
    return hipGetLastError();
}

// ------------------------------------------------------------------ transpose
// 64 x 64 bit-matrix transpose across a wave: lane r holds row r (bit c =
// column c); afterwards lane c holds column c (bit r = row r).  Six butterfly
// stages exchange blocks of 32, 16, ..., 1 bits with lane r ^ s.
__device__ __forceinline__ uint64_t transpose64(uint64_t w) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t M[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                           0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int s = 32 >> k;
        const uint64_t p = __shfl_xor(w, s, kWave);
        if ((lane & s) == 0)
            w = (w & M[k]) | ((p & M[k]) << s);
        else
            w = ((p >> s) & M[k]) | (w & ~M[k]);
    }
    return w;
}

constexpr int kTrRowBlocks = 8;   // 64-row blocks per tile
constexpr int kTrWordCols = 16;   // mask word columns per tile

__global__ __launch_bounds__(256) void k_transpose(const uint64_t* __restrict__ mask, int64_t n,
                                                   int64_t m, int64_t W, int64_t Wn,
                                                   int64_t ncol_tiles, uint64_t* __restrict__ maskT,
                                                   int32_t* __restrict__ col_cnt) {
    __shared__ uint64_t tile[64][kTrWordCols + 1];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    const int64_t rt = blockIdx.x / ncol_tiles, ct = blockIdx.x % ncol_tiles;
    uint64_t out[4][kTrRowBlocks];
    const int lr = threadIdx.x >> 2;          // row of the tile this thread loads
    const int lq = (threadIdx.x & 3) * 4;     // first of its 4 words
#pragma unroll
    for (int rho = 0; rho < kTrRowBlocks; ++rho) {
        const int64_t I = rt * kTrRowBlocks + rho;
        const int64_t i = 64 * I + lr;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t wc = ct * kTrWordCols + lq + q;
            tile[lr][lq + q] = (I < Wn && i < n && wc < W) ? mask[i * W + wc] : 0ull;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) out[k][rho] = transpose64(tile[lane][wv * 4 + k]);
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t wc = ct * kTrWordCols + wv * 4 + k;
        const int64_t j = 64 * wc + lane;
        if (j >= m) continue;
        int cnt = 0;
#pragma unroll
        for (int rho = 0; rho < kTrRowBlocks; ++rho) {
            const int64_t I = rt * kTrRowBlocks + rho;
            if (I < Wn) {
                maskT[j * Wn + I] = out[k][rho];
                cnt += __popcll(out[k][rho]);
            }
        }
        if (cnt) atomicAdd(&col_cnt[j], cnt);
    }
}

hipError_t launch_transpose(const uint64_t* mask, int64_t n, int64_t m, uint64_t* maskT,
                            int32_t* col_cnt, hipStream_t st) {
    const int64_t W = (m + 63) / 64, Wn = (n + 63) / 64;
    const int64_t nct = (W + kTrWordCols - 1) / kTrWordCols;
    const int64_t nrt = (Wn + kTrRowBlocks - 1) / kTrRowBlocks;
    hipLaunchKernelGGL(k_transpose, dim3((unsigned)(nct * nrt)), dim3(256), 0, st, mask, n, m, W, Wn,
                       nct, maskT, col_cnt);
    return hipGetLastError();
}

// ------------------------------------------------------------------ scan
// Exclusive scan of int32 counts into int64 offsets ptr[0..n], ptr[n] = total.
__device__ __forceinline__ int64_t wave_incl_scan64(int64_t v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int64_t o = __shfl_up(v, off, kWave);
        if (lane >= off) v += o;
    }
    return v;
}

// Exclusive scan over a 256-thread block; *total receives the block total.
__device__ __forceinline__ int64_t block_excl_scan256(int64_t v, int64_t* sh, int64_t* total) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    const int64_t incl = wave_incl_scan64(v);
    __syncthreads();
    if (lane == kWave - 1) sh[wv] = incl;
    __syncthreads();
    int64_t off = 0;
    for (int k = 0; k < wv; ++k) off += sh[k];
    *total = sh[0] + sh[1] + sh[2] + sh[3];
    return off + incl - v;
}

__global__ __launch_bounds__(256) void k_scan_sums(const int32_t* cnt, int64_t n, int64_t* bsum) {
    __shared__ int64_t sh[4];
    const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
    int64_t v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) v += (base + k < n) ? cnt[base + k] : 0;
    int64_t tot;
    block_excl_scan256(v, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// In-place exclusive scan of nb block sums by one block; writes the total to *ptr_end.
__global__ __launch_bounds__(256) void k_scan_top(int64_t* bsum, int64_t nb, int64_t* ptr_end) {
    __shared__ int64_t sh[4];
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t b0 = base + threadIdx.x * 4;
        int64_t e[4], v = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            e[k] = (b0 + k < nb) ? bsum[b0 + k] : 0;
            v += e[k];
        }
        int64_t tot;
        int64_t off = block_excl_scan256(v, sh, &tot) + carry;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (b0 + k < nb) bsum[b0 + k] = off;
            off += e[k];
        }
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *ptr_end = carry;
}

__global__ __launch_bounds__(256) void k_scan_apply(const int32_t* cnt, int64_t n, const int64_t* boff,
                                                    int64_t* ptr) {
    __shared__ int64_t sh[4];
    const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
    int64_t e[4], v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        e[k] = (base + k < n) ? cnt[base + k] : 0;
        v += e[k];
    }
    int64_t tot;
    int64_t off = block_excl_scan256(v, sh, &tot) + boff[blockIdx.x];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < n) ptr[base + k] = off;
        off += e[k];
    }
}

// scratch: ceil(n / 1024) int64.
hipError_t launch_scan(const int32_t* cnt, int64_t n, int64_t* ptr, int64_t* scratch,
                       hipStream_t st) {
    const int64_t nb = (n + 1023) / 1024;
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(256), 0, st, cnt, n, scratch);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, st, scratch, nb, ptr + n);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, st, cnt, n, scratch, ptr);
    return hipGetLastError();
}

// ------------------------------------------------------------------ fill
// Value of K~_ij = K_ij / p*_ij in FP64 (eq. (pois)), K_ij = exp(-C_ij/eps)
// with C recomputed from the coordinates; also its log, -C/eps - log p*.
template <bool UOT, int D>
__device__ __forceinline__ double entry_value(const ProbParams& pp, double kappa, int64_t i,
                                              int64_t j, double* logv) {
    const double c = sqdist<D>(pp.x + i * pp.d, pp.y + j * pp.d, pp.d);
    const double C = c * pp.inv_cmax;
    const double Ce = C / pp.eps;
    const double K = exp(-Ce);
    double P;
    if (UOT)
        P = fmin(1.0, kappa * exp((pp.row_fac[i] + pp.col_fac[j]) - C * pp.inv_tau));
    else
        P = fmin(1.0, pp.row_fac[i] * pp.col_fac[j]);
    *logv = -Ce - log(P);
    return K / P;
}

// One wave per line (row for the CSR, column for the CSC).  Phase 1: a
// prefix-popcount of the line's mask words gives each kept entry its slot, in
// ascending order; the index is written out and queued in LDS.  Phase 2: the
// whole wave computes the queued values, one entry per lane (a line's entries
// are too sparse among its words to keep the lanes busy in phase 1).
constexpr int kFillQueue = 512;

template <int PREC>
__device__ __forceinline__ void store_value(void* val, int64_t pos, double v, double lv) {
    if (PREC == P_F64) ((double*)val)[pos] = v;
    if (PREC == P_F32) ((float*)val)[pos] = (float)v;
    if (PREC == P_LOG) ((float*)val)[pos] = (float)lv;
}

template <int ROLE, bool UOT, int PREC, int D>
__global__ __launch_bounds__(256) void k_fill(ProbParams pp, const double* __restrict__ stats,
                                              const uint64_t* __restrict__ bits, int64_t nlines,
                                              int64_t words, const int64_t* __restrict__ ptr,
                                              int32_t* __restrict__ idx, void* __restrict__ val,
                                              int64_t cap) {
    __shared__ int32_t queue[4][kFillQueue];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    const int64_t line = (int64_t)blockIdx.x * 4 + wv;
    const bool active = line < nlines;
    const double kappa = UOT ? pp.s / stats[ST_Z] : 0.0;
    const uint64_t* row = bits + (active ? line : 0) * words;
    const int64_t base = active ? ptr[line] : 0;
    int64_t run = base;
    for (int64_t w0 = 0; w0 < words; w0 += kWave) {
        const int64_t widx = w0 + lane;
        uint64_t word = (active && widx < words) ? row[widx] : 0ull;
        const int c = __popcll(word);
        const int incl = wave_inclusive_scan(c);
        int64_t pos = run + (incl - c);
        while (word) {
            const int b = __ffsll((unsigned long long)word) - 1;
            word &= word - 1;
            const int64_t other = 64 * widx + b;
            const int64_t local = pos - base;
            if (pos < cap) idx[pos] = (int32_t)other;
            if (local < kFillQueue) {
                queue[wv][local] = (int32_t)other;
            } else if (pos < cap) {
                const int64_t i = ROLE == 0 ? line : other;
                const int64_t j = ROLE == 0 ? other : line;
                double lv;
                const double v = entry_value<UOT, D>(pp, kappa, i, j, &lv);
                store_value<PREC>(val, pos, v, lv);
            }
            ++pos;
        }
        run += __shfl(incl, kWave - 1, kWave);
    }
    __syncthreads();
    const int64_t cnt = run - base;
    const int64_t nq = cnt < kFillQueue ? cnt : kFillQueue;
    for (int64_t e = lane; e < nq; e += kWave) {
        const int64_t pos = base + e;
        if (pos >= cap) break;
        const int64_t other = queue[wv][e];
        const int64_t i = ROLE == 0 ? line : other;
        const int64_t j = ROLE == 0 ? other : line;
        double lv;
        const double v = entry_value<UOT, D>(pp, kappa, i, j, &lv);
        store_value<PREC>(val, pos, v, lv);
    }
}

template <int ROLE, bool UOT, int PREC, int D>
static void run_fill4(const ProbParams& pp, const double* stats, const uint64_t* bits,
                      int64_t nlines, int64_t words, const int64_t* ptr, int32_t* idx, void* val,
                      int64_t cap, hipStream_t st) {
    hipLaunchKernelGGL((k_fill<ROLE, UOT, PREC, D>), dim3((unsigned)((nlines + 3) / 4)), dim3(256),
                       0, st, pp, stats, bits, nlines, words, ptr, idx, val, cap);
}

template <int D>
static void run_fill(int role, int prec, const ProbParams& pp, const double* stats,
                     const uint64_t* bits, int64_t nlines, int64_t words, const int64_t* ptr,
                     int32_t* idx, void* val, int64_t cap, hipStream_t st) {
#define SS_FILL_CASE(R, U, P)                                                                    \
    if (role == R && (pp.uot != 0) == U && prec == P)                                            \
        run_fill4<R, U, P, D>(pp, stats, bits, nlines, words, ptr, idx, val, cap, st);
    SS_FILL_CASE(0, false, P_F64) SS_FILL_CASE(0, false, P_F32) SS_FILL_CASE(0, false, P_LOG)
    SS_FILL_CASE(0, true, P_F64) SS_FILL_CASE(0, true, P_F32) SS_FILL_CASE(0, true, P_LOG)
    SS_FILL_CASE(1, false, P_F64) SS_FILL_CASE(1, false, P_F32) SS_FILL_CASE(1, false, P_LOG)
    SS_FILL_CASE(1, true, P_F64) SS_FILL_CASE(1, true, P_F32) SS_FILL_CASE(1, true, P_LOG)
#undef SS_FILL_CASE
}

hipError_t launch_fill_entries(int role, int precision, const ProbParams& pp, const double* stats,
                               const uint64_t* bits, int64_t nlines, int64_t words,
                               const int64_t* ptr, int32_t* idx, void* val, int64_t cap,
                               hipStream_t st) {
    if (nlines <= 0) return hipSuccess;
    SS_DISPATCH_D(pp.d, run_fill, role, precision, pp, stats, bits, nlines, words, ptr, idx, val,
                  cap, st);
    return hipGetLastError();
}

// ------------------------------------------------------------------ empty lines
// which = 0: rows (a, stats slots *_A / EMPTY_ROWS); 1: columns.
__global__ void k_empty_split(const double* a, const int32_t* cnt, int64_t n, double* act,
                              double* dropped, double* flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool on = cnt[i] > 0;
    act[i] = on ? a[i] : 0.0;
    dropped[i] = on ? 0.0 : a[i];
    flag[i] = (!on && a[i] > 0.0) ? 1.0 : 0.0;
}

__global__ void k_scale_by(const double* in, int64_t n, const double* den, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i] / *den;
}

__global__ void k_copy_f64(const double* in, int64_t n, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}

// tmp: 2n doubles; scratch: tree-sum scratch.
hipError_t launch_empty_policy(const double* a, const int32_t* cnt, int64_t n, int renormalize,
                               int which, double* a_eff, double* tmp, double* scratch,
                               double* stats, hipStream_t st) {
    double* dropped = tmp;
    double* flag = tmp + n;
    hipLaunchKernelGGL(k_empty_split, dim3(grid_for(n)), dim3(kBlock), 0, st, a, cnt, n, a_eff,
                       dropped, flag);
    const int s_act = which == 0 ? ST_SUM_A_ACTIVE : ST_SUM_B_ACTIVE;
    const int s_drop = which == 0 ? ST_DROPPED_A : ST_DROPPED_B;
    const int s_flag = which == 0 ? ST_EMPTY_ROWS : ST_EMPTY_COLS;
    hipError_t e = launch_tree_sum(a_eff, n, scratch, stats + s_act, st);
    if (e == hipSuccess) e = launch_tree_sum(dropped, n, scratch, stats + s_drop, st);
    if (e == hipSuccess) e = launch_tree_sum(flag, n, scratch, stats + s_flag, st);
    if (e != hipSuccess) return e;
    if (renormalize)
        hipLaunchKernelGGL(k_scale_by, dim3(grid_for(n)), dim3(kBlock), 0, st, a_eff, n,
                           stats + s_act, a_eff);
    return hipGetLastError();
}

}  // namespace ss
