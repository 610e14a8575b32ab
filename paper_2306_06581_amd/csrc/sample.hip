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
//
// Exact pruning: with a centre c and R = max_j |y_j - c|, the triangle
// inequality bounds row i by ub_i = (|x_i - c| + R)^2 >= max_j c_ij (a
// relative margin of 1e-9 covers the rounding of every term for d <= 64).
// The full row of the x point farthest from c gives a lower bound L0 on the
// maximum, so only rows with ub_i >= L0 can hold it; those rows are scanned
// with the same distance code as the brute-force maximum, so the result is
// that maximum, bit for bit.  Clouds without such structure leave every row
// a survivor and cost one brute-force pass.
constexpr int kCenterPoints = 16384;  // the centre is the mean of the first points of y

struct CmaxScratch {
    double center[64];
    unsigned long long r2;   // max_j |y_j - c|^2 as bits
    unsigned long long far;  // (float bits of |x_i - c|^2) << 32 | i, maximised
    int count;               // survivor rows
    int pad;
};

__device__ __forceinline__ double center_sqdist(const double* p, const double* c, int d) {
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
        const double u = p[k] - c[k];
        acc = acc + u * u;
    }
    return acc;
}

__global__ __launch_bounds__(256) void k_cm_center(const double* __restrict__ y, int64_t m, int d,
                                                   CmaxScratch* cs) {
    __shared__ double sh[16];
    const int64_t np = m < kCenterPoints ? m : kCenterPoints;
    for (int k = 0; k < d; ++k) {
        double acc = 0.0;
        for (int64_t j = threadIdx.x; j < np; j += blockDim.x) acc += y[j * d + k];
        acc = block_sum(acc, sh);
        if (threadIdx.x == 0) cs->center[k] = acc / (double)np;
    }
    if (threadIdx.x == 0) {
        cs->r2 = 0ull;
        cs->far = 0ull;
        cs->count = 0;
    }
}

__global__ __launch_bounds__(256) void k_cm_radius(const double* __restrict__ y, int64_t m, int d,
                                                   CmaxScratch* cs) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double r2 = j < m ? center_sqdist(y + j * d, cs->center, d) : 0.0;
    r2 = group_max<kWave>(r2);
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(&cs->r2, (unsigned long long)__double_as_longlong(r2));
}

__global__ __launch_bounds__(256) void k_cm_far(const double* __restrict__ x, int64_t n, int d,
                                                CmaxScratch* cs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long key = 0ull;
    if (i < n) {
        const float d2 = (float)center_sqdist(x + i * d, cs->center, d);
        key = ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned long long)i;
    }
    key = group_max<kWave>(key);
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(&cs->far, key);
}

// Lower bound: the full row of the farthest x point, into stats[ST_CMAX].
template <int D>
__global__ __launch_bounds__(256) void k_cm_row(const double* __restrict__ x, const double* __restrict__ y,
                                                int64_t m, int d, const CmaxScratch* cs,
                                                double* stats) {
    const int64_t i = (int64_t)(cs->far & 0xffffffffull);
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double mx = j < m ? sqdist<D>(x + i * d, y + j * d, d) : 0.0;
    mx = group_max<kWave>(mx);
    if ((threadIdx.x & (kWave - 1)) == 0)
        atomicMax((unsigned long long*)&stats[ST_CMAX], (unsigned long long)__double_as_longlong(mx));
}

// Rows whose bound reaches the lower bound.
__global__ __launch_bounds__(256) void k_cm_survivors(const double* __restrict__ x, int64_t n, int d,
                                                      CmaxScratch* cs, const double* stats,
                                                      int32_t* __restrict__ rows) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double R = sqrt(__longlong_as_double((long long)cs->r2));
    const double di = sqrt(center_sqdist(x + i * d, cs->center, d));
    const double ub = (di + R) * (di + R) * (1.0 + 1e-9);
    if (ub >= stats[ST_CMAX] && i != (int64_t)(cs->far & 0xffffffffull))
        rows[atomicAdd(&cs->count, 1)] = (int32_t)i;
}

// Maximum over the survivor rows: items (64 survivor rows, 256 columns),
// grid-stride; the item's rows go to LDS, thread = column, rows in order.  The
// distance is the brute-force one, sqdist(x_i, y_j).
constexpr int kCmaxRows = 64;

template <int D>
__global__ __launch_bounds__(256) void k_cmax_rows(const double* __restrict__ x, const double* __restrict__ y,
                                                   int64_t m, int d, const int32_t* __restrict__ rows,
                                                   const CmaxScratch* cs, double* stats) {
    __shared__ double xr[kCmaxRows * 64];  // d <= 64
    const int64_t ncc = (m + 255) / 256;
    const int64_t count = cs->count;
    const int64_t items = (count + kCmaxRows - 1) / kCmaxRows * ncc;
    double mx = 0.0;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int64_t rg = it / ncc, cc = it - rg * ncc;
        const int64_t s0 = rg * kCmaxRows;
        const int nr = (int)(count - s0 < kCmaxRows ? count - s0 : kCmaxRows);
        __syncthreads();  // the previous item's rows are no longer read
        for (int t = threadIdx.x; t < nr * d; t += blockDim.x)
            xr[t] = x[(int64_t)rows[s0 + t / d] * d + t % d];
        __syncthreads();
        const int64_t j = cc * 256 + threadIdx.x;
        if (j < m) {
            const double* yj = y + j * d;
            for (int r = 0; r < nr; ++r) {
                const double c = sqdist<D>(xr + r * d, yj, d);
                mx = c > mx ? c : mx;
            }
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
            case 5: KERNEL<5>(__VA_ARGS__); break;            \
            case 10: KERNEL<10>(__VA_ARGS__); break;          \
            default: KERNEL<0>(__VA_ARGS__); break;           \
        }                                                     \
    } while (0)

template <int D>
static void run_cmax(const double* x, const double* y, int64_t n, int64_t m, int d, double* stats,
                     CmaxScratch* cs, int32_t* rows, hipStream_t st) {
    hipLaunchKernelGGL(k_cm_row<D>, dim3(grid_for(m)), dim3(256), 0, st, x, y, m, d, cs, stats);
    hipLaunchKernelGGL(k_cm_survivors, dim3(grid_for(n)), dim3(256), 0, st, x, n, d, cs, stats,
                       rows);
    hipLaunchKernelGGL(k_cmax_rows<D>, dim3(1024), dim3(256), 0, st, x, y, m, d, rows, cs, stats);
}

hipError_t launch_cmax(const double* x, const double* y, int64_t n, int64_t m, int d,
                       double* stats, void* scratch, hipStream_t st) {
    CmaxScratch* cs = (CmaxScratch*)scratch;
    int32_t* rows = (int32_t*)(cs + 1);
    hipLaunchKernelGGL(k_cm_center, dim3(1), dim3(256), 0, st, y, m, d, cs);
    hipLaunchKernelGGL(k_cm_radius, dim3(grid_for(m)), dim3(256), 0, st, y, m, d, cs);
    hipLaunchKernelGGL(k_cm_far, dim3(grid_for(n)), dim3(256), 0, st, x, n, d, cs);
    SS_DISPATCH_D(d, run_cmax, x, y, n, m, d, stats, cs, rows, st);
    return hipGetLastError();
}

size_t cmax_scratch_bytes(int64_t n) { return sizeof(CmaxScratch) + (size_t)n * 4; }

// ------------------------------------------------------------------ OT prep
__global__ void k_sqrt2(const double* a, const double* b, int64_t n, int64_t m, double* ra,
                        double* rb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ra[i] = sqrt(a[i]);
    if (i < m) rb[i] = sqrt(b[i]);
}

// alpha_i = kappa sqrt(a_i), kappa = s / (S_a S_b)   (eq. (pij-ot) times s).
// With shrinkage (Sec. 4) the factor carries the weight 1 - g of eq. (pij-ot).
__global__ void k_alpha(double* ra, int64_t n, double s, double w, const double* stats) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double kappa = s / (stats[ST_SA] * stats[ST_SB]);
    if (i < n) ra[i] = (kappa * ra[i]) * w;
}

hipError_t launch_ot_prep(const double* a, const double* b, int64_t n, int64_t m, double s,
                          double shrink_w, double* ra, double* rb, double* scratch,
                          double* stats, hipStream_t st) {
    const int64_t t = n > m ? n : m;
    hipLaunchKernelGGL(k_sqrt2, dim3(grid_for(t)), dim3(kBlock), 0, st, a, b, n, m, ra, rb);
    hipError_t e = launch_tree_sum(ra, n, scratch, stats + ST_SA, st);
    if (e != hipSuccess) return e;
    e = launch_tree_sum(rb, m, scratch, stats + ST_SB, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_alpha, dim3(grid_for(n)), dim3(kBlock), 0, st, ra, n, s, shrink_w, stats);
    return hipGetLastError();
}

// ------------------------------------------------------------------ UOT prep
// la_i = th_u log a_i, lb_j = th_u log b_j (th_u = lam/(2lam+eps)); ea_i = exp(la_i),
// eb_j = exp(lb_j); with the specified logarithm and exponential (elemfn.hpp),
// since la and lb enter the keep decisions.
__global__ void k_uot_logs(const double* a, const double* b, int64_t n, int64_t m, double thu,
                           double* la, double* lb, double* ea, double* eb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double l = thu * log_spec(a[i]);
        la[i] = l;
        ea[i] = exp_spec(l);
    }
    if (i < m) {
        const double l = thu * log_spec(b[i]);
        lb[i] = l;
        eb[i] = exp_spec(l);
    }
}

hipError_t launch_uot_prep(const double* a, const double* b, int64_t n, int64_t m, double lam,
                           double eps, double* la, double* lb, double* ea, double* eb,
                           hipStream_t st) {
    const double thu = lam / (2.0 * lam + eps);
    const int64_t t = n > m ? n : m;
    hipLaunchKernelGGL(k_uot_logs, dim3(grid_for(t)), dim3(kBlock), 0, st, a, b, n, m, thu, la, lb,
                       ea, eb);
    return hipGetLastError();
}

// q_ij = exp((la_i + lb_j) - C_ij inv_tau): eq. (pij-uot) numerator, from the
// squared distance c_ij, with the specified exponential and cost (it decides
// the entry).
__device__ __forceinline__ double uot_q_of(const ProbParams& pp, double c, int64_t i, int64_t j) {
    const double C = cost_spec(c, pp.cost, pp.inv_cmax, pp.wfr_w);
    return exp_spec((pp.row_fac[i] + pp.col_fac[j]) - C * pp.inv_tau);
}

// The cost factor exp(-C_ij inv_tau) of q_ij bounded from above by 2^(-t) with
// t from the squared distance alone: t = c inv_cmax inv_tau log2(e) for the
// squared Euclidean costs (equality), and for WFR, where cos z <= exp(-z^2/2)
// on [0, pi/2], cos(z)^(2 inv_tau) <= exp(-z^2 inv_tau) with z^2 = c w^2;
// t = +inf where z is surely past pi/2 (blocked: q = 0).
__device__ __forceinline__ double uot_bound_exponent(const ProbParams& pp, double c) {
    if (pp.cost == kCostWfr) {
        const double z2 = c * (pp.wfr_w * pp.wfr_w);
        if (z2 >= (kHalfPi * kHalfPi) * (1.0 + 1e-12)) return INFINITY;
        return z2 * pp.inv_tau * kLog2e;
    }
    return c * (pp.inv_cmax * pp.inv_tau) * kLog2e;
}

// Z = sum_ij q_ij: per-thread sums over a column tile in column order, a fixed
// block tree, then the tree sum of the block partials.
//
// SHORT (g = inv_cmax inv_tau with g max c <= 1/2): q_ij = ea_i eb_j
// exp(-g c_ij), and exp(-g c) = e^(-1/4) e^u with u = 1/4 - g c in
// [-1/4, 1/4] is a degree-11 Taylor polynomial in u (truncation below
// 1.6e-16 relative), so no range reduction is needed: 12 fused multiply-adds
// a pair instead of a general exponential.
template <int D, bool SHORT>
__global__ __launch_bounds__(256) void k_uot_z(ProbParams pp, int64_t n, int64_t m, int64_t ncol_tiles,
                                               const double* __restrict__ eb, double g,
                                               double e_quarter, double* partials) {
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
        if constexpr (SHORT) {
            // 1/k!, k = 0..11
            constexpr double f0 = 1.0, f1 = 1.0, f2 = 1.0 / 2, f3 = 1.0 / 6, f4 = 1.0 / 24,
                             f5 = 1.0 / 120, f6 = 1.0 / 720, f7 = 1.0 / 5040, f8 = 1.0 / 40320,
                             f9 = 1.0 / 362880, f10 = 1.0 / 3628800, f11 = 1.0 / 39916800;
            for (int64_t j = j0; j < j1; ++j) {
                const double c = sqdist<D>(D > 0 ? xi : xp, pp.y + j * pp.d, pp.d);
                const double u = fma(-g, c, 0.25);
                double p = f11;
                p = fma(p, u, f10);
                p = fma(p, u, f9);
                p = fma(p, u, f8);
                p = fma(p, u, f7);
                p = fma(p, u, f6);
                p = fma(p, u, f5);
                p = fma(p, u, f4);
                p = fma(p, u, f3);
                p = fma(p, u, f2);
                p = fma(p, u, f1);
                p = fma(p, u, f0);
                acc = fma(p, eb[j], acc);
            }
            acc = acc * (pp.row_bnd[i] * e_quarter);
        } else {
            const double la = pp.row_fac[i];
            for (int64_t j = j0; j < j1; ++j) {
                const double c = sqdist<D>(D > 0 ? xi : xp, pp.y + j * pp.d, pp.d);
                const double C = cost_value(c, pp.cost, pp.inv_cmax, pp.wfr_w);
                acc = acc + exp((la + pp.col_fac[j]) - C * pp.inv_tau);
            }
        }
    }
    const double tot = block_sum256(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// WFR: q = ea eb cos(z)^(2 inv_tau) (ea = exp(la), eb = exp(lb)), cos z from its Taylor series in
// t = z^2 = c w^2 < (pi/2)^2 up to t^11 (truncation below 1e-19; no square
// root, no range reduction).  Blocked pairs (z >= pi/2) add nothing, and
// neither does a pair whose series rounds to <= 0.  Most pairs are blocked,
// so the pairs that are not are compacted before the logarithm and
// exponential: each wave scans its 64 rows against the tile's columns one
// column at a time, appends the unblocked pairs (t and the weight ea eb) to
// its own LDS queue in lane order (a ballot and prefix count: a fixed order),
// and whenever 64 are queued every lane evaluates one.  Sums stay in a fixed
// order for a given launch shape.
//
// Same support (SYM: n = m and y equal to x bit for bit, checked on the
// device before the host reads the cost scale): c_ij = c_ji, so Z =
// sum_i ea_i eb_i + sum_{i<j} (ea_i eb_j + ea_j eb_i) cos(z_ij)^(2 inv_tau).
// The grid holds only the tiles with a pair j >= i (column tile major, its row
// tiles 0 .. ceil(j1 / 256) - 1 in order, so consecutive blocks, which go to
// different XCDs, share a column tile), and only pairs j >= i are evaluated:
// half the scan and half the logarithms and exponentials.
constexpr double kWfrC[12] = {1.0,
                              1.0 / 2,
                              1.0 / 24,
                              1.0 / 720,
                              1.0 / 40320,
                              1.0 / 3628800,
                              1.0 / 479001600,
                              1.0 / 87178291200.0,
                              1.0 / 20922789888000.0,
                              1.0 / 6402373705728000.0,
                              1.0 / 2432902008176640000.0,
                              1.0 / 1124000727777607680000.0};

// The normaliser's logarithm and exponential come from the small tables of
// common.hpp (TabLog; Z needs its sum to 1e-13, not bit-exactness).
__device__ __forceinline__ double wfr_q(double t, double w, double k2, const TabLog& T) {
    const double u = -t;  // cos z = sum_k u^k / (2k)!
    double p = kWfrC[11];
#pragma unroll
    for (int k = 10; k >= 0; --k) p = fma(p, u, kWfrC[k]);
    // w is the pair's weight ea eb; cos z below 2^-1000 gives a term far
    // below the sum's rounding
    if (!(p > 0x1p-1000)) return 0.0;
    const double x = k2 * tab_log(p, T);
    return x < -740.0 ? 0.0 : w * tab_exp(x, T);
}

// stats[ST_SAME_SUPPORT] = 0 if any coordinate of y differs from x's (bit
// for bit); launch_same_support sets it to 1 first.  Every writer stores the
// same value, so the outcome does not depend on their order.
__global__ void k_same_support(const double* __restrict__ x, const double* __restrict__ y,
                               int64_t len, double* stats) {
    bool diff = false;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
         e += (int64_t)gridDim.x * blockDim.x)
        diff = diff || __double_as_longlong(x[e]) != __double_as_longlong(y[e]);
    if (__syncthreads_or(diff) && threadIdx.x == 0) stats[ST_SAME_SUPPORT] = 0.0;
}

// Columns per LDS stage of the WFR normaliser: their coordinates and log
// factors are read once per block, then by every wave as broadcasts.
constexpr int kZwChunk = 256;

// Row tiles of column tile ct in the same-support grid.
__host__ __device__ inline int64_t zw_sym_rows(int64_t ct, int64_t nrt) {
    const int64_t r = (ct + 1) * (kCostTileCols / 256);
    return r < nrt ? r : nrt;
}

template <int D, bool SYM>
__global__ __launch_bounds__(256) void k_uot_z_wfr(ProbParams pp, int64_t n, int64_t m,
                                                   int64_t ncol_tiles, const double* __restrict__ ea,
                                                   const double* __restrict__ eb,
                                                   double* partials) {
    constexpr int DD = D > 0 ? D : 1;
    __shared__ double sh[4];
    __shared__ double qt[4][128], qs[4][128];
    __shared__ double ys[kZwChunk][DD + 2];  // coordinates, then the column's eb and ea
    __shared__ TabLog tabs;
    tab_log_init(tabs);
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr bool sym = SYM;
    int64_t rt, ct;
    if constexpr (SYM) {
        const int64_t nrt = (n + 255) / 256;
        int64_t b = blockIdx.x;
        ct = 0;
        while (b >= zw_sym_rows(ct, nrt)) {
            b -= zw_sym_rows(ct, nrt);
            ++ct;
        }
        rt = b;
    } else {
        rt = blockIdx.x / ncol_tiles;
        ct = blockIdx.x % ncol_tiles;
    }
    const int64_t i = rt * 256 + threadIdx.x;
    const int64_t j0 = ct * kCostTileCols;
    const int64_t j1 = (j0 + kCostTileCols < m) ? j0 + kCostTileCols : m;
    const bool live = i < n;
    double xi[DD];
    const double* xp = pp.x + (live ? i : 0) * pp.d;
#pragma unroll
    for (int k = 0; k < DD; ++k) xi[k] = D > 0 ? xp[k] : 0.0;
    const double eai = live ? ea[i] : 0.0;
    const double ebi = live && sym ? eb[i] : 0.0;
    const double w2 = pp.wfr_w * pp.wfr_w;
    const double k2 = 2.0 * pp.inv_tau;
    double acc = 0.0;
    int nq = 0;  // queued pairs of this wave (wave-uniform)
    for (int64_t c0 = j0; c0 < j1; c0 += kZwChunk) {
        const int nc = (int)(j1 - c0 < kZwChunk ? j1 - c0 : kZwChunk);
        if constexpr (D > 0) {
            __syncthreads();  // the previous chunk is read
            if (threadIdx.x < nc) {
                const double* yp = pp.y + (c0 + threadIdx.x) * D;
#pragma unroll
                for (int k = 0; k < D; ++k) ys[threadIdx.x][k] = yp[k];
                ys[threadIdx.x][D] = eb[c0 + threadIdx.x];
                ys[threadIdx.x][D + 1] = ea[c0 + threadIdx.x];
            }
            __syncthreads();
        }
        for (int jj = 0; jj < nc; ++jj) {
            const int64_t j = c0 + jj;
            double c, ebj, eaj;
            if constexpr (D > 0) {
                // fused: the normaliser needs its sum to 1e-13, not the
                // mask's operation order (a pair it would block differently
                // lies at z = pi/2, where its term is 0)
                double d0 = xi[0] - ys[jj][0];
                c = d0 * d0;
#pragma unroll
                for (int k = 1; k < D; ++k) {
                    const double u = xi[k] - ys[jj][k];
                    c = fma(u, u, c);
                }
                ebj = ys[jj][D];
                eaj = ys[jj][D + 1];
            } else {
                c = sqdist<D>(xp, pp.y + j * pp.d, pp.d);
                ebj = eb[j];
                eaj = ea[j];
            }
            const double t = c * w2;
            const bool on = live && t < kHalfPi * kHalfPi && (!sym || j >= i);
            const uint64_t bal = __ballot(on);
            if (on) {
                const int pos = nq + __popcll(bal & ((1ull << lane) - 1));
                qt[wv][pos] = t;
                qs[wv][pos] = !sym || j == i ? eai * ebj : eai * ebj + eaj * ebi;
            }
            nq += __popcll(bal);
            if (nq >= 64) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                acc = acc + wfr_q(qt[wv][lane], qs[wv][lane], k2, tabs);
                const double t2 = qt[wv][64 + lane], s2 = qs[wv][64 + lane];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                nq -= 64;
                if (lane < nq) {
                    qt[wv][lane] = t2;
                    qs[wv][lane] = s2;
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < nq) acc = acc + wfr_q(qt[wv][lane], qs[wv][lane], k2, tabs);
    const double tot = block_sum256(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

template <int D>
static void run_uot_z(const ProbParams& pp, int64_t n, int64_t m, const double* eb, double g,
                      bool short_range, bool same, double* partials, int64_t nct, int64_t nrt,
                      int64_t nsym, hipStream_t st) {
    const double eq = exp(-0.25);
    if (short_range)
        hipLaunchKernelGGL((k_uot_z<D, true>), dim3((unsigned)(nct * nrt)), dim3(256), 0, st, pp, n,
                           m, nct, eb, g, eq, partials);
    else if (pp.cost == kCostWfr && same)
        hipLaunchKernelGGL((k_uot_z_wfr<D, true>), dim3((unsigned)nsym), dim3(256), 0, st, pp, n, m,
                           nct, pp.row_bnd, eb, partials);
    else if (pp.cost == kCostWfr)
        hipLaunchKernelGGL((k_uot_z_wfr<D, false>), dim3((unsigned)(nct * nrt)), dim3(256), 0, st,
                           pp, n, m, nct, pp.row_bnd, eb, partials);
    else
        hipLaunchKernelGGL((k_uot_z<D, false>), dim3((unsigned)(nct * nrt)), dim3(256), 0, st, pp, n,
                           m, nct, eb, g, eq, partials);
}

hipError_t launch_same_support(const double* x, const double* y, int64_t n, int64_t m, int d,
                               double* stats, hipStream_t st) {
    hipError_t e = launch_fill_f64(stats + ST_SAME_SUPPORT, 1, n == m ? 1.0 : 0.0, st);
    if (e != hipSuccess) return e;
    if (n == m && x != y)
        hipLaunchKernelGGL(k_same_support, dim3(256), dim3(256), 0, st, x, y, n * d, stats);
    return hipGetLastError();
}

hipError_t launch_uot_z(const ProbParams& pp, int64_t n, int64_t m, const double* eb, double cmax,
                        bool same_support, double* partials, double* scratch, double* stats,
                        hipStream_t st) {
    const int64_t nct = (m + kCostTileCols - 1) / kCostTileCols;
    const int64_t nrt = (n + 255) / 256;
    const double g = pp.inv_cmax * pp.inv_tau;
    // the short-range exponential needs the squared Euclidean cost
    const bool short_range = pp.cost != kCostWfr && g * cmax <= 0.5;
    const bool same = pp.cost == kCostWfr && same_support && n == m;
    int64_t nsym = 0;
    for (int64_t ct = 0; ct < nct; ++ct) nsym += zw_sym_rows(ct, nrt);
    SS_DISPATCH_D(pp.d, run_uot_z, pp, n, m, eb, g, short_range, same, partials, nct, nrt, nsym,
                  st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_tree_sum(partials, same ? nsym : nct * nrt, scratch, stats + ST_Z, st);
}

// ------------------------------------------------------------------ Z by expansion
// With x~ = x - c and y~ = y - c for a centre c, c_ij = |x~_i|^2 + |y~_j|^2 -
// 2 x~_i . y~_j, so q_ij = A_i B_j exp(2 g x~_i . y~_j) with
// A_i = exp(la_i - g |x~_i|^2), B_j = exp(lb_j - g |y~_j|^2), and
// exp(2 g x~.y~) = sum_alpha (2g)^|alpha| / alpha! x~^alpha y~^alpha (the
// multinomial form of the exponential series).  Cut at |alpha| <= K (the host
// picks K so that the remainder is below 2^-64 of the smallest term), Z =
// sum_alpha coef_alpha S_alpha T_alpha with S_alpha = sum_i A_i x~_i^alpha,
// T_alpha = sum_j B_j y~_j^alpha: O((n + m) M) work for M monomials instead
// of nm exponentials.  Every sum runs in a fixed order.
__global__ __launch_bounds__(256) void k_cm_radii(const double* __restrict__ x,
                                                  const double* __restrict__ y, int64_t n,
                                                  int64_t m, int d, const CmaxScratch* cs,
                                                  double* __restrict__ center_out, double* stats) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < d) center_out[t] = cs->center[t];
    double rx = t < n ? center_sqdist(x + t * d, cs->center, d) : 0.0;
    double ry = t < m ? center_sqdist(y + t * d, cs->center, d) : 0.0;
    rx = group_max<kWave>(rx);
    ry = group_max<kWave>(ry);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicMax((unsigned long long*)&stats[ST_RX2], (unsigned long long)__double_as_longlong(rx));
        atomicMax((unsigned long long*)&stats[ST_RY2], (unsigned long long)__double_as_longlong(ry));
    }
}

hipError_t launch_center_radii(const double* x, const double* y, int64_t n, int64_t m, int d,
                               const void* cmax_scratch, double* center_out, double* stats,
                               hipStream_t st) {
    const int64_t t = n > m ? n : m;
    hipLaunchKernelGGL(k_cm_radii, dim3(grid_for(t > d ? t : d)), dim3(256), 0, st, x, y, n, m, d,
                       (const CmaxScratch*)cmax_scratch, center_out, stats);
    return hipGetLastError();
}

constexpr int kZPts = 32;   // points staged per round

// Block partials of S_alpha (side 0: x, la) or T_alpha (side 1: y, lb) over a
// grid-stride of point chunks; thread t owns monomials t, t + 256, ...
template <int D>
__global__ __launch_bounds__(256) void k_zexp_part(ZExpArgs A, int side) {
    __shared__ double pw[kZPts][8][kZMaxDegree + 1];
    __shared__ double w[kZPts];
    const double* pts = side == 0 ? A.x : A.y;
    const double* lw = side == 0 ? A.la : A.lb;
    const int64_t np = side == 0 ? A.n : A.m;
    const int d = D > 0 ? D : A.d;
    double acc[kZMaxMono / 256];
#pragma unroll
    for (int s = 0; s < kZMaxMono / 256; ++s) acc[s] = 0.0;
    for (int64_t p0 = (int64_t)blockIdx.x * kZPts; p0 < np; p0 += (int64_t)gridDim.x * kZPts) {
        __syncthreads();   // the previous chunk is no longer read
        for (int t = threadIdx.x; t < kZPts * d; t += blockDim.x) {
            const int p = t / d, k = t - p * d;
            const int64_t i = p0 + p;
            const double v = i < np ? pts[i * d + k] - A.center[k] : 0.0;
            double e = 1.0;
            for (int q = 0; q <= A.K; ++q) {
                pw[p][k][q] = e;
                e *= v;
            }
        }
        __syncthreads();
        if (threadIdx.x < kZPts) {
            const int p = threadIdx.x;
            const int64_t i = p0 + p;
            double r2 = 0.0;
            for (int k = 0; k < d; ++k) r2 = r2 + pw[p][k][1] * pw[p][k][1];
            w[p] = i < np ? exp(lw[i] - A.g * r2) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kZMaxMono / 256; ++s) {
            const int a = threadIdx.x + 256 * s;
            if (a < A.M) {
                const uint8_t* ex = A.exps + (int64_t)a * 8;
                uint8_t e[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) e[k] = ex[k];
                double sum = 0.0;
                for (int p = 0; p < kZPts; ++p) {
                    double f = w[p];
#pragma unroll
                    for (int k = 0; k < (D > 0 ? D : 8); ++k)
                        if (D > 0 || k < d) f *= pw[p][k][e[k]];
                    sum += f;
                }
                acc[s] += sum;
            }
        }
    }
#pragma unroll
    for (int s = 0; s < kZMaxMono / 256; ++s) {
        const int a = threadIdx.x + 256 * s;
        if (a < A.M) A.part[((int64_t)side * gridDim.x + blockIdx.x) * A.M + a] = acc[s];
    }
}

// sums[side][alpha] = sum over the blocks' partials: one block per (alpha,
// side), a thread-strided pass and the fixed block tree.
__global__ __launch_bounds__(256) void k_zexp_sum(ZExpArgs A, int nblocks) {
    __shared__ double sh[16];
    const int a = blockIdx.x;
    const int side = blockIdx.y;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        s += A.part[((int64_t)side * nblocks + b) * A.M + a];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) A.sums[side * A.M + a] = s;
}

// Z = sum_alpha coef_alpha S_alpha T_alpha (one block, fixed tree).
__global__ __launch_bounds__(256) void k_zexp_final(ZExpArgs A, double* stats) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (int a = threadIdx.x; a < A.M; a += blockDim.x)
        acc += A.coef[a] * (A.sums[a] * A.sums[A.M + a]);
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) stats[ST_Z] = acc;
}

template <int D>
static void run_zexp(const ZExpArgs& a, hipStream_t st) {
    for (int side = 0; side < 2; ++side)
        hipLaunchKernelGGL(k_zexp_part<D>, dim3(kZBlocks), dim3(256), 0, st, a, side);
}

hipError_t launch_uot_zexp(const ZExpArgs& a, double* stats, hipStream_t st) {
    if (a.d > 8 || a.M > kZMaxMono || a.K > kZMaxDegree) return hipErrorInvalidValue;
    switch (a.d) {
        case 2: run_zexp<2>(a, st); break;
        case 3: run_zexp<3>(a, st); break;
        case 5: run_zexp<5>(a, st); break;
        default: run_zexp<0>(a, st); break;
    }
    hipLaunchKernelGGL(k_zexp_sum, dim3((unsigned)a.M, 2), dim3(256), 0, st, a, kZBlocks);
    hipLaunchKernelGGL(k_zexp_final, dim3(1), dim3(256), 0, st, a, stats);
    return hipGetLastError();
}

// Column factor of a rigorous upper bound on p*: for every (i, j),
// p*_ij <= ea_i * fb_j + c (1 + 2^-30) with fb_j = (1 - g)(s/Z) exp(lb_j)
// (1 + 2^-30) and c the uniform part of shrinkage; the margins cover the
// rounding of the sum, exponential and products (all < 1e-12).
__global__ void k_uot_bounds(const double* lb, int64_t m, double s, double w,
                             const double* stats, double* fb) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const double kappa = w * (s / stats[ST_Z]);
    fb[j] = kappa * exp_spec(lb[j]) * (1.0 + 0x1p-30);
}

hipError_t launch_uot_bounds(const double* lb, int64_t m, double s, double shrink_w,
                             const double* stats, double* fb, hipStream_t st) {
    hipLaunchKernelGGL(k_uot_bounds, dim3(grid_for(m)), dim3(kBlock), 0, st, lb, m, s, shrink_w,
                       stats, fb);
    return hipGetLastError();
}

// ------------------------------------------------------------------ mask
// Block tile: 16 rows x 64 mask words (4096 columns).  Wave w owns hash
// groups 2w, 2w+1 of the tile (512 columns each): one Philox call per lane per
// group and row gives the 16-bit high halves of eight columns 64 apart.
//
// Two phases per wave, so that the hash loop stays small (few registers,
// high occupancy) and no wave idles while one lane evaluates an exact p*:
//  1. filter: hash the high halves and keep as a candidate every entry that
//     can still be sampled, hi < 2^16 P with P the decision's probability
//     (OT) or its cost-free bound (UOT), scaled by 2^16 (1 + 2^-40) so that
//     the filter only ever adds candidates; candidates go to a per-wave list
//     in LDS (ballot + lane prefix count, no atomics);
//  2. decide: when the list may overflow, and at the end, every lane takes
//     one listed entry and runs the exact decision (the same test and
//     arithmetic as a pair-by-pair evaluation: the OT comparison of U with
//     p*; for UOT the cost-free bound, the cost factor's bound for the
//     unnormalised and WFR costs, then the exact p* and U).  Kept entries set
//     their bit in the wave's own words of the tile.
// An entry that the filter drops has hi >= 2^16 P, so U >= P: it is never
// kept.  The mask is therefore the same as a pair-by-pair evaluation's.
// WFR (which takes no shrinkage): the filter also bounds the cost factor, F <= 2^-t
// with t = z^2 inv_tau log2(e) (uot_bound_exponent), from an FP32 squared
// distance c32 with its rounding taken out, c >= c32 (1 - 2^-20) - 2^-20
// (|x|^2 + |y|^2) (coordinates rounded to FP32, differences and the sum
// rounded); with log2 hi >= e + m for hi = 2^e (1 + m) (read off the bits of
// hi as a float), an entry is a candidate only if hi = 0 or
// e + m + t < log2(2^16 P) (both sides bounded outward), which drops the
// pairs whose cost factor rules them out before the exact decision (about
// 70 in 71 of the cost-free candidates at the WFR workload's sparsity).
// A list entry is 32 bits: row (4), slot of the wave (4), lane (6), high half.
// The FP32 bit pattern of 2^23 + hi, hi the coarse half of `slot`: the half's
// two bytes and the bytes 0x00, 0x4B of the constant in one byte permute
// (selectors 0-3 take the word's bytes, 4-7 the constant's).
__device__ __forceinline__ uint32_t half_f23(const Words4& w, int slot) {
    const int t = slot >> 1;
    const uint32_t x = t == 0 ? w.w[0] : t == 1 ? w.w[1] : t == 2 ? w.w[2] : w.w[3];
    return __builtin_amdgcn_perm(0x4B000000u, x, (slot & 1) ? 0x07040302u : 0x07040100u);
}
// An FP32 upper bound of a factor v >= 0 in [2^-126, inf] (v = 0 and the
// FP32 denormals included); -inf and NaN stay as they are.
__device__ __forceinline__ float fac_up(double v) {
    if (!(v > 0x1p-126)) return v >= 0.0 ? 0x1p-126f : (float)v;
    float f = (float)v;  // nearest; above FLT_MAX by more than half an ulp: inf
    if ((double)f < v) f = __int_as_float(__float_as_int(f) + 1);  // FLT_MAX -> inf
    return f;
}
// An FP32 upper bound of log2 v for a double v (+ 2^-8 for the rounding of
// the conversion and of v_log_f32); -inf for v <= 0 and NaN.
__device__ __forceinline__ float log2_up(double v) {
    if (!(v > 0.0)) return -INFINITY;
    if (v == INFINITY) return INFINITY;
    int e;
    const double f = frexp(v, &e);  // f in [1/2, 1)
    return (float)e + __builtin_amdgcn_logf((float)f) + 0x1p-8f;
}

constexpr int kMaskRows = 16;
constexpr int kMaskCand = 1024;  // list entries per wave (>= 512 + one row's 512)

// One tile: rows rt * 16 split .. + 16 split - 1 of one problem, mask words
// ct * 64 .. ct * 64 + 63; adds the popcounts to row_cnt.  All 256 threads
// call it.  With split = 1 every wave takes the tile's 16 rows and 16 of its
// words; with split = 2 or 4 (rows of at most 32 or 16 words) 4 / split waves
// cover a row's words and the waves take split blocks of 16 rows.  `cand`
// holds kMaskCand entries per wave.  WFR = false: the cost is not the WFR
// cost (its cosine and logarithm are left out of the kernel).
template <bool UOT, int D, bool WFR>
__device__ __forceinline__ void mask_tile(const ProbParams& pp, int64_t n, int64_t m, int64_t W,
                                          int64_t rt, int64_t ct, int split,
                                          uint64_t* __restrict__ mask,
                                          int32_t* __restrict__ row_cnt, double kappa,
                                          uint64_t (*tile)[64], uint32_t (*cand)[kMaskCand]) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    const int wpr = 4 / split;  // waves across a row's words
    const int cp = wv % wpr;    // this wave's 16-word part of the row
    const int64_t row0 = rt * kMaskRows * split + (wv / wpr) * kMaskRows;
    const int nrows = (int)(n - row0 < kMaskRows ? (n - row0 > 0 ? n - row0 : 0) : kMaskRows);
    // the wave's 16 words of each row start empty
#pragma unroll
    for (int e = lane; e < kMaskRows * 16; e += kWave) tile[e >> 4][wv * 16 + (e & 15)] = 0;
    const double* __restrict__ rsrc = UOT ? pp.row_bnd : pp.row_fac;
    const double* __restrict__ csrc = UOT ? pp.col_bnd : pp.col_fac;
    // the uniform part of shrinkage (0 without it); for the UOT bound with
    // the bound's margin
    const double pc = UOT ? pp.shrink_c * (1.0 + 0x1p-30) : pp.shrink_c;
    // filter scale 2^16 (1 + 2^-40)
    constexpr double kScale = 0x1p16 * (1.0 + 0x1p-40);
    // lane r < 16 holds row r's factor, scaled
    const double rowv = lane < nrows ? rsrc[row0 + lane] * kScale : 0.0;
    // The filter in FP32: hi is a candidate when 2^23 + hi < fma(r, c, b)
    // with r, c the scaled row and column factors rounded up into
    // [2^-126, inf] and b = 2^23 + 2^16 pc + 1 rounded up.  A kept entry has
    // hi < 2^16 P; the exact sum r c + b is at least 2^23 + 2^16 P + 1, and
    // its rounding (ulp 1 below 2^24) loses at most 1/2, so every kept entry
    // is a candidate, hi = 0 always, and no product is NaN (only the columns
    // past m carry -inf, and are never candidates).
    const float bias32 = fac_up(0x1p23 + pc * kScale + 1.0);
    const float row32 = fac_up(rowv);
    // the cost as a value the compiler sees: without WFR one of the two
    // squared Euclidean kinds, so the WFR branches fold away
    ProbParams lp = pp;
    if constexpr (!WFR)
        lp.cost = pp.cost == SS_COST_SQEUCLID ? SS_COST_SQEUCLID : SS_COST_SQEUCLID_MAXNORM;
    uint32_t* const list = cand[wv];
    int cnt = 0;  // wave-uniform
    // WFR (no shrinkage: the host rejects it with this cost): lane r < 16
    // holds row r's FP32 coordinates, its squared norm less 2^-16 of it and
    // an upper bound of log2 of its factor (the kernels of a fixed
    // dimension; D = 0 reads pp.d at run time and keeps the cost-free
    // filter).  A pair's squared distance is bounded below by
    // |x|^2 (1 - 2^-16) + |y|^2 (1 - 2^-16) - 2 x.y in FP32: with u = 2^-24
    // and S = |x|^2 + |y|^2, rounding the coordinates to FP32 moves c by at
    // most 4 u S, the fused sums of at most 10 terms by 20 u S and the last
    // roundings by 4 u S, far inside the 2^-16 S taken off.  A norm of 2^100
    // or more (or NaN) takes -inf, so its pairs are always candidates and
    // nothing overflows.
    constexpr bool kCfb = WFR && D > 0;
    constexpr int CD = kCfb ? D : 1;
    float xr_l[CD], nxs_l = 0.0f, lr_l = -INFINITY;
    float alpha = 0.0f;
    if constexpr (kCfb) {
        float nx = 0.0f;
#pragma unroll
        for (int k = 0; k < CD; ++k) {
            xr_l[k] = lane < nrows ? (float)pp.x[(row0 + lane) * D + k] : 0.0f;
            nx = fmaf(xr_l[k], xr_l[k], nx);
        }
        nxs_l = nx < 0x1p100f ? nx * (1.0f - 0x1p-16f) : -INFINITY;
        lr_l = log2_up(rowv);
        // t per unit squared distance, rounded down
        alpha = (float)(pp.wfr_w * pp.wfr_w * pp.inv_tau * kLog2e) * (1.0f - 0x1p-20f);
    }
    const int64_t g_end = (W + 7) / 8;  // hash groups of 512 columns (8 words)
    const int64_t g_first = ct * 8 + cp * 2;
    const int ng = (int)(g_end - g_first < 2 ? (g_end - g_first > 0 ? g_end - g_first : 0) : 2);
    for (int gg = 0; gg < ng; ++gg) {
        const int64_t g = g_first + gg;
        const uint32_t q = (uint32_t)(g * 64 + lane);
        // column factors of this group; -inf past the last column makes the
        // filter's bound -inf (or NaN for a zero row factor): never a candidate
        double cf[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int64_t j = 512 * g + 64 * s + lane;
            cf[s] = j < m ? csrc[j] : -INFINITY;
        }
        float cf32[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) cf32[s] = fac_up(cf[s]);
        // cost-factor bound data of the lane's eight columns (WFR)
        float yc[8][CD], nys[8], lcol[8];
        if constexpr (kCfb) {
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int64_t j = 512 * g + 64 * s + lane;
                float ny = 0.0f;
#pragma unroll
                for (int k = 0; k < CD; ++k) {
                    yc[s][k] = j < m ? (float)pp.y[j * D + k] : 0.0f;
                    ny = fmaf(yc[s][k], yc[s][k], ny);
                }
                nys[s] = ny < 0x1p100f ? ny * (1.0f - 0x1p-16f) : -INFINITY;
                lcol[s] = log2_up(cf[s]);
            }
        }
        for (int r = 0; r < nrows; ++r) {
            const int64_t i = row0 + r;
            const float rowf =
                __int_as_float(__builtin_amdgcn_readlane(__float_as_int(row32), r));
            const Words4 h = philox10(q, (uint32_t)i, pp.problem_index, 0u, pp.k0, pp.k1);
            float xr[CD], nxs = 0.0f, lr = 0.0f;
            if constexpr (kCfb) {
#pragma unroll
                for (int k = 0; k < CD; ++k)
                    xr[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xr_l[k]), r));
                nxs = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(nxs_l), r));
                lr = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lr_l), r));
            }
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                uint32_t hs;
                bool c;
                if constexpr (kCfb) {
                    hs = coarse_half(h, s);
                    float dot = xr[0] * yc[s][0];
#pragma unroll
                    for (int k = 1; k < CD; ++k) dot = fmaf(xr[k], yc[s][k], dot);
                    const float clo = fmaf(-2.0f, dot, nxs + nys[s]);
                    // e + m of hs (as an unsigned float, exact below 2^24) plus t
                    const float bits = (float)__float_as_uint((float)hs);
                    const float v = fmaf(bits, 0x1p-23f, fmaf(alpha, clo, -127.0f));
                    // NaN (an infinite norm) is a candidate too
                    c = !(v >= lr + lcol[s]) || hs == 0u;
                } else {
                    const uint32_t hb = half_f23(h, s);
                    c = __uint_as_float(hb) < fmaf(rowf, cf32[s], bias32);
                    hs = hb & 0xFFFFu;
                }
                const uint64_t bal = __ballot(c);
                if (bal) {
                    if (c) {
                        const int pos = cnt + (int)__builtin_amdgcn_mbcnt_hi(
                                                  (uint32_t)(bal >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                        list[pos] = ((uint32_t)r << 26) | ((uint32_t)(gg * 8 + s) << 22) |
                                    ((uint32_t)lane << 16) | hs;
                    }
                    cnt += __popcll(bal);
                }
            }
            if (cnt <= kMaskCand - 512 && (r + 1 < nrows || gg + 1 < ng)) continue;
            // ---- decide the listed entries, one per lane (the list was written
            // by other lanes of this wave: LDS operations of a wave complete in
            // order; the wait and clobber also keep the compiler's order)
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            for (int base = 0; base < cnt; base += kWave) {
                const int e = base + lane;
                if (e >= cnt) break;
                const uint32_t it = list[e];
                const uint32_t hw = it & 0xFFFFu;
                const int er = (int)(it >> 26), slot = (int)(it >> 22) & 15,
                          lc = (int)(it >> 16) & 63;
                const int es = slot & 7;
                const int64_t eg = g_first + (slot >> 3);
                const int64_t ej = 512 * eg + 64 * es + lc;
                const int64_t ei = row0 + er;
                const uint32_t eq = (uint32_t)(eg * 64 + lc);
                bool keep = false;
                if (ej < m) {
                    const double Pr = rsrc[ei] * csrc[ej];
                    const double P = Pr + pc;
                    if (!UOT) {
                        keep = keep_decision(hw, P, eq, (uint32_t)ei, pp.problem_index, pp.k0, pp.k1,
                                             es);
                    } else if ((double)hw * 0x1p-16 < P) {
                        // P bounds p* without the cost factor.  Candidates first take
                        // the cost factor's bound in FP32 (margin 2^-12 for the
                        // rounding of its argument and of the exponential), and only
                        // those below it pay for the exact p*.  Where the FP32 bound
                        // underflows, only hi = 0 can still fall below p*, so that
                        // case goes to the exact test as well.  (With the
                        // max-normalised cost, C <= 1, the cost factor is at least
                        // exp(-inv_tau) and the refinement does not pay.)
                        const double c = sqdist<D>(pp.x + ei * pp.d, pp.y + ej * pp.d, pp.d);
                        bool exact = true;
                        if (lp.cost != SS_COST_SQEUCLID_MAXNORM) {
                            const double t = uot_bound_exponent(lp, c);
                            const double ex = t < 200.0 ? (double)__builtin_amdgcn_exp2f(-(float)t) : 0.0;
                            const double Pt = Pr * ex * (1.0 + 0x1p-12) + pc;
                            exact = (double)hw * 0x1p-16 < Pt || hw == 0u;
                        }
                        if (exact) {
                            const double q_ij = uot_q_of(lp, c, ei, ej);
                            const double pst = fmin(1.0, kappa * q_ij + pp.shrink_c);
                            keep = keep_decision(hw, pst, eq, (uint32_t)ei, pp.problem_index, pp.k0,
                                                 pp.k1, es);
                        }
                    }
                }
                if (keep)
                    atomicOr((unsigned long long*)&tile[er][wv * 16 + slot], 1ull << lc);
            }
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // list slots are rewritten next
            cnt = 0;
        }
    }
    __syncthreads();
    if (split == 1) {
        // a row's 64 words from the four waves' parts, one row per instruction
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
    } else {
        // each wave writes its own 16 rows x 16 words, four rows per
        // instruction, and adds its part of each row's count (integer adds:
        // the order does not matter)
#pragma unroll
        for (int rr = 0; rr < kMaskRows / 4; ++rr) {
            const int r = 4 * rr + lane / 16;
            const int64_t i = row0 + r;
            const int64_t widx = ct * 64 + cp * 16 + (lane & 15);
            const bool ok = i < n && widx < W;
            const uint64_t w = tile[r][wv * 16 + (lane & 15)];
            if (ok) mask[i * W + widx] = w;
            int c = ok ? __popcll(w) : 0;
            c = group_sum<16>(c);
            if ((lane & 15) == 0 && c) atomicAdd(&row_cnt[i], c);
        }
    }
}

// Six waves per SIMD (the LDS of six blocks fills a compute unit): the hash
// loop then fits in 80 registers; only the decision phase reloads a few
// spilled values.  The WFR decision (FP64 cosine and logarithm) needs more,
// so its kernel keeps the compiler's register count instead of spilling in
// the hash loop.
template <bool UOT, int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_mask(
    ProbParams pp, int64_t n, int64_t m, int64_t W, int64_t ncol_tiles, uint64_t* __restrict__ mask,
    int32_t* __restrict__ row_cnt, const double* __restrict__ stats) {
    __shared__ uint64_t tile[kMaskRows][64];
    __shared__ uint32_t cand[4][kMaskCand];
    const int64_t rt = blockIdx.x / ncol_tiles, ct = blockIdx.x % ncol_tiles;
    const double kappa = UOT ? pp.shrink_w * (pp.s / stats[ST_Z]) : 0.0;
    mask_tile<UOT, D, false>(pp, n, m, W, rt, ct, 1, mask, row_cnt, kappa, tile, cand);
}

template <int D>
__global__ __launch_bounds__(256) void k_mask_wfr(ProbParams pp, int64_t n, int64_t m, int64_t W,
                                                  int64_t ncol_tiles, uint64_t* __restrict__ mask,
                                                  int32_t* __restrict__ row_cnt,
                                                  const double* __restrict__ stats) {
    __shared__ uint64_t tile[kMaskRows][64];
    __shared__ uint32_t cand[4][kMaskCand];
    const int64_t rt = blockIdx.x / ncol_tiles, ct = blockIdx.x % ncol_tiles;
    const double kappa = pp.shrink_w * (pp.s / stats[ST_Z]);
    mask_tile<true, D, true>(pp, n, m, W, rt, ct, 1, mask, row_cnt, kappa, tile, cand);
}

template <bool UOT, int D, bool WFR>
static void run_mask(const ProbParams& pp, int64_t n, int64_t m, uint64_t* mask, int32_t* row_cnt,
                     const double* stats, hipStream_t st) {
    const int64_t W = (m + 63) / 64;
    const int64_t nct = (W + 63) / 64;
    const int64_t nrt = (n + kMaskRows - 1) / kMaskRows;
    const dim3 grid((unsigned)(nct * nrt));
    if constexpr (WFR)
        hipLaunchKernelGGL((k_mask_wfr<D>), grid, dim3(256), 0, st, pp, n, m, W, nct, mask,
                           row_cnt, stats);
    else
        hipLaunchKernelGGL((k_mask<UOT, D>), grid, dim3(256), 0, st, pp, n, m, W, nct, mask,
                           row_cnt, stats);
}

template <int D>
static void run_mask_d(const ProbParams& pp, int64_t n, int64_t m, uint64_t* mask,
                       int32_t* row_cnt, const double* stats, hipStream_t st) {
    if (pp.uot)
        if (pp.cost == kCostWfr)
            run_mask<true, D, true>(pp, n, m, mask, row_cnt, stats, st);
        else
            run_mask<true, D, false>(pp, n, m, mask, row_cnt, stats, st);
    else
        run_mask<false, 2, false>(pp, n, m, mask, row_cnt, stats, st);  // OT never reads coordinates
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

// One tile: 64-row blocks rt * 8 .. rt * 8 + 7, mask word columns ct * 16 ..
// ct * 16 + 15; adds the popcounts to col_cnt.  All 256 threads call it.
__device__ __forceinline__ void transpose_tile(const uint64_t* __restrict__ mask, int64_t n,
                                               int64_t m, int64_t W, int64_t Wn, int64_t rt,
                                               int64_t ct, uint64_t* __restrict__ maskT,
                                               int32_t* __restrict__ col_cnt,
                                               uint64_t (*tile)[kTrWordCols + 1]) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    uint64_t out[4][kTrRowBlocks];
    const int lr = threadIdx.x >> 2;          // row of the tile this thread loads
    const int lq = (threadIdx.x & 3) * 4;     // first of its 4 words
    // the words of row block rho + 1 are in flight while block rho is
    // transposed: the barriers wait for LDS only, not for those loads
    uint64_t nx[4];
    // a row's 4 words in two 16-byte loads when they all exist (an aligned
    // base and W even keep them 16-byte aligned)
    const bool wfull = ((uintptr_t)mask & 15) == 0 && (W & 1) == 0 &&
                       ct * kTrWordCols + lq + 4 <= W;
    auto load_block = [&](int rho) __attribute__((always_inline)) {
        const int64_t I = rt * kTrRowBlocks + rho;
        const int64_t i = 64 * I + lr;
        if (wfull && I < Wn && i < n) {
            const ulonglong2* src = (const ulonglong2*)(mask + i * W + ct * kTrWordCols + lq);
            const ulonglong2 a = src[0], b = src[1];
            nx[0] = a.x;
            nx[1] = a.y;
            nx[2] = b.x;
            nx[3] = b.y;
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t wc = ct * kTrWordCols + lq + q;
                nx[q] = (I < Wn && i < n && wc < W) ? mask[i * W + wc] : 0ull;
            }
        }
    };
    load_block(0);
#pragma unroll
    for (int rho = 0; rho < kTrRowBlocks; ++rho) {
#pragma unroll
        for (int q = 0; q < 4; ++q) tile[lr][lq + q] = nx[q];
        if (rho + 1 < kTrRowBlocks) load_block(rho + 1);
        lds_barrier();
#pragma unroll
        for (int k = 0; k < 4; ++k) out[k][rho] = transpose64(tile[lane][wv * 4 + k]);
        lds_barrier();
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t wc = ct * kTrWordCols + wv * 4 + k;
        const int64_t j = 64 * wc + lane;
        if (j >= m) continue;
        int cnt = 0;
        if (((uintptr_t)maskT & 15) == 0 && (Wn & 1) == 0 &&
            rt * kTrRowBlocks + kTrRowBlocks <= Wn) {
            // the column's 8 words in four 16-byte stores (aligned base, Wn even)
            ulonglong2* dst = (ulonglong2*)(maskT + j * Wn + rt * kTrRowBlocks);
#pragma unroll
            for (int h = 0; h < kTrRowBlocks / 2; ++h) {
                ulonglong2 t;
                t.x = out[k][2 * h];
                t.y = out[k][2 * h + 1];
                dst[h] = t;
                cnt += __popcll(t.x) + __popcll(t.y);
            }
        } else {
#pragma unroll
            for (int rho = 0; rho < kTrRowBlocks; ++rho) {
                const int64_t I = rt * kTrRowBlocks + rho;
                if (I < Wn) {
                    maskT[j * Wn + I] = out[k][rho];
                    cnt += __popcll(out[k][rho]);
                }
            }
        }
        if (cnt) atomicAdd(&col_cnt[j], cnt);
    }
}

__global__ __launch_bounds__(256) void k_transpose(const uint64_t* __restrict__ mask, int64_t n,
                                                   int64_t m, int64_t W, int64_t Wn,
                                                   int64_t ncol_tiles, uint64_t* __restrict__ maskT,
                                                   int32_t* __restrict__ col_cnt) {
    __shared__ uint64_t tile[64][kTrWordCols + 1];
    const int64_t rt = blockIdx.x / ncol_tiles, ct = blockIdx.x % ncol_tiles;
    transpose_tile(mask, n, m, W, Wn, rt, ct, maskT, col_cnt, tile);
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
// The specified exponential, logarithm and cost (elemfn.hpp) make every
// stored value a fixed sequence of IEEE operations.
template <bool UOT, int D>
__device__ __forceinline__ double entry_value(const ProbParams& pp, double kappa, int64_t i,
                                              int64_t j, double* logv) {
    const double c = sqdist<D>(pp.x + i * pp.d, pp.y + j * pp.d, pp.d);
    const double C = cost_spec(c, pp.cost, pp.inv_cmax, pp.wfr_w);
    const double Ce = C / pp.eps;
    const double K = exp_spec(-Ce);
    double P;
    if (UOT)
        P = fmin(1.0, kappa * exp_spec((pp.row_fac[i] + pp.col_fac[j]) - C * pp.inv_tau) + pp.shrink_c);
    else
        P = fmin(1.0, pp.row_fac[i] * pp.col_fac[j] + pp.shrink_c);
    *logv = -Ce - log_spec(P);
    return K / P;
}

template <int PREC>
__device__ __forceinline__ void store_value(void* val, int64_t pos, double v, double lv) {
    if (PREC == P_F64) ((double*)val)[pos] = v;
    if (PREC == P_F32) ((float*)val)[pos] = (float)v;
    if (PREC == P_LOG) ((float*)val)[pos] = (float)lv;
}

// Single-problem fill in two passes, so that neither waits on the other's
// latency: the index pass streams the mask at high occupancy (no FP64 work),
// the value pass takes each line's entries two per lane.
//
// Index pass: one wave per line; the words are read 16 per lane ahead of the
// prefix-popcount, and every kept entry's index goes to its slot (ascending).
__global__ __launch_bounds__(256) void k_fill_idx(const uint64_t* __restrict__ bits,
                                                  int64_t nlines, int64_t words,
                                                  const int64_t* __restrict__ ptr,
                                                  int32_t* __restrict__ idx, int64_t cap) {
    constexpr int NB = 16;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t line = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (line >= nlines) return;  // the whole wave
    const uint64_t* __restrict__ row = bits + line * words;
    int64_t run = ptr[line];
    for (int64_t g0 = 0; g0 < words; g0 += NB * kWave) {
        uint64_t wd[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const int64_t widx = g0 + k * kWave + lane;
            wd[k] = widx < words ? row[widx] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            uint64_t word = wd[k];
            const int64_t widx = g0 + k * kWave + lane;
            const int c = __popcll(word);
            const int incl = wave_inclusive_scan(c);
            int64_t pos = run + (incl - c);
            while (word) {
                const int b = __ffsll((unsigned long long)word) - 1;
                word &= word - 1;
                if (pos < cap) idx[pos] = (int32_t)(64 * widx + b);
                ++pos;
            }
            run += __shfl(incl, kWave - 1, kWave);
        }
    }
}

// Value pass: one wave per line, two entries per lane at a time.  WFR =
// false: the cost is a squared Euclidean kind (the WFR branches fold away).
template <int ROLE, bool UOT, int PREC, int D, bool WFR>
__global__ __launch_bounds__(256) void k_fill_val(ProbParams pp, const double* __restrict__ stats,
                                                  int64_t nlines, const int64_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ idx,
                                                  void* __restrict__ val, int64_t cap) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t line = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (line >= nlines) return;
    const double kappa = UOT ? pp.shrink_w * (pp.s / stats[ST_Z]) : 0.0;
    ProbParams lp = pp;
    if constexpr (!WFR)
        lp.cost = pp.cost == SS_COST_SQEUCLID ? SS_COST_SQEUCLID
                  : pp.cost == SS_COST_EUCLID ? SS_COST_EUCLID
                                              : SS_COST_SQEUCLID_MAXNORM;
    const int64_t e0 = ptr[line];
    const int64_t e1 = ptr[line + 1] < cap ? ptr[line + 1] : cap;
    for (int64_t e = e0 + lane; e < e1; e += 2 * kWave) {
        const int64_t e2 = e + kWave;
        const bool two = e2 < e1;
        const int64_t oa = idx[e];
        const int64_t ob = two ? idx[e2] : oa;
        double la, lb;
        const double va = entry_value<UOT, D>(lp, kappa, ROLE == 0 ? line : oa,
                                              ROLE == 0 ? oa : line, &la);
        const double vb = entry_value<UOT, D>(lp, kappa, ROLE == 0 ? line : ob,
                                              ROLE == 0 ? ob : line, &lb);
        store_value<PREC>(val, e, va, la);
        if (two) store_value<PREC>(val, e2, vb, lb);
    }
}

template <int ROLE, bool UOT, int PREC, int D>
static void run_fill4(const ProbParams& pp, const double* stats, const uint64_t* bits,
                      int64_t nlines, int64_t words, const int64_t* ptr, int32_t* idx, void* val,
                      int64_t cap, hipStream_t st) {
    const dim3 grid((unsigned)((nlines + 3) / 4));
    hipLaunchKernelGGL(k_fill_idx, grid, dim3(256), 0, st, bits, nlines, words, ptr, idx, cap);
    if (pp.cost == kCostWfr)
        hipLaunchKernelGGL((k_fill_val<ROLE, UOT, PREC, D, true>), grid, dim3(256), 0, st, pp,
                           stats, nlines, ptr, idx, val, cap);
    else
        hipLaunchKernelGGL((k_fill_val<ROLE, UOT, PREC, D, false>), grid, dim3(256), 0, st, pp,
                           stats, nlines, ptr, idx, val, cap);
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

// ================================================================== batches
// The sampling stages of a batch of OT problems, one launch per stage over
// all problems: block b works on tile b - pre[k] of the problem k that owns
// it (pre = prefix of the per-problem tile counts, searched by every block);
// the fills, one wave per line, read the line's problem from a table.

// Last k in [0, count) with pre[k] <= key.
__device__ __forceinline__ int owner_of(const int64_t* __restrict__ pre, int count, int64_t key) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= key)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Perfect binary tree (adjacent pairs) over v[0..4096), zero padded past n,
// with 1024 threads; the result (in every thread) equals the tree sum of the
// vector padded to any power of two >= n.  sh: 1024 doubles.  Callers may
// have just written v: the first barrier orders those writes.
__device__ double block_tree4096(const double* v, int64_t n, double* sh) {
    const int tid = threadIdx.x;
    __syncthreads();  // v was just written by other threads
    double e[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) e[k] = (tid * 4 + k < n) ? v[tid * 4 + k] : 0.0;
    sh[tid] = (e[0] + e[1]) + (e[2] + e[3]);
    __syncthreads();
    for (int s = 1; s < 1024; s <<= 1) {
        if ((tid & (2 * s - 1)) == 0) sh[tid] = sh[tid] + sh[tid + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Block maximum (1024 threads); the result is in every thread.
__device__ __forceinline__ double block_max1024(double x, double* sh) {
    x = group_max<kWave>(x);
    __syncthreads();  // sh is free
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = x;
    __syncthreads();
    double r = sh[0];
    for (int w = 1; w < 1024 / kWave; ++w) r = sh[w] > r ? sh[w] : r;
    return r;
}

// Exact cost maximum of every problem, one block of 1024 threads per problem,
// pruned like the single-problem scan: with c the mean of y (fixed-order tree
// sums) and R = max_j |y_j - c|, row i reaches at most (|x_i - c| + R)^2 (the
// triangle inequality, with a 1e-9 relative margin for rounding); the full
// row of the x farthest from c gives a lower bound L, and only rows whose
// bound reaches L are scanned, with the brute-force distance code.  The row
// holding the maximum always survives, so the result is the brute-force
// maximum bit for bit.
template <int D>
__global__ __launch_bounds__(1024) void k_b_cmax(BatchArgs A) {
    __shared__ double v[kBatchMaxSide];
    __shared__ double sh[1024];
    __shared__ double cen[64];
    __shared__ int surv[kBatchMaxSide];
    __shared__ int nsurv, far_row;
    const int k = blockIdx.x;
    const BProb P = A.prob[k];
    const int d = A.d;
    const int tid = threadIdx.x;
    const double* x = A.x + P.xo * d;
    const double* y = A.y + P.yo * d;
    // centre: mean of y per coordinate
    for (int c = 0; c < d; ++c) {
        for (int64_t j = tid; j < P.m; j += 1024) v[j] = y[j * d + c];
        const double sum = block_tree4096(v, P.m, sh);
        __syncthreads();  // every thread has the sum before v is rewritten
        if (tid == 0) cen[c] = sum / (double)P.m;
    }
    __syncthreads();
    // R^2 = max_j |y_j - c|^2; |x_i - c| into v
    double r2 = 0.0;
    for (int64_t j = tid; j < P.m; j += 1024) {
        double acc = 0.0;
        for (int c = 0; c < d; ++c) {
            const double t = y[j * d + c] - cen[c];
            acc = acc + t * t;
        }
        r2 = acc > r2 ? acc : r2;
    }
    const double R = sqrt(block_max1024(r2, sh));
    double rmax = -1.0;
    for (int64_t i = tid; i < P.n; i += 1024) {
        double acc = 0.0;
        for (int c = 0; c < d; ++c) {
            const double t = x[i * d + c] - cen[c];
            acc = acc + t * t;
        }
        v[i] = sqrt(acc);
        rmax = v[i] > rmax ? v[i] : rmax;
    }
    rmax = block_max1024(rmax, sh);
    if (tid == 0) {
        far_row = (int)P.n;
        nsurv = 0;
    }
    __syncthreads();
    // the farthest row (smallest index among ties)
    for (int64_t i = tid; i < P.n; i += 1024)
        if (v[i] == rmax) atomicMin(&far_row, (int)i);
    __syncthreads();
    const int64_t f = far_row;
    double lb = 0.0;
    for (int64_t j = tid; j < P.m; j += 1024) {
        const double c = sqdist<D>(x + f * d, y + j * d, d);
        lb = c > lb ? c : lb;
    }
    const double L = block_max1024(lb, sh);
    // survivors (any order: the maximum is order-free)
    for (int64_t i = tid; i < P.n; i += 1024) {
        const double b = (v[i] + R) * (v[i] + R) * (1.0 + 1e-9);
        if (b >= L) surv[atomicAdd(&nsurv, 1)] = (int)i;
    }
    __syncthreads();
    const int ns = nsurv;
    double mx = L;
    if constexpr (D > 0) {
        // each thread keeps its (at most four) columns in registers; the
        // survivors' coordinates go through LDS (v is free now) in chunks and
        // are read as broadcasts, so the scan has no global load in its loop
        constexpr int kCols = kBatchMaxSide / 1024;
        double yr[kCols][D];
#pragma unroll
        for (int t = 0; t < kCols; ++t) {
            const int64_t j = tid + 1024 * t;
#pragma unroll
            for (int c = 0; c < D; ++c) yr[t][c] = j < P.m ? y[j * D + c] : 0.0;
        }
        constexpr int cap = kBatchMaxSide / D;  // survivors per chunk
        for (int q0 = 0; q0 < ns; q0 += cap) {
            const int nq = ns - q0 < cap ? ns - q0 : cap;
            __syncthreads();  // v's previous contents are read
            for (int e = tid; e < nq * D; e += 1024) v[e] = x[(int64_t)surv[q0 + e / D] * D + e % D];
            __syncthreads();
            for (int q = 0; q < nq; ++q) {
                double xi[D];
#pragma unroll
                for (int c = 0; c < D; ++c) xi[c] = v[q * D + c];
#pragma unroll
                for (int t = 0; t < kCols; ++t) {
                    if (tid + 1024 * t < P.m) {
                        const double c = sqdist<D>(xi, yr[t], D);
                        mx = c > mx ? c : mx;
                    }
                }
            }
        }
    } else {
        for (int q = 0; q < ns; ++q) {
            const int64_t i = surv[q];
            for (int64_t j = tid; j < P.m; j += 1024) {
                const double c = sqdist<D>(x + i * d, y + j * d, d);
                mx = c > mx ? c : mx;
            }
        }
    }
    mx = block_max1024(mx, sh);
    if (tid == 0) A.stat[k].cmax = mx;
}

// One block (1024 threads) per problem: C scale, S_a, S_b (tree sums of
// sqrt a, sqrt b), alpha_i = s sqrt(a_i) / (S_a S_b), sqrt(b_j)  (eq. (pij-ot)).
__global__ __launch_bounds__(1024) void k_b_prep(BatchArgs A) {
    __shared__ double v[kBatchMaxSide];
    __shared__ double sh[1024];
    const int k = blockIdx.x;
    const BProb P = A.prob[k];
    const double cmax = A.stat[k].cmax;
    for (int64_t i = threadIdx.x; i < P.n; i += blockDim.x) v[i] = sqrt(A.a[P.xo + i]);
    const double sa = block_tree4096(v, P.n, sh);
    for (int64_t j = threadIdx.x; j < P.m; j += blockDim.x) v[j] = sqrt(A.b[P.yo + j]);
    const double sb = block_tree4096(v, P.m, sh);
    const double kappa = P.s / (sa * sb);
    for (int64_t i = threadIdx.x; i < P.n; i += blockDim.x)
        A.row_fac[P.xo + i] = kappa * sqrt(A.a[P.xo + i]);
    for (int64_t j = threadIdx.x; j < P.m; j += blockDim.x) A.col_fac[P.yo + j] = v[j];
    if (threadIdx.x == 0) {
        A.stat[k].inv_cmax = (A.cost == 0 && cmax > 0.0) ? 1.0 / cmax : 1.0;
        A.stat[k].sa = sa;
        A.stat[k].sb = sb;
    }
}

__global__ __launch_bounds__(256) void k_b_mask(BatchArgs A) {
    __shared__ uint64_t tile[kMaskRows][64];
    __shared__ uint32_t cand[4][kMaskCand];
    const int k = owner_of(A.tile_mask, A.count, blockIdx.x);
    const BProb P = A.prob[k];
    const int64_t t = blockIdx.x - A.tile_mask[k];
    const int64_t nct = (P.W + 63) / 64;
    ProbParams pp;
    pp.uot = 0;
    pp.shrink_w = 1.0;
    pp.shrink_c = 0.0;
    pp.cost = SS_COST_SQEUCLID_MAXNORM;   // C = c * inv_cmax (inv_cmax = 1 for the plain cost)
    pp.wfr_w = 0.0;
    pp.row_fac = A.row_fac + P.xo;
    pp.col_fac = A.col_fac + P.yo;
    pp.problem_index = P.pidx;
    pp.k0 = A.k0;
    pp.k1 = A.k1;
    mask_tile<false, 2, false>(pp, P.n, P.m, P.W, t / nct, t % nct, batch_mask_split(P.W),
                               A.mask + P.mo, A.row_cnt + P.xo, 0.0, tile, cand);
}

__global__ __launch_bounds__(256) void k_b_transpose(BatchArgs A) {
    __shared__ uint64_t tile[64][kTrWordCols + 1];
    const int k = owner_of(A.tile_tr, A.count, blockIdx.x);
    const BProb P = A.prob[k];
    const int64_t t = blockIdx.x - A.tile_tr[k];
    const int64_t nct = (P.W + kTrWordCols - 1) / kTrWordCols;
    transpose_tile(A.mask + P.mo, P.n, P.m, P.W, P.Wn, t / nct, t % nct, A.maskT + P.mto,
                   A.col_cnt + P.yo, tile);
}

// Problem of every row and every column (one block per problem).
__global__ __launch_bounds__(256) void k_b_owner(BatchArgs A) {
    const int k = blockIdx.x;
    for (int64_t l = A.row_off[k] + threadIdx.x; l < A.row_off[k + 1]; l += blockDim.x)
        A.owner[l] = k;
    for (int64_t l = A.col_off[k] + threadIdx.x; l < A.col_off[k + 1]; l += blockDim.x)
        A.owner[A.rows + l] = k;
}

// Batched fill in two passes (a batch line has at most 64 mask words:
// SS_BATCH_MAX_SIDE = 4096).  Index pass: the prefix-popcount over a line's
// words gives its local indices in ascending order; kBIdxLines lines per
// wave, 16 lanes a line and four words a lane, so a wave runs four lines'
// chains of dependent loads (owner, problem, words, offset) at once.
constexpr int kBIdxLines = 4;

template <int ROLE>
__global__ __launch_bounds__(256) void k_b_fill_idx(BatchArgs A) {
    constexpr int LL = kWave / kBIdxLines;  // lanes a line
    constexpr int WPL = kWave / LL;         // words a lane
    static_assert(LL * WPL == 64 && SS_BATCH_MAX_SIDE <= 64 * 64, "a line's words fit its lanes");
    const int lane = threadIdx.x & (kWave - 1);
    const int sub = lane % LL;
    const int64_t lines = ROLE == 0 ? A.rows : A.cols;
    const int64_t L = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kBIdxLines + lane / LL;
    // lanes of a line past the end take part in the scan with no words
    const bool live = L < lines;
    uint64_t w[WPL];
    int64_t base = 0;
    if (live) {
        const int k = A.owner[(ROLE == 0 ? 0 : A.rows) + L];
        const BProb P = A.prob[k];
        const int64_t local = L - (ROLE == 0 ? A.row_off : A.col_off)[k];
        const int64_t words = ROLE == 0 ? P.W : P.Wn;
        const uint64_t* bits =
            ROLE == 0 ? A.mask + P.mo + local * P.W : A.maskT + P.mto + local * P.Wn;
        base = (ROLE == 0 ? A.row_ptr : A.col_ptr)[L];
#pragma unroll
        for (int q = 0; q < WPL; ++q) {
            const int wi = sub * WPL + q;
            w[q] = wi < words ? bits[wi] : 0ull;
        }
    } else {
#pragma unroll
        for (int q = 0; q < WPL; ++q) w[q] = 0ull;
    }
    int c = 0;
#pragma unroll
    for (int q = 0; q < WPL; ++q) c += __popcll(w[q]);
    // inclusive scan over the line's lanes (every lane of the wave takes part)
    int incl = c;
#pragma unroll
    for (int d = 1; d < LL; d <<= 1) {
        const int t = __shfl_up(incl, d, LL);
        if (sub >= d) incl += t;
    }
    int64_t pos = base + (incl - c);
    uint16_t* idx = ROLE == 0 ? A.col_idx : A.row_idx;
#pragma unroll
    for (int q = 0; q < WPL; ++q) {
        uint64_t word = w[q];
        const int col0 = 64 * (sub * WPL + q);
        while (word) {
            const int b = __ffsll((unsigned long long)word) - 1;
            word &= word - 1;
            if (pos < A.cap) idx[pos] = (uint16_t)(col0 + b);
            ++pos;
        }
    }
}

// Value pass: one wave per line, two entries per lane at a time.
constexpr int kBValLines = 4;  // lines per wave of the batched value pass

template <int ROLE, int PREC, int D>
__global__ __launch_bounds__(256) void k_b_fill_val(BatchArgs A) {
    // kBValLines lines per wave, kWave / kBValLines lanes each: a line of
    // these problems holds ~8 ln n entries, so a wave per line spent most of
    // its time on the line's chain of dependent loads (owner, problem, offsets,
    // indices, coordinates); four lines a wave run four chains at once
    constexpr int LL = kWave / kBValLines;
    const int lane = threadIdx.x & (kWave - 1);
    const int sub = lane % LL;
    const int64_t lines = ROLE == 0 ? A.rows : A.cols;
    const int64_t L = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kBValLines + lane / LL;
    if (L >= lines) return;  // no wave-wide operation follows
    const int k = A.owner[(ROLE == 0 ? 0 : A.rows) + L];
    const BProb P = A.prob[k];
    const int64_t local = L - (ROLE == 0 ? A.row_off : A.col_off)[k];
    ProbParams pp;
    pp.uot = 0;
    pp.shrink_w = 1.0;
    pp.shrink_c = 0.0;
    pp.cost = SS_COST_SQEUCLID_MAXNORM;   // C = c * inv_cmax (inv_cmax = 1 for the plain cost)
    pp.wfr_w = 0.0;
    pp.s = P.s;
    pp.eps = A.eps;
    pp.inv_cmax = A.stat[k].inv_cmax;
    pp.row_fac = A.row_fac + P.xo;
    pp.col_fac = A.col_fac + P.yo;
    pp.x = A.x + P.xo * A.d;
    pp.y = A.y + P.yo * A.d;
    pp.d = A.d;
    const int64_t* ptr = ROLE == 0 ? A.row_ptr : A.col_ptr;
    const uint16_t* idx = ROLE == 0 ? A.col_idx : A.row_idx;
    void* val = ROLE == 0 ? A.val : A.val_t;
    const int64_t e0 = ptr[L];
    const int64_t e1 = ptr[L + 1] < A.cap ? ptr[L + 1] : A.cap;
    for (int64_t e = e0 + sub; e < e1; e += 2 * LL) {
        const int64_t e2 = e + LL;
        const bool two = e2 < e1;
        const int64_t oa = idx[e];
        const int64_t ob = two ? idx[e2] : oa;
        double la, lb;
        const double va = entry_value<false, D>(pp, 0.0, ROLE == 0 ? local : oa,
                                                ROLE == 0 ? oa : local, &la);
        const double vb = entry_value<false, D>(pp, 0.0, ROLE == 0 ? local : ob,
                                                ROLE == 0 ? ob : local, &lb);
        store_value<PREC>(val, e, va, la);
        if (two) store_value<PREC>(val, e2, vb, lb);
    }
}

__global__ __launch_bounds__(1024) void k_b_empty(BatchArgs A) {
    __shared__ double v[kBatchMaxSide];
    __shared__ double sh[1024];
    const int k = blockIdx.x;
    const BProb P = A.prob[k];
    double res[2][3];
    for (int side = 0; side < 2; ++side) {
        const int64_t n = side == 0 ? P.n : P.m;
        const int64_t o = side == 0 ? P.xo : P.yo;
        const double* a = side == 0 ? A.a : A.b;
        const int32_t* cnt = side == 0 ? A.row_cnt : A.col_cnt;
        double* eff = side == 0 ? A.a_eff : A.b_eff;
        for (int q = 0; q < 3; ++q) {
            for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
                const bool on = cnt[o + i] > 0;
                const double ai = a[o + i];
                v[i] = q == 0 ? (on ? ai : 0.0) : q == 1 ? (on ? 0.0 : ai) : ((!on && ai > 0.0) ? 1.0 : 0.0);
            }
            res[side][q] = block_tree4096(v, n, sh);
        }
        const bool renorm = A.empty_policy == SS_EMPTY_RENORMALIZE;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            const double act = cnt[o + i] > 0 ? a[o + i] : 0.0;
            eff[o + i] = renorm ? act / res[side][0] : act;
        }
    }
    if (threadIdx.x == 0) {
        BStat& S = A.stat[k];
        S.sum_a_act = res[0][0];
        S.dropped_a = res[0][1];
        S.empty_rows = res[0][2];
        S.sum_b_act = res[1][0];
        S.dropped_b = res[1][1];
        S.empty_cols = res[1][2];
        S.nnz = A.row_ptr[P.xo + P.n] - A.row_ptr[P.xo];
    }
}

template <int D>
static void run_b_cmax(const BatchArgs& a, int64_t nt, hipStream_t st) {
    (void)nt;
    hipLaunchKernelGGL(k_b_cmax<D>, dim3((unsigned)a.count), dim3(1024), 0, st, a);
}

template <int PREC, int D>
static void run_b_fill(const BatchArgs& a, hipStream_t st) {
    constexpr int64_t pi = 4 * kBIdxLines;  // lines per block of the index pass
    const dim3 gr((unsigned)((a.rows + pi - 1) / pi)), gc((unsigned)((a.cols + pi - 1) / pi));
    constexpr int64_t per = 4 * kBValLines;  // lines per block of the value pass
    const dim3 vr((unsigned)((a.rows + per - 1) / per)), vc((unsigned)((a.cols + per - 1) / per));
    hipLaunchKernelGGL((k_b_fill_idx<0>), gr, dim3(256), 0, st, a);
    hipLaunchKernelGGL((k_b_fill_val<0, PREC, D>), vr, dim3(256), 0, st, a);
    hipLaunchKernelGGL((k_b_fill_idx<1>), gc, dim3(256), 0, st, a);
    hipLaunchKernelGGL((k_b_fill_val<1, PREC, D>), vc, dim3(256), 0, st, a);
}

template <int D>
static void run_b_fill_d(int precision, const BatchArgs& a, hipStream_t st) {
    if (precision == P_F64)
        run_b_fill<P_F64, D>(a, st);
    else
        run_b_fill<P_F32, D>(a, st);
}

hipError_t launch_batch_sample(int precision, const BatchArgs& a, int64_t ntile_cmax,
                               int64_t ntile_mask, int64_t ntile_tr, int64_t* scan_scratch,
                               hipStream_t st) {
    hipError_t e = launch_fill_f64(a.gstats, ST_COUNT, 0.0, st);
    if (e == hipSuccess) e = launch_fill_u32((uint32_t*)a.stat, (int64_t)a.count * sizeof(BStat) / 4, 0u, st);
    if (e == hipSuccess) e = launch_fill_i32(a.row_cnt, a.rows, 0, st);
    if (e == hipSuccess) e = launch_fill_i32(a.col_cnt, a.cols, 0, st);
    if (e == hipSuccess) e = launch_validate(a.a, a.rows, a.x, a.rows * a.d, a.gstats, st);
    if (e == hipSuccess) e = launch_validate(a.b, a.cols, a.y, a.cols * a.d, a.gstats, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_b_owner, dim3(a.count), dim3(256), 0, st, a);
    SS_DISPATCH_D(a.d, run_b_cmax, a, ntile_cmax, st);
    hipLaunchKernelGGL(k_b_prep, dim3(a.count), dim3(1024), 0, st, a);
    hipLaunchKernelGGL(k_b_mask, dim3((unsigned)ntile_mask), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_b_transpose, dim3((unsigned)ntile_tr), dim3(256), 0, st, a);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_scan(a.row_cnt, a.rows, a.row_ptr, scan_scratch, st);
    if (e == hipSuccess) e = launch_scan(a.col_cnt, a.cols, a.col_ptr, scan_scratch, st);
    if (e != hipSuccess) return e;
    SS_DISPATCH_D(a.d, run_b_fill_d, precision, a, st);
    hipLaunchKernelGGL(k_b_empty, dim3(a.count), dim3(1024), 0, st, a);
    return hipGetLastError();
}

}  // namespace ss
