// Learned warm start: a DeepSets network predicting the initial scalings of
// Alg. 1 for every problem of a batch, its training step (forward, backward,
// Adam) on the GPU.  Hidden width 256, BF16 weights and activations into the
// matrix cores, FP32 accumulation.
//
// Points enter in kernel units: centred on the mean of all points of their
// problem and divided by sqrt(eps C_s), C_s = max_ij |x_i - y_j|^2 for the
// max-normalised cost (1 for the plain cost), so that the Gibbs kernel of eq.
// (rot) reads exp(-|x' - y'|^2).  For the side predicting the scalings of
// points z_i (weights w_i) given the opposite measure (o_j, q_j), j < m:
//   phi_j = ReLU(P [o_j, m q_j] + p),  e = mean_j phi_j,  g = U e + c1
//   h1_i  = ReLU(W1 z_i + g),  h2_i = ReLU(W2 h1_i + c2),  psi_i = w3 . h2_i + c3
//   log y0_i = log w_i + psi_i
// Sinkhorn's first update reads only v^0 and (u, v) -> (c u, v / c) leaves
// the plan unchanged (eq. (rot-solu)), so the loss of a side is the centred
// squared error mean_M (d - mean_M d)^2, d = psi - (log y* - log w), over the
// points M with a finite target; the batch loss is the mean over all sides.
//
// Kernels (all sums in a fixed order; no atomics on values):
//   k_ws_cmax       one block per problem: max squared distance (pruned)
//   k_ws_prep       one block per problem: centre and kernel length
//   k_ws_embed_part (side, chunk of opposite points) blocks: partial phi sums
//                   on the FP32 matrix cores
//   k_ws_embed      one block per side: e, g; the side's tile tables
//   k_ws_head_fwd   forward head for prediction: both layers transposed on the
//                   matrix cores, W2 in registers, loads a group ahead
//   k_ws_head_train persistent blocks over 16-point tiles of all sides.  W2
//                   stays in LDS (padded rows); h2 = ReLU(h1 W2^T + c2) on
//                   MFMA 16x16x32 BF16.  Recomputes the forward,
//                   dz2 = dpsi w3 [z2 > 0], dh1 = dz2 W2 (MFMA, W2^T from
//                   global), dz1 = dh1 [h1 > 0]; per-block sums of dW1, dc2,
//                   dw3, dc3, per-tile sums of dg; h1 and dz2 rows go to
//                   scratch for dW2.
//   k_ws_centre     one block per side: loss, dL/dpsi
//   k_ws_dw2        dW2 = sum_i dz2_i^T h1_i: chunks of points, MFMA, partials
//   k_ws_embed_bwd  one block per side: dg, de = U^T dg, dP, dp partials
//   k_ws_du         dU = sum_sides dg e^T
//   k_ws_reduce     the gradient vector from all partials
//   k_ws_adam       Adam (Kingma & Ba, ICLR 2015), BF16 copies of the weights
#include <math.h>

#include "common.hpp"
#include "internal.hpp"

namespace ss {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kH = 256;            // hidden width
constexpr int kTile = 16;          // points per head tile
constexpr int kPad = kH + 8;       // padded LDS row (bf16 elements): spreads banks
constexpr int kChunk = 2048;       // points per dW2 block
constexpr int kSub = 32;           // points per dW2 MFMA step
constexpr int kSubPad = kSub + 8;

// parameter layout (FP32 master, BF16 copy): P, p, W1, U, c1, W2, c2, w3, c3
constexpr int OFF_P = 0, OFF_p = 1024, OFF_W1 = 1280, OFF_U = 2048, OFF_c1 = 67584,
              OFF_W2 = 67840, OFF_c2 = 133376, OFF_w3 = 133632, OFF_c3 = 133888;
constexpr int kParams = 133889;
static_assert(kParams == SS_MLP_PARAMS, "parameter layout");
// per-block training partial: dW1 (768), dc2 (256), dw3 (256), dc3 (1)
constexpr int kBlkPart = 768 + 256 + 256 + 1;
// per-side embedding partial: dP (1024), dp (256)
constexpr int kSidePart = 1280;

__device__ __forceinline__ float bf(const __bf16* w, int i) { return (float)w[i]; }

__device__ __forceinline__ const double* side_pts(const MlpArgs& A, const WSide& S) {
    return S.which == 0 ? A.x : A.y;
}

// Phi pre-activation of hidden unit t for opposite point f (4 features).
__device__ __forceinline__ float phi_pre(const __bf16* wb, int t, const float* f) {
    float z = bf(wb, OFF_p + t);
#pragma unroll
    for (int c = 0; c < 4; ++c) z = fmaf(bf(wb, OFF_P + 4 * t + c), f[c], z);
    return z;
}

__device__ __forceinline__ void opp_feature(const MlpArgs& A, const WSide& S, int64_t j, float* f) {
    const double* o = S.which == 0 ? A.y : A.x;
    const double* q = S.which == 0 ? A.b : A.a;
    const float* xf = A.xform + 4 * S.prob;
    const int64_t r = S.opp_off + j;
    f[0] = ((float)o[3 * r + 0] - xf[0]) * xf[3];
    f[1] = ((float)o[3 * r + 1] - xf[1]) * xf[3];
    f[2] = ((float)o[3 * r + 2] - xf[2]) * xf[3];
    f[3] = (float)((double)S.nopp * q[r]);
}

// ---------------------------------------------------------------- inputs
// C_s = max |x_i - y_j|^2 per problem (FP32, a feature scale), one block of
// 1024 threads per problem, exact with pruning: with c the centre of the
// bounding box of all points, R = max_j |y_j - c| and r_i = |x_i - c|, every
// pair of row i has |x_i - y_j| <= r_i + R.  The row with the largest r_i
// gives a lower bound L (its exact maximum); only rows with
// (r_i + R)^2 (1 + 2^-16) >= L can hold a larger pair (the margin covers the
// FP32 rounding of the bounds and of the pair distances), and they are
// scanned exactly.  Pair distances are formed as in a full scan,
// (d0 d0 + d1 d1) + d2 d2 from FP32 coordinates, and the maximum is
// order-free, so the result equals the full scan's.
constexpr int kCmaxThreads = 1024;

__device__ __forceinline__ float ws_d2(float a0, float a1, float a2, float b0, float b1,
                                       float b2) {
    const float d0 = a0 - b0, d1 = a1 - b1, d2 = a2 - b2;
    return d0 * d0 + d1 * d1 + d2 * d2;
}

__device__ __forceinline__ float block_max_f(float v, float* sh) {
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    float r = sh[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmaxf(r, sh[w]);
    return r;
}

__global__ __launch_bounds__(kCmaxThreads) void k_ws_cmax(MlpArgs A) {
    __shared__ float sh[16];
    __shared__ float rx[kBatchMaxSide];
    __shared__ float xsurv[kBatchMaxSide][3];
    __shared__ int nrows;
    const int k = blockIdx.x, t = threadIdx.x;
    const WSide S = A.sides[2 * k];
    const int64_t n = S.npts, m = S.nopp;
    const double* x = A.x + 3 * S.pts_off;
    const double* y = A.y + 3 * S.opp_off;
    // bounding box of x and y (min and max are order-free)
    float c[3];
    for (int d = 0; d < 3; ++d) {
        float lo = INFINITY, hi = -INFINITY;
        for (int64_t i = t; i < n; i += blockDim.x) {
            const float v = (float)x[3 * i + d];
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
        }
        for (int64_t j = t; j < m; j += blockDim.x) {
            const float v = (float)y[3 * j + d];
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
        }
        hi = block_max_f(hi, sh);
        lo = -block_max_f(-lo, sh);
        c[d] = 0.5f * (lo + hi);
    }
    float ry = 0.0f;
    for (int64_t j = t; j < m; j += blockDim.x)
        ry = fmaxf(ry, ws_d2((float)y[3 * j], (float)y[3 * j + 1], (float)y[3 * j + 2], c[0], c[1],
                             c[2]));
    const float R = sqrtf(block_max_f(ry, sh));
    float best = -1.0f;
    int besti = 0;
    for (int64_t i = t; i < n; i += blockDim.x) {
        const float r = sqrtf(ws_d2((float)x[3 * i], (float)x[3 * i + 1], (float)x[3 * i + 2], c[0],
                                    c[1], c[2]));
        rx[i] = r;
        if (r > best) {
            best = r;
            besti = (int)i;
        }
    }
    // the row of the largest r_i (any of the largest: the bound only needs one)
    const float bmax = block_max_f(best, sh);
    __syncthreads();
    if (t == 0) nrows = n;
    __syncthreads();
    if (best == bmax) atomicMin(&nrows, besti);
    __syncthreads();
    const int64_t istar = nrows;
    const float a0 = (float)x[3 * istar], a1 = (float)x[3 * istar + 1], a2 = (float)x[3 * istar + 2];
    float lm = 0.0f;
    for (int64_t j = t; j < m; j += blockDim.x)
        lm = fmaxf(lm, ws_d2(a0, a1, a2, (float)y[3 * j], (float)y[3 * j + 1], (float)y[3 * j + 2]));
    const float L = block_max_f(lm, sh);
    // rows that may hold a larger pair (list order is free: the maximum is)
    __syncthreads();
    if (t == 0) nrows = 0;
    __syncthreads();
    for (int64_t i = t; i < n; i += blockDim.x) {
        const float ub = (rx[i] + R) * (rx[i] + R) * (1.0f + 0x1p-16f);
        if (ub >= L && i != istar) {
            const int q = atomicAdd(&nrows, 1);
            xsurv[q][0] = (float)x[3 * i];
            xsurv[q][1] = (float)x[3 * i + 1];
            xsurv[q][2] = (float)x[3 * i + 2];
        }
    }
    __syncthreads();
    const int nr = nrows;
    // each thread's columns in registers, the surviving rows from LDS
    constexpr int CPT = kBatchMaxSide / kCmaxThreads;
    float b[CPT][3];
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int64_t j = t + (int64_t)u * blockDim.x;
        const int64_t jj = j < m ? j : m - 1;  // past the end: repeats column m - 1
        b[u][0] = (float)y[3 * jj];
        b[u][1] = (float)y[3 * jj + 1];
        b[u][2] = (float)y[3 * jj + 2];
    }
    float mx = L;
    for (int q = 0; q < nr; ++q) {
        const float a0 = xsurv[q][0], a1 = xsurv[q][1], a2 = xsurv[q][2];
#pragma unroll
        for (int u = 0; u < CPT; ++u) mx = fmaxf(mx, ws_d2(a0, a1, a2, b[u][0], b[u][1], b[u][2]));
    }
    mx = block_max_f(mx, sh);
    if (t == 0) A.xform[4 * k + 3] = mx;
}

// One block per problem: the mean of all its points (fixed order) and the
// kernel-length factor 1 / sqrt(eps C_s) (C_s from k_ws_cmax, or 1).
__global__ __launch_bounds__(256) void k_ws_prep(MlpArgs A) {
    __shared__ double sh[16];
    const int k = blockIdx.x;
    const WSide S = A.sides[2 * k];
    // the side of each embedding chunk of this problem's two sides
    for (int h = 0; h < 2; ++h) {
        const WSide& Sh = A.sides[2 * k + h];
        for (int c = threadIdx.x; c < Sh.nemb; c += blockDim.x) A.emb_side[Sh.emb0 + c] = 2 * k + h;
    }
    const int64_t n = S.npts, m = S.nopp;
    const double* x = A.x + 3 * S.pts_off;
    const double* y = A.y + 3 * S.opp_off;
    double c[3];
    for (int d = 0; d < 3; ++d) {
        double v = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) v += x[3 * i + d];
        for (int64_t j = threadIdx.x; j < m; j += blockDim.x) v += y[3 * j + d];
        c[d] = block_sum(v, sh) / (double)(n + m);
    }
    if (threadIdx.x == 0) {
        float* xf = A.xform + 4 * k;
        float cs = A.cost == 0 ? xf[3] : 1.0f;
        if (!(cs > 0.0f)) cs = 1.0f;
        xf[0] = (float)c[0];
        xf[1] = (float)c[1];
        xf[2] = (float)c[2];
        xf[3] = (float)(1.0 / sqrt(A.eps * (double)cs));
    }
}

// ---------------------------------------------------------------- embedding
// columns of U per LDS stage of g = U e + c1
constexpr int kEmbUCols = 64;

// Partial sums of phi over one chunk of kWsEmbPart opposite points of a side
// (chunks keep the blocks' work equal whatever the sides' sizes).
// phi_j = ReLU(P f_j + p) as (hidden unit) x (point) tiles on the FP32 MFMA
// 16x16x4 (k = the 4 features): wave wv owns units [64 wv, 64 wv + 64);
// A fragments P[unit][feature], the bias p as the accumulator input; lane
// (lr, lg) of a product holds units 16 ut + 4 lg + r of point lr and sums
// their ReLUs over its points; the 16 point classes are then added in class
// order.
__global__ __launch_bounds__(256, 4) void k_ws_embed_part(MlpArgs A) {
    __shared__ __align__(16) float4 fs[kWsEmbPart];
    __shared__ float red[16][kH];
    const int c = blockIdx.x, t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6, lr = lane & 15, lg = lane >> 4;
    const int s = A.emb_side[c];
    const WSide S = A.sides[s];
    const __bf16* wb = (const __bf16*)A.wbf;
    const int64_t j0 = (c - S.emb0) * (int64_t)kWsEmbPart;
    const int cnt = (int)(S.nopp - j0 < kWsEmbPart ? S.nopp - j0 : kWsEmbPart);
    {
        float f[kWsEmbPart / 256][4];
#pragma unroll
        for (int k = 0; k < kWsEmbPart / 256; ++k)
            if (t + 256 * k < cnt) opp_feature(A, S, j0 + t + 256 * k, f[k]);
#pragma unroll
        for (int k = 0; k < kWsEmbPart / 256; ++k)
            if (t + 256 * k < cnt) fs[t + 256 * k] = make_float4(f[k][0], f[k][1], f[k][2], f[k][3]);
    }
    float pa[4];
    floatx4 pb[4], acc[4];
#pragma unroll
    for (int ut = 0; ut < 4; ++ut) {
        const int u = 64 * wv + 16 * ut;
        pa[ut] = bf(wb, OFF_P + 4 * (u + lr) + lg);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            pb[ut][r] = bf(wb, OFF_p + u + 4 * lg + r);
            acc[ut][r] = 0.0f;
        }
    }
    __syncthreads();
    // two 16-point tiles per step: eight independent products; points past
    // the chunk's end add zero
    for (int p0 = 0; p0 < cnt; p0 += 32) {
        float fb[2];
        bool live[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            live[h] = p0 + 16 * h + lr < cnt;
            fb[h] = ((const float*)fs)[4 * (p0 + 16 * h + lr) + lg];
        }
        floatx4 d[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int ut = 0; ut < 4; ++ut)
                d[h][ut] = __builtin_amdgcn_mfma_f32_16x16x4f32(pa[ut], fb[h], pb[ut], 0, 0, 0);
        if (p0 + 32 <= cnt) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int ut = 0; ut < 4; ++ut)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[ut][r] += fmaxf(d[h][ut][r], 0.0f);
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int ut = 0; ut < 4; ++ut)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        acc[ut][r] += live[h] ? fmaxf(d[h][ut][r], 0.0f) : 0.0f;
        }
    }
#pragma unroll
    for (int ut = 0; ut < 4; ++ut)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[lr][64 * wv + 16 * ut + 4 * lg + r] = acc[ut][r];
    __syncthreads();
    float sum = 0.0f;
    for (int q = 0; q < 16; ++q) sum += red[q][t];
    A.embp[(int64_t)c * kH + t] = sum;
}

// One block per side: e = (chunk sums in chunk order) / m, g = U e + c1, and
// the side's tile tables for the forward head.  Every loop issues its loads
// together before using them (a side has at most 8 chunks and 4096 points).
__global__ __launch_bounds__(256) void k_ws_embed(MlpArgs A) {
    __shared__ float e_s[kH];
    __shared__ __align__(16) __bf16 us[kH][kEmbUCols + 8];
    const int s = blockIdx.x, t = threadIdx.x;
    const WSide S = A.sides[s];
    const __bf16* wb = (const __bf16*)A.wbf;
    constexpr int kMaxChunks = (kBatchMaxSide + kWsEmbPart - 1) / kWsEmbPart;
    float ps[kMaxChunks];
#pragma unroll
    for (int c = 0; c < kMaxChunks; ++c)
        ps[c] = c < S.nemb ? A.embp[(S.emb0 + c) * kH + t] : 0.0f;
    float sum = 0.0f;
#pragma unroll
    for (int c = 0; c < kMaxChunks; ++c)
        if (c < S.nemb) sum += ps[c];
    const float e = sum / (float)S.nopp;
    e_s[t] = e;
    A.emb[(int64_t)s * kH + t] = e;
    // g = U e + c1: U staged in LDS by column chunks (16-byte row pieces),
    // each unit accumulating its row in column order
    float g = bf(wb, OFF_c1 + t);
    constexpr int kPieces = kH * kEmbUCols / 8;  // 16-byte pieces per chunk
    for (int c0 = 0; c0 < kH; c0 += kEmbUCols) {
        bf16x8 pc[kPieces / 256];
#pragma unroll
        for (int k = 0; k < kPieces / 256; ++k) {
            const int i = t + 256 * k, u = i / (kEmbUCols / 8), q = 8 * (i % (kEmbUCols / 8));
            pc[k] = *(const bf16x8*)(wb + OFF_U + u * kH + c0 + q);
        }
        __syncthreads();  // e_s written / the previous chunk read
#pragma unroll
        for (int k = 0; k < kPieces / 256; ++k) {
            const int i = t + 256 * k, u = i / (kEmbUCols / 8), q = 8 * (i % (kEmbUCols / 8));
            *(bf16x8*)&us[u][q] = pc[k];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kEmbUCols; q += 8) {
            const bf16x8 r = *(const bf16x8*)&us[t][q];
#pragma unroll
            for (int c = 0; c < 8; ++c) g = fmaf((float)r[c], e_s[c0 + q + c], g);
        }
    }
    A.gvec[(int64_t)s * kH + t] = g;
    // this side's own points in kernel units and the logs of their masses,
    // tile-padded with zeros, and its tile records, for the forward head
    // (the arithmetic of the head's coordinate transform, done once per point)
    const float* xf = A.xform + 4 * S.prob;
    const double* __restrict__ pts = side_pts(A, S) + 3 * S.pts_off;
    const double* __restrict__ w = (S.which == 0 ? A.a : A.b) + S.pts_off;
    float4* __restrict__ tp = (float4*)A.tpts + S.tile0 * kTile;
    double* __restrict__ tl = A.tlw + S.tile0 * kTile;
    const int npad = (int)(S.ntiles * kTile);
    constexpr int kPer = 4;  // points per thread per round, loads first
    for (int i0 = 0; i0 < npad; i0 += 256 * kPer) {
        double q[kPer][4];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int i = i0 + t + 256 * k;
            const bool live = i < S.npts;
            q[k][0] = live ? pts[3 * i + 0] : 0.0;
            q[k][1] = live ? pts[3 * i + 1] : 0.0;
            q[k][2] = live ? pts[3 * i + 2] : 0.0;
            q[k][3] = live ? w[i] : 1.0;
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int i = i0 + t + 256 * k;
            if (i >= npad) continue;
            float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            double lw = 0.0;
            if (i < S.npts) {
                v.x = ((float)q[k][0] - xf[0]) * xf[3];
                v.y = ((float)q[k][1] - xf[1]) * xf[3];
                v.z = ((float)q[k][2] - xf[2]) * xf[3];
                lw = log(q[k][3]);
            }
            tp[i] = v;
            tl[i] = lw;
        }
    }
    for (int64_t k = t; k < S.ntiles; k += blockDim.x) {
        WTile rec;
        rec.pt = S.pt0 + k * kTile;
        rec.row = S.pts_off + k * kTile;
        rec.side = s;
        rec.nrow = (int)(S.npts - k * kTile < kTile ? S.npts - k * kTile : kTile);
        rec.which = S.which;
        rec.pad = 0;
        A.tiles[S.tile0 + k] = rec;
    }
}

// ---------------------------------------------------------------- head
__global__ __launch_bounds__(256) void k_ws_head_train(MlpArgs A) {
    extern __shared__ __align__(16) unsigned char dsm[];
    __bf16* w2s = (__bf16*)dsm;                 // [kH][kPad]  W2 rows (out n, in k)
    __bf16* h1s = w2s + kH * kPad;              // [kTile][kPad]
    __bf16* dz2s = h1s + kTile * kPad;          // [kTile][kPad] (training)
    __shared__ float xs[kTile][3];
    __shared__ float dps[kTile];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const __bf16* wb = (const __bf16*)A.wbf;
    // W2 into LDS once per block
    for (int i = tid; i < kH * (kH / 8); i += 256) {
        const int n = i / (kH / 8), k8 = (i % (kH / 8)) * 8;
        *(bf16x8*)(w2s + n * kPad + k8) = *(const bf16x8*)(wb + OFF_W2 + n * kH + k8);
    }
    // per-block training sums (thread t owns hidden unit t of dc2/dw3; dW1 row t)
    float bw1[3] = {0.f, 0.f, 0.f}, bc2 = 0.f, bw3 = 0.f, bc3 = 0.f;
    const float w1t[3] = {bf(wb, OFF_W1 + 3 * tid), bf(wb, OFF_W1 + 3 * tid + 1),
                          bf(wb, OFF_W1 + 3 * tid + 2)};
    __syncthreads();
    for (int64_t tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
        // the side owning this tile
        int lo = 0, hi = A.nsides - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (A.sides[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
        }
        const WSide S = A.sides[lo];
        const int64_t i0 = (tile - S.tile0) * kTile;
        const int nrow = (int)(S.npts - i0 < kTile ? S.npts - i0 : kTile);
        const double* z = side_pts(A, S);
        if (tid < kTile * 3) {
            const int r = tid / 3, c = tid % 3;
            const float* xf = A.xform + 4 * S.prob;
            xs[r][c] = r < nrow ? ((float)z[3 * (S.pts_off + i0 + r) + c] - xf[c]) * xf[3] : 0.0f;
        }
        if (tid < kTile) dps[tid] = tid < nrow ? A.dpsi[S.pt0 + i0 + tid] : 0.0f;
        __syncthreads();
        // h1 rows (thread = hidden unit)
        const float g = A.gvec[(int64_t)lo * kH + tid];
        for (int r = 0; r < kTile; ++r) {
            float z1 = g;
#pragma unroll
            for (int c = 0; c < 3; ++c) z1 = fmaf(w1t[c], xs[r][c], z1);
            h1s[r * kPad + tid] = (__bf16)(r < nrow ? fmaxf(z1, 0.0f) : 0.0f);
        }
        __syncthreads();
        // z2 = h1 W2^T: wave wv owns output columns [64 wv, 64 wv + 64)
        floatx4 acc[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < kH / 32; ++ks) {
            const int kk = 32 * ks + 8 * (lane >> 4);
            const bf16x8 a = *(const bf16x8*)(h1s + (lane & 15) * kPad + kk);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                const int n = 64 * wv + 16 * ct + (lane & 15);
                const bf16x8 b = *(const bf16x8*)(w2s + n * kPad + kk);
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[ct], 0, 0, 0);
            }
        }
        // h2 = ReLU(z2 + c2) (psi itself comes from the forward head)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int n = 64 * wv + 16 * ct + (lane & 15);
            const float c2 = bf(wb, OFF_c2 + n);
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[ct][r] = fmaxf(acc[ct][r] + c2, 0.0f);
        }
        __syncthreads();
        // ---- backward of the tile
        float gc2[4] = {0.f, 0.f, 0.f, 0.f}, gw3[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int n = 64 * wv + 16 * ct + (lane & 15);
            const float w3 = bf(wb, OFF_w3 + n);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 4 * (lane >> 4) + r;
                const float h2 = acc[ct][r];
                const float d = dps[row];
                const float dz = h2 > 0.0f ? d * w3 : 0.0f;
                gc2[ct] += dz;
                gw3[ct] = fmaf(d, h2, gw3[ct]);
                dz2s[row * kPad + n] = (__bf16)dz;
            }
        }
        __syncthreads();
        // dh1 = dz2 W2 (B operand: W2^T rows from global, k = output index n)
        floatx4 dacc[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) dacc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
        const __bf16* w2t = (const __bf16*)A.w2t;
#pragma unroll
        for (int ks = 0; ks < kH / 32; ++ks) {
            const int kk = 32 * ks + 8 * (lane >> 4);
            const bf16x8 a = *(const bf16x8*)(dz2s + (lane & 15) * kPad + kk);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                const int c = 64 * wv + 16 * ct + (lane & 15);
                const bf16x8 b = *(const bf16x8*)(w2t + c * kH + kk);
                dacc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, dacc[ct], 0, 0, 0);
            }
        }
        __syncthreads();  // every wave has read dz2s
        {
            __bf16* h1g = (__bf16*)A.h1g;
            __bf16* dz2g = (__bf16*)A.dz2g;
            for (int r = 0; r < nrow; ++r) {
                const int64_t pt = S.pt0 + i0 + r;
                h1g[pt * kH + tid] = h1s[r * kPad + tid];
                dz2g[pt * kH + tid] = dz2s[r * kPad + tid];
            }
        }
        __syncthreads();  // dz2s is reused below
        // dz1 = dh1 [h1 > 0]; sums over the tile's rows per hidden unit
        float gdg[4] = {0.f, 0.f, 0.f, 0.f}, gw1[4][3];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            gw1[ct][0] = gw1[ct][1] = gw1[ct][2] = 0.f;
            const int c = 64 * wv + 16 * ct + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 4 * (lane >> 4) + r;
                const float h1 = (float)h1s[row * kPad + c];
                const float dz1 = h1 > 0.0f ? dacc[ct][r] : 0.0f;
                gdg[ct] += dz1;
#pragma unroll
                for (int q = 0; q < 3; ++q) gw1[ct][q] = fmaf(dz1, xs[row][q], gw1[ct][q]);
            }
        }
        // reduce over the 4 row groups of the wave (lanes 16 apart)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            float* v[6] = {&gc2[ct], &gw3[ct], &gdg[ct], &gw1[ct][0], &gw1[ct][1], &gw1[ct][2]};
#pragma unroll
            for (int u = 0; u < 6; ++u) {
                float x = *v[u];
                x += __shfl_xor(x, 16, 64);
                x += __shfl_xor(x, 32, 64);
                *v[u] = x;
            }
        }
        // lanes 0..15 of each wave hold columns 64 wv + 16 ct + lane: hand the
        // per-unit values to thread = unit through LDS (dz2s as floats)
        float* red = (float*)dz2s;  // [6][kH]
        if (lane < 16) {
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                const int c = 64 * wv + 16 * ct + lane;
                red[0 * kH + c] = gc2[ct];
                red[1 * kH + c] = gw3[ct];
                red[2 * kH + c] = gdg[ct];
                red[3 * kH + c] = gw1[ct][0];
                red[4 * kH + c] = gw1[ct][1];
                red[5 * kH + c] = gw1[ct][2];
            }
        }
        __syncthreads();
        bc2 += red[0 * kH + tid];
        bw3 += red[1 * kH + tid];
        A.dgp[tile * kH + tid] = red[2 * kH + tid];
        bw1[0] += red[3 * kH + tid];
        bw1[1] += red[4 * kH + tid];
        bw1[2] += red[5 * kH + tid];
        if (tid == 0) {
            float sd = 0.f;
            for (int r = 0; r < kTile; ++r) sd += dps[r];
            bc3 += sd;
        }
        __syncthreads();
    }
    float* part = A.blkp + (int64_t)blockIdx.x * kBlkPart;
    part[3 * tid + 0] = bw1[0];
    part[3 * tid + 1] = bw1[1];
    part[3 * tid + 2] = bw1[2];
    part[768 + tid] = bc2;
    part[1024 + tid] = bw3;
    if (tid == 0) part[1280] = bc3;
}

// Forward head for prediction: the forward arithmetic of k_ws_head_train per point,
// arranged for the matrix cores.  Both layers are computed transposed, as
// (hidden unit) x (point) tiles, so that a lane's accumulators hold several
// hidden units of one point and the output layer reduces in registers:
//  * first layer: W1 [x; 0] on the FP32 MFMA 16x16x4 (k = 3 is the zero
//    fourth coordinate), plus the side's bias g, ReLU, BF16 rows into LDS;
//  * second layer: W2 h1 on MFMA 16x16x32 BF16 with FP32 accumulation.  Wave
//    wv owns hidden units [64 wv, 64 wv + 64); its A fragments of W2 (4 unit
//    tiles x 8 k-steps of 8 BF16, 128 VGPRs) are loaded once per block;
//  * output: w3 . ReLU(h2 + c2) summed over a lane's 16 units, the 16 partial
//    sums of a point (4 waves x 4 lane groups) added in a fixed order.
// A block takes a contiguous range of 16-point tiles and works through it in
// groups of kSubT tiles (the rows of a group may come from several sides:
// only the first layer's bias belongs to a side).  Points come in kernel
// units from the tile-padded table k_ws_embed writes, so every load of a
// group has an address known a group ahead: the tile records two groups
// ahead, the coordinates and biases one group ahead, all in flight while
// the matrix cores work.
constexpr int kHeadGroup = 2;  // tiles per group: 2 fits 256 VGPRs at two waves per SIMD

template <int kSubT>
__global__ __launch_bounds__(256, 2) void k_ws_head_fwd(MlpArgs A) {
    constexpr int kRows = kSubT * kTile;  // points of a group
    __shared__ __align__(16) __bf16 h1s[kRows * kPad];
    __shared__ __align__(16) float xs[2][kRows][4];
    __shared__ __align__(16) float gl[2][kSubT][kH];
    __shared__ __align__(16) float cw[2][kH];  // c2, w3
    __shared__ float psum[4][4][kRows];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const __bf16* wb = (const __bf16*)A.wbf;
    const int64_t t0 = A.ntiles * blockIdx.x / gridDim.x;
    const int64_t t1 = A.ntiles * (blockIdx.x + 1) / gridDim.x;
    if (t0 >= t1) return;
    bf16x8 bw[4][kH / 32];
#pragma unroll
    for (int ut = 0; ut < 4; ++ut) {
        const int u = 64 * wv + 16 * ut + lr;
#pragma unroll
        for (int ks = 0; ks < kH / 32; ++ks)
            bw[ut][ks] = *(const bf16x8*)(wb + OFF_W2 + u * kH + 32 * ks + 8 * lg);
    }
    // first-layer A fragments: W1[unit][k], k = lane group (k = 3 is zero)
    float w1f[4];
#pragma unroll
    for (int ut = 0; ut < 4; ++ut) {
        const int u = 64 * wv + 16 * ut + lr;
        w1f[ut] = lg < 3 ? bf(wb, OFF_W1 + 3 * u + lg) : 0.0f;
    }
    cw[0][tid] = bf(wb, OFF_c2 + tid);
    cw[1][tid] = bf(wb, OFF_w3 + tid);
    const float c3 = bf(wb, OFF_c3);
    const float* tpts = A.tpts;
    // loads of group `tile`: its side indices (from the tile records), its
    // coordinates (thread tid < 4 kRows: row tid / 4, axis tid % 4), its
    // biases (unit tid) and its output records (thread tid < kRows); tiles
    // past the block's range read as side 0 / zero
    auto side_at = [&](int64_t tile) { return tile < t1 ? A.tiles[tile].side : 0; };
    auto coord_at = [&](int64_t tile) {
        return tid < 4 * kRows && tile * kTile * 4 + tid < t1 * kTile * 4
                   ? tpts[tile * kTile * 4 + tid] : 0.0f;
    };
    auto rec_at = [&](int64_t tile, WTile* r) {
        if (tid < kRows && tile + tid / kTile < t1) *r = A.tiles[tile + tid / kTile];
    };
    int sideN[kSubT];
    WTile recN;
    recN.nrow = 0;
    // the first group's coordinates and biases go to buffer 0
    {
#pragma unroll
        for (int q = 0; q < kSubT; ++q) sideN[q] = side_at(t0 + q);
#pragma unroll
        for (int q = 0; q < kSubT; ++q) gl[0][q][tid] = A.gvec[(int64_t)sideN[q] * kH + tid];
        if (tid < kRows * 4) xs[0][tid >> 2][tid & 3] = coord_at(t0);
    }
    rec_at(t0, &recN);
    // the second group's sides, coordinates and biases are in flight
#pragma unroll
    for (int q = 0; q < kSubT; ++q) sideN[q] = side_at(t0 + kSubT + q);
    float gN[kSubT];
#pragma unroll
    for (int q = 0; q < kSubT; ++q) gN[q] = A.gvec[(int64_t)sideN[q] * kH + tid];
    float xN = coord_at(t0 + kSubT);
#pragma unroll
    for (int q = 0; q < kSubT; ++q) sideN[q] = side_at(t0 + 2 * kSubT + q);
    __syncthreads();
    int buf = 0;
    for (int64_t tile = t0; tile < t1; tile += kSubT) {
        // this group's output record (loaded a group ago) and mass logs (read
        // after the products); the next group's record
        const WTile rec = recN;
        const bool store = tid < kRows && tile + tid / kTile < t1;
        const double lw = store ? A.tlw[tile * kTile + tid] : 0.0;
        rec_at(tile + kSubT, &recN);
        // first layer, bias g as the accumulator input: rows past a side's
        // end come from zero coordinates and are never stored (points do not
        // mix)
#pragma unroll
        for (int pt = 0; pt < kSubT; ++pt) {
            const float xb = xs[buf][kTile * pt + lr][lg];
#pragma unroll
            for (int ut = 0; ut < 4; ++ut) {
                const float4 g = *(const float4*)&gl[buf][pt][64 * wv + 16 * ut + 4 * lg];
                const floatx4 d = __builtin_amdgcn_mfma_f32_16x16x4f32(
                    w1f[ut], xb, floatx4{g.x, g.y, g.z, g.w}, 0, 0, 0);
                typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
                bf16x4 h;
                h[0] = (__bf16)fmaxf(d[0], 0.0f);
                h[1] = (__bf16)fmaxf(d[1], 0.0f);
                h[2] = (__bf16)fmaxf(d[2], 0.0f);
                h[3] = (__bf16)fmaxf(d[3], 0.0f);
                *(bf16x4*)(h1s + (kTile * pt + lr) * kPad + 64 * wv + 16 * ut + 4 * lg) = h;
            }
        }
        __syncthreads();
        // the next group's coordinates and biases into the other buffer (its
        // previous contents were read before the barrier above), the loads
        // for the group after it issued
        if (tid < kRows * 4) xs[buf ^ 1][tid >> 2][tid & 3] = xN;
#pragma unroll
        for (int q = 0; q < kSubT; ++q) gl[buf ^ 1][q][tid] = gN[q];
#pragma unroll
        for (int q = 0; q < kSubT; ++q) gN[q] = A.gvec[(int64_t)sideN[q] * kH + tid];
        xN = coord_at(tile + 2 * kSubT);
#pragma unroll
        for (int q = 0; q < kSubT; ++q) sideN[q] = side_at(tile + 3 * kSubT + q);
        // second layer, c2 as the accumulator input
        floatx4 acc[kSubT][4];
#pragma unroll
        for (int ut = 0; ut < 4; ++ut) {
            const float4 c2 = *(const float4*)&cw[0][64 * wv + 16 * ut + 4 * lg];
#pragma unroll
            for (int pt = 0; pt < kSubT; ++pt) acc[pt][ut] = floatx4{c2.x, c2.y, c2.z, c2.w};
        }
#pragma unroll
        for (int ks = 0; ks < kH / 32; ++ks) {
            bf16x8 hb[kSubT];
#pragma unroll
            for (int pt = 0; pt < kSubT; ++pt)
                hb[pt] = *(const bf16x8*)(h1s + (kTile * pt + lr) * kPad + 32 * ks + 8 * lg);
#pragma unroll
            for (int pt = 0; pt < kSubT; ++pt)
#pragma unroll
                for (int ut = 0; ut < 4; ++ut)
                    acc[pt][ut] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[ut][ks], hb[pt],
                                                                          acc[pt][ut], 0, 0, 0);
        }
        // lane (lr, lg) holds units 64 wv + 16 ut + 4 lg + r of point lr
        float part[kSubT];
#pragma unroll
        for (int pt = 0; pt < kSubT; ++pt) part[pt] = 0.0f;
#pragma unroll
        for (int ut = 0; ut < 4; ++ut) {
            const float4 w3 = *(const float4*)&cw[1][64 * wv + 16 * ut + 4 * lg];
#pragma unroll
            for (int pt = 0; pt < kSubT; ++pt) {
                float s = part[pt];
                s = fmaf(fmaxf(acc[pt][ut][0], 0.0f), w3.x, s);
                s = fmaf(fmaxf(acc[pt][ut][1], 0.0f), w3.y, s);
                s = fmaf(fmaxf(acc[pt][ut][2], 0.0f), w3.z, s);
                s = fmaf(fmaxf(acc[pt][ut][3], 0.0f), w3.w, s);
                part[pt] = s;
            }
        }
#pragma unroll
        for (int pt = 0; pt < kSubT; ++pt) psum[wv][lg][kTile * pt + lr] = part[pt];
        __syncthreads();
        // psum is next written after the next group's first barrier, which
        // wave 0 reaches only after these reads
        if (store && tid % kTile < rec.nrow) {
            float psi = 0.0f;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const float pw = (psum[w][0][tid] + psum[w][1][tid]) +
                                 (psum[w][2][tid] + psum[w][3][tid]);
                psi += pw;
            }
            psi += c3;
            const int r = tid % kTile;
            A.psi[rec.pt + r] = psi;
            double* out = rec.which == 0 ? A.out_u : A.out_v;
            if (out) out[rec.row + r] = lw + (double)psi;
        }
        buf ^= 1;
    }
}

// ---------------------------------------------------------------- centring
__global__ __launch_bounds__(256) void k_ws_centre(MlpArgs A) {
    __shared__ double sh[16];
    const int s = blockIdx.x;
    const WSide S = A.sides[s];
    const double* w = S.which == 0 ? A.a : A.b;
    const double* tl = S.which == 0 ? A.tgt_u : A.tgt_v;
    double sd = 0.0, cnt = 0.0;
    for (int64_t i = threadIdx.x; i < S.npts; i += blockDim.x) {
        const int64_t r = S.pts_off + i;
        const double t = tl[r] - log(w[r]);
        if (isfinite(t)) {
            sd += (double)A.psi[S.pt0 + i] - t;
            cnt += 1.0;
        }
    }
    sd = block_sum(sd, sh);
    cnt = block_sum(cnt, sh);
    const double dbar = cnt > 0.0 ? sd / cnt : 0.0;
    double sq = 0.0;
    for (int64_t i = threadIdx.x; i < S.npts; i += blockDim.x) {
        const int64_t r = S.pts_off + i;
        const double t = tl[r] - log(w[r]);
        float dp = 0.0f;
        if (isfinite(t)) {
            const double d = (double)A.psi[S.pt0 + i] - t - dbar;
            sq += d * d;
            dp = (float)(2.0 * d / cnt / (double)A.nsides);
        }
        A.dpsi[S.pt0 + i] = dp;
    }
    sq = block_sum(sq, sh);
    if (threadIdx.x == 0) A.loss[s] = cnt > 0.0 ? sq / cnt : 0.0;
}

// ---------------------------------------------------------------- dW2
// Block b: points [b * kChunk, (b+1) * kChunk) of the concatenated point list;
// 16 waves, wave w owns rows n in [16 w, 16 w + 16) of dW2 (all 256 columns).
__global__ __launch_bounds__(1024) void k_ws_dw2(MlpArgs A) {
    __shared__ __align__(16) __bf16 dzT[kH][kSubPad];
    __shared__ __align__(16) __bf16 h1T[kH][kSubPad];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t p0 = (int64_t)blockIdx.x * kChunk;
    const int64_t p1 = p0 + kChunk < A.npts ? p0 + kChunk : A.npts;
    const __bf16* dz2 = (const __bf16*)A.dz2g;
    const __bf16* h1 = (const __bf16*)A.h1g;
    floatx4 acc[16];
#pragma unroll
    for (int ct = 0; ct < 16; ++ct) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int64_t q = p0; q < p1; q += kSub) {
        // stage kSub points transposed: thread -> point q + tid / 32, units 8 (tid % 32)..
        {
            const int r = tid / 32, n0 = (tid % 32) * 8;
            const int64_t pt = q + r;
            bf16x8 vd, vh;
            if (pt < p1) {
                vd = *(const bf16x8*)(dz2 + pt * kH + n0);
                vh = *(const bf16x8*)(h1 + pt * kH + n0);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) vd[e] = vh[e] = (__bf16)0.0f;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                dzT[n0 + e][r] = vd[e];
                h1T[n0 + e][r] = vh[e];
            }
        }
        __syncthreads();
        const int kk = 8 * (lane >> 4);
        const bf16x8 a = *(const bf16x8*)(&dzT[16 * wv + (lane & 15)][kk]);
#pragma unroll
        for (int ct = 0; ct < 16; ++ct) {
            const bf16x8 b = *(const bf16x8*)(&h1T[16 * ct + (lane & 15)][kk]);
            acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[ct], 0, 0, 0);
        }
        __syncthreads();
    }
    float* part = A.w2p + (int64_t)blockIdx.x * (kH * kH);
#pragma unroll
    for (int ct = 0; ct < 16; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = 16 * wv + 4 * (lane >> 4) + r, k = 16 * ct + (lane & 15);
            part[n * kH + k] = acc[ct][r];
        }
}

// ---------------------------------------------------------------- embedding backward
__global__ __launch_bounds__(256) void k_ws_embed_bwd(MlpArgs A) {
    __shared__ float dg_s[kH];
    const int s = blockIdx.x, t = threadIdx.x;
    const WSide S = A.sides[s];
    const __bf16* wb = (const __bf16*)A.wbf;
    float dg = 0.0f;
    for (int64_t k = 0; k < S.ntiles; ++k) dg += A.dgp[(S.tile0 + k) * kH + t];
    dg_s[t] = dg;
    A.dgs[(int64_t)s * kH + t] = dg;
    __syncthreads();
    float de = 0.0f;  // (U^T dg)_t
    for (int r = 0; r < kH; ++r) de = fmaf(bf(wb, OFF_U + r * kH + t), dg_s[r], de);
    const float scale = de / (float)S.nopp;
    const float pb = bf(wb, OFF_p + t);
    float pw[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) pw[c] = bf(wb, OFF_P + 4 * t + c);
    float gP[4] = {0.f, 0.f, 0.f, 0.f}, gp = 0.f;
#pragma unroll 4
    for (int64_t j = 0; j < S.nopp; ++j) {
        float f[4];
        opp_feature(A, S, j, f);
        float z = pb;  // phi_pre with unit t's weights in registers
#pragma unroll
        for (int c = 0; c < 4; ++c) z = fmaf(pw[c], f[c], z);
        if (z > 0.0f) {
            gp += scale;
#pragma unroll
            for (int c = 0; c < 4; ++c) gP[c] = fmaf(scale, f[c], gP[c]);
        }
    }
    float* part = A.sidep + (int64_t)s * kSidePart;
#pragma unroll
    for (int c = 0; c < 4; ++c) part[4 * t + c] = gP[c];
    part[1024 + t] = gp;
}

// dU[t][c] = sum_s dg_s[t] e_s[c]: block t, thread c.
__global__ __launch_bounds__(256) void k_ws_du(MlpArgs A) {
    const int t = blockIdx.x, c = threadIdx.x;
    float acc = 0.0f;
    for (int s = 0; s < A.nsides; ++s) acc = fmaf(A.dgs[(int64_t)s * kH + t], A.emb[(int64_t)s * kH + c], acc);
    A.grad[OFF_U + t * kH + c] = acc;
}

// Every other gradient entry from its partials, in index order.
__global__ __launch_bounds__(256) void k_ws_reduce(MlpArgs A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kParams) return;
    float v = 0.0f;
    if (i < OFF_p) {
        for (int s = 0; s < A.nsides; ++s) v += A.sidep[(int64_t)s * kSidePart + i];
    } else if (i < OFF_W1) {
        for (int s = 0; s < A.nsides; ++s) v += A.sidep[(int64_t)s * kSidePart + 1024 + (i - OFF_p)];
    } else if (i < OFF_U) {
        for (int b = 0; b < A.nblk; ++b) v += A.blkp[(int64_t)b * kBlkPart + (i - OFF_W1)];
    } else if (i < OFF_c1) {
        return;  // k_ws_du
    } else if (i < OFF_W2) {
        for (int s = 0; s < A.nsides; ++s) v += A.dgs[(int64_t)s * kH + (i - OFF_c1)];
    } else if (i < OFF_c2) {
        for (int b = 0; b < A.nchunk; ++b) v += A.w2p[(int64_t)b * kH * kH + (i - OFF_W2)];
    } else if (i < OFF_w3) {
        for (int b = 0; b < A.nblk; ++b) v += A.blkp[(int64_t)b * kBlkPart + 768 + (i - OFF_c2)];
    } else if (i < OFF_c3) {
        for (int b = 0; b < A.nblk; ++b) v += A.blkp[(int64_t)b * kBlkPart + 1024 + (i - OFF_w3)];
    } else {
        for (int b = 0; b < A.nblk; ++b) v += A.blkp[(int64_t)b * kBlkPart + 1280];
    }
    A.grad[i] = v;
}

// Adam step t on the FP32 master weights; refreshes the BF16 copies.
__global__ __launch_bounds__(256) void k_ws_adam(float* __restrict__ w, float* __restrict__ m1,
                                                  float* __restrict__ m2,
                                                  const float* __restrict__ grad, __bf16* wbf,
                                                  __bf16* w2t, float lr, float bc1, float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kParams) return;
    if (grad) {
        const float g = grad[i];
        const float a = 0.9f * m1[i] + 0.1f * g;
        const float b = 0.999f * m2[i] + 0.001f * g * g;
        m1[i] = a;
        m2[i] = b;
        w[i] -= lr * (a / bc1) / (sqrtf(b / bc2) + 1e-8f);
    }
    const __bf16 q = (__bf16)w[i];
    wbf[i] = q;
    if (i >= OFF_W2 && i < OFF_c2) {
        const int n = (i - OFF_W2) / kH, k = (i - OFF_W2) % kH;
        w2t[k * kH + n] = q;
    }
}

// ---------------------------------------------------------------- launchers
constexpr size_t kHeadLds = (size_t)(kH + 2 * kTile) * kPad * 2;

hipError_t mlp_init() {
    static hipError_t status = hipFuncSetAttribute((const void*)&k_ws_head_train,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)kHeadLds);
    return status;
}

int mlp_head_grid() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

int mlp_chunks(int64_t npts) { return (int)((npts + kChunk - 1) / kChunk); }

hipError_t launch_mlp_sync(float* w, __bf16* wbf, __bf16* w2t, hipStream_t st) {
    hipLaunchKernelGGL(k_ws_adam, dim3((kParams + 255) / 256), dim3(256), 0, st, w, nullptr,
                       nullptr, nullptr, wbf, w2t, 0.0f, 1.0f, 1.0f);
    return hipGetLastError();
}

hipError_t launch_mlp_predict(const MlpArgs& a, hipStream_t st) {
    const int nprob = a.nsides / 2;
    hipError_t e = launch_fill_u32((uint32_t*)a.xform, (int64_t)nprob * 4, 0u, st);
    if (e != hipSuccess) return e;
    if (a.cost == 0) hipLaunchKernelGGL(k_ws_cmax, dim3(nprob), dim3(kCmaxThreads), 0, st, a);
    hipLaunchKernelGGL(k_ws_prep, dim3(nprob), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_ws_embed_part, dim3(a.nemb), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_ws_embed, dim3(a.nsides), dim3(256), 0, st, a);
    const int64_t grid2 = 2 * (int64_t)a.nblk;  // two blocks per compute unit
    const int grid = a.ntiles < grid2 ? (int)a.ntiles : (int)grid2;
    hipLaunchKernelGGL(k_ws_head_fwd<kHeadGroup>, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Forward, loss, backward; the gradient lands in a.grad.
hipError_t launch_mlp_grad(const MlpArgs& a, hipStream_t st) {
    hipError_t e = launch_mlp_predict(a, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ws_centre, dim3(a.nsides), dim3(256), 0, st, a);
    MlpArgs b = a;
    b.nblk = a.ntiles < a.nblk ? (int)a.ntiles : a.nblk;
    // blocks past the tile count never run: their partials must read as zero
    e = launch_fill_u32((uint32_t*)a.blkp, (int64_t)a.nblk * kBlkPart, 0u, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ws_head_train, dim3(b.nblk), dim3(256), kHeadLds, st, b);
    hipLaunchKernelGGL(k_ws_dw2, dim3(a.nchunk), dim3(1024), 0, st, b);
    hipLaunchKernelGGL(k_ws_embed_bwd, dim3(a.nsides), dim3(256), 0, st, b);
    hipLaunchKernelGGL(k_ws_du, dim3(kH), dim3(256), 0, st, b);
    hipLaunchKernelGGL(k_ws_reduce, dim3((kParams + 255) / 256), dim3(256), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* w, float* m1, float* m2, const float* grad, __bf16* wbf,
                           __bf16* w2t, float lr, int step, hipStream_t st) {
    const float bc1 = 1.0f - powf(0.9f, (float)step), bc2 = 1.0f - powf(0.999f, (float)step);
    hipLaunchKernelGGL(k_ws_adam, dim3((kParams + 255) / 256), dim3(256), 0, st, w, m1, m2, grad,
                       wbf, w2t, lr, bc1, bc2);
    return hipGetLastError();
}

}  // namespace ss
