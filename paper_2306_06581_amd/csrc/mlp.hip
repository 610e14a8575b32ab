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
// Kernels (all sums in a fixed order; no atomics):
//   k_ws_cmax       (problem, row chunk) blocks: max squared distance
//   k_ws_prep       one block per problem: centre and kernel length
//   k_ws_embed      one block per side: e, g
//   k_ws_head<T>    persistent blocks over 16-point tiles of all sides.  W2
//                   stays in LDS (padded rows); h2 = ReLU(h1 W2^T + c2) on
//                   MFMA 16x16x32 BF16.  Forward: psi (and log w + psi).
//                   Training: recomputes the forward, dz2 = dpsi w3 [z2 > 0],
//                   dh1 = dz2 W2 (MFMA, W2^T from global), dz1 = dh1 [h1 > 0];
//                   per-block sums of dW1, dc2, dw3, dc3, per-tile sums of dg;
//                   h1 and dz2 rows go to scratch for dW2.
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
// Opposite points per LDS stage of the embedding.
constexpr int kEmbChunk = 1024;

__global__ __launch_bounds__(256) void k_ws_embed(MlpArgs A) {
    __shared__ float e_s[kH];
    __shared__ float4 fs[kEmbChunk];
    const int s = blockIdx.x, t = threadIdx.x;
    const WSide S = A.sides[s];
    const __bf16* wb = (const __bf16*)A.wbf;
    // unit t's weights in registers (phi_pre's arithmetic, in its order)
    const float pb = bf(wb, OFF_p + t);
    float pw[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) pw[c] = bf(wb, OFF_P + 4 * t + c);
    float acc = 0.0f;
    // the opposite points' features are formed once per stage (not once per
    // hidden unit) and read from LDS by every unit, in point order
    for (int64_t j0 = 0; j0 < S.nopp; j0 += kEmbChunk) {
        const int cnt = (int)(S.nopp - j0 < kEmbChunk ? S.nopp - j0 : kEmbChunk);
        __syncthreads();  // the previous stage is read
        for (int q = t; q < cnt; q += blockDim.x) {
            float f[4];
            opp_feature(A, S, j0 + q, f);
            fs[q] = make_float4(f[0], f[1], f[2], f[3]);
        }
        __syncthreads();
#pragma unroll 4
        for (int q = 0; q < cnt; ++q) {
            const float4 f = fs[q];
            float z = pb;
            z = fmaf(pw[0], f.x, z);
            z = fmaf(pw[1], f.y, z);
            z = fmaf(pw[2], f.z, z);
            z = fmaf(pw[3], f.w, z);
            acc += fmaxf(z, 0.0f);
        }
    }
    const float e = acc / (float)S.nopp;
    e_s[t] = e;
    A.emb[(int64_t)s * kH + t] = e;
    __syncthreads();
    float g = bf(wb, OFF_c1 + t);
    for (int c = 0; c < kH; ++c) g = fmaf(bf(wb, OFF_U + t * kH + c), e_s[c], g);
    A.gvec[(int64_t)s * kH + t] = g;
}

// ---------------------------------------------------------------- head
template <bool TRAIN>
__global__ __launch_bounds__(256) void k_ws_head(MlpArgs A) {
    extern __shared__ __align__(16) unsigned char dsm[];
    __bf16* w2s = (__bf16*)dsm;                 // [kH][kPad]  W2 rows (out n, in k)
    __bf16* h1s = w2s + kH * kPad;              // [kTile][kPad]
    __bf16* dz2s = h1s + kTile * kPad;          // [kTile][kPad] (training)
    __shared__ float xs[kTile][3];
    __shared__ float psum[4][kTile];
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
    const float c3 = bf(wb, OFF_c3);
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
        if (TRAIN && tid < kTile) dps[tid] = tid < nrow ? A.dpsi[S.pt0 + i0 + tid] : 0.0f;
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
        // h2 = ReLU(z2 + c2); psi partial sums over this wave's columns
        float rowp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int n = 64 * wv + 16 * ct + (lane & 15);
            const float c2 = bf(wb, OFF_c2 + n), w3 = bf(wb, OFF_w3 + n);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float h2 = fmaxf(acc[ct][r] + c2, 0.0f);
                acc[ct][r] = h2;
                rowp[r] = fmaf(h2, w3, rowp[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float v = rowp[r];
            v += __shfl_xor(v, 1, 64);
            v += __shfl_xor(v, 2, 64);
            v += __shfl_xor(v, 4, 64);
            v += __shfl_xor(v, 8, 64);
            rowp[r] = v;
        }
        if ((lane & 15) == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) psum[wv][4 * (lane >> 4) + r] = rowp[r];
        }
        __syncthreads();
        if (!TRAIN) {
            if (tid < nrow) {
                const float psi = ((psum[0][tid] + psum[1][tid]) + (psum[2][tid] + psum[3][tid])) + c3;
                A.psi[S.pt0 + i0 + tid] = psi;
                if (A.out_u || A.out_v) {
                    double* out = S.which == 0 ? A.out_u : A.out_v;
                    const double* w = S.which == 0 ? A.a : A.b;
                    if (out) out[S.pts_off + i0 + tid] = log(w[S.pts_off + i0 + tid]) + (double)psi;
                }
            }
            __syncthreads();
            continue;
        }
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
    if (TRAIN) {
        float* part = A.blkp + (int64_t)blockIdx.x * kBlkPart;
        part[3 * tid + 0] = bw1[0];
        part[3 * tid + 1] = bw1[1];
        part[3 * tid + 2] = bw1[2];
        part[768 + tid] = bc2;
        part[1024 + tid] = bw3;
        if (tid == 0) part[1280] = bc3;
    }
}

// Forward head for prediction: the same arithmetic as k_ws_head<false>, with
// W2 held in registers instead of LDS.  Wave wv owns output columns
// [64 wv, 64 wv + 64); its B fragments of W2 (4 column tiles x 8 k-steps of
// 8 BF16 each, 128 VGPRs) are loaded once per block, so a 16-point tile
// reads only its h1 rows from LDS and the matrix cores, not LDS bandwidth,
// bound the tile (32 MFMA 16x16x32 per wave).  A block takes a contiguous
// range of tiles, so the owning side is found once and then advanced, and
// the next tile's coordinates are loaded while the current one computes.
__global__ __launch_bounds__(256, 2) void k_ws_head_fwd(MlpArgs A) {
    __shared__ __align__(16) __bf16 h1s[kTile * kPad];
    __shared__ float xs[kTile][3];
    __shared__ float psum[4][kTile];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const __bf16* wb = (const __bf16*)A.wbf;
    const int64_t t0 = A.ntiles * blockIdx.x / gridDim.x;
    const int64_t t1 = A.ntiles * (blockIdx.x + 1) / gridDim.x;
    if (t0 >= t1) return;
    bf16x8 bw[4][kH / 32];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int n = 64 * wv + 16 * ct + (lane & 15);
#pragma unroll
        for (int ks = 0; ks < kH / 32; ++ks)
            bw[ct][ks] = *(const bf16x8*)(wb + OFF_W2 + n * kH + 32 * ks + 8 * (lane >> 4));
    }
    float c2v[4], w3v[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int n = 64 * wv + 16 * ct + (lane & 15);
        c2v[ct] = bf(wb, OFF_c2 + n);
        w3v[ct] = bf(wb, OFF_w3 + n);
    }
    const float w1t[3] = {bf(wb, OFF_W1 + 3 * tid), bf(wb, OFF_W1 + 3 * tid + 1),
                          bf(wb, OFF_W1 + 3 * tid + 2)};
    const float c3 = bf(wb, OFF_c3);
    // the side of the first tile
    int lo = 0, hi = A.nsides - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A.sides[mid].tile0 <= t0) lo = mid; else hi = mid - 1;
    }
    WSide S = A.sides[lo];
    float g = A.gvec[(int64_t)lo * kH + tid];
    // coordinate (row tid / 3, axis tid % 3) of a tile, loaded one tile ahead
    auto coord = [&](int64_t tile, const WSide& Sx) -> float {
        const int64_t i0 = (tile - Sx.tile0) * kTile;
        const int r = tid / 3, c = tid % 3;
        if (tid >= kTile * 3 || i0 + r >= Sx.npts) return 0.0f;
        const float* xf = A.xform + 4 * Sx.prob;
        return ((float)side_pts(A, Sx)[3 * (Sx.pts_off + i0 + r) + c] - xf[c]) * xf[3];
    };
    float xnext = coord(t0, S);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t i0 = (tile - S.tile0) * kTile;
        const int nrow = (int)(S.npts - i0 < kTile ? S.npts - i0 : kTile);
        __syncthreads();  // the previous tile's h1s and psum are read
        if (tid < kTile * 3) xs[tid / 3][tid % 3] = xnext;
        __syncthreads();
        for (int r = 0; r < kTile; ++r) {
            float z1 = g;
#pragma unroll
            for (int c = 0; c < 3; ++c) z1 = fmaf(w1t[c], xs[r][c], z1);
            h1s[r * kPad + tid] = (__bf16)(r < nrow ? fmaxf(z1, 0.0f) : 0.0f);
        }
        // the next tile's side and coordinates, in flight during the products
        WSide Sn = S;
        int lon = lo;
        if (tile + 1 < t1) {
            while (lon + 1 < A.nsides && A.sides[lon + 1].tile0 <= tile + 1) ++lon;
            if (lon != lo) Sn = A.sides[lon];
            xnext = coord(tile + 1, Sn);
        }
        __syncthreads();
        floatx4 acc[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < kH / 32; ++ks) {
            const bf16x8 a = *(const bf16x8*)(h1s + (lane & 15) * kPad + 32 * ks + 8 * (lane >> 4));
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[ct][ks], acc[ct], 0, 0, 0);
        }
        float rowp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
#pragma unroll
            for (int r = 0; r < 4; ++r) rowp[r] = fmaf(fmaxf(acc[ct][r] + c2v[ct], 0.0f), w3v[ct], rowp[r]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float v = rowp[r];
            v += __shfl_xor(v, 1, 64);
            v += __shfl_xor(v, 2, 64);
            v += __shfl_xor(v, 4, 64);
            v += __shfl_xor(v, 8, 64);
            rowp[r] = v;
        }
        if ((lane & 15) == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) psum[wv][4 * (lane >> 4) + r] = rowp[r];
        }
        __syncthreads();
        if (tid < nrow) {
            const float psi = ((psum[0][tid] + psum[1][tid]) + (psum[2][tid] + psum[3][tid])) + c3;
            A.psi[S.pt0 + i0 + tid] = psi;
            if (A.out_u || A.out_v) {
                double* out = S.which == 0 ? A.out_u : A.out_v;
                const double* w = S.which == 0 ? A.a : A.b;
                if (out) out[S.pts_off + i0 + tid] = log(w[S.pts_off + i0 + tid]) + (double)psi;
            }
        }
        if (lon != lo) {
            lo = lon;
            S = Sn;
            g = A.gvec[(int64_t)lo * kH + tid];
        }
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
    static hipError_t status = [] {
        hipError_t e = hipFuncSetAttribute((const void*)&k_ws_head<false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kHeadLds);
        const hipError_t e2 = hipFuncSetAttribute((const void*)&k_ws_head<true>,
                                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  (int)kHeadLds);
        return e != hipSuccess ? e : e2;
    }();
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
    hipLaunchKernelGGL(k_ws_embed, dim3(a.nsides), dim3(256), 0, st, a);
    const int64_t grid2 = 2 * (int64_t)a.nblk;  // two blocks per compute unit
    const int grid = a.ntiles < grid2 ? (int)a.ntiles : (int)grid2;
    hipLaunchKernelGGL(k_ws_head_fwd, dim3(grid), dim3(256), 0, st, a);
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
    hipLaunchKernelGGL(k_ws_head<true>, dim3(b.nblk), dim3(256), kHeadLds, st, b);
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
