// Internal interfaces between the host driver (api.cpp) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sparsink.h"

namespace ss {

// Device-resident state of one Sinkhorn loop.  Written only by block 0 of
// the iteration launches, read by every block of later launches.
struct IterState {
    int32_t cnt_u;       // iteration of the last v-launch (read by u-launches)
    int32_t cnt_v;       // iteration of the last u-launch (read by v-launches)
    int32_t stop_iter;   // 0 while running; else t of the returned iterate
    int32_t nonfinite;   // set when a scaling became NaN/Inf
    double err_col;      // column residual of the previous iterate (marginal rule)
    double err_row;      // |du| of the current iteration (delta rule)
    double err_final;    // err of the returned iterate
    double err_last;     // err of the latest iterate tested (the host's replay schedule)
};

// Grid cap of the iteration kernels (grid-stride over lines): 8 blocks per CU.
constexpr int kMaxLoopBlocks = 2048;

// Per-solve scalars produced on the device and copied to the host once.
enum StatSlot {
    ST_CMAX = 0,
    ST_SA,
    ST_SB,
    ST_Z,
    ST_SUM_A_ACTIVE,
    ST_SUM_B_ACTIVE,
    ST_DROPPED_A,
    ST_DROPPED_B,
    ST_TRANSPORT,
    ST_NEGENT,
    ST_SPARSEOBJ,
    ST_KL_A,
    ST_KL_B,
    ST_ROWSUM,
    ST_COLSUM,
    ST_BAD_INPUT,   // > 0 if an input was negative or non-finite
    ST_EMPTY_ROWS,  // rows with no entry and a_i > 0 (stored as double)
    ST_EMPTY_COLS,
    ST_RX2,         // max_i |x_i - c|^2 about the cost-scan centre c
    ST_RY2,         // max_j |y_j - c|^2
    ST_SAME_SUPPORT,  // WFR normaliser: 1 when n = m and y is x bit for bit, else 0
    ST_COUNT = 32
};

enum Precision { P_F64 = 0, P_F32 = 1, P_LOG = 2 };

// Parameters of the sampling probabilities and entry values.
struct ProbParams {
    int uot;            // 0: eq. (pij-ot), 1: eq. (pij-uot)
    double s;           // budget
    double eps;
    double inv_cmax;    // C = c * inv_cmax
    double inv_tau;     // 1 / (2 lam + eps)            (UOT)
    double kappa;       // s / Z                        (UOT; device value in stats)
    double shrink_w;    // 1 - g: weight of eq. (pij-ot)/(pij-uot) in the shrunk p
    double shrink_c;    // s g / (nm): the uniform part of s p (0 without shrinkage)
    int cost;           // SS_COST_*; kCostWfr: C from cost_value with wfr_w
    double wfr_w;       // 1 / (2 eta)
    const double* row_fac;  // OT: alpha_i;  UOT: th_u log a_i
    const double* col_fac;  // OT: sqrt b_j; UOT: th_u log b_j
    const double* row_bnd;  // UOT: exp(row_fac_i)
    const double* col_bnd;  // UOT: kappa * exp(col_fac_j) * (1 + 2^-30)
    const double* x;
    const double* y;
    int d;
    uint32_t problem_index;
    uint32_t k0, k1;
};

struct Workspace;

// ---- ibp.hip (Spar-IBP)
constexpr int kIbpMaxMeasures = 64;

// Arguments of the two launches of one Spar-IBP step.  Measure k's sketch
// holds its entries at [k * cap, k * cap + nnz_k) of the entry arrays, its
// row (column) offsets at row_ptr + k (n + 1) (col_ptr + k (n + 1)), relative
// to k * cap.  Vectors of all measures are laid out measure-major (k * n + i).
// Protocol (IterState fields reused): a column launch runs step
// t = cnt_u + 1, its block 0 first closes step t - 1 (error, history, stop)
// and sets cnt_v = t; a row launch runs step cnt_v and its block 0 sets
// cnt_u.  No launch reads a field its own grid writes, except stop_iter and
// nonfinite, whose early sight only skips work that is no longer needed.
struct IbpArgs {
    int64_t n;
    int32_t count;
    int32_t nb_rows;          // grid of the row launch = number of partials
    int64_t cap;              // entry stride between measures
    const int64_t* row_ptr;   // count x (n + 1)
    const int32_t* col_idx;
    const void* val;          // FP64 or FP32
    const int64_t* col_ptr;
    const int32_t* row_idx;
    const void* val_t;
    const double* b;          // count x n
    double* u;                // count x n
    double* v[2];             // count x n, by step parity
    double* q[2];             // n, by step parity (q[0] starts as 1/n)
    double* partials;         // nb_rows
    IterState* st;
    double* err_hist;
    int32_t max_iter;
    double tol;
    double w[kIbpMaxMeasures];
};

hipError_t launch_ibp_prep(const double* b, int64_t n, double s, double shrink_w, double* row_fac,
                           double* col_fac, double* scratch, double* stats, hipStream_t st);
hipError_t launch_ibp_empty(const int32_t* cnt, int64_t n, unsigned long long* out,
                            hipStream_t st);
hipError_t launch_ibp_init(double* u, int64_t nu, double* q0, int64_t n, hipStream_t st);
// Grid of the row launch (the number of residual partials) for n points and
// count measures.
int ibp_row_blocks(int64_t n, int count);
// Raises the dynamic LDS limit of the LDS-staged step kernels (once, before
// any launch or capture).
hipError_t ibp_lds_init();
hipError_t launch_ibp_iteration(int precision, const IbpArgs& A, hipStream_t st);

// ---- sample.hip
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
hipError_t launch_validate(const double* a, int64_t n, const double* x, int64_t nx, double* stats,
                           hipStream_t st);
hipError_t launch_tree_sum(const double* in, int64_t n, double* scratch, double* out,
                           hipStream_t st);
// max_ij c_ij into stats[ST_CMAX] (which must start at 0); `scratch` holds
// cmax_scratch_bytes(n) bytes.
hipError_t launch_cmax(const double* x, const double* y, int64_t n, int64_t m, int d,
                       double* stats, void* scratch, hipStream_t st);
size_t cmax_scratch_bytes(int64_t n);
// After launch_cmax: copies the centre c of the cost scan to center_out[d]
// and maximises |x_i - c|^2, |y_j - c|^2 into stats[ST_RX2], stats[ST_RY2]
// (which must start at 0).
hipError_t launch_center_radii(const double* x, const double* y, int64_t n, int64_t m, int d,
                               const void* cmax_scratch, double* center_out, double* stats,
                               hipStream_t st);

// Z (eq. (pij-uot) normaliser) for the squared Euclidean costs by the
// truncated expansion of exp(2 g x~.y~) in monomials of degree <= K about the
// centre (g = inv_cmax inv_tau): Z = sum_alpha coef_alpha S_alpha T_alpha.
// exps: M x 8 exponents (d <= 8); coef: M; part: 2 x kZBlocks x M scratch,
// sums: 2 x M.  Writes stats[ST_Z].
constexpr int kZBlocks = 512;
constexpr int kZMaxMono = 1024;
constexpr int kZMaxDegree = 24;
struct ZExpArgs {
    const double* x;
    const double* y;
    const double* la;   // th_u log a (row factor)
    const double* lb;   // th_u log b
    int64_t n, m;
    int d, K, M;
    double g;
    const double* center;
    const uint8_t* exps;
    const double* coef;
    double* part;
    double* sums;
};
hipError_t launch_uot_zexp(const ZExpArgs& a, double* stats, hipStream_t st);
hipError_t launch_ot_prep(const double* a, const double* b, int64_t n, int64_t m, double s,
                          double shrink_w, double* ra, double* rb, double* scratch,
                          double* stats, hipStream_t st);
hipError_t launch_uot_prep(const double* a, const double* b, int64_t n, int64_t m, double lam,
                           double eps, double* la, double* lb, double* ea, double* eb,
                           hipStream_t st);
// Z (eq. (pij-uot) normaliser) into stats[ST_Z]; eb_j = exp(col_fac_j); cmax
// is the cost maximum (chooses the short-range exponential when it applies).
// same_support: stats[ST_SAME_SUPPORT] as read by the host (WFR: only the
// pairs j >= i are evaluated).
hipError_t launch_uot_z(const ProbParams& pp, int64_t n, int64_t m, const double* eb, double cmax,
                        bool same_support, double* partials, double* scratch, double* stats,
                        hipStream_t st);
// stats[ST_SAME_SUPPORT] = 1 if n = m and y is x bit for bit, else 0.
hipError_t launch_same_support(const double* x, const double* y, int64_t n, int64_t m, int d,
                               double* stats, hipStream_t st);
hipError_t launch_uot_bounds(const double* lb, int64_t m, double s, double shrink_w,
                             const double* stats, double* fb, hipStream_t st);
hipError_t launch_mask(const ProbParams& pp, int64_t n, int64_t m, uint64_t* mask,
                       int32_t* row_cnt, const double* stats, hipStream_t st);
hipError_t launch_transpose(const uint64_t* mask, int64_t n, int64_t m, uint64_t* maskT,
                            int32_t* col_cnt, hipStream_t st);
hipError_t launch_scan(const int32_t* cnt, int64_t n, int64_t* ptr, int64_t* scratch,
                       hipStream_t st);
hipError_t launch_fill_entries(int role, int precision, const ProbParams& pp, const double* stats,
                               const uint64_t* bits, int64_t nlines, int64_t words,
                               const int64_t* ptr, int32_t* idx, void* val, int64_t cap,
                               hipStream_t st);
hipError_t launch_empty_policy(const double* a, const int32_t* cnt, int64_t n, int renormalize,
                               int which, double* a_eff, double* tmp, double* scratch,
                               double* stats, hipStream_t st);

// Fixed-order sums of up to 8 partial arrays into stats slots (one block).
struct ReduceSpec {
    int nq;
    const double* src[8];
    int64_t len[8];
    int slot[8];
};
hipError_t launch_reduce_stats(const ReduceSpec& r, double* stats, hipStream_t st);

// ---- iterate.hip
// Device-side parameters of a lane plan (see build_plan).
struct PlanInfo {
    int64_t T;      // quad weight per step
    int64_t K;      // number of steps
    int64_t Q;      // quads of all lines
    int64_t W1;     // line weights summed with the single-pass floor
    int64_t tcap;   // largest step weight of the chosen policy
    int64_t kmin;   // fewest steps of the chosen policy
    int32_t minw;   // line weight floor of the chosen policy
    int32_t pad;
};

// Lane plan of one sparse matrix for the iteration kernel: the lines are cut
// into steps, each step's (slice, line) segments are laid out in quads of 4
// entries and packed into lanes of J quads (at most two segments a lane), and
// the entries are repacked lane by lane.  Built once per solve, on the device.
struct IterPlan {
    int block = 0;          // threads per block
    int ns = 0;             // slices of the gathered vector
    int64_t slice = 0;      // elements per slice
    int grid = 0;           // blocks per launch (resident blocks, <= kMaxLoopBlocks)
    int64_t kmax = 0;       // bound on the number of steps
    int64_t lanes_max = 0;  // bound on the number of lanes
    int32_t* split = nullptr;      // [nlines][ns + 1] entry offsets at the slice boundaries
    int32_t* quads = nullptr;      // [nlines] quads of each line (sum over its segments)
    int32_t* weight = nullptr;     // [nlines] step weight of each line
    int64_t* wptr = nullptr;       // [nlines + 1] exclusive scan of weights
    int32_t* rstart = nullptr;     // [kmax + 1] first line of each step
    PlanInfo* info = nullptr;
    int64_t* scan = nullptr;       // scan scratch
    int32_t* qs = nullptr;         // [nlines * ns] first packed quad of each segment in its step
    int32_t* qe = nullptr;         // [nlines * ns] end of the segment's packed quads
    int32_t* steplanes = nullptr;  // [kmax] lanes of each step
    int64_t* stepoff = nullptr;    // [kmax + 1] exclusive scan of steplanes
    int32_t* lmeta = nullptr;      // [lanes_max] slice << 8 | quad where the second segment starts
    void* pval = nullptr;          // [lanes_max * E] packed values
    uint16_t* poff = nullptr;      // [lanes_max * E] packed byte offsets inside the slice
};

struct IterArgs {
    const int64_t* ptr;   // line pointers (empty-line test)
    int64_t nlines;
    int64_t nx;           // length of the gathered vector
    int nslices;
    const int32_t* rstart;
    const int64_t* stepoff;
    const int32_t* qs;
    const int32_t* qe;
    const int32_t* lmeta;
    const PlanInfo* info;
    const void* pval;
    const uint16_t* poff;
    const double* marg;   // a_eff (u role) or b_eff (v role)
    const double* lmarg;  // log of marg (log domain; else unused)
    const void* xin;      // gathered vector: v^(t-1) (u role), u^t (v role)
    void* yout;           // new scaling / potential
    float* yg;            // log domain: FP32 copy of yout for the next gather (else NULL)
    const void* yprev;    // previous value of the same scaling
    double theta;         // lam/(lam+eps); 1 for OT
    double* partials;     // this launch's residual partials (one per block)
    const double* prev_partials;  // the previous launch's partials
    int prev_nblocks;
    IterState* st;
    double* err_hist;
    int role;             // 0 = u-update (closes the previous iterate), 1 = v-update
    int stop_rule;
    int max_iter;
    double tol;
};
hipError_t iterate_init();
int iterate_block_size(int64_t nlines);
int slice_elems(int precision, int block);
int iterate_slices(int precision, int block, int64_t nx);
// Fills the sizes of a plan (block, ns, slice, grid, kmax, lanes_max) for a
// matrix of nlines lines over a gathered vector of nx entries holding at most
// cap entries; returns false when nx is beyond the slice limit.
bool plan_shape(int precision, int block, int64_t nlines, int64_t nx, int64_t cap, IterPlan* p);
size_t plan_value_bytes(int precision, const IterPlan& p);
size_t plan_offset_bytes(int precision, const IterPlan& p);
int iterate_grid(int precision, int block);  // valid after iterate_init()
hipError_t build_plan(int precision, const IterPlan& p, const int64_t* ptr, const int32_t* idx,
                      const void* val, int64_t nlines, hipStream_t st);
hipError_t launch_iterate(int precision, int block, int grid, const IterArgs& a, hipStream_t st);
// out[i] = log(in[i]) (log of a marginal; -inf for 0)
hipError_t launch_log_vec(const double* in, double* out, int64_t n, hipStream_t st);
hipError_t launch_init_scaling(int precision, void* y, float* yg, const double* init_log,
                               int64_t n, hipStream_t st);
hipError_t launch_export_scaling(int precision, const void* y, double* out, int64_t n,
                                 hipStream_t st);

// ---- objective.hip
struct ObjArgs {
    const int64_t* ptr;
    const int32_t* idx;
    const void* val;
    int64_t nlines;
    const void* ys;       // scaling of the line (u for rows, v for columns)
    const void* zs;       // scaling of the other side
    const double* marg;   // a (rows) / b (columns), original masses
    const double* x;      // coordinates of the line side
    const double* y;      // coordinates of the other side
    int d;
    double inv_cmax;
    double eps;
    int cost;             // SS_COST_*
    double wfr_w;         // 1 / (2 eta) (WFR)
    int uot;
    int role;             // 0 rows (transport, entropy, KL_a), 1 columns (KL_b)
    double* partials;     // 4 * nblocks
    IterState* st;
    double* stats;
};
hipError_t launch_objective(int precision, const ObjArgs& a, hipStream_t st);

// Gradient of the sparse problem's value in the points of one side (envelope
// theorem, squared Euclidean cost): out[line * d + k] += coef * sum over the
// line's entries of T~ (xl[line][k] - xo[other][k]).
struct GradArgs {
    const int64_t* ptr;
    const int32_t* idx;
    const void* val;
    int64_t nlines;
    const void* ys;       // scaling of the line side
    const void* zs;       // scaling of the other side
    const double* xl;     // coordinates of the line side
    const double* xo;     // coordinates of the other side
    int d;
    int euclid;           // 1: C = |x - y| (entries weighted by 1 / |x - y|)
    double coef;
    double* out;
};
hipError_t launch_plan_grad(int precision, const GradArgs& a, hipStream_t st);

// ---- dense.hip
struct DenseArgs {
    const double* xl;     // coordinates of the line side (n_l x d)
    const double* xo;     // coordinates of the other side (n_o x d)
    int64_t nl, no;
    int d;
    double scale;         // inv_cmax / eps: K = exp(-c * scale)
    double inv_cmax, eps; // FP64 mode: K = exp(-((c * inv_cmax) / eps))
    int cost;             // SS_COST_*; WFR: K = cos(sqrt(c) w)^(2/eps), 0 past pi/2
    double wfr_w;         // 1 / (2 eta)
    const double* marg;
    const void* xin;      // other side's scaling
    void* yout;
    const void* yprev;
    double theta;
    double* partials;
    const double* prev_partials;
    int prev_nblocks;
    IterState* st;
    double* err_hist;
    int role, stop_rule, max_iter;
    double tol;
    const double* stats;
};
hipError_t launch_dense_half(int precision, const DenseArgs& a, void* part, hipStream_t st);
int dense_blocks(int64_t nlines);
size_t dense_partial_bytes(int64_t nl, int64_t no);
struct DenseObjArgs {
    const double* x;
    const double* y;
    int64_t n, m;
    int d;
    double inv_cmax, eps;
    int cost;
    double wfr_w;
    const void* u;
    const void* v;
    const double* a;
    const double* b;
    int uot, precision;
    double* partials;
    double* rowsum;       // n
    double* colsum;       // m (written by the column pass)
    IterState* st;
    double* stats;
    const double* statsc;
};
hipError_t launch_dense_objective(const DenseObjArgs& a, hipStream_t st);

// ---- batches (sample.hip: sampling stages; batch.hip: loop, objective)
constexpr int kBatchMaxSide = 4096;

// 16-row blocks of one batched mask tile: a tile's four waves each cover 16
// words of a row, so a problem whose rows have at most 16 (32) words gives
// the spare waves further row blocks, 4 (2) per tile.
__host__ __device__ constexpr int batch_mask_split(int64_t W) { return W <= 16 ? 4 : W <= 32 ? 2 : 1; }

// Per problem, written by the host.
struct BProb {
    int64_t n, m;      // points of x and y
    int64_t xo, yo;    // first row / column in the concatenated arrays
    int64_t mo, mto;   // first word of its mask / transposed mask
    int64_t W, Wn;     // words per mask row (ceil(m/64)) / per transposed row (ceil(n/64))
    double s;          // budget
    uint32_t pidx;     // hash counter word
    int32_t pad;
};

// Per problem, written by the device.
struct BStat {
    double cmax, inv_cmax, sa, sb;
    double sum_a_act, sum_b_act, dropped_a, dropped_b, empty_rows, empty_cols;
    double transport, negent, sparseobj, err;
    int64_t nnz;
    int32_t iters, status;
    int32_t warm, pad;  // warm start: 1 kept, 0 replaced by the plain start, -1 none given
};

struct BatchArgs {
    int count, d;
    const BProb* prob;          // [count]
    BStat* stat;                // [count]
    const int64_t* tile_cmax;   // [count + 1] prefix of cost-scan tiles
    const int64_t* tile_mask;   // [count + 1] prefix of mask tiles
    const int64_t* tile_tr;     // [count + 1] prefix of transpose tiles
    const int64_t* row_off;     // [count + 1] prefix of n
    const int64_t* col_off;     // [count + 1] prefix of m
    int32_t* owner;             // [rows + cols]: problem of each row, then of each column
    int64_t rows, cols;         // sum n, sum m
    const double *x, *y, *a, *b;
    double *row_fac, *col_fac;  // alpha_i, sqrt(b_j)
    double *a_eff, *b_eff;
    uint64_t *mask, *maskT;
    int32_t *row_cnt, *col_cnt;
    int64_t *row_ptr, *col_ptr;
    uint16_t *col_idx, *row_idx;
    void *val, *val_t;
    int64_t cap;
    int cost;                   // SS_COST_*
    int empty_policy;           // SS_EMPTY_RENORMALIZE or SS_EMPTY_ZERO
    double eps;
    uint32_t k0, k1;
    double* gstats;             // ST_COUNT slots (input validation)
};

struct BIterArgs {
    int count;
    const int32_t* order;       // problems, largest first
    int32_t* queue;             // next position in `order` (zeroed before the launch)
    const BProb* prob;
    BStat* stat;
    const int64_t *row_ptr, *col_ptr;
    const uint16_t *col_idx, *row_idx;
    const void *val, *val_t;
    const double *a_eff, *b_eff;
    int64_t rows, cols, cap;
    int nmax, mmax;             // largest n, m (LDS sizing)
    const double *init_log_u, *init_log_v;
    void *u, *v;                // iterate of every problem (FP64 or FP32)
    double *u_out, *v_out;      // optional FP64 copies
    int max_iter;
    double tol;
};

struct BObjArgs {
    int d;
    const BProb* prob;
    BStat* stat;
    const int64_t* row_ptr;
    const uint16_t* col_idx;
    const void* val;
    const void *u, *v;
    const double *x, *y;
    int64_t rows, cols, cap;
    const int64_t* col_ptr;
    double* part;  // [count][kBObjSplit][3] block partials
};
constexpr int kBObjSplit = 8;  // objective blocks per problem

hipError_t launch_batch_sample(int precision, const BatchArgs& a, int64_t ntile_cmax,
                               int64_t ntile_mask, int64_t ntile_tr, int64_t* scan_scratch,
                               hipStream_t st);
hipError_t batch_init();
size_t batch_iter_lds(int precision, int nmax, int mmax);
int batch_iter_grid(int precision, int lanes, int block, int nmax, int mmax);
hipError_t launch_batch_iterate(int precision, int lanes, int block, int grid, const BIterArgs& a,
                                hipStream_t st);
hipError_t launch_batch_objective(int precision, int count, const BObjArgs& a, hipStream_t st);
// out[i] = log y[i] (y FP64 or FP32 by precision): a batch iterate as a warm start.
hipError_t launch_batch_log_scaling(int precision, const void* y, double* out, int64_t n,
                                    hipStream_t st);

// ---- mlp.hip (learned warm start)
// One side of a problem: the points whose scalings are predicted and the
// opposite measure.
struct WSide {
    int64_t npts, pts_off;   // points, first row in their concatenated array
    int64_t nopp, opp_off;   // opposite measure
    int64_t tile0, ntiles;   // head tiles of this side
    int64_t pt0;             // first position in the list of all sides' points
    int64_t emb0;            // first embedding chunk (of kWsEmbPart opposite points)
    int32_t nemb;            // embedding chunks
    int32_t which;           // 0: points from x / a (u side), 1: from y / b (v side)
    int32_t prob;            // problem index
    int32_t pad;
};

// Opposite points per block of the embedding's partial sums.
constexpr int kWsEmbPart = 512;

// One 16-point head tile: where its points and outputs sit.
struct WTile {
    int64_t pt;              // first position in the list of all sides' points
    int64_t row;             // first row in the side's concatenated point array
    int32_t side;            // side index
    int32_t nrow;            // points in the tile (16 except at a side's end)
    int32_t which;           // as WSide::which
    int32_t pad;
};

struct MlpArgs {
    const WSide* sides;
    WTile* tiles;            // [tile]
    int nemb;                // embedding chunks over all sides
    int32_t* emb_side;       // [chunk]: its side
    float* embp;             // [chunk][256]: partial ReLU sums of the embedding
    float* tpts;             // [tile][16][4]: points in kernel units, 4th 0, tail 0
    double* tlw;             // [tile][16]: log of the point's mass, tail 0
    int nsides;
    int64_t ntiles, npts;
    int nblk;                // head blocks (<= resident)
    int nchunk;              // dW2 blocks
    const double *x, *y, *a, *b;
    const double *tgt_u, *tgt_v;
    double *out_u, *out_v;
    float* xform;            // [problem][4]: centre (3), 1 / sqrt(eps C_s)
    double eps;
    int cost;                // SS_COST_*
    const void* wbf;         // BF16 weights
    const void* w2t;         // BF16 W2 transposed
    float *emb, *gvec;       // [side][256]
    float *psi, *dpsi;       // [point]
    void *h1g, *dz2g;        // BF16 [point][256]
    float *dgp;              // [tile][256]
    float *blkp;             // [block][1281]
    float *w2p;              // [chunk][65536]
    float *sidep;            // [side][1280]
    float *dgs;              // [side][256]
    float *grad;             // [SS_MLP_PARAMS]
    double* loss;            // [side]
};

hipError_t mlp_init();
int mlp_head_grid();
int mlp_chunks(int64_t npts);
hipError_t launch_mlp_sync(float* w, __bf16* wbf, __bf16* w2t, hipStream_t st);
hipError_t launch_mlp_predict(const MlpArgs& a, hipStream_t st);
hipError_t launch_mlp_grad(const MlpArgs& a, hipStream_t st);
hipError_t launch_mlp_adam(float* w, float* m1, float* m2, const float* grad, __bf16* wbf,
                           __bf16* w2t, float lr, int step, hipStream_t st);

}  // namespace ss
