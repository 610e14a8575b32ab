// Host driver of the C ABI declared in include/sparsink.h: argument checks,
// workspace carving, stage orchestration on the caller's stream, the
// graph-captured Sinkhorn loop, and the result assembly.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <functional>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/sparsink.h"
#include "internal.hpp"

using namespace ss;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess)                                                           \
            return fail(SS_E_HIP, "%s failed: %s", #expr, hipGetErrorString(_e));      \
    } while (0)

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Byte offsets of every region of the caller's workspace.
struct Layout {
    size_t mask, maskT, row_cnt, col_cnt, row_ptr, col_ptr, scan, col_idx, row_idx, val, val_t;
    size_t row_fac, col_fac, row_bnd, col_bnd, a_eff, b_eff, la_eff, lb_eff, tmp, tree, u[2], v[2];
    size_t ug[2], vg[2];
    size_t partials, loop_part[2], state, stats, hstage, dense_part, rowsum, colsum;
    // UOT normaliser by expansion: centre, monomial table, partials, sums
    size_t zcenter, zexps, zcoef, zpart, zsums;
    // lane plans of the iteration kernel: [0] rows (u-update), [1] columns
    struct PlanOff {
        size_t split, quads, weight, wptr, rstart, info, scan, qs, qe, steplanes, stepoff, lmeta;
        size_t pval, poff;
    } po[2];
    IterPlan plan[2];
    int64_t loop_part_len;
    size_t total;
    int64_t cap;
    int64_t partials_len;
};

int64_t entry_capacity(double s, int64_t n, int64_t m) {
    const double nm = (double)n * (double)m;
    double c = floor(s + 8.0 * sqrt(s) + 64.0);
    if (c > nm) c = nm;
    return (int64_t)c;
}

size_t esize(int precision) { return precision == SS_F64 ? 8 : 4; }
size_t ysize(int precision) { return precision == SS_F32 ? 4 : 8; }

int block_for(const ss_options* O, int64_t nlines) {
    return O->block_threads ? O->block_threads : iterate_block_size(nlines);
}

// Shapes of the two lane plans; false when a dimension is beyond the slice
// limit of the iteration kernel.
bool plan_shapes(const ss_problem* P, const ss_options* O, int64_t cap, IterPlan* pl) {
    const int pr = O->precision;
    return plan_shape(pr, block_for(O, P->n), P->n, P->m, cap, &pl[0]) &&
           plan_shape(pr, block_for(O, P->m), P->m, P->n, cap, &pl[1]);
}

Layout plan(const ss_problem* P, const ss_options* O) {
    Layout L;
    const int64_t n = P->n, m = P->m;
    const int64_t W = (m + 63) / 64, Wn = (n + 63) / 64;
    const int64_t nm = n > m ? n : m;
    L.cap = entry_capacity(O->s, n, m);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    // The sampling masks are dead once the CSR and CSC are filled; the packed
    // entry arrays of the lane plans reuse their memory.
    plan_shapes(P, O, L.cap, L.plan);
    {
        const size_t base = off;
        L.mask = take((size_t)n * W * 8);
        L.maskT = take((size_t)m * Wn * 8);
        const size_t end_masks = off;
        off = base;
        for (int d = 0; d < 2; ++d) {
            L.po[d].pval = take(plan_value_bytes(O->precision, L.plan[d]));
            L.po[d].poff = take(plan_offset_bytes(O->precision, L.plan[d]));
        }
        if (off < end_masks) off = end_masks;
    }
    L.row_cnt = take((size_t)n * 4);
    L.col_cnt = take((size_t)m * 4);
    L.row_ptr = take((size_t)(n + 1) * 8);
    L.col_ptr = take((size_t)(m + 1) * 8);
    L.scan = take((size_t)((nm + 1023) / 1024 + 1) * 8);
    // entry arrays carry 16 entries of padding: the iteration kernel reads
    // whole 16-byte quads around each line
    L.col_idx = take((size_t)(L.cap + 16) * 4);
    L.row_idx = take((size_t)(L.cap + 16) * 4);
    L.val = take((size_t)(L.cap + 16) * esize(O->precision));
    L.val_t = take((size_t)(L.cap + 16) * esize(O->precision));
    L.row_fac = take((size_t)n * 8);
    L.col_fac = take((size_t)m * 8);
    L.row_bnd = take((size_t)n * 8);
    L.col_bnd = take((size_t)m * 8);
    L.a_eff = take((size_t)n * 8);
    L.b_eff = take((size_t)m * 8);
    // log domain: logs of the effective marginals, formed once per solve
    L.la_eff = take(O->precision == SS_F32_LOG ? (size_t)n * 8 : 0);
    L.lb_eff = take(O->precision == SS_F32_LOG ? (size_t)m * 8 : 0);
    // sampling scratch; at the start it holds the pruned cost maximum's state
    const size_t tmp_bytes = (size_t)2 * nm * 8;
    L.tmp = take(tmp_bytes > cmax_scratch_bytes(n) ? tmp_bytes : cmax_scratch_bytes(n));
    const int64_t cost_blocks = ((n + 255) / 256) * ((m + 2047) / 2048);
    const int64_t tree_len = (cost_blocks > nm ? cost_blocks : nm);
    L.tree = take((size_t)(2 * ((tree_len + 1023) / 1024) + 2) * 8);
    for (int k = 0; k < 2; ++k) {
        L.u[k] = take((size_t)n * ysize(O->precision));
        L.v[k] = take((size_t)m * ysize(O->precision));
        // log domain: FP32 copies of the potentials for the sparse gathers
        L.ug[k] = take(O->precision == SS_F32_LOG ? (size_t)n * 4 : 0);
        L.vg[k] = take(O->precision == SS_F32_LOG ? (size_t)m * 4 : 0);
    }
    // block partials: iteration kernels (<= nm lines / 4 per block), objective
    // (5 per block of 16 lines), UOT normaliser, dense objective.
    int64_t pl = 5 * ((nm + 15) / 16) + 64;
    if (cost_blocks > pl) pl = cost_blocks;
    pl += 8 * ((nm + 255) / 256) + 3 * 4096 + 64;
    L.partials_len = pl;
    L.partials = take((size_t)pl * 8);
    L.loop_part_len = ((nm + 255) / 256 > kMaxLoopBlocks ? (nm + 255) / 256 : kMaxLoopBlocks) + 64;
    L.loop_part[0] = take((size_t)L.loop_part_len * 8);
    L.loop_part[1] = take((size_t)L.loop_part_len * 8);
    for (int d = 0; d < 2; ++d) {
        const IterPlan& p = L.plan[d];
        const int64_t nl = d == 0 ? n : m;
        const int64_t kmax = p.kmax;
        const int64_t scan_len = nl > kmax ? nl : kmax;
        L.po[d].split = take((size_t)nl * (size_t)(p.ns + 1) * 4);
        L.po[d].quads = take((size_t)nl * 4);
        L.po[d].weight = take((size_t)nl * 4);
        L.po[d].wptr = take((size_t)(nl + 1) * 8);
        L.po[d].rstart = take((size_t)(kmax + 1) * 4);
        L.po[d].info = take(sizeof(PlanInfo));
        L.po[d].scan = take((size_t)((scan_len + 1023) / 1024 + 1) * 8);
        L.po[d].qs = take((size_t)nl * (size_t)p.ns * 4);
        L.po[d].qe = take((size_t)nl * (size_t)p.ns * 4);
        L.po[d].steplanes = take((size_t)kmax * 4);
        L.po[d].stepoff = take((size_t)(kmax + 1) * 8);
        L.po[d].lmeta = take((size_t)p.lanes_max * 4);
    }

    L.state = take(sizeof(IterState));
    L.stats = take(ST_COUNT * 8);
    L.hstage = take(64);
    L.dense_part = take((size_t)64 * nm * 12);  // <= 64 column segments per line
    const bool uot = isfinite(O->lambda);
    L.zcenter = take(uot ? 64 * 8 : 0);
    L.zexps = take(uot ? (size_t)kZMaxMono * 8 : 0);
    L.zcoef = take(uot ? (size_t)kZMaxMono * 8 : 0);
    L.zpart = take(uot ? (size_t)2 * kZBlocks * kZMaxMono * 8 : 0);
    L.zsums = take(uot ? (size_t)2 * kZMaxMono * 8 : 0);
    L.rowsum = take((size_t)64 * n * 8);
    L.colsum = take((size_t)64 * m * 8);
    L.total = off;
    return L;
}

template <typename T>
T* at(void* ws, size_t off) {
    return (T*)((char*)ws + off);
}

int check_args(const ss_problem* P, const ss_options* O, bool dense) {
    if (!P || !O) return fail(SS_E_INVALID_ARG, "problem and options must not be NULL");
    if (P->n <= 0 || P->m <= 0) return fail(SS_E_INVALID_ARG, "n and m must be positive");
    if (P->n >= ((int64_t)1 << 31) || P->m >= ((int64_t)1 << 31))
        return fail(SS_E_INVALID_ARG, "n and m must be below 2^31");
    if (P->d <= 0 || P->d > 64) return fail(SS_E_INVALID_ARG, "d must be in [1, 64]");
    if (dense && P->d > 16) return fail(SS_E_INVALID_ARG, "dense_sinkhorn supports d <= 16");
    if (!P->x || !P->y || !P->a || !P->b)
        return fail(SS_E_INVALID_ARG, "x, y, a, b must not be NULL");
    if (!(O->eps > 0.0) || !isfinite(O->eps)) return fail(SS_E_INVALID_ARG, "eps must be > 0");
    if (!dense && (!(O->s > 0.0) || !isfinite(O->s)))
        return fail(SS_E_INVALID_ARG, "s must be a positive finite number");
    if (!(O->tol >= 0.0)) return fail(SS_E_INVALID_ARG, "tol must be >= 0");
    if (O->max_iter < 1) return fail(SS_E_INVALID_ARG, "max_iter must be >= 1");
    if (O->precision < SS_F64 || O->precision > SS_F32_LOG)
        return fail(SS_E_INVALID_ARG, "unknown precision %d", O->precision);
    if (O->cost != SS_COST_SQEUCLID_MAXNORM && O->cost != SS_COST_SQEUCLID &&
        O->cost != SS_COST_WFR && O->cost != SS_COST_EUCLID)
        return fail(SS_E_INVALID_ARG, "unknown cost %d", O->cost);
    if (O->cost == SS_COST_EUCLID) {
        // the dense kernels and the UOT probability's bounds and normaliser
        // are written for the squared distances
        if (dense) return fail(SS_E_INVALID_ARG, "dense_sinkhorn takes the squared Euclidean or WFR cost");
        if (isfinite(O->lambda))
            return fail(SS_E_INVALID_ARG, "the Euclidean cost takes OT sampling (lambda = +INFINITY)");
    }
    if (O->cost == SS_COST_WFR) {
        if (!(O->eta > 0.0) || !isfinite(O->eta))
            return fail(SS_E_INVALID_ARG, "the WFR cost needs a finite eta > 0");
        // the OT probability ignores K, and shrinkage would sample the
        // structural zeros of K: the sparse solvers need the UOT probability
        if (!dense && !isfinite(O->lambda))
            return fail(SS_E_INVALID_ARG, "the WFR cost needs finite lambda (UOT sampling)");
        if (!dense && O->shrink != 0.0)
            return fail(SS_E_INVALID_ARG, "the WFR cost takes shrink = 0");
    }
    if (O->stop_rule != SS_STOP_MARGINAL_L1 && O->stop_rule != SS_STOP_SCALING_DELTA_L1)
        return fail(SS_E_INVALID_ARG, "unknown stop rule %d", O->stop_rule);
    if (O->empty_policy < SS_EMPTY_AUTO || O->empty_policy > SS_EMPTY_FAIL)
        return fail(SS_E_INVALID_ARG, "unknown empty policy %d", O->empty_policy);
    const int bt = O->block_threads;
    if (!(bt == 0 || bt == 256 || bt == 1024))
        return fail(SS_E_INVALID_ARG, "block_threads must be 0, 256 or 1024");
    if (!(O->lambda > 0.0)) return fail(SS_E_INVALID_ARG, "lambda must be > 0 (or +INFINITY)");
    if (!(O->shrink >= 0.0 && O->shrink <= 1.0))
        return fail(SS_E_INVALID_ARG, "shrink must be in [0, 1]");
    if (!dense) {
        // the sparse iteration cuts the gathered vector into at most a fixed
        // number of LDS slices
        IterPlan pl[2];
        if (!plan_shapes(P, O, entry_capacity(O->s, P->n, P->m), pl))
            return fail(SS_E_INVALID_ARG, "n or m too large for block_threads %d", bt);
    }
    return SS_OK;
}

int check_ws(const ss_problem* P, const ss_options* O, void* ws, size_t ws_bytes, Layout* L) {
    *L = plan(P, O);
    if (!ws) return fail(SS_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(SS_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < L->total)
        return fail(SS_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, L->total);
    return SS_OK;
}

struct Timer {
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    bool ok = false;
    // enabled = false: no events are created and every time reads 0
    explicit Timer(bool enabled = true) {
        if (!enabled) return;
        ok = true;
        for (auto& e : ev)
            if (hipEventCreate(&e) != hipSuccess) ok = false;
    }
    ~Timer() {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    void mark(int k, hipStream_t st) {
        if (ok) (void)hipEventRecord(ev[k], st);
    }
    float ms(int a, int b) {
        float t = 0.f;
        if (ok) (void)hipEventElapsedTime(&t, ev[a], ev[b]);
        return t;
    }
};

// Two pinned host slots for the loop state per host thread, kept for the
// thread's lifetime (a copy into pinned memory is asynchronous, so the host
// can enqueue the next replay before it reads the previous one's state);
// nullptr if pinned memory is unavailable.
static IterState* pinned_state_slots() {
    thread_local IterState* slots = nullptr;
    thread_local bool tried = false;
    if (!tried) {
        tried = true;
        void* p = nullptr;
        if (hipHostMalloc(&p, 2 * sizeof(IterState), hipHostMallocDefault) == hipSuccess)
            slots = (IterState*)p;
    }
    return slots;
}

// Graph kinds with an executable cached per host thread and device.
enum GraphKind { GK_LOOP = 0, GK_TIMING, GK_SAMPLE, GK_BATCH_LOOP, GK_OTHER, GK_COUNT };
constexpr int kGraphDevices = 64;

// Per host thread and device: the stream graphs are captured on and one
// executable graph per kind, kept for the thread's life like the pinned loop
// slots (never destroyed: they may outlive the runtime at process exit).  A
// solve then creates no stream, and when its graph has the shape of the
// previous one of its kind (same launches, new arguments) the executable is
// updated in place instead of instantiated.
struct ThreadGraphs {
    hipStream_t cs;
    hipGraphExec_t exec[GK_COUNT];
};

static ThreadGraphs* thread_graphs() {
    thread_local ThreadGraphs tg[kGraphDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kGraphDevices) return nullptr;
    ThreadGraphs& g = tg[dev];
    if (!g.cs && hipStreamCreateWithFlags(&g.cs, hipStreamNonBlocking) != hipSuccess) {
        g.cs = nullptr;
        return nullptr;
    }
    return &g;
}

// Records `rec(stream)` into a graph on the thread's capture stream and
// returns an executable for it in *exec: the thread's executable of `kind`
// updated in place when the shapes match, else a new one that replaces it.
// The caller must have waited for every earlier launch of that executable
// (every entry point synchronises before it returns).
hipError_t capture_exec(int kind, const std::function<hipError_t(hipStream_t)>& rec,
                        hipGraphExec_t* exec) {
    *exec = nullptr;
    ThreadGraphs* tg = thread_graphs();
    if (!tg) return hipErrorInvalidDevice;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(tg->cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t e1 = rec(tg->cs);
        const hipError_t e2 = hipStreamEndCapture(tg->cs, &graph);
        e = e1 != hipSuccess ? e1 : e2;
    }
    if (e == hipSuccess && tg->exec[kind]) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateSuccess;
        if (hipGraphExecUpdate(tg->exec[kind], graph, &bad, &res) == hipSuccess &&
            res == hipGraphExecUpdateSuccess) {
            *exec = tg->exec[kind];
        } else {
            (void)hipGetLastError();  // a refused update is not an error of the solve
            (void)hipGraphExecDestroy(tg->exec[kind]);
            tg->exec[kind] = nullptr;
        }
    }
    if (e == hipSuccess && !*exec) {
        e = hipGraphInstantiate(&tg->exec[kind], graph, nullptr, nullptr, 0);
        if (e == hipSuccess) *exec = tg->exec[kind];
        else tg->exec[kind] = nullptr;
    }
    if (graph) (void)hipGraphDestroy(graph);
    return e;
}

// Runs the Sinkhorn loop: `iter(k, stream)` enqueues iteration k (its
// ping-pong parity is k & 1).  With graph_iters > 0 an even number of
// iterations is captured once and replayed.  Replays are pipelined: replay
// r + 1 is enqueued before the host reads the stop state that replay r copies
// into a pinned slot, so the device never waits for the host between
// replays.  The replay in flight when the stop is seen runs its launches as
// no-ops (they return at entry); the stream is synchronised before return.
// `tol` (the stop tolerance, or 0) only steers the lookahead.
int run_loop(const std::function<hipError_t(int, hipStream_t)>& iter, int graph_iters,
             int max_iter, double tol, IterState* d_state, IterState* h_state,
             hipStream_t stream) {
    const int total = max_iter + 1;  // the last launch only closes the residual
    if (graph_iters > 0) {
        int G = graph_iters + (graph_iters & 1);
        if (G > total + (total & 1)) G = total + (total & 1);
        hipGraphExec_t exec = nullptr;
        hipError_t e = capture_exec(GK_LOOP, [&](hipStream_t cs) {
            hipError_t er = hipSuccess;
            for (int k = 0; k < G && er == hipSuccess; ++k) er = iter(k, cs);
            return er;
        }, &exec);
        int rc = SS_OK;
        if (e != hipSuccess) rc = fail(SS_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
        const int nrep = (total + G - 1) / G;
        IterState* slot = pinned_state_slots();
        hipEvent_t ev[2] = {nullptr, nullptr};
        bool piped = slot != nullptr;
        for (auto& x : ev)
            if (piped && hipEventCreateWithFlags(&x, hipEventDisableTiming) != hipSuccess) piped = false;
        if (rc == SS_OK && piped) {
            auto enqueue = [&](int r) -> hipError_t {
                hipError_t er = hipGraphLaunch(exec, stream);
                if (er == hipSuccess)
                    er = hipMemcpyAsync(&slot[r & 1], d_state, sizeof(IterState),
                                        hipMemcpyDeviceToHost, stream);
                if (er == hipSuccess) er = hipEventRecord(ev[r & 1], stream);
                return er;
            };
            // Lookahead is skipped for the replay after the one the residual
            // trend says will stop: its launches would all be no-ops.  The
            // trend (geometric decay of the latest err over the last two
            // replays read) only schedules replays; the stop test stays on
            // the device.
            double e1 = -1.0, e2 = -1.0;  // proxies after the last two replays read
            auto likely_last = [&]() {
                if (!(tol > 0.0) || !(e1 > 0.0) || !(e2 > e1)) return false;
                const double reps = std::log(tol / e1) / std::log(e1 / e2);
                return reps <= 1.0;
            };
            int queued = 0;
            e = enqueue(queued++);
            for (int r = 0; e == hipSuccess && r < nrep; ++r) {
                if (queued == r + 1 && queued < nrep && !likely_last()) e = enqueue(queued++);
                if (e == hipSuccess) e = hipEventSynchronize(ev[r & 1]);
                if (e != hipSuccess) break;
                *h_state = slot[r & 1];
                if (h_state->stop_iter != 0 || h_state->nonfinite != 0) break;
                e2 = e1;
                e1 = h_state->err_last;
                if (queued == r + 1 && queued < nrep) e = enqueue(queued++);
            }
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            if (e != hipSuccess) rc = fail(SS_E_HIP, "loop failed: %s", hipGetErrorString(e));
        } else {
            for (int done = 0; rc == SS_OK && done < total; done += G) {
                e = hipGraphLaunch(exec, stream);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(h_state, d_state, sizeof(IterState), hipMemcpyDeviceToHost,
                                       stream);
                if (e == hipSuccess) e = hipStreamSynchronize(stream);
                if (e != hipSuccess) rc = fail(SS_E_HIP, "loop failed: %s", hipGetErrorString(e));
                if (h_state->stop_iter != 0 || h_state->nonfinite != 0) break;
            }
        }
        for (auto& x : ev)
            if (x) (void)hipEventDestroy(x);
        return rc;
    }
    const int poll = 8;
    for (int t = 1; t <= total; ++t) {
        HIP_TRY(iter((t - 1) & 1, stream));
        if (t % poll == 0 || t == total) {
            HIP_TRY(hipMemcpyAsync(h_state, d_state, sizeof(IterState), hipMemcpyDeviceToHost,
                                   stream));
            HIP_TRY(hipStreamSynchronize(stream));
            if (h_state->stop_iter != 0 || h_state->nonfinite != 0) break;
        }
    }
    return SS_OK;
}

struct Ctx {
    const ss_problem* P;
    const ss_options* O;
    Layout L;
    void* ws;
    hipStream_t st;
    bool uot;
    double stats[ST_COUNT];
    int64_t nnz;
    double inv_cmax;
    // host copy of the monomial table of the normaliser's expansion (kept
    // until the sampling stage synchronises)
    std::vector<uint8_t> zexps;
    std::vector<double> zcoef;
    // UOT: a normaliser given by the caller of ss_sample (0: the library's own)
    double z_in = 0.0;
};

// Degree K of the normaliser's expansion: the remainder of the exponential
// series at |t| <= T is below T^(K+1)/(K+1)! e^T, relative to a term of at
// least e^-T; K is the smallest degree with that ratio below 2^-64.  False
// when no K <= kZMaxDegree works or the monomials exceed kZMaxMono.
bool zexp_degree(double g, double rx2, double ry2, int d, int* K_out, int* M_out) {
    if (!(g >= 0.0) || !isfinite(g) || d > 8) return false;
    const double T = 2.0 * g * sqrt(rx2) * sqrt(ry2) * (1.0 + 1e-9);
    if (!isfinite(T)) return false;
    double term = T * exp(2.0 * T);   // T^(K+1)/(K+1)! e^(2T) at K = 0
    for (int K = 0; K <= kZMaxDegree; ++K) {
        if (K > 0) term *= T / (double)(K + 1);
        if (term <= 0x1p-64) {
            // monomials of degree <= K in d variables: C(K + d, d)
            double M = 1.0;
            for (int i = 1; i <= d; ++i) M = M * (double)(K + i) / (double)i;
            if (M > kZMaxMono) return false;
            *K_out = K;
            *M_out = (int)llround(M);
            return true;
        }
    }
    return false;
}

// Every multi-index alpha with |alpha| <= K (d <= 8 exponents per entry) and
// coef_alpha = (2g)^|alpha| / alpha!.
void zexp_table(int d, int K, double g, std::vector<uint8_t>* exps, std::vector<double>* coef) {
    exps->clear();
    coef->clear();
    uint8_t a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    std::function<void(int, int)> rec = [&](int k, int left) {
        if (k == d) {
            double c = 1.0;
            for (int i = 0; i < d; ++i)
                for (int q = 1; q <= a[i]; ++q) c *= (2.0 * g) / (double)q;
            exps->insert(exps->end(), a, a + 8);
            coef->push_back(c);
            return;
        }
        for (int e = 0; e <= left; ++e) {
            a[k] = (uint8_t)e;
            rec(k + 1, left - e);
        }
        a[k] = 0;
    };
    rec(0, K);
}

// Zeroes state and statistics, checks the inputs, computes max c_ij.
int stage_start(Ctx& c) {
    const ss_problem* P = c.P;
    double* stats = at<double>(c.ws, c.L.stats);
    HIP_TRY(launch_fill_f64(stats, ST_COUNT, 0.0, c.st));
    HIP_TRY(launch_fill_u32(at<uint32_t>(c.ws, c.L.state), sizeof(IterState) / 4, 0u, c.st));
    HIP_TRY(launch_validate(P->a, P->n, P->x, P->n * P->d, stats, c.st));
    HIP_TRY(launch_validate(P->b, P->m, P->y, P->m * P->d, stats, c.st));
    HIP_TRY(launch_cmax(P->x, P->y, P->n, P->m, P->d, stats, at<void>(c.ws, c.L.tmp), c.st));
    if (c.uot)
        HIP_TRY(launch_center_radii(P->x, P->y, P->n, P->m, P->d, at<void>(c.ws, c.L.tmp),
                                    at<double>(c.ws, c.L.zcenter), stats, c.st));
    if (c.uot && c.O->cost == SS_COST_WFR)
        HIP_TRY(launch_same_support(P->x, P->y, P->n, P->m, P->d, stats, c.st));
    HIP_TRY(hipMemcpyAsync(c.stats, stats, sizeof(c.stats), hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    if (c.stats[ST_BAD_INPUT] != 0.0)
        return fail(SS_E_INVALID_ARG, "a, b must be finite and >= 0 and x, y finite");
    const double cmax = c.stats[ST_CMAX];
    c.inv_cmax = (c.O->cost == SS_COST_SQEUCLID_MAXNORM && cmax > 0.0) ? 1.0 / cmax : 1.0;
    return SS_OK;
}

ProbParams make_params(const Ctx& c) {
    ProbParams pp;
    const ss_options* O = c.O;
    pp.uot = c.uot ? 1 : 0;
    pp.s = O->s;
    pp.eps = O->eps;
    pp.inv_cmax = c.inv_cmax;
    pp.inv_tau = c.uot ? 1.0 / (2.0 * O->lambda + O->eps) : 0.0;
    pp.kappa = 0.0;
    // Sec. 4 shrinkage: s p = (1 - g) s p_ij + s g / (nm)
    pp.shrink_w = 1.0 - O->shrink;
    pp.shrink_c = O->s * O->shrink / ((double)c.P->n * (double)c.P->m);
    pp.cost = O->cost;
    pp.wfr_w = 0.5 / O->eta;
    pp.row_fac = at<double>(c.ws, c.L.row_fac);
    pp.col_fac = at<double>(c.ws, c.L.col_fac);
    pp.row_bnd = at<double>(c.ws, c.L.row_bnd);
    pp.col_bnd = at<double>(c.ws, c.L.col_bnd);
    pp.x = c.P->x;
    pp.y = c.P->y;
    pp.d = c.P->d;
    pp.problem_index = c.P->problem_index;
    pp.k0 = (uint32_t)(O->seed & 0xFFFFFFFFull);
    pp.k1 = (uint32_t)(O->seed >> 32);
    return pp;
}

// Probabilities, mask, CSR and CSC, empty-line policy (step 1 of Alg. 3/4).
int stage_sample(Ctx& c) {
    const ss_problem* P = c.P;
    const ss_options* O = c.O;
    const int64_t n = P->n, m = P->m;
    const int64_t W = (m + 63) / 64, Wn = (n + 63) / 64;
    void* ws = c.ws;
    hipStream_t st = c.st;
    double* stats = at<double>(ws, c.L.stats);
    double* tree = at<double>(ws, c.L.tree);
    ProbParams pp = make_params(c);
    if (!c.uot) {
        HIP_TRY(launch_ot_prep(P->a, P->b, n, m, O->s, pp.shrink_w, (double*)pp.row_fac,
                               (double*)pp.col_fac, tree, stats, st));
    } else {
        // exp(col_fac) goes to col_bnd until the bounds below replace it
        HIP_TRY(launch_uot_prep(P->a, P->b, n, m, O->lambda, O->eps, (double*)pp.row_fac,
                                (double*)pp.col_fac, (double*)pp.row_bnd, (double*)pp.col_bnd, st));
        // Z: by the truncated expansion where the cost is squared Euclidean
        // and the degree stays small, else pair by pair
        int K = 0, M = 0;
        if (O->cost != SS_COST_WFR &&
            zexp_degree(c.inv_cmax * pp.inv_tau, c.stats[ST_RX2], c.stats[ST_RY2], P->d, &K, &M)) {
            zexp_table(P->d, K, c.inv_cmax * pp.inv_tau, &c.zexps, &c.zcoef);
            uint8_t* dexps = at<uint8_t>(ws, c.L.zexps);
            double* dcoef = at<double>(ws, c.L.zcoef);
            HIP_TRY(hipMemcpyAsync(dexps, c.zexps.data(), c.zexps.size(), hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(dcoef, c.zcoef.data(), c.zcoef.size() * 8, hipMemcpyHostToDevice,
                                   st));
            ZExpArgs za;
            za.x = P->x;
            za.y = P->y;
            za.la = pp.row_fac;
            za.lb = pp.col_fac;
            za.n = n;
            za.m = m;
            za.d = P->d;
            za.K = K;
            za.M = M;
            za.g = c.inv_cmax * pp.inv_tau;
            za.center = at<double>(ws, c.L.zcenter);
            za.exps = dexps;
            za.coef = dcoef;
            za.part = at<double>(ws, c.L.zpart);
            za.sums = at<double>(ws, c.L.zsums);
            HIP_TRY(launch_uot_zexp(za, stats, st));
        } else {
            HIP_TRY(launch_uot_z(pp, n, m, pp.col_bnd, c.stats[ST_CMAX],
                                 c.stats[ST_SAME_SUPPORT] != 0.0, at<double>(ws, c.L.partials),
                                 tree, stats, st));
        }
        if (c.z_in > 0.0) HIP_TRY(launch_fill_f64(stats + ST_Z, 1, c.z_in, st));
        HIP_TRY(launch_uot_bounds(pp.col_fac, m, O->s, pp.shrink_w, stats, (double*)pp.col_bnd,
                                  st));
    }
    int32_t* row_cnt = at<int32_t>(ws, c.L.row_cnt);
    int32_t* col_cnt = at<int32_t>(ws, c.L.col_cnt);
    HIP_TRY(launch_fill_i32(row_cnt, n, 0, st));
    HIP_TRY(launch_fill_i32(col_cnt, m, 0, st));
    uint64_t* mask = at<uint64_t>(ws, c.L.mask);
    uint64_t* maskT = at<uint64_t>(ws, c.L.maskT);
    HIP_TRY(launch_mask(pp, n, m, mask, row_cnt, stats, st));
    HIP_TRY(launch_transpose(mask, n, m, maskT, col_cnt, st));
    int64_t* row_ptr = at<int64_t>(ws, c.L.row_ptr);
    int64_t* col_ptr = at<int64_t>(ws, c.L.col_ptr);
    HIP_TRY(launch_scan(row_cnt, n, row_ptr, at<int64_t>(ws, c.L.scan), st));
    HIP_TRY(launch_scan(col_cnt, m, col_ptr, at<int64_t>(ws, c.L.scan), st));
    int64_t tot[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(&tot[0], row_ptr + n, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&tot[1], col_ptr + m, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (tot[0] != tot[1]) return fail(SS_E_HIP, "CSR and CSC sizes differ (%lld vs %lld)",
                                      (long long)tot[0], (long long)tot[1]);
    c.nnz = tot[0];
    if (c.nnz > c.L.cap)
        return fail(SS_E_CAPACITY, "sampled %lld entries exceed the capacity %lld",
                    (long long)c.nnz, (long long)c.L.cap);
    HIP_TRY(launch_fill_entries(0, O->precision, pp, stats, mask, n, W, row_ptr,
                                at<int32_t>(ws, c.L.col_idx), at<void>(ws, c.L.val), c.L.cap, st));
    HIP_TRY(launch_fill_entries(1, O->precision, pp, stats, maskT, m, Wn, col_ptr,
                                at<int32_t>(ws, c.L.row_idx), at<void>(ws, c.L.val_t), c.L.cap,
                                st));
    int policy = O->empty_policy;
    if (policy == SS_EMPTY_AUTO) policy = c.uot ? SS_EMPTY_ZERO : SS_EMPTY_RENORMALIZE;
    const int renorm = policy == SS_EMPTY_RENORMALIZE;
    HIP_TRY(launch_empty_policy(P->a, row_cnt, n, renorm, 0, at<double>(ws, c.L.a_eff),
                                at<double>(ws, c.L.tmp), tree, stats, st));
    HIP_TRY(launch_empty_policy(P->b, col_cnt, m, renorm, 1, at<double>(ws, c.L.b_eff),
                                at<double>(ws, c.L.tmp), tree, stats, st));
    if (policy == SS_EMPTY_FAIL) {
        HIP_TRY(hipMemcpyAsync(c.stats, stats, sizeof(c.stats), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (c.stats[ST_EMPTY_ROWS] > 0 || c.stats[ST_EMPTY_COLS] > 0)
            return fail(SS_E_EMPTY, "%.0f empty rows and %.0f empty columns",
                        c.stats[ST_EMPTY_ROWS], c.stats[ST_EMPTY_COLS]);
    }
    return SS_OK;
}

// Captures `iters` iterations (iters even, every launch active), replays the
// graph once to warm up, resets the state and scalings, replays it again
// between two events, and reports the mean time of one kernel launch
// (2 launches per iteration for the sparse loop, `launches_per_iter` in general).
int time_graph(const std::function<hipError_t(int, hipStream_t)>& iter, int iters, void* u0,
               void* v0, float* ug0, float* vg0, int prec, int64_t n, int64_t m,
               const ss_options* O, IterState* d_state, hipStream_t st, double* ms_out,
               int launches_per_iter = 2) {
    if (!ms_out) return fail(SS_E_INVALID_ARG, "ms_out must not be NULL");
    hipGraphExec_t exec = nullptr;
    hipError_t e = capture_exec(GK_TIMING, [&](hipStream_t cs) {
        hipError_t er = hipSuccess;
        for (int k = 0; k < iters && er == hipSuccess; ++k) er = iter(k, cs);
        return er;
    }, &exec);
    hipEvent_t a = nullptr, b = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    float ms = 0.f;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        e = launch_fill_u32((uint32_t*)d_state, sizeof(IterState) / 4, 0u, st);
        if (e == hipSuccess) e = launch_init_scaling(prec, u0, ug0, O->init_log_u, n, st);
        if (e == hipSuccess) e = launch_init_scaling(prec, v0, vg0, O->init_log_v, m, st);
        if (e == hipSuccess && rep == 1) e = hipEventRecord(a, st);
        if (e == hipSuccess) e = hipGraphLaunch(exec, st);
        if (e == hipSuccess && rep == 1) e = hipEventRecord(b, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return fail(SS_E_HIP, "timing graph failed: %s", hipGetErrorString(e));
    *ms_out = (double)ms / (double)(iters * launches_per_iter);
    return SS_OK;
}

void fill_result(const Ctx& c, const IterState& hs, ss_result* R, int64_t nnz) {
    const double* s = c.stats;
    const ss_options* O = c.O;
    const double kl = c.uot ? O->lambda * (s[ST_KL_A] + s[ST_KL_B]) : 0.0;
    R->transport = s[ST_TRANSPORT];
    R->neg_entropy = s[ST_NEGENT];
    R->kl_a = c.uot ? s[ST_KL_A] : 0.0;
    R->kl_b = c.uot ? s[ST_KL_B] : 0.0;
    R->estimate = s[ST_TRANSPORT] + O->eps * s[ST_NEGENT] + kl;
    R->sparse_objective = O->eps * s[ST_SPARSEOBJ] + kl;
    R->marginal_err = hs.err_final;
    R->cmax = s[ST_CMAX];
    R->z_norm = c.uot ? s[ST_Z] : 0.0;
    R->dropped_mass_a = s[ST_DROPPED_A];
    R->dropped_mass_b = s[ST_DROPPED_B];
    R->nnz = nnz;
    R->empty_rows = (int64_t)s[ST_EMPTY_ROWS];
    R->empty_cols = (int64_t)s[ST_EMPTY_COLS];
    R->iters = hs.stop_iter;
    R->warm_start = (O->init_log_u || O->init_log_v) ? 1 : -1;
}

// time_iters > 0: after sampling, run exactly time_iters iterations (tol = 0)
// as one captured graph, once to warm up and once timed with HIP events, and
// return the mean duration of one iteration-kernel launch in *ms_out.
// Where a solve adds the envelope gradients of its sparse value (the
// divergence): gx += cx * d/dx, gy += cy * d/dy (gy may equal gx).
struct GradSink {
    double* gx;
    double* gy;
    double cx, cy;
};

// noalloc: no HIP object is created (no events, graphs or streams) and the
// loop runs as plain launches; the workspace is whatever the caller passed.
int spar_sink_impl(const ss_problem* P, const ss_options* O, void* ws, size_t ws_bytes,
                   void* stream, ss_result* R, bool uot, int time_iters = 0,
                   double* ms_out = nullptr, const GradSink* gs = nullptr, bool noalloc = false) {
    int rc = check_args(P, O, false);
    if (rc != SS_OK) return rc;
    if (!R) return fail(SS_E_INVALID_ARG, "result must not be NULL");
    if (uot && !isfinite(O->lambda)) return fail(SS_E_INVALID_ARG, "spar_sink_uot needs finite lambda");
    if (!uot && isfinite(O->lambda)) return fail(SS_E_INVALID_ARG, "spar_sink_ot needs lambda = +INFINITY");
    Ctx c;
    c.P = P;
    c.O = O;
    c.ws = ws;
    c.st = (hipStream_t)stream;
    c.uot = uot;
    rc = check_ws(P, O, ws, ws_bytes, &c.L);
    if (rc != SS_OK) return rc;
    memset(R, 0, sizeof *R);
    Timer tm(!noalloc);
    tm.mark(0, c.st);
    rc = stage_start(c);
    if (rc != SS_OK) return rc;
    tm.mark(1, c.st);
    rc = stage_sample(c);
    if (rc != SS_OK) return rc;
    tm.mark(2, c.st);

    const int64_t n = P->n, m = P->m;
    const int prec = O->precision;
    void* u[2] = {at<void>(ws, c.L.u[0]), at<void>(ws, c.L.u[1])};
    void* v[2] = {at<void>(ws, c.L.v[0]), at<void>(ws, c.L.v[1])};
    const bool lg = prec == SS_F32_LOG;
    float* ug[2] = {lg ? at<float>(ws, c.L.ug[0]) : nullptr, lg ? at<float>(ws, c.L.ug[1]) : nullptr};
    float* vg[2] = {lg ? at<float>(ws, c.L.vg[0]) : nullptr, lg ? at<float>(ws, c.L.vg[1]) : nullptr};
    HIP_TRY(launch_init_scaling(prec, u[0], ug[0], O->init_log_u, n, c.st));
    HIP_TRY(launch_init_scaling(prec, v[0], vg[0], O->init_log_v, m, c.st));
    if (lg) {
        HIP_TRY(launch_log_vec(at<double>(ws, c.L.a_eff), at<double>(ws, c.L.la_eff), n, c.st));
        HIP_TRY(launch_log_vec(at<double>(ws, c.L.b_eff), at<double>(ws, c.L.lb_eff), m, c.st));
    }
    IterState* d_state = at<IterState>(ws, c.L.state);
    const double theta = uot ? O->lambda / (O->lambda + O->eps) : 1.0;
    HIP_TRY(iterate_init());
    IterPlan pl[2];
    for (int d = 0; d < 2; ++d) {
        IterPlan p = c.L.plan[d];
        const Layout::PlanOff& po = c.L.po[d];
        p.grid = iterate_grid(prec, p.block);
        p.split = at<int32_t>(ws, po.split);
        p.quads = at<int32_t>(ws, po.quads);
        p.weight = at<int32_t>(ws, po.weight);
        p.wptr = at<int64_t>(ws, po.wptr);
        p.rstart = at<int32_t>(ws, po.rstart);
        p.info = at<PlanInfo>(ws, po.info);
        p.scan = at<int64_t>(ws, po.scan);
        p.qs = at<int32_t>(ws, po.qs);
        p.qe = at<int32_t>(ws, po.qe);
        p.steplanes = at<int32_t>(ws, po.steplanes);
        p.stepoff = at<int64_t>(ws, po.stepoff);
        p.lmeta = at<int32_t>(ws, po.lmeta);
        p.pval = at<void>(ws, po.pval);
        p.poff = at<uint16_t>(ws, po.poff);
        pl[d] = p;
    }
    HIP_TRY(build_plan(prec, pl[0], at<int64_t>(ws, c.L.row_ptr), at<int32_t>(ws, c.L.col_idx),
                       at<void>(ws, c.L.val), n, c.st));
    HIP_TRY(build_plan(prec, pl[1], at<int64_t>(ws, c.L.col_ptr), at<int32_t>(ws, c.L.row_idx),
                       at<void>(ws, c.L.val_t), m, c.st));
    IterArgs ua[2], va[2];
    for (int k = 0; k < 2; ++k) {
        IterArgs a;
        a.ptr = at<int64_t>(ws, c.L.row_ptr);
        a.nlines = n;
        a.nx = m;
        a.nslices = pl[0].ns;
        a.rstart = pl[0].rstart;
        a.stepoff = pl[0].stepoff;
        a.qs = pl[0].qs;
        a.qe = pl[0].qe;
        a.lmeta = pl[0].lmeta;
        a.info = pl[0].info;
        a.pval = pl[0].pval;
        a.poff = pl[0].poff;
        a.marg = at<double>(ws, c.L.a_eff);
        a.lmarg = lg ? at<double>(ws, c.L.la_eff) : nullptr;
        a.xin = lg ? (const void*)vg[k] : v[k];
        a.yout = u[(k + 1) & 1];
        a.yg = ug[(k + 1) & 1];
        a.yprev = u[k];
        a.theta = theta;
        a.partials = at<double>(ws, c.L.loop_part[0]);
        a.prev_partials = at<double>(ws, c.L.loop_part[1]);
        a.prev_nblocks = pl[1].grid;
        a.st = d_state;
        a.err_hist = O->err_hist;
        a.role = 0;
        a.stop_rule = O->stop_rule;
        a.max_iter = O->max_iter;
        a.tol = O->tol;
        ua[k] = a;
        a.ptr = at<int64_t>(ws, c.L.col_ptr);
        a.nlines = m;
        a.nx = n;
        a.nslices = pl[1].ns;
        a.rstart = pl[1].rstart;
        a.stepoff = pl[1].stepoff;
        a.qs = pl[1].qs;
        a.qe = pl[1].qe;
        a.lmeta = pl[1].lmeta;
        a.info = pl[1].info;
        a.pval = pl[1].pval;
        a.poff = pl[1].poff;
        a.marg = at<double>(ws, c.L.b_eff);
        a.lmarg = lg ? at<double>(ws, c.L.lb_eff) : nullptr;
        a.xin = lg ? (const void*)ug[(k + 1) & 1] : u[(k + 1) & 1];
        a.yout = v[(k + 1) & 1];
        a.yg = vg[(k + 1) & 1];
        a.yprev = v[k];
        a.partials = at<double>(ws, c.L.loop_part[1]);
        a.prev_partials = at<double>(ws, c.L.loop_part[0]);
        a.prev_nblocks = pl[0].grid;
        a.role = 1;
        va[k] = a;
    }
    // one pointer captured: the std::function below stores it in place
    struct LoopLaunch {
        int prec;
        const IterPlan* pl;
        const IterArgs* ua;
        const IterArgs* va;
    } const ll = {prec, pl, ua, va};
    auto iter = [q = &ll](int k, hipStream_t s) -> hipError_t {
        hipError_t e = launch_iterate(q->prec, q->pl[0].block, q->pl[0].grid, q->ua[k & 1], s);
        if (e == hipSuccess) e = launch_iterate(q->prec, q->pl[1].block, q->pl[1].grid, q->va[k & 1], s);
        return e;
    };
    if (time_iters > 0) {
        for (int k = 0; k < 2; ++k) {
            // a negative tolerance never stops the loop: an error that
            // reaches exactly 0 would otherwise end every later launch at entry
            ua[k].tol = va[k].tol = -1.0;
            ua[k].max_iter = va[k].max_iter = time_iters;
            ua[k].err_hist = va[k].err_hist = nullptr;
        }
        return time_graph(iter, time_iters, u[0], v[0], ug[0], vg[0], prec, n, m, O, d_state, c.st,
                          ms_out);
    }
    const int G = noalloc ? -1 : O->graph_iters == 0 ? 16 : O->graph_iters;
    IterState hs;
    memset(&hs, 0, sizeof hs);
    rc = run_loop(iter, G, O->max_iter, O->tol, d_state, &hs, c.st);
    if (rc != SS_OK) return rc;
    tm.mark(3, c.st);
    if (hs.nonfinite) return fail(SS_E_NONFINITE, "a scaling became NaN or Inf");
    if (hs.stop_iter <= 0) return fail(SS_E_HIP, "loop ended without a result");
    const int p = hs.stop_iter & 1;

    ObjArgs oa;
    oa.ptr = at<int64_t>(ws, c.L.row_ptr);
    oa.idx = at<int32_t>(ws, c.L.col_idx);
    oa.val = at<void>(ws, c.L.val);
    oa.nlines = n;
    oa.ys = u[p];
    oa.zs = v[p];
    oa.marg = P->a;
    oa.x = P->x;
    oa.y = P->y;
    oa.d = P->d;
    oa.inv_cmax = c.inv_cmax;
    oa.cost = O->cost;
    oa.wfr_w = 0.5 / O->eta;
    oa.eps = O->eps;
    oa.uot = uot ? 1 : 0;
    oa.role = 0;
    oa.partials = at<double>(ws, c.L.partials);
    oa.st = d_state;
    oa.stats = at<double>(ws, c.L.stats);
    HIP_TRY(launch_objective(prec, oa, c.st));
    oa.ptr = at<int64_t>(ws, c.L.col_ptr);
    oa.idx = at<int32_t>(ws, c.L.row_idx);
    oa.val = at<void>(ws, c.L.val_t);
    oa.nlines = m;
    oa.ys = v[p];
    oa.zs = u[p];
    oa.marg = P->b;
    oa.x = P->y;
    oa.y = P->x;
    oa.role = 1;
    HIP_TRY(launch_objective(prec, oa, c.st));
    if (gs) {
        // squared Euclidean cost: dC_ij/dx_i = 2 inv_cmax (x_i - y_j); Euclidean
        // cost: (x_i - y_j) / |x_i - y_j| (0 where the points coincide); the
        // column side symmetrically
        const bool eu = O->cost == SS_COST_EUCLID;
        const double gscale = eu ? 1.0 : 2.0 * c.inv_cmax;
        GradArgs ga;
        ga.euclid = eu ? 1 : 0;
        ga.ptr = at<int64_t>(ws, c.L.row_ptr);
        ga.idx = at<int32_t>(ws, c.L.col_idx);
        ga.val = at<void>(ws, c.L.val);
        ga.nlines = n;
        ga.ys = u[p];
        ga.zs = v[p];
        ga.xl = P->x;
        ga.xo = P->y;
        ga.d = P->d;
        ga.coef = gscale * gs->cx;
        ga.out = gs->gx;
        HIP_TRY(launch_plan_grad(prec, ga, c.st));
        ga.ptr = at<int64_t>(ws, c.L.col_ptr);
        ga.idx = at<int32_t>(ws, c.L.row_idx);
        ga.val = at<void>(ws, c.L.val_t);
        ga.nlines = m;
        ga.ys = v[p];
        ga.zs = u[p];
        ga.xl = P->y;
        ga.xo = P->x;
        ga.coef = gscale * gs->cy;
        ga.out = gs->gy;
        HIP_TRY(launch_plan_grad(prec, ga, c.st));
    }
    HIP_TRY(launch_export_scaling(prec, u[p], O->u_out, n, c.st));
    HIP_TRY(launch_export_scaling(prec, v[p], O->v_out, m, c.st));
    HIP_TRY(hipMemcpyAsync(c.stats, at<double>(ws, c.L.stats), sizeof(c.stats),
                           hipMemcpyDeviceToHost, c.st));
    tm.mark(4, c.st);
    HIP_TRY(hipStreamSynchronize(c.st));
    fill_result(c, hs, R, c.nnz);
    R->t_prep_ms = tm.ms(0, 1);
    R->t_sample_ms = tm.ms(1, 2);
    R->t_iter_ms = tm.ms(2, 3);
    R->t_obj_ms = tm.ms(3, 4);
    R->status = hs.err_final <= O->tol ? SS_OK : SS_NOT_CONVERGED;
    return R->status;
}


// ------------------------------------------------------------------ batches
struct BLayout {
    size_t prob, stat, tile_cmax, tile_mask, tile_tr, row_off, col_off, owner, order, queue, gstats;
    size_t row_fac, col_fac, a_eff, b_eff, mask, maskT, row_cnt, col_cnt, row_ptr, col_ptr, scan;
    size_t col_idx, row_idx, val, val_t, u, v, obj_part;
    size_t hlog, handoff, handoff_bytes;  // straggler hand-off: log scalings, solver workspace
    size_t total;
    int64_t rows, cols, cap, nt_cmax, nt_mask, nt_tr;
    int nmax, mmax;
};

int check_batch(const ss_batch* B, const ss_options* O) {
    if (!B || !O) return fail(SS_E_INVALID_ARG, "batch and options must not be NULL");
    if (B->count < 1) return fail(SS_E_INVALID_ARG, "count must be >= 1");
    if (B->d <= 0 || B->d > 64) return fail(SS_E_INVALID_ARG, "d must be in [1, 64]");
    if (!B->n || !B->m || !B->s) return fail(SS_E_INVALID_ARG, "n, m, s must not be NULL");
    if (!B->x || !B->y || !B->a || !B->b)
        return fail(SS_E_INVALID_ARG, "x, y, a, b must not be NULL");
    for (int k = 0; k < B->count; ++k) {
        if (B->n[k] < 1 || B->n[k] > SS_BATCH_MAX_SIDE || B->m[k] < 1 || B->m[k] > SS_BATCH_MAX_SIDE)
            return fail(SS_E_INVALID_ARG, "problem %d: n and m must be in [1, %d]", k, SS_BATCH_MAX_SIDE);
        if (!(B->s[k] > 0.0) || !isfinite(B->s[k]))
            return fail(SS_E_INVALID_ARG, "problem %d: s must be a positive finite number", k);
    }
    if (!(O->eps > 0.0) || !isfinite(O->eps)) return fail(SS_E_INVALID_ARG, "eps must be > 0");
    if (!(O->tol >= 0.0)) return fail(SS_E_INVALID_ARG, "tol must be >= 0");
    if (O->max_iter < 1) return fail(SS_E_INVALID_ARG, "max_iter must be >= 1");
    if (isfinite(O->lambda)) return fail(SS_E_INVALID_ARG, "batches solve OT: lambda must be +INFINITY");
    if (O->shrink != 0.0) return fail(SS_E_INVALID_ARG, "batches sample with shrink = 0 only");
    if (O->precision != SS_F64 && O->precision != SS_F32)
        return fail(SS_E_INVALID_ARG, "batches support precision SS_F64 or SS_F32");
    if (O->cost != SS_COST_SQEUCLID_MAXNORM && O->cost != SS_COST_SQEUCLID)
        return fail(SS_E_INVALID_ARG, "unknown cost %d", O->cost);
    if (O->stop_rule != SS_STOP_MARGINAL_L1)
        return fail(SS_E_INVALID_ARG, "batches support the marginal stop rule only");
    if (O->empty_policy != SS_EMPTY_AUTO && O->empty_policy != SS_EMPTY_RENORMALIZE &&
        O->empty_policy != SS_EMPTY_ZERO)
        return fail(SS_E_INVALID_ARG, "batches support empty_policy AUTO, RENORMALIZE or ZERO");
    if (O->err_hist) return fail(SS_E_INVALID_ARG, "err_hist must be NULL for batches");
    return SS_OK;
}

BLayout bplan(const ss_batch* B, const ss_options* O) {
    BLayout L;
    const int K = B->count;
    L.rows = L.cols = L.cap = 0;
    L.nt_cmax = L.nt_mask = L.nt_tr = 0;
    L.nmax = L.mmax = 0;
    int64_t mask_words = 0, maskT_words = 0;
    for (int k = 0; k < K; ++k) {
        const int64_t n = B->n[k], m = B->m[k];
        const int64_t W = (m + 63) / 64, Wn = (n + 63) / 64;
        L.rows += n;
        L.cols += m;
        L.cap += entry_capacity(B->s[k], n, m);
        mask_words += n * W;
        maskT_words += m * Wn;
        L.nt_cmax += ((n + 255) / 256) * ((m + 2047) / 2048);
        L.nt_mask += ((n + 15) / 16) * ((W + 63) / 64);
        L.nt_tr += ((Wn + 7) / 8) * ((W + 15) / 16);
        if (n > L.nmax) L.nmax = (int)n;
        if (m > L.mmax) L.mmax = (int)m;
    }
    const size_t es = O->precision == SS_F64 ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    L.prob = take((size_t)K * sizeof(BProb));
    L.stat = take((size_t)K * sizeof(BStat));
    L.tile_cmax = take((size_t)(K + 1) * 8);
    L.tile_mask = take((size_t)(K + 1) * 8);
    L.tile_tr = take((size_t)(K + 1) * 8);
    L.row_off = take((size_t)(K + 1) * 8);
    L.col_off = take((size_t)(K + 1) * 8);
    L.owner = take((size_t)(L.rows + L.cols) * 4);
    L.order = take((size_t)K * 4);
    L.queue = take(64);
    L.gstats = take(ST_COUNT * 8);
    L.row_fac = take((size_t)L.rows * 8);
    L.col_fac = take((size_t)L.cols * 8);
    L.a_eff = take((size_t)L.rows * 8);
    L.b_eff = take((size_t)L.cols * 8);
    L.mask = take((size_t)mask_words * 8);
    L.maskT = take((size_t)maskT_words * 8);
    L.row_cnt = take((size_t)L.rows * 4);
    L.col_cnt = take((size_t)L.cols * 4);
    L.row_ptr = take((size_t)(L.rows + 1) * 8);
    L.col_ptr = take((size_t)(L.cols + 1) * 8);
    const int64_t big = L.rows > L.cols ? L.rows : L.cols;
    L.scan = take((size_t)((big + 1023) / 1024 + 1) * 8);
    L.col_idx = take((size_t)(L.cap + 64) * 2);
    L.row_idx = take((size_t)(L.cap + 64) * 2);
    L.val = take((size_t)(L.cap + 64) * es);
    L.val_t = take((size_t)(L.cap + 64) * es);
    L.u = take((size_t)L.rows * es);
    L.v = take((size_t)L.cols * es);
    L.obj_part = take((size_t)K * kBObjSplit * 3 * 8);
    // hand-off of stragglers to the single-problem solver: its workspace for
    // the largest sides and budget of the batch (every region grows with n,
    // m and s) and the log scalings that start it
    double smax = 0.0;
    for (int k = 0; k < K; ++k) smax = B->s[k] > smax ? B->s[k] : smax;
    ss_problem hp;
    memset(&hp, 0, sizeof hp);
    hp.n = L.nmax;
    hp.m = L.mmax;
    hp.d = B->d;
    ss_options ho = *O;
    ho.s = smax;
    L.hlog = take((size_t)(L.nmax + L.mmax) * 8);
    L.handoff_bytes = plan(&hp, &ho).total;
    L.handoff = take(L.handoff_bytes);
    L.total = off;
    return L;
}

struct BHost {
    std::vector<BProb> prob;
    std::vector<int64_t> tc, tm, tt, ro, co;
    std::vector<int32_t> order;
};

void build_batch_tables(const ss_batch* B, BHost* H) {
    const int K = B->count;
    H->prob.resize(K);
    H->tc.assign(K + 1, 0);
    H->tm.assign(K + 1, 0);
    H->tt.assign(K + 1, 0);
    H->ro.assign(K + 1, 0);
    H->co.assign(K + 1, 0);
    int64_t mo = 0, mto = 0;
    for (int k = 0; k < K; ++k) {
        BProb& P = H->prob[k];
        P.n = B->n[k];
        P.m = B->m[k];
        P.W = (P.m + 63) / 64;
        P.Wn = (P.n + 63) / 64;
        P.xo = H->ro[k];
        P.yo = H->co[k];
        P.mo = mo;
        P.mto = mto;
        P.s = B->s[k];
        P.pidx = B->problem_index ? B->problem_index[k] : (uint32_t)k;
        P.pad = 0;
        mo += P.n * P.W;
        mto += P.m * P.Wn;
        H->ro[k + 1] = H->ro[k] + P.n;
        H->co[k + 1] = H->co[k] + P.m;
        H->tc[k + 1] = H->tc[k] + ((P.n + 255) / 256) * ((P.m + 2047) / 2048);
        const int64_t rows_per_tile = 16 * batch_mask_split(P.W);
        H->tm[k + 1] = H->tm[k] + ((P.n + rows_per_tile - 1) / rows_per_tile) * ((P.W + 63) / 64);
        H->tt[k + 1] = H->tt[k] + ((P.Wn + 7) / 8) * ((P.W + 15) / 16);
    }
    // longest first: entries grow with s, iterations roughly with size
    H->order.resize(K);
    for (int k = 0; k < K; ++k) H->order[k] = k;
    std::stable_sort(H->order.begin(), H->order.end(), [&](int x, int y) {
        return B->s[x] * (double)(B->n[x] + B->m[x]) > B->s[y] * (double)(B->n[y] + B->m[y]);
    });
}

struct BCtx {
    const ss_batch* B;
    const ss_options* O;
    void* ws;
    hipStream_t st;
    BLayout L;
    BHost H;
    BatchArgs ba;
    BIterArgs ia;
    BObjArgs oa;
};

// Uploads the tables and fills the kernel arguments.
int batch_setup(BCtx& c) {
    const ss_batch* B = c.B;
    const ss_options* O = c.O;
    void* ws = c.ws;
    build_batch_tables(B, &c.H);
    const int K = B->count;
    HIP_TRY(hipMemcpyAsync(at<void>(ws, c.L.prob), c.H.prob.data(), (size_t)K * sizeof(BProb),
                           hipMemcpyHostToDevice, c.st));
    HIP_TRY(hipMemcpyAsync(at<void>(ws, c.L.tile_cmax), c.H.tc.data(), (K + 1) * 8, hipMemcpyHostToDevice, c.st));
    HIP_TRY(hipMemcpyAsync(at<void>(ws, c.L.tile_mask), c.H.tm.data(), (K + 1) * 8, hipMemcpyHostToDevice, c.st));
    HIP_TRY(hipMemcpyAsync(at<void>(ws, c.L.tile_tr), c.H.tt.data(), (K + 1) * 8, hipMemcpyHostToDevice, c.st));
    HIP_TRY(hipMemcpyAsync(at<void>(ws, c.L.row_off), c.H.ro.data(), (K + 1) * 8, hipMemcpyHostToDevice, c.st));
    HIP_TRY(hipMemcpyAsync(at<void>(ws, c.L.col_off), c.H.co.data(), (K + 1) * 8, hipMemcpyHostToDevice, c.st));
    HIP_TRY(hipMemcpyAsync(at<void>(ws, c.L.order), c.H.order.data(), (size_t)K * 4, hipMemcpyHostToDevice, c.st));

    BatchArgs& a = c.ba;
    a.count = K;
    a.d = B->d;
    a.prob = at<BProb>(ws, c.L.prob);
    a.stat = at<BStat>(ws, c.L.stat);
    a.tile_cmax = at<int64_t>(ws, c.L.tile_cmax);
    a.tile_mask = at<int64_t>(ws, c.L.tile_mask);
    a.tile_tr = at<int64_t>(ws, c.L.tile_tr);
    a.row_off = at<int64_t>(ws, c.L.row_off);
    a.col_off = at<int64_t>(ws, c.L.col_off);
    a.owner = at<int32_t>(ws, c.L.owner);
    a.rows = c.L.rows;
    a.cols = c.L.cols;
    a.x = B->x;
    a.y = B->y;
    a.a = B->a;
    a.b = B->b;
    a.row_fac = at<double>(ws, c.L.row_fac);
    a.col_fac = at<double>(ws, c.L.col_fac);
    a.a_eff = at<double>(ws, c.L.a_eff);
    a.b_eff = at<double>(ws, c.L.b_eff);
    a.mask = at<uint64_t>(ws, c.L.mask);
    a.maskT = at<uint64_t>(ws, c.L.maskT);
    a.row_cnt = at<int32_t>(ws, c.L.row_cnt);
    a.col_cnt = at<int32_t>(ws, c.L.col_cnt);
    a.row_ptr = at<int64_t>(ws, c.L.row_ptr);
    a.col_ptr = at<int64_t>(ws, c.L.col_ptr);
    a.col_idx = at<uint16_t>(ws, c.L.col_idx);
    a.row_idx = at<uint16_t>(ws, c.L.row_idx);
    a.val = at<void>(ws, c.L.val);
    a.val_t = at<void>(ws, c.L.val_t);
    a.cap = c.L.cap;
    a.cost = O->cost;
    a.empty_policy = O->empty_policy == SS_EMPTY_AUTO ? SS_EMPTY_RENORMALIZE : O->empty_policy;
    a.eps = O->eps;
    a.k0 = (uint32_t)(O->seed & 0xFFFFFFFFull);
    a.k1 = (uint32_t)(O->seed >> 32);
    a.gstats = at<double>(ws, c.L.gstats);

    BIterArgs& it = c.ia;
    it.count = K;
    it.order = at<int32_t>(ws, c.L.order);
    it.queue = at<int32_t>(ws, c.L.queue);
    it.prob = a.prob;
    it.stat = a.stat;
    it.row_ptr = a.row_ptr;
    it.col_ptr = a.col_ptr;
    it.col_idx = a.col_idx;
    it.row_idx = a.row_idx;
    it.val = a.val;
    it.val_t = a.val_t;
    it.a_eff = a.a_eff;
    it.b_eff = a.b_eff;
    it.rows = a.rows;
    it.cols = a.cols;
    it.cap = a.cap;
    it.nmax = c.L.nmax;
    it.mmax = c.L.mmax;
    it.init_log_u = O->init_log_u;
    it.init_log_v = O->init_log_v;
    it.u = at<void>(ws, c.L.u);
    it.v = at<void>(ws, c.L.v);
    it.u_out = O->u_out;
    it.v_out = O->v_out;
    it.max_iter = O->max_iter;
    it.tol = O->tol;

    BObjArgs& ob = c.oa;
    ob.d = B->d;
    ob.prob = a.prob;
    ob.stat = a.stat;
    ob.row_ptr = a.row_ptr;
    ob.col_idx = a.col_idx;
    ob.val = a.val;
    ob.u = it.u;
    ob.v = it.v;
    ob.x = B->x;
    ob.y = B->y;
    ob.rows = a.rows;
    ob.cols = a.cols;
    ob.cap = a.cap;
    ob.col_ptr = a.col_ptr;
    ob.part = at<double>(ws, c.L.obj_part);
    return SS_OK;
}

hipError_t batch_sample(const BCtx& c, hipStream_t s) {
    return launch_batch_sample(c.O->precision, c.ba, c.L.nt_cmax, c.L.nt_mask, c.L.nt_tr,
                               at<int64_t>(c.ws, c.L.scan), s);
}

hipError_t batch_iterate(const BCtx& c, const BIterArgs& ia, const ss_schedule& sc, hipStream_t s) {
    hipError_t e = launch_fill_u32((uint32_t*)ia.queue, 1, 0u, s);
    if (e != hipSuccess) return e;
    const int grid = batch_iter_grid(c.O->precision, sc.lanes_per_line, sc.block_threads,
                                     c.L.nmax, c.L.mmax);
    if (grid <= 0) return hipErrorInvalidConfiguration;
    return launch_batch_iterate(c.O->precision, sc.lanes_per_line, sc.block_threads, grid, ia, s);
}

// Captures fn into a graph (the thread's executable of `kind`), replays it
// once on st and waits for it.
hipError_t run_captured(int kind, const std::function<hipError_t(hipStream_t)>& fn,
                        hipStream_t st) {
    hipGraphExec_t exec = nullptr;
    hipError_t e = capture_exec(kind, fn, &exec);
    if (e == hipSuccess) e = hipGraphLaunch(exec, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

const int kLanesCand[4] = {4, 8, 16, 32};
const int kBlockCand[3] = {256, 512, 1024};

int batch_autotune(BCtx& c, ss_schedule* best, float* cand_ms, int32_t* ncand) {
    BIterArgs ia = c.ia;
    ia.tol = -1.0;  // never stops early: every candidate runs its 16 iterations
    ia.max_iter = 16;
    ia.u_out = ia.v_out = nullptr;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best_ms = INFINITY;
    int nc = 0;
    hipError_t e = hipSuccess;
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {  // pass 0 warms up
        nc = 0;
        for (int li = 0; li < 4 && e == hipSuccess; ++li)
            for (int bi = 0; bi < 3 && e == hipSuccess; ++bi) {
                const ss_schedule sc = {kLanesCand[li], kBlockCand[bi]};
                e = hipEventRecord(e0, c.st);
                if (e == hipSuccess) e = batch_iterate(c, ia, sc, c.st);
                if (e == hipSuccess) e = hipEventRecord(e1, c.st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (pass == 1) {
                    if (cand_ms && ncand && nc < *ncand) cand_ms[nc] = ms;
                    if (ms < best_ms) {
                        best_ms = ms;
                        *best = sc;
                    }
                }
                ++nc;
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(SS_E_HIP, "autotuning failed: %s", hipGetErrorString(e));
    if (ncand) *ncand = nc;
    return SS_OK;
}

// The schedule spar_sink_batched uses when the caller passes none: the one
// ss_autotune_batched picks on MI355X for batches of a few hundred problems
// with sides up to 4096 (8 lanes per line, 1024 threads).  The library keeps
// no tuning state; a caller who wants tuning runs ss_autotune_batched once
// and passes its result.
constexpr ss_schedule kDefaultSchedule = {8, 1024};

int batch_start(BCtx& c, const ss_batch* B, const ss_options* O, void* ws, size_t ws_bytes,
                void* stream) {
    int rc = check_batch(B, O);
    if (rc != SS_OK) return rc;
    c.B = B;
    c.O = O;
    c.ws = ws;
    c.st = (hipStream_t)stream;
    c.L = bplan(B, O);
    if (!ws) return fail(SS_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(SS_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < c.L.total)
        return fail(SS_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, c.L.total);
    HIP_TRY(batch_init());
    return batch_setup(c);
}


// ------------------------------------------------------------------ warm start
struct WLayout {
    size_t sides, tiles, tpts, tlw, emb_side, embp, xform, emb, gvec, psi, dpsi, h1g, dz2g, dgp, blkp, w2p, sidep, dgs, grad, loss;
    size_t total;
    int nsides, nblk, nchunk, nemb;
    int64_t ntiles, npts;
};

int check_ws_batch(const ss_batch* B) {
    if (!B) return fail(SS_E_INVALID_ARG, "batch must not be NULL");
    if (B->count < 1) return fail(SS_E_INVALID_ARG, "count must be >= 1");
    if (B->d != 3) return fail(SS_E_INVALID_ARG, "the warm-start network takes d = 3");
    if (!B->n || !B->m) return fail(SS_E_INVALID_ARG, "n, m must not be NULL");
    if (!B->x || !B->y || !B->a || !B->b)
        return fail(SS_E_INVALID_ARG, "x, y, a, b must not be NULL");
    for (int k = 0; k < B->count; ++k)
        if (B->n[k] < 1 || B->n[k] > SS_BATCH_MAX_SIDE || B->m[k] < 1 || B->m[k] > SS_BATCH_MAX_SIDE)
            return fail(SS_E_INVALID_ARG, "problem %d: n and m must be in [1, %d]", k, SS_BATCH_MAX_SIDE);
    return SS_OK;
}

constexpr int kWsTile = 16, kWsChunk = 2048, kWsH = 256;

void ws_sides(const ss_batch* B, std::vector<WSide>* out) {
    out->clear();
    int64_t ro = 0, co = 0, tile = 0, pt = 0, emb = 0;
    for (int k = 0; k < B->count; ++k) {
        for (int side = 0; side < 2; ++side) {
            WSide S;
            S.which = side;
            S.prob = k;
            S.npts = side == 0 ? B->n[k] : B->m[k];
            S.pts_off = side == 0 ? ro : co;
            S.nopp = side == 0 ? B->m[k] : B->n[k];
            S.opp_off = side == 0 ? co : ro;
            S.tile0 = tile;
            S.ntiles = (S.npts + kWsTile - 1) / kWsTile;
            S.pt0 = pt;
            S.emb0 = emb;
            S.nemb = (int32_t)((S.nopp + kWsEmbPart - 1) / kWsEmbPart);
            S.pad = 0;
            emb += S.nemb;
            tile += S.ntiles;
            pt += S.npts;
            out->push_back(S);
        }
        ro += B->n[k];
        co += B->m[k];
    }
}

WLayout wplan(const ss_batch* B) {
    WLayout L;
    std::vector<WSide> sides;
    ws_sides(B, &sides);
    L.nsides = (int)sides.size();
    L.ntiles = sides.back().tile0 + sides.back().ntiles;
    L.npts = sides.back().pt0 + sides.back().npts;
    L.nemb = (int)(sides.back().emb0 + sides.back().nemb);
    L.nblk = kMaxLoopBlocks;  // bound; the launch uses the compute-unit count
    L.nchunk = (int)((L.npts + kWsChunk - 1) / kWsChunk);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    L.sides = take(sides.size() * sizeof(WSide));
    L.tiles = take((size_t)L.ntiles * sizeof(WTile));
    L.tpts = take((size_t)L.ntiles * kWsTile * 4 * 4);
    L.tlw = take((size_t)L.ntiles * kWsTile * 8);
    L.emb_side = take((size_t)L.nemb * 4);
    L.embp = take((size_t)L.nemb * kWsH * 4);
    L.xform = take((size_t)B->count * 4 * 4);
    L.emb = take((size_t)L.nsides * kWsH * 4);
    L.gvec = take((size_t)L.nsides * kWsH * 4);
    L.psi = take((size_t)L.npts * 4);
    L.dpsi = take((size_t)L.npts * 4);
    L.h1g = take((size_t)L.npts * kWsH * 2);
    L.dz2g = take((size_t)L.npts * kWsH * 2);
    L.dgp = take((size_t)L.ntiles * kWsH * 4);
    L.blkp = take((size_t)L.nblk * (768 + 256 + 256 + 1) * 4);
    L.w2p = take((size_t)L.nchunk * kWsH * kWsH * 4);
    L.sidep = take((size_t)L.nsides * 1280 * 4);
    L.dgs = take((size_t)L.nsides * kWsH * 4);
    L.grad = take((size_t)SS_MLP_PARAMS * 4);
    L.loss = take((size_t)L.nsides * 8);
    L.total = off;
    return L;
}

int ws_args(const ss_mlp* M, const ss_batch* B, double eps, int cost, void* ws, size_t ws_bytes,
            hipStream_t st, WLayout* L, std::vector<WSide>* sides, MlpArgs* a) {
    int rc = check_ws_batch(B);
    if (rc != SS_OK) return rc;
    if (!(eps > 0.0) || !isfinite(eps)) return fail(SS_E_INVALID_ARG, "eps must be > 0");
    if (cost != SS_COST_SQEUCLID_MAXNORM && cost != SS_COST_SQEUCLID)
        return fail(SS_E_INVALID_ARG, "unknown cost %d", cost);
    if (!M || !M->params || !M->bf16 || !M->w2t) return fail(SS_E_INVALID_ARG, "mlp buffers must not be NULL");
    *L = wplan(B);
    if (!ws) return fail(SS_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(SS_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < L->total)
        return fail(SS_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, L->total);
    HIP_TRY(mlp_init());
    ws_sides(B, sides);
    HIP_TRY(hipMemcpyAsync(at<void>(ws, L->sides), sides->data(), sides->size() * sizeof(WSide),
                           hipMemcpyHostToDevice, st));
    const int grid = mlp_head_grid();
    if (grid <= 0) return fail(SS_E_HIP, "no device");
    a->sides = at<WSide>(ws, L->sides);
    a->tiles = at<WTile>(ws, L->tiles);
    a->tpts = at<float>(ws, L->tpts);
    a->tlw = at<double>(ws, L->tlw);
    a->nemb = L->nemb;
    a->emb_side = at<int32_t>(ws, L->emb_side);
    a->embp = at<float>(ws, L->embp);
    a->nsides = L->nsides;
    a->ntiles = L->ntiles;
    a->npts = L->npts;
    a->nblk = grid < L->nblk ? grid : L->nblk;
    a->nchunk = L->nchunk;
    a->x = B->x;
    a->y = B->y;
    a->a = B->a;
    a->b = B->b;
    a->tgt_u = a->tgt_v = nullptr;
    a->out_u = a->out_v = nullptr;
    a->xform = at<float>(ws, L->xform);
    a->eps = eps;
    a->cost = cost;
    a->wbf = M->bf16;
    a->w2t = M->w2t;
    a->emb = at<float>(ws, L->emb);
    a->gvec = at<float>(ws, L->gvec);
    a->psi = at<float>(ws, L->psi);
    a->dpsi = at<float>(ws, L->dpsi);
    a->h1g = at<void>(ws, L->h1g);
    a->dz2g = at<void>(ws, L->dz2g);
    a->dgp = at<float>(ws, L->dgp);
    a->blkp = at<float>(ws, L->blkp);
    a->w2p = at<float>(ws, L->w2p);
    a->sidep = at<float>(ws, L->sidep);
    a->dgs = at<float>(ws, L->dgs);
    a->grad = at<float>(ws, L->grad);
    a->loss = at<double>(ws, L->loss);
    return SS_OK;
}

}  // namespace

extern "C" {

int ss_mlp_sync(ss_mlp* M, void* stream) {
    if (!M || !M->params || !M->bf16 || !M->w2t) return fail(SS_E_INVALID_ARG, "mlp buffers must not be NULL");
    HIP_TRY(launch_mlp_sync(M->params, (__bf16*)M->bf16, (__bf16*)M->w2t, (hipStream_t)stream));
    return SS_OK;
}

int ss_warmstart_workspace_size(const ss_batch* batch, size_t* bytes) {
    int rc = check_ws_batch(batch);
    if (rc != SS_OK) return rc;
    if (!bytes) return fail(SS_E_INVALID_ARG, "bytes must not be NULL");
    *bytes = wplan(batch).total;
    return SS_OK;
}

int ss_warmstart_predict(const ss_mlp* M, const ss_batch* B, double eps, int32_t cost,
                         double* log_u0, double* log_v0, void* ws, size_t ws_bytes, void* stream) {
    const hipStream_t st = (hipStream_t)stream;
    WLayout L;
    std::vector<WSide> sides;
    MlpArgs a;
    int rc = ws_args(M, B, eps, cost, ws, ws_bytes, st, &L, &sides, &a);
    if (rc != SS_OK) return rc;
    a.out_u = log_u0;
    a.out_v = log_v0;
    HIP_TRY(launch_mlp_predict(a, st));
    HIP_TRY(hipStreamSynchronize(st));  // the side table's host copy goes out of scope
    return SS_OK;
}

int ss_warmstart_train_step(ss_mlp* M, const ss_batch* B, double eps, int32_t cost,
                            const double* tgt_log_u, const double* tgt_log_v, float lr, void* ws,
                            size_t ws_bytes, void* stream, float* loss, float* grad_out) {
    if (!tgt_log_u || !tgt_log_v) return fail(SS_E_INVALID_ARG, "targets must not be NULL");
    if (!(lr >= 0.0f) || !isfinite(lr)) return fail(SS_E_INVALID_ARG, "lr must be >= 0");
    if (lr > 0.0f && (!M || !M->adam_m || !M->adam_v))
        return fail(SS_E_INVALID_ARG, "Adam moments must not be NULL");
    const hipStream_t st = (hipStream_t)stream;
    WLayout L;
    std::vector<WSide> sides;
    MlpArgs a;
    int rc = ws_args(M, B, eps, cost, ws, ws_bytes, st, &L, &sides, &a);
    if (rc != SS_OK) return rc;
    a.tgt_u = tgt_log_u;
    a.tgt_v = tgt_log_v;
    HIP_TRY(launch_mlp_grad(a, st));
    if (grad_out)
        HIP_TRY(hipMemcpyAsync(grad_out, a.grad, (size_t)SS_MLP_PARAMS * 4, hipMemcpyDeviceToDevice, st));
    if (lr > 0.0f) {
        M->step += 1;
        HIP_TRY(launch_mlp_adam(M->params, M->adam_m, M->adam_v, a.grad, (__bf16*)M->bf16,
                                (__bf16*)M->w2t, lr, M->step, st));
    }
    std::vector<double> ls(L.nsides);
    HIP_TRY(hipMemcpyAsync(ls.data(), a.loss, ls.size() * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (loss) {
        double tot = 0.0;
        for (double v : ls) tot += v;
        *loss = (float)(tot / (double)L.nsides);
    }
    return SS_OK;
}

}  // extern "C"

namespace {

}  // namespace

extern "C" {

int ss_batch_workspace_size(const ss_batch* batch, const ss_options* opts, size_t* bytes) {
    int rc = check_batch(batch, opts);
    if (rc != SS_OK) return rc;
    if (!bytes) return fail(SS_E_INVALID_ARG, "bytes must not be NULL");
    *bytes = bplan(batch, opts).total;
    return SS_OK;
}

int ss_autotune_batched(const ss_batch* B, const ss_options* O, void* ws, size_t ws_bytes,
                        void* stream, ss_schedule* best, float* cand_ms, int32_t* ncand) {
    if (!best) return fail(SS_E_INVALID_ARG, "best must not be NULL");
    BCtx c;
    int rc = batch_start(c, B, O, ws, ws_bytes, stream);
    if (rc != SS_OK) return rc;
    HIP_TRY(batch_sample(c, c.st));
    return batch_autotune(c, best, cand_ms, ncand);
}

}  // extern "C"

// Scratch of spar_sink_ot_noalloc: a static device array, one copy per GPU
// the library runs on, held until the process ends.  In host code its name is
// only a host-side stand-in; the array's device address on each GPU comes from
// hipGetSymbolAddress, taken once per device (with that device current, on the
// entry point's first call there) and used for every kernel argument.
static __device__ __align__(256) unsigned char scratch[SS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// *ws = the current device's copy of `scratch`.
static int noalloc_scratch(void** ws) {
    int dev = -1;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SS_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(SS_E_HIP, "device %d is beyond the %d the scratch table holds", dev, kMaxDevices);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t r = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (r != hipSuccess || !p)
            return fail(SS_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(r));
        if ((uintptr_t)p % 256 != 0) return fail(SS_E_HIP, "scratch is not 256-byte aligned");
        g_scratch_ptr[dev] = p;
    }
    *ws = g_scratch_ptr[dev];
    return SS_OK;
}

// Straggler hand-off: iterations of the batch loop before stragglers are
// counted, and the most stragglers handed to the single-problem solver (one
// problem there takes every compute unit for (iters - kHandoffIters) x ~10
// us; one block of the batch loop takes ~50 us an iteration at n = 4096, so a
// hand-off pays while only a few problems remain).
constexpr int kHandoffIters = 64;
constexpr int kHandoffMax = 2;

namespace {

// spar_sink_batched; `before_loop` (may be null) is an event the stream
// waits for between the sampling stage and the loop (the warm start's
// producer on another stream).
// Host checks of the arguments batched_run takes beside the batch.
int check_run_args(const ss_schedule* schedule, const ss_result* outs) {
    if (!outs) return fail(SS_E_INVALID_ARG, "outs must not be NULL");
    if (schedule) {
        bool ok = false;
        for (int l : kLanesCand) ok = ok || l == schedule->lanes_per_line;
        bool okb = false;
        for (int b : kBlockCand) okb = okb || b == schedule->block_threads;
        if (!ok || !okb)
            return fail(SS_E_INVALID_ARG, "schedule: lanes_per_line in {4,8,16,32}, block_threads in {256,512,1024}");
    }
    return SS_OK;
}

int batched_run(const ss_batch* B, const ss_options* O, const ss_schedule* schedule, void* ws,
                size_t ws_bytes, void* stream, ss_result* outs, hipEvent_t before_loop) {
    int rc = check_run_args(schedule, outs);
    if (rc != SS_OK) return rc;
    BCtx c;
    rc = batch_start(c, B, O, ws, ws_bytes, stream);
    if (rc != SS_OK) return rc;
    Timer tm;
    tm.mark(0, c.st);
    HIP_TRY(run_captured(GK_SAMPLE, [&](hipStream_t s) { return batch_sample(c, s); }, c.st));
    tm.mark(1, c.st);
    const ss_schedule sc = schedule ? *schedule : kDefaultSchedule;
    if (before_loop) HIP_TRY(hipStreamWaitEvent(c.st, before_loop, 0));
    tm.mark(2, c.st);
    // The loop runs at most kHandoffIters iterations first.  When at most
    // kHandoffMax problems are still short of the tolerance, each continues
    // on the single-problem solver (every compute unit on one problem) from
    // its current iterate, with the same sketch; otherwise the batch loop is
    // run again from the start to max_iter.
    const int K = B->count;
    std::vector<int> strag;
    if (O->max_iter > kHandoffIters) {
        BIterArgs ia = c.ia;
        ia.max_iter = kHandoffIters;
        HIP_TRY(run_captured(GK_BATCH_LOOP, [&](hipStream_t s) { return batch_iterate(c, ia, sc, s); },
                             c.st));
        std::vector<BStat> st0(K);
        HIP_TRY(hipMemcpyAsync(st0.data(), at<void>(ws, c.L.stat), (size_t)K * sizeof(BStat),
                               hipMemcpyDeviceToHost, c.st));
        HIP_TRY(hipStreamSynchronize(c.st));
        for (int k = 0; k < K; ++k)
            if (st0[k].status == SS_NOT_CONVERGED && st0[k].iters == kHandoffIters)
                strag.push_back(k);
        if ((int)strag.size() > kHandoffMax) {
            strag.clear();
            HIP_TRY(run_captured(GK_BATCH_LOOP,
                                 [&](hipStream_t s) { return batch_iterate(c, c.ia, sc, s); }, c.st));
        }
    } else {
        HIP_TRY(run_captured(GK_BATCH_LOOP,
                             [&](hipStream_t s) { return batch_iterate(c, c.ia, sc, s); }, c.st));
    }
    tm.mark(3, c.st);
    HIP_TRY(run_captured(
        GK_OTHER, [&](hipStream_t s) { return launch_batch_objective(O->precision, B->count, c.oa, s); },
        c.st));
    tm.mark(4, c.st);
    std::vector<BStat> stat(K);
    double gst[ST_COUNT];
    int64_t tot[2];
    HIP_TRY(hipMemcpyAsync(stat.data(), at<void>(ws, c.L.stat), (size_t)K * sizeof(BStat),
                           hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipMemcpyAsync(gst, at<void>(ws, c.L.gstats), sizeof gst, hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipMemcpyAsync(&tot[0], at<int64_t>(ws, c.L.row_ptr) + c.L.rows, 8, hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipMemcpyAsync(&tot[1], at<int64_t>(ws, c.L.col_ptr) + c.L.cols, 8, hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    if (gst[ST_BAD_INPUT] != 0.0)
        return fail(SS_E_INVALID_ARG, "a, b must be finite and >= 0 and x, y finite");
    if (tot[0] > c.L.cap || tot[1] > c.L.cap)
        return fail(SS_E_CAPACITY, "sampled entries %lld exceed the capacity %lld", (long long)tot[0],
                    (long long)c.L.cap);
    // stage times: sampling graph, schedule choice (autotuning when not cached),
    // iteration graph, objective graph
    const float t_sample = tm.ms(0, 1), t_tune = tm.ms(1, 2), t_iter = tm.ms(2, 3),
                t_obj = tm.ms(3, 4);
    int worst = SS_OK;
    for (int k = 0; k < K; ++k) {
        const BStat& S = stat[k];
        ss_result& R = outs[k];
        memset(&R, 0, sizeof R);
        R.transport = S.transport;
        R.neg_entropy = S.negent;
        R.estimate = S.transport + O->eps * S.negent;
        R.sparse_objective = O->eps * S.sparseobj;
        R.marginal_err = S.err;
        R.cmax = S.cmax;
        R.dropped_mass_a = S.dropped_a;
        R.dropped_mass_b = S.dropped_b;
        R.nnz = S.nnz;
        R.empty_rows = (int64_t)S.empty_rows;
        R.empty_cols = (int64_t)S.empty_cols;
        R.iters = S.iters;
        R.status = S.status;
        R.warm_start = S.warm;
        R.t_prep_ms = t_tune;
        R.t_sample_ms = t_sample;
        R.t_iter_ms = t_iter;
        R.t_obj_ms = t_obj;
        if (S.status < 0 && (worst >= 0)) worst = S.status;
        if (S.status == SS_NOT_CONVERGED && worst == SS_OK) worst = SS_NOT_CONVERGED;
    }
    // hand-offs: the single-problem solver continues each straggler from its
    // iterate (log u, log v of the batch loop) for the remaining iterations
    float t_hand = 0.f;
    if (!strag.empty()) {
        Timer th;
        th.mark(0, c.st);
        for (int k : strag) {
            const BProb& bp = c.H.prob[k];
            double* lu = at<double>(ws, c.L.hlog);
            double* lv = lu + c.L.nmax;
            const int prec = O->precision == SS_F64 ? P_F64 : P_F32;
            const size_t es = O->precision == SS_F64 ? 8 : 4;
            HIP_TRY(launch_batch_log_scaling(prec, at<char>(ws, c.L.u) + bp.xo * es, lu, bp.n, c.st));
            HIP_TRY(launch_batch_log_scaling(prec, at<char>(ws, c.L.v) + bp.yo * es, lv, bp.m, c.st));
            ss_problem hp;
            memset(&hp, 0, sizeof hp);
            hp.n = bp.n;
            hp.m = bp.m;
            hp.d = B->d;
            hp.x = B->x + bp.xo * B->d;
            hp.y = B->y + bp.yo * B->d;
            hp.a = B->a + bp.xo;
            hp.b = B->b + bp.yo;
            hp.problem_index = bp.pidx;
            ss_options ho = *O;
            ho.s = B->s[k];
            ho.max_iter = O->max_iter - kHandoffIters;
            ho.init_log_u = lu;
            ho.init_log_v = lv;
            ho.u_out = O->u_out ? O->u_out + bp.xo : nullptr;
            ho.v_out = O->v_out ? O->v_out + bp.yo : nullptr;
            ho.err_hist = nullptr;
            ho.block_threads = 0;
            ho.graph_iters = 0;
            ss_result R;
            memset(&R, 0, sizeof R);
            const int hr = spar_sink_impl(&hp, &ho, at<void>(ws, c.L.handoff), c.L.handoff_bytes,
                                          c.st, &R, false);
            if (hr < 0) return fail(hr, "problem %d: hand-off to the single-problem solver failed", k);
            R.iters += kHandoffIters;
            R.t_prep_ms = outs[k].t_prep_ms;
            R.t_sample_ms = outs[k].t_sample_ms;
            R.t_obj_ms = outs[k].t_obj_ms;
            R.warm_start = outs[k].warm_start;  // the batch loop's judgement of the start
            outs[k] = R;
        }
        th.mark(1, c.st);
        HIP_TRY(hipStreamSynchronize(c.st));
        t_hand = th.ms(0, 1);
    }
    worst = SS_OK;
    for (int k = 0; k < K; ++k) {
        outs[k].t_iter_ms = t_iter + t_hand;
        if (outs[k].status < 0 && worst >= 0) worst = outs[k].status;
        if (outs[k].status == SS_NOT_CONVERGED && worst == SS_OK) worst = SS_NOT_CONVERGED;
    }
    if (worst < 0) return fail(worst, "a problem of the batch failed: %s", "see outs[k].status");
    return worst;
}

// Per host thread and device: a second stream for work that overlaps the
// caller's stream, and two events, created on first use and kept for the
// thread's life (default priority).
struct SideStream {
    hipStream_t s;
    hipEvent_t ev[2];
};

static SideStream* side_stream() {
    thread_local SideStream ss[kGraphDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kGraphDevices) return nullptr;
    SideStream& x = ss[dev];
    if (!x.s) {
        if (hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking) != hipSuccess) {
            x.s = nullptr;
            return nullptr;
        }
        for (auto& e : x.ev)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    }
    return &x;
}

// Workspace of spar_sink_batched_learned: the batch's, the network's and the
// two start vectors, each 256-byte aligned.
struct LearnedLayout {
    size_t batch, pred, lu, lv, total;
};

int learned_plan(const ss_batch* B, const ss_options* O, LearnedLayout* L) {
    int rc = check_batch(B, O);
    if (rc != SS_OK) return rc;
    rc = check_ws_batch(B);
    if (rc != SS_OK) return rc;
    int64_t rows = 0, cols = 0;
    for (int k = 0; k < B->count; ++k) {
        rows += B->n[k];
        cols += B->m[k];
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    L->batch = take(bplan(B, O).total);
    L->pred = take(wplan(B).total);
    L->lu = take((size_t)rows * 8);
    L->lv = take((size_t)cols * 8);
    L->total = off;
    return SS_OK;
}

}  // namespace

extern "C" {

int spar_sink_batched(const ss_batch* B, const ss_options* O, const ss_schedule* schedule, void* ws,
                      size_t ws_bytes, void* stream, ss_result* outs) {
    return batched_run(B, O, schedule, ws, ws_bytes, stream, outs, nullptr);
}

int ss_batch_learned_workspace_size(const ss_batch* batch, const ss_options* opts, size_t* bytes) {
    if (!bytes) return fail(SS_E_INVALID_ARG, "bytes must not be NULL");
    LearnedLayout L;
    const int rc = learned_plan(batch, opts, &L);
    if (rc != SS_OK) return rc;
    *bytes = L.total;
    return SS_OK;
}

int spar_sink_batched_learned(const ss_batch* B, const ss_options* O, const ss_schedule* schedule,
                              const ss_mlp* mlp, void* ws, size_t ws_bytes, void* stream,
                              ss_result* outs) {
    if (!O) return fail(SS_E_INVALID_ARG, "options must not be NULL");
    if (O->init_log_u || O->init_log_v)
        return fail(SS_E_INVALID_ARG, "the network gives the start: init_log_u/v must be NULL");
    LearnedLayout L;
    int rc = learned_plan(B, O, &L);
    if (rc != SS_OK) return rc;
    rc = check_run_args(schedule, outs);
    if (rc != SS_OK) return rc;
    if (!mlp || !mlp->params || !mlp->bf16 || !mlp->w2t)
        return fail(SS_E_INVALID_ARG, "mlp buffers must not be NULL");
    if (O->cost != SS_COST_SQEUCLID_MAXNORM && O->cost != SS_COST_SQEUCLID)
        return fail(SS_E_INVALID_ARG, "unknown cost %d", O->cost);
    if (!ws) return fail(SS_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(SS_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total)
        return fail(SS_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    SideStream* side = side_stream();
    if (!side) return fail(SS_E_HIP, "no side stream");
    const hipStream_t st = (hipStream_t)stream;
    // the prediction starts after the caller's earlier work on `stream` (its
    // inputs) and runs beside the sampling stage
    HIP_TRY(hipEventRecord(side->ev[0], st));
    HIP_TRY(hipStreamWaitEvent(side->s, side->ev[0], 0));
    WLayout WL;
    std::vector<WSide> sides;  // its host copy stays alive until the solve returns
    MlpArgs a;
    rc = ws_args(mlp, B, O->eps, O->cost, at<void>(ws, L.pred), L.total - L.pred, side->s, &WL,
                 &sides, &a);
    if (rc != SS_OK) return rc;
    a.out_u = at<double>(ws, L.lu);
    a.out_v = at<double>(ws, L.lv);
    HIP_TRY(launch_mlp_predict(a, side->s));
    HIP_TRY(hipEventRecord(side->ev[1], side->s));
    ss_options o = *O;
    o.init_log_u = a.out_u;
    o.init_log_v = a.out_v;
    rc = batched_run(B, &o, schedule, at<void>(ws, L.batch), L.pred - L.batch, stream, outs,
                     side->ev[1]);
    // the stream waited for the prediction before its loop and was
    // synchronised; an early error leaves the side stream to finish here
    (void)hipStreamSynchronize(side->s);
    return rc;
}

int ss_version(void) { return 100; }

const char* ss_last_error(void) { return g_last_error.c_str(); }

const char* ss_status_string(int status) {
    switch (status) {
        case SS_OK: return "ok";
        case SS_NOT_CONVERGED: return "not converged: max_iter reached with err > tol";
        case SS_E_INVALID_ARG: return "invalid argument";
        case SS_E_HIP: return "HIP runtime error";
        case SS_E_WORKSPACE: return "workspace missing, misaligned or too small";
        case SS_E_NONFINITE: return "non-finite scaling";
        case SS_E_EMPTY: return "empty row or column with empty_policy FAIL";
        case SS_E_CAPACITY: return "sampled entries exceed the workspace capacity";
        default: return "unknown status";
    }
}

int ss_workspace_size(const ss_problem* problem, const ss_options* opts, size_t* bytes) {
    int rc = check_args(problem, opts, false);
    if (rc != SS_OK) return rc;
    if (!bytes) return fail(SS_E_INVALID_ARG, "bytes must not be NULL");
    *bytes = plan(problem, opts).total;
    return SS_OK;
}

int ss_sample(const ss_problem* P, const ss_options* O, ss_sparse* out, void* ws, size_t ws_bytes,
              void* stream) {
    int rc = check_args(P, O, false);
    if (rc != SS_OK) return rc;
    if (!out) return fail(SS_E_INVALID_ARG, "out must not be NULL");
    if (!(out->z_in >= 0.0) || !isfinite(out->z_in))
        return fail(SS_E_INVALID_ARG, "out->z_in must be 0 or a positive finite normaliser");
    Ctx c;
    c.P = P;
    c.O = O;
    c.ws = ws;
    c.st = (hipStream_t)stream;
    c.uot = isfinite(O->lambda);
    c.z_in = c.uot ? out->z_in : 0.0;
    rc = check_ws(P, O, ws, ws_bytes, &c.L);
    if (rc != SS_OK) return rc;
    rc = stage_start(c);
    if (rc != SS_OK) return rc;
    rc = stage_sample(c);
    if (rc != SS_OK) return rc;
    const int64_t n = P->n, m = P->m;
    const int64_t W = (m + 63) / 64;
    const bool wants_entries = out->col_idx || out->val || out->row_idx || out->val_t;
    if (wants_entries && out->capacity < c.nnz)
        return fail(SS_E_CAPACITY, "out->capacity %lld < nnz %lld", (long long)out->capacity,
                    (long long)c.nnz);
    const size_t es = esize(O->precision);
    auto cp = [&](void* dst, size_t off, size_t bytes) -> hipError_t {
        if (!dst || bytes == 0) return hipSuccess;
        return hipMemcpyAsync(dst, at<char>(ws, off), bytes, hipMemcpyDeviceToDevice, c.st);
    };
    HIP_TRY(cp(out->mask, c.L.mask, (size_t)n * W * 8));
    HIP_TRY(cp(out->row_ptr, c.L.row_ptr, (size_t)(n + 1) * 8));
    HIP_TRY(cp(out->col_idx, c.L.col_idx, (size_t)c.nnz * 4));
    HIP_TRY(cp(out->val, c.L.val, (size_t)c.nnz * es));
    HIP_TRY(cp(out->col_ptr, c.L.col_ptr, (size_t)(m + 1) * 8));
    HIP_TRY(cp(out->row_idx, c.L.row_idx, (size_t)c.nnz * 4));
    HIP_TRY(cp(out->val_t, c.L.val_t, (size_t)c.nnz * es));
    HIP_TRY(cp(out->row_fac, c.L.row_fac, (size_t)n * 8));
    HIP_TRY(cp(out->col_fac, c.L.col_fac, (size_t)m * 8));
    HIP_TRY(hipMemcpyAsync(c.stats, at<double>(ws, c.L.stats), sizeof(c.stats),
                           hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    out->nnz = c.nnz;
    out->cmax = c.stats[ST_CMAX];
    out->z_norm = c.uot ? c.stats[ST_Z] : 0.0;
    return SS_OK;
}

int spar_sink_ot(const ss_problem* P, const ss_options* O, void* ws, size_t ws_bytes, void* stream,
                 ss_result* R) {
    return spar_sink_impl(P, O, ws, ws_bytes, stream, R, false);
}

int spar_sink_uot(const ss_problem* P, const ss_options* O, void* ws, size_t ws_bytes,
                  void* stream, ss_result* R) {
    return spar_sink_impl(P, O, ws, ws_bytes, stream, R, true);
}

int spar_sink_ot_noalloc(const ss_problem* P, const ss_options* O, void* stream, ss_result* R) {
    void* ws = nullptr;
    int rc = noalloc_scratch(&ws);
    if (rc != SS_OK) return rc;
    size_t need = 0;
    rc = ss_workspace_size(P, O, &need);
    if (rc != SS_OK) return rc;
    if (need > (size_t)SS_NOALLOC_SCRATCH_BYTES)
        return fail(SS_E_WORKSPACE,
                    "the problem needs %zu bytes of scratch; spar_sink_ot_noalloc has %zu "
                    "(use spar_sink_ot with a workspace)",
                    need, (size_t)SS_NOALLOC_SCRATCH_BYTES);
    return spar_sink_impl(P, O, ws, (size_t)SS_NOALLOC_SCRATCH_BYTES, stream, R, false, 0,
                          nullptr, nullptr, true);
}

int ss_time_iterations(const ss_problem* P, const ss_options* O, void* ws, size_t ws_bytes,
                       void* stream, int32_t iters, double* ms_per_launch) {
    if (iters < 2 || (iters & 1)) return fail(SS_E_INVALID_ARG, "iters must be even and >= 2");
    if (!O) return fail(SS_E_INVALID_ARG, "options must not be NULL");
    ss_result R;
    return spar_sink_impl(P, O, ws, ws_bytes, stream, &R, isfinite(O->lambda), iters,
                          ms_per_launch);
}

int dense_sinkhorn(const ss_problem* P, const ss_options* O, void* ws, size_t ws_bytes,
                   void* stream, ss_result* R) {
    int rc = check_args(P, O, true);
    if (rc != SS_OK) return rc;
    if (!R) return fail(SS_E_INVALID_ARG, "result must not be NULL");
    Ctx c;
    c.P = P;
    c.O = O;
    c.ws = ws;
    c.st = (hipStream_t)stream;
    c.uot = isfinite(O->lambda);
    rc = check_ws(P, O, ws, ws_bytes, &c.L);
    if (rc != SS_OK) return rc;
    memset(R, 0, sizeof *R);
    Timer tm;
    tm.mark(0, c.st);
    rc = stage_start(c);
    if (rc != SS_OK) return rc;
    tm.mark(1, c.st);
    tm.mark(2, c.st);
    const int64_t n = P->n, m = P->m;
    const int prec = O->precision;
    void* u[2] = {at<void>(ws, c.L.u[0]), at<void>(ws, c.L.u[1])};
    void* v[2] = {at<void>(ws, c.L.v[0]), at<void>(ws, c.L.v[1])};
    HIP_TRY(launch_init_scaling(prec, u[0], nullptr, O->init_log_u, n, c.st));
    HIP_TRY(launch_init_scaling(prec, v[0], nullptr, O->init_log_v, m, c.st));
    IterState* d_state = at<IterState>(ws, c.L.state);
    const double theta = c.uot ? O->lambda / (O->lambda + O->eps) : 1.0;
    DenseArgs ua[2], va[2];
    for (int k = 0; k < 2; ++k) {
        DenseArgs a;
        a.xl = P->x;
        a.xo = P->y;
        a.nl = n;
        a.no = m;
        a.d = P->d;
        a.scale = c.inv_cmax / O->eps;
        a.inv_cmax = c.inv_cmax;
        a.cost = O->cost;
        a.wfr_w = 0.5 / O->eta;
        a.eps = O->eps;
        a.marg = P->a;
        a.xin = v[k];
        a.yout = u[(k + 1) & 1];
        a.yprev = u[k];
        a.theta = theta;
        a.partials = at<double>(ws, c.L.loop_part[0]);
        a.prev_partials = at<double>(ws, c.L.loop_part[1]);
        a.prev_nblocks = dense_blocks(m);
        a.st = d_state;
        a.err_hist = O->err_hist;
        a.role = 0;
        a.stop_rule = O->stop_rule;
        a.max_iter = O->max_iter;
        a.tol = O->tol;
        a.stats = at<double>(ws, c.L.stats);
        ua[k] = a;
        a.partials = at<double>(ws, c.L.loop_part[1]);
        a.prev_partials = at<double>(ws, c.L.loop_part[0]);
        a.prev_nblocks = dense_blocks(n);
        a.xl = P->y;
        a.xo = P->x;
        a.nl = m;
        a.no = n;
        a.marg = P->b;
        a.xin = u[(k + 1) & 1];
        a.yout = v[(k + 1) & 1];
        a.yprev = v[k];
        a.role = 1;
        va[k] = a;
    }
    void* part = at<void>(ws, c.L.dense_part);
    auto iter = [&](int k, hipStream_t s) -> hipError_t {
        hipError_t e = launch_dense_half(prec, ua[k & 1], part, s);
        if (e == hipSuccess) e = launch_dense_half(prec, va[k & 1], part, s);
        return e;
    };
    const int G = O->graph_iters == 0 ? 8 : O->graph_iters;
    IterState hs;
    memset(&hs, 0, sizeof hs);
    rc = run_loop(iter, G, O->max_iter, O->tol, d_state, &hs, c.st);
    if (rc != SS_OK) return rc;
    tm.mark(3, c.st);
    if (hs.nonfinite) return fail(SS_E_NONFINITE, "a scaling became NaN or Inf");
    if (hs.stop_iter <= 0) return fail(SS_E_HIP, "loop ended without a result");
    const int p = hs.stop_iter & 1;
    DenseObjArgs oa;
    oa.x = P->x;
    oa.y = P->y;
    oa.n = n;
    oa.m = m;
    oa.d = P->d;
    oa.inv_cmax = c.inv_cmax;
    oa.cost = O->cost;
    oa.wfr_w = 0.5 / O->eta;
    oa.eps = O->eps;
    oa.u = u[p];
    oa.v = v[p];
    oa.a = P->a;
    oa.b = P->b;
    oa.uot = c.uot ? 1 : 0;
    oa.precision = prec;
    oa.partials = at<double>(ws, c.L.partials);
    oa.rowsum = at<double>(ws, c.L.rowsum);
    oa.colsum = at<double>(ws, c.L.colsum);
    oa.st = d_state;
    oa.stats = at<double>(ws, c.L.stats);
    oa.statsc = oa.stats;
    HIP_TRY(launch_dense_objective(oa, c.st));
    HIP_TRY(launch_export_scaling(prec, u[p], O->u_out, n, c.st));
    HIP_TRY(launch_export_scaling(prec, v[p], O->v_out, m, c.st));
    HIP_TRY(hipMemcpyAsync(c.stats, at<double>(ws, c.L.stats), sizeof(c.stats),
                           hipMemcpyDeviceToHost, c.st));
    tm.mark(4, c.st);
    HIP_TRY(hipStreamSynchronize(c.st));
    fill_result(c, hs, R, n * m);
    R->t_prep_ms = tm.ms(0, 1);
    R->t_sample_ms = 0.f;
    R->t_iter_ms = tm.ms(2, 3);
    R->t_obj_ms = tm.ms(3, 4);
    R->status = hs.err_final <= O->tol ? SS_OK : SS_NOT_CONVERGED;
    return R->status;
}

}  // extern "C"

// ---------------------------------------------------------------- Spar-IBP
namespace {

struct IbpLayout {
    size_t mask, maskT, row_cnt, col_cnt, scan, tmp, tree, stats, row_fac, col_fac;
    size_t row_ptr, col_ptr, col_idx, row_idx, val, val_t;
    size_t u, v[2], q[2], partials, state, empty;
    int64_t cap;   // entries per measure (and the stride between measures)
    int nb_rows;
    size_t total;
};

IbpLayout ibp_plan(const ss_ibp_problem* P, const ss_options* O) {
    IbpLayout L;
    const int64_t n = P->n, K = P->count;
    const int64_t W = (n + 63) / 64;
    L.cap = entry_capacity(O->s, n, n);
    L.nb_rows = ibp_row_blocks(n, (int)K);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    const size_t es = esize(O->precision);
    L.mask = take((size_t)n * W * 8);
    L.maskT = take((size_t)n * W * 8);
    L.row_cnt = take((size_t)n * 4);
    L.col_cnt = take((size_t)n * 4);
    L.scan = take((size_t)((n + 1023) / 1024 + 1) * 8);
    L.tmp = take(cmax_scratch_bytes(n) > (size_t)16 * n ? cmax_scratch_bytes(n) : (size_t)16 * n);
    L.tree = take((size_t)(2 * ((n + 1023) / 1024) + 2) * 8);
    L.stats = take(ST_COUNT * 8);
    L.row_fac = take((size_t)n * 8);
    L.col_fac = take((size_t)n * 8);
    L.row_ptr = take((size_t)K * (n + 1) * 8);
    L.col_ptr = take((size_t)K * (n + 1) * 8);
    L.col_idx = take((size_t)K * L.cap * 4);
    L.row_idx = take((size_t)K * L.cap * 4);
    L.val = take((size_t)K * L.cap * es);
    L.val_t = take((size_t)K * L.cap * es);
    L.u = take((size_t)K * n * 8);
    L.v[0] = take((size_t)K * n * 8);
    L.v[1] = take((size_t)K * n * 8);
    L.q[0] = take((size_t)n * 8);
    L.q[1] = take((size_t)n * 8);
    L.partials = take((size_t)L.nb_rows * 8);
    L.state = take(sizeof(IterState));
    L.empty = take(2 * sizeof(unsigned long long));
    L.total = off;
    return L;
}

int check_ibp(const ss_ibp_problem* P, const ss_options* O) {
    if (!P || !O) return fail(SS_E_INVALID_ARG, "problem and options must not be NULL");
    if (P->n <= 0 || P->n >= ((int64_t)1 << 31)) return fail(SS_E_INVALID_ARG, "n must be in [1, 2^31)");
    if (P->d <= 0 || P->d > 64) return fail(SS_E_INVALID_ARG, "d must be in [1, 64]");
    if (P->count < 1 || P->count > SS_IBP_MAX_MEASURES)
        return fail(SS_E_INVALID_ARG, "count must be in [1, %d]", SS_IBP_MAX_MEASURES);
    if (!P->x || !P->b || !P->w) return fail(SS_E_INVALID_ARG, "x, b, w must not be NULL");
    double sw = 0.0;
    for (int k = 0; k < P->count; ++k) {
        if (!(P->w[k] >= 0.0) || !isfinite(P->w[k]))
            return fail(SS_E_INVALID_ARG, "weight %d must be finite and >= 0", k);
        sw += P->w[k];
    }
    if (fabs(sw - 1.0) > 1e-12) return fail(SS_E_INVALID_ARG, "weights must sum to 1 (%.17g)", sw);
    if (!(O->eps > 0.0) || !isfinite(O->eps)) return fail(SS_E_INVALID_ARG, "eps must be > 0");
    if (!(O->s > 0.0) || !isfinite(O->s))
        return fail(SS_E_INVALID_ARG, "s must be a positive finite number");
    if (!(O->tol >= 0.0)) return fail(SS_E_INVALID_ARG, "tol must be >= 0");
    if (O->max_iter < 1) return fail(SS_E_INVALID_ARG, "max_iter must be >= 1");
    if (O->precision != SS_F64 && O->precision != SS_F32)
        return fail(SS_E_INVALID_ARG, "spar_ibp supports precision SS_F64 or SS_F32");
    if (O->cost != SS_COST_SQEUCLID_MAXNORM && O->cost != SS_COST_SQEUCLID)
        return fail(SS_E_INVALID_ARG, "unknown cost %d", O->cost);
    if (isfinite(O->lambda)) return fail(SS_E_INVALID_ARG, "spar_ibp needs lambda = +INFINITY");
    if (!(O->shrink >= 0.0 && O->shrink <= 1.0))
        return fail(SS_E_INVALID_ARG, "shrink must be in [0, 1]");
    if (O->init_log_u || O->init_log_v)
        return fail(SS_E_INVALID_ARG, "spar_ibp takes no warm start");
    return SS_OK;
}

struct IbpCtx {
    const ss_ibp_problem* P;
    const ss_options* O;
    IbpLayout L;
    void* ws;
    hipStream_t st;
    double stats[ST_COUNT];
    double inv_cmax;
    int64_t nnz;
};

int ibp_start(IbpCtx& c, const ss_ibp_problem* P, const ss_options* O, void* ws, size_t ws_bytes,
              void* stream) {
    int rc = check_ibp(P, O);
    if (rc != SS_OK) return rc;
    c.P = P;
    c.O = O;
    c.ws = ws;
    c.st = (hipStream_t)stream;
    c.L = ibp_plan(P, O);
    c.nnz = 0;
    if (!ws) return fail(SS_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(SS_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < c.L.total)
        return fail(SS_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, c.L.total);
    double* stats = at<double>(ws, c.L.stats);
    HIP_TRY(launch_fill_f64(stats, ST_COUNT, 0.0, c.st));
    HIP_TRY(launch_fill_u32(at<uint32_t>(ws, c.L.state), sizeof(IterState) / 4, 0u, c.st));
    HIP_TRY(launch_fill_u32(at<uint32_t>(ws, c.L.empty), 4, 0u, c.st));
    HIP_TRY(launch_validate(P->b, (int64_t)P->count * P->n, P->x, P->n * P->d, stats, c.st));
    HIP_TRY(launch_cmax(P->x, P->x, P->n, P->n, P->d, stats, at<void>(ws, c.L.tmp), c.st));
    HIP_TRY(hipMemcpyAsync(c.stats, stats, sizeof(c.stats), hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    if (c.stats[ST_BAD_INPUT] != 0.0)
        return fail(SS_E_INVALID_ARG, "b must be finite and >= 0 and x finite");
    const double cmax = c.stats[ST_CMAX];
    c.inv_cmax = (O->cost == SS_COST_SQEUCLID_MAXNORM && cmax > 0.0) ? 1.0 / cmax : 1.0;
    return SS_OK;
}

// eq. (pois-k): the sketch of measure k into its CSR / CSC region.
int ibp_sample_one(IbpCtx& c, int k) {
    const ss_ibp_problem* P = c.P;
    const ss_options* O = c.O;
    const int64_t n = P->n, W = (n + 63) / 64;
    void* ws = c.ws;
    hipStream_t st = c.st;
    double* stats = at<double>(ws, c.L.stats);
    ProbParams pp;
    memset(&pp, 0, sizeof pp);
    pp.uot = 0;
    pp.s = O->s;
    pp.eps = O->eps;
    pp.inv_cmax = c.inv_cmax;
    pp.shrink_w = 1.0 - O->shrink;
    pp.shrink_c = O->s * O->shrink / ((double)n * (double)n);
    pp.row_fac = at<double>(ws, c.L.row_fac);
    pp.col_fac = at<double>(ws, c.L.col_fac);
    pp.x = P->x;
    pp.y = P->x;
    pp.d = P->d;
    pp.problem_index = (uint32_t)k;
    pp.k0 = (uint32_t)(O->seed & 0xFFFFFFFFull);
    pp.k1 = (uint32_t)(O->seed >> 32);
    HIP_TRY(launch_ibp_prep(P->b + (int64_t)k * n, n, O->s, pp.shrink_w, (double*)pp.row_fac,
                            (double*)pp.col_fac, at<double>(ws, c.L.tree), stats, st));
    int32_t* row_cnt = at<int32_t>(ws, c.L.row_cnt);
    int32_t* col_cnt = at<int32_t>(ws, c.L.col_cnt);
    HIP_TRY(launch_fill_i32(row_cnt, n, 0, st));
    HIP_TRY(launch_fill_i32(col_cnt, n, 0, st));
    uint64_t* mask = at<uint64_t>(ws, c.L.mask);
    uint64_t* maskT = at<uint64_t>(ws, c.L.maskT);
    HIP_TRY(launch_mask(pp, n, n, mask, row_cnt, stats, st));
    HIP_TRY(launch_transpose(mask, n, n, maskT, col_cnt, st));
    int64_t* row_ptr = at<int64_t>(ws, c.L.row_ptr) + (int64_t)k * (n + 1);
    int64_t* col_ptr = at<int64_t>(ws, c.L.col_ptr) + (int64_t)k * (n + 1);
    HIP_TRY(launch_scan(row_cnt, n, row_ptr, at<int64_t>(ws, c.L.scan), st));
    HIP_TRY(launch_scan(col_cnt, n, col_ptr, at<int64_t>(ws, c.L.scan), st));
    int64_t tot[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(&tot[0], row_ptr + n, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&tot[1], col_ptr + n, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (tot[0] != tot[1])
        return fail(SS_E_HIP, "measure %d: CSR and CSC sizes differ (%lld vs %lld)", k,
                    (long long)tot[0], (long long)tot[1]);
    if (tot[0] > c.L.cap)
        return fail(SS_E_CAPACITY, "measure %d: sampled %lld entries exceed the capacity %lld", k,
                    (long long)tot[0], (long long)c.L.cap);
    c.nnz += tot[0];
    const size_t es = esize(O->precision);
    const int64_t base = (int64_t)k * c.L.cap;
    HIP_TRY(launch_fill_entries(0, O->precision, pp, stats, mask, n, W, row_ptr,
                                at<int32_t>(ws, c.L.col_idx) + base,
                                at<char>(ws, c.L.val) + (size_t)base * es, c.L.cap, st));
    HIP_TRY(launch_fill_entries(1, O->precision, pp, stats, maskT, n, W, col_ptr,
                                at<int32_t>(ws, c.L.row_idx) + base,
                                at<char>(ws, c.L.val_t) + (size_t)base * es, c.L.cap, st));
    unsigned long long* empty = at<unsigned long long>(ws, c.L.empty);
    HIP_TRY(launch_ibp_empty(row_cnt, n, empty, st));
    HIP_TRY(launch_ibp_empty(col_cnt, n, empty + 1, st));
    return SS_OK;
}

IbpArgs ibp_args(const IbpCtx& c) {
    IbpArgs A;
    memset(&A, 0, sizeof A);
    void* ws = c.ws;
    A.n = c.P->n;
    A.count = c.P->count;
    A.nb_rows = c.L.nb_rows;
    A.cap = c.L.cap;
    A.row_ptr = at<int64_t>(ws, c.L.row_ptr);
    A.col_idx = at<int32_t>(ws, c.L.col_idx);
    A.val = at<void>(ws, c.L.val);
    A.col_ptr = at<int64_t>(ws, c.L.col_ptr);
    A.row_idx = at<int32_t>(ws, c.L.row_idx);
    A.val_t = at<void>(ws, c.L.val_t);
    A.b = c.P->b;
    A.u = at<double>(ws, c.L.u);
    A.v[0] = at<double>(ws, c.L.v[0]);
    A.v[1] = at<double>(ws, c.L.v[1]);
    A.q[0] = at<double>(ws, c.L.q[0]);
    A.q[1] = at<double>(ws, c.L.q[1]);
    A.partials = at<double>(ws, c.L.partials);
    A.st = at<IterState>(ws, c.L.state);
    A.err_hist = c.O->err_hist;
    A.max_iter = c.O->max_iter;
    A.tol = c.O->tol;
    for (int k = 0; k < c.P->count; ++k) A.w[k] = c.P->w[k];
    return A;
}

}  // namespace

extern "C" {

int ss_ibp_workspace_size(const ss_ibp_problem* problem, const ss_options* opts, size_t* bytes) {
    int rc = check_ibp(problem, opts);
    if (rc != SS_OK) return rc;
    if (!bytes) return fail(SS_E_INVALID_ARG, "bytes must not be NULL");
    *bytes = ibp_plan(problem, opts).total;
    return SS_OK;
}

int ss_ibp_sample(const ss_ibp_problem* P, const ss_options* O, int32_t k, ss_sparse* out,
                  void* ws, size_t ws_bytes, void* stream) {
    if (!out) return fail(SS_E_INVALID_ARG, "out must not be NULL");
    IbpCtx c;
    int rc = ibp_start(c, P, O, ws, ws_bytes, stream);
    if (rc != SS_OK) return rc;
    if (k < 0 || k >= P->count) return fail(SS_E_INVALID_ARG, "k must be in [0, count)");
    rc = ibp_sample_one(c, k);
    if (rc != SS_OK) return rc;
    const int64_t n = P->n, W = (n + 63) / 64;
    const bool wants_entries = out->col_idx || out->val || out->row_idx || out->val_t;
    if (wants_entries && out->capacity < c.nnz)
        return fail(SS_E_CAPACITY, "out->capacity %lld < nnz %lld", (long long)out->capacity,
                    (long long)c.nnz);
    const size_t es = esize(O->precision);
    const int64_t base = (int64_t)k * c.L.cap;
    auto cp = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        if (!dst || bytes == 0) return hipSuccess;
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c.st);
    };
    HIP_TRY(cp(out->mask, at<char>(ws, c.L.mask), (size_t)n * W * 8));
    HIP_TRY(cp(out->row_ptr, at<int64_t>(ws, c.L.row_ptr) + (int64_t)k * (n + 1), (size_t)(n + 1) * 8));
    HIP_TRY(cp(out->col_idx, at<int32_t>(ws, c.L.col_idx) + base, (size_t)c.nnz * 4));
    HIP_TRY(cp(out->val, at<char>(ws, c.L.val) + (size_t)base * es, (size_t)c.nnz * es));
    HIP_TRY(cp(out->col_ptr, at<int64_t>(ws, c.L.col_ptr) + (int64_t)k * (n + 1), (size_t)(n + 1) * 8));
    HIP_TRY(cp(out->row_idx, at<int32_t>(ws, c.L.row_idx) + base, (size_t)c.nnz * 4));
    HIP_TRY(cp(out->val_t, at<char>(ws, c.L.val_t) + (size_t)base * es, (size_t)c.nnz * es));
    HIP_TRY(cp(out->row_fac, at<double>(ws, c.L.row_fac), (size_t)n * 8));
    HIP_TRY(cp(out->col_fac, at<double>(ws, c.L.col_fac), (size_t)n * 8));
    HIP_TRY(hipStreamSynchronize(c.st));
    out->nnz = c.nnz;
    out->cmax = c.stats[ST_CMAX];
    out->z_norm = 0.0;
    return SS_OK;
}

int spar_ibp(const ss_ibp_problem* P, const ss_options* O, double* q_out, void* ws,
             size_t ws_bytes, void* stream, ss_ibp_result* R) {
    if (!R) return fail(SS_E_INVALID_ARG, "result must not be NULL");
    if (!q_out) return fail(SS_E_INVALID_ARG, "q_out must not be NULL");
    IbpCtx c;
    int rc = ibp_start(c, P, O, ws, ws_bytes, stream);
    if (rc != SS_OK) return rc;
    memset(R, 0, sizeof *R);
    Timer tm;
    tm.mark(0, c.st);
    for (int k = 0; k < P->count; ++k) {
        rc = ibp_sample_one(c, k);
        if (rc != SS_OK) return rc;
    }
    tm.mark(1, c.st);
    const int64_t n = P->n, K = P->count;
    HIP_TRY(ibp_lds_init());
    IbpArgs A = ibp_args(c);
    HIP_TRY(launch_ibp_init(A.u, K * n, A.q[0], n, c.st));
    const int prec = O->precision == SS_F64 ? P_F64 : P_F32;
    auto iter = [&](int, hipStream_t s) -> hipError_t { return launch_ibp_iteration(prec, A, s); };
    const int G = O->graph_iters == 0 ? 16 : O->graph_iters;
    IterState hs;
    memset(&hs, 0, sizeof hs);
    rc = run_loop(iter, G, O->max_iter, O->tol, A.st, &hs, c.st);
    if (rc != SS_OK) return rc;
    tm.mark(2, c.st);
    if (hs.nonfinite) return fail(SS_E_NONFINITE, "the barycenter became NaN or Inf");
    if (hs.stop_iter <= 0) return fail(SS_E_HIP, "loop ended without a result");
    const int p = hs.stop_iter & 1;
    HIP_TRY(hipMemcpyAsync(q_out, A.q[p], (size_t)n * 8, hipMemcpyDeviceToDevice, c.st));
    if (O->u_out)
        HIP_TRY(hipMemcpyAsync(O->u_out, A.u, (size_t)K * n * 8, hipMemcpyDeviceToDevice, c.st));
    if (O->v_out)
        HIP_TRY(hipMemcpyAsync(O->v_out, A.v[p], (size_t)K * n * 8, hipMemcpyDeviceToDevice, c.st));
    unsigned long long empty[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(empty, at<unsigned long long>(ws, c.L.empty), sizeof empty,
                           hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    R->err = hs.err_final;
    R->cmax = c.stats[ST_CMAX];
    R->nnz = c.nnz;
    R->empty_rows = (int64_t)empty[0];
    R->empty_cols = (int64_t)empty[1];
    R->iters = hs.stop_iter;
    R->t_sample_ms = tm.ms(0, 1);
    R->t_iter_ms = tm.ms(1, 2);
    R->status = hs.err_final <= O->tol ? SS_OK : SS_NOT_CONVERGED;
    return R->status;
}

int ss_ibp_time_iterations(const ss_ibp_problem* P, const ss_options* O, void* ws,
                           size_t ws_bytes, void* stream, int32_t iters, double* ms_per_iter,
                           int64_t* nnz) {
    if (iters < 1) return fail(SS_E_INVALID_ARG, "iters must be >= 1");
    if (!ms_per_iter) return fail(SS_E_INVALID_ARG, "ms_per_iter must not be NULL");
    IbpCtx c;
    int rc = ibp_start(c, P, O, ws, ws_bytes, stream);
    if (rc != SS_OK) return rc;
    for (int k = 0; k < P->count; ++k) {
        rc = ibp_sample_one(c, k);
        if (rc != SS_OK) return rc;
    }
    if (nnz) *nnz = c.nnz;
    HIP_TRY(ibp_lds_init());
    IbpArgs A = ibp_args(c);
    A.tol = -1.0;  // never stops early (an exactly zero change would end the later launches)
    A.max_iter = iters;
    A.err_hist = nullptr;
    const int prec = O->precision == SS_F64 ? P_F64 : P_F32;
    hipGraphExec_t exec = nullptr;
    hipError_t e = capture_exec(GK_TIMING, [&](hipStream_t cs) {
        hipError_t er = hipSuccess;
        for (int k = 0; k < iters && er == hipSuccess; ++k) er = launch_ibp_iteration(prec, A, cs);
        return er;
    }, &exec);
    hipEvent_t a = nullptr, b = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    float ms = 0.f;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        e = launch_fill_u32((uint32_t*)A.st, sizeof(IterState) / 4, 0u, c.st);
        if (e == hipSuccess) e = launch_ibp_init(A.u, (int64_t)P->count * P->n, A.q[0], P->n, c.st);
        if (e == hipSuccess && rep == 1) e = hipEventRecord(a, c.st);
        if (e == hipSuccess) e = hipGraphLaunch(exec, c.st);
        if (e == hipSuccess && rep == 1) e = hipEventRecord(b, c.st);
        if (e == hipSuccess) e = hipStreamSynchronize(c.st);
    }
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return fail(SS_E_HIP, "timing graph failed: %s", hipGetErrorString(e));
    IterState hs;
    HIP_TRY(hipMemcpy(&hs, A.st, sizeof hs, hipMemcpyDeviceToHost));
    if (hs.nonfinite) return fail(SS_E_NONFINITE, "the barycenter became NaN or Inf");
    *ms_per_iter = (double)ms / (double)iters;
    return SS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- divergence
namespace {

int check_divergence(const ss_problem* P, const ss_options* O) {
    int rc = check_args(P, O, false);
    if (rc != SS_OK) return rc;
    if (isfinite(O->lambda)) return fail(SS_E_INVALID_ARG, "the divergence is built from OT terms");
    if (O->cost != SS_COST_SQEUCLID && O->cost != SS_COST_EUCLID)
        return fail(SS_E_INVALID_ARG,
                    "the divergence needs an unnormalised cost (SS_COST_EUCLID or SS_COST_SQEUCLID)");
    // the self terms are n x n and m x m problems with the same options
    const ss_problem pxx = {P->n, P->n, P->d, P->problem_index, P->x, P->x, P->a, P->a};
    const ss_problem pyy = {P->m, P->m, P->d, P->problem_index, P->y, P->y, P->b, P->b};
    rc = check_args(&pxx, O, false);
    if (rc != SS_OK) return rc;
    return check_args(&pyy, O, false);
}

}  // namespace

extern "C" {

int ss_divergence_workspace_size(const ss_problem* P, const ss_options* O, size_t* bytes) {
    int rc = check_divergence(P, O);
    if (rc != SS_OK) return rc;
    if (!bytes) return fail(SS_E_INVALID_ARG, "bytes must not be NULL");
    const ss_problem pxx = {P->n, P->n, P->d, P->problem_index, P->x, P->x, P->a, P->a};
    const ss_problem pyy = {P->m, P->m, P->d, P->problem_index, P->y, P->y, P->b, P->b};
    size_t b0 = plan(P, O).total, b1 = plan(&pxx, O).total, b2 = plan(&pyy, O).total;
    *bytes = b0 > b1 ? (b0 > b2 ? b0 : b2) : (b1 > b2 ? b1 : b2);
    return SS_OK;
}

int ss_sinkhorn_divergence(const ss_problem* P, const ss_options* O, double* grad_x,
                           double* grad_y, void* ws, size_t ws_bytes, void* stream,
                           ss_divergence* R) {
    int rc = check_divergence(P, O);
    if (rc != SS_OK) return rc;
    if (!R) return fail(SS_E_INVALID_ARG, "result must not be NULL");
    if ((grad_x == nullptr) != (grad_y == nullptr))
        return fail(SS_E_INVALID_ARG, "grad_x and grad_y are both given or both NULL");
    memset(R, 0, sizeof *R);
    hipStream_t st = (hipStream_t)stream;
    // per-term outputs and warm starts do not apply to the three solves
    ss_options o = *O;
    o.init_log_u = o.init_log_v = nullptr;
    o.u_out = o.v_out = o.err_hist = nullptr;
    const uint32_t pi = P->problem_index;
    const ss_problem pxy = {P->n, P->m, P->d, pi, P->x, P->y, P->a, P->b};
    const ss_problem pxx = {P->n, P->n, P->d, pi + 1u, P->x, P->x, P->a, P->a};
    const ss_problem pyy = {P->m, P->m, P->d, pi + 2u, P->y, P->y, P->b, P->b};
    if (grad_x) {
        HIP_TRY(launch_fill_f64(grad_x, P->n * P->d, 0.0, st));
        HIP_TRY(launch_fill_f64(grad_y, P->m * P->d, 0.0, st));
    }
    const GradSink g_xy = {grad_x, grad_y, 1.0, 1.0};
    const GradSink g_xx = {grad_x, grad_x, -0.5, -0.5};
    const GradSink g_yy = {grad_y, grad_y, -0.5, -0.5};
    ss_result r[3];
    const ss_problem* probs[3] = {&pxy, &pxx, &pyy};
    const GradSink* sinks[3] = {&g_xy, &g_xx, &g_yy};
    int worst = SS_OK;
    for (int t = 0; t < 3; ++t) {
        rc = spar_sink_impl(probs[t], &o, ws, ws_bytes, stream, &r[t], false, 0, nullptr,
                            grad_x ? sinks[t] : nullptr);
        if (rc < 0) return rc;
        if (rc > worst) worst = rc;
    }
    R->value = r[0].estimate - 0.5 * (r[1].estimate + r[2].estimate);
    R->value_sparse = r[0].sparse_objective - 0.5 * (r[1].sparse_objective + r[2].sparse_objective);
    R->ot_xy = r[0].estimate;
    R->ot_xx = r[1].estimate;
    R->ot_yy = r[2].estimate;
    R->sparse_xy = r[0].sparse_objective;
    R->sparse_xx = r[1].sparse_objective;
    R->sparse_yy = r[2].sparse_objective;
    R->nnz = r[0].nnz + r[1].nnz + r[2].nnz;
    R->iters_xy = r[0].iters;
    R->iters_xx = r[1].iters;
    R->iters_yy = r[2].iters;
    R->status = worst;
    return worst;
}

}  // extern "C"
