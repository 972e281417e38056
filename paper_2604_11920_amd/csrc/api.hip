// Host runtime of the C ABI declared in lsqr_mi355x.h.
//
// Owns validation, device buffers (through the caller's allocator), the
// transpose, depth-run, scale and quantisation set-up, the iteration schedule
// on the caller's stream (hipGraph replay of blocks of iterations), the FP64
// iterative refinement of the quantised forms, and read-back of the stop
// state and residual history.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <thread>
#include <vector>

#include "ctx.h"
#include "runs_host.h"

using namespace lsqr;

namespace lsqr {

static thread_local std::string g_err;

lsqr_status fail(lsqr_ctx *c, lsqr_status s, const std::string &msg)
{
    if (c) c->err = msg;
    else g_err = msg;
    return s;
}

}  // namespace lsqr

namespace {

lsqr_status validate_host_csr(const lsqr_csr *G)
{
    const int64_t m = G->m, n = G->n;
    if (G->row_ptr[0] != 0 || G->row_ptr[m] != G->nnz)
        return fail(nullptr, LSQR_E_BAD_CSR, "row_ptr[0] must be 0 and row_ptr[m] must equal nnz");
    for (int64_t i = 0; i < m; ++i)
        if (G->row_ptr[i + 1] < G->row_ptr[i])
            return fail(nullptr, LSQR_E_BAD_CSR, "row_ptr is not non-decreasing");
    // rows are independent: split them over host threads
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (G->nnz < (1 << 20)) nt = 1;
    std::vector<int> bad(nt, 0);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            int b = 0;
            for (int64_t i = m * t / nt; i < m * (t + 1) / nt; ++i)
                for (int64_t p = G->row_ptr[i]; p < G->row_ptr[i + 1]; ++p) {
                    const int32_t cc = G->col_idx[p];
                    if (cc < 0 || cc >= n) b |= 2;
                    if (p > G->row_ptr[i] && cc <= G->col_idx[p - 1]) b |= 4;
                    if (!isfinite(G->val[p])) b |= 8;
                }
            bad[t] = b;
        });
    int all = 0;
    for (unsigned t = 0; t < nt; ++t) { th[t].join(); all |= bad[t]; }
    if (all & 2) return fail(nullptr, LSQR_E_BAD_CSR, "column index out of range");
    if (all & 4) return fail(nullptr, LSQR_E_BAD_CSR, "columns not strictly increasing within a row");
    if (all & 8) return fail(nullptr, LSQR_E_NONFINITE, "non-finite value in G");
    return LSQR_OK;
}

int pick_lanes(double avg)
{
    if (avg >= 384) return 64;
    if (avg >= 96) return 32;
    if (avg >= 24) return 16;
    if (avg >= 8) return 8;
    return 4;
}

bool valid_lanes(int l) { return l == 4 || l == 8 || l == 16 || l == 32 || l == 64; }

int cap_blocks(int64_t work, int per, int cap)
{
    int64_t b = (work + per - 1) / per;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

// FP32 values of the transposed product four depths to a word (one 16-byte
// load per lane and run), like the 16-bit codes; else depth pairs.
#ifndef LSQR_F32_FOUR_DEPTHS
#define LSQR_F32_FOUR_DEPTHS 1
#endif
constexpr bool kF32FourDepths = LSQR_F32_FOUR_DEPTHS;
// 16-bit codes of the transposed product: depths per lane and load (4: one
// 8-byte load, 8: one 16-byte load; 8 measured 2-3 % faster on the
// paper-shaped system, BF16 423 -> 412 us, for 215 M padding codes against 80 M).
#ifndef LSQR_Q_DEPTHS
#define LSQR_Q_DEPTHS 8
#endif
constexpr int kQDepths = LSQR_Q_DEPTHS;

// The node-run values of `src` (CSR order, elem_bytes each) in the layout of
// W depths to a word: every run from a position that is a multiple of W,
// zeros before its first depth's offset in the word and after its end, W
// zeros after the last run; the layout's quarter offsets and destinations
// are kept in the context.
static lsqr_status build_four_depth(lsqr_ctx *c, const NodeRuns &NR, int nz, const void *src,
                                    int elem_bytes, int W, void **out)
{
    hipStream_t st = c->st;
    const int64_t nn = c->P.n / nz;
    std::vector<uint32_t> dst4;
    std::vector<int64_t> nvq4;
    if (!pair_layout_host(NR, nn, dst4, nvq4, c->npad4, W))
        return fail(c, LSQR_E_UNSUPPORTED, "the wide depth layout needs fewer than 2^32 padded values");
    c->nvqp4 = ctx_alloc<int64_t>(c, 4 * nn + 1);
    c->ndstp4 = ctx_alloc<uint32_t>(c, c->nnruns);
    void *vals = ctx_alloc_bytes(c, (size_t)(c->npad4 + W) * elem_bytes);
    if (!c->nvqp4 || !c->ndstp4 || !vals) return fail(c, LSQR_E_OOM, "device allocation failed");
    *out = vals;
    HIP_TRY(c, hipMemcpy(c->nvqp4, nvq4.data(), (4 * nn + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->ndstp4, dst4.data(), c->nnruns * sizeof(uint32_t), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemsetAsync(vals, 0, (size_t)(c->npad4 + W) * elem_bytes, st));
    launch_gather_runs(st, c->nnruns, c->nsrc, c->ndstp4, c->ndesc, src, vals, elem_bytes);
    return LSQR_OK;
}

lsqr_status setup_engine(lsqr_ctx *c, Engine &E, int vec, const RowFmt &R, const ColFmt &C)
{
    const int64_t m = c->P.m, n = c->P.n, mb = m + 2 * n;
    const size_t vs = vt_size(vec);
    E.vec = vec;
    E.R = R;
    E.C = C;
    E.g_fwd = cap_blocks(std::max<int64_t>(m * R.lpr, 2 * n), kBlock, 2048);
    // pipelined CSR rows: as many workgroups as the device holds at once, on
    // contiguous row ranges balanced in entries
    const int gp = m > 0 ? fwd_pipe_grid(vec, R) : 0;
    const int gl = m > 0 ? fwd_lcol_grid(vec, R) : 0;
    if (gl > 0) {
        // row groups: as many workgroups as the device holds at once, on
        // contiguous group ranges balanced in entries
        E.g_fwd = gl;
        E.wrow = ctx_alloc<int32_t>(c, (int64_t)gl + 1);
        if (!E.wrow) return fail(c, LSQR_E_OOM, "device allocation failed");
        launch_group_parts(c->st, R.rp, R.gp, R.ngroups, gl, E.wrow);
        E.R.wrow = E.wrow;
        E.R.wgrid = gl;
    } else if (gp > 0) {
        E.g_fwd = gp;
        const int parts = fwd_pipe_parts(gp);
        E.wrow = ctx_alloc<int32_t>(c, (int64_t)parts + 1);
        if (!E.wrow) return fail(c, LSQR_E_OOM, "device allocation failed");
        launch_wave_rows(c->st, R.rp, m, parts, E.wrow);
        E.R.wrow = E.wrow;
        E.R.wgrid = gp;
    }
    if (C.nrp) {
        // node runs: a workgroup per node, no more workgroups
        // than the device holds at once (one round, measured 3 % faster)
        const int ga = adj_nruns_grid(vec, C);
        const int64_t cap = ga > 0 ? std::min(ga, 2048) : 2048;
        E.g_adj = (int)std::max<int64_t>(1, std::min<int64_t>(n / c->P.nz, cap));
    } else {
        E.g_adj = cap_blocks(n * C.lpc, kBlock, 2048);
    }
    E.g_upd = cap_blocks(n, kBlock, 1024);
    E.T[0] = ctx_alloc_bytes(c, mb * vs);
    E.T[1] = ctx_alloc_bytes(c, mb * vs);
    if (R.sigma) E.Ts = ctx_alloc_bytes(c, std::max<int64_t>(m, 1) * vs);
    E.q = ctx_alloc_bytes(c, n * vs);
    E.v = ctx_alloc_bytes(c, n * vs);
    E.z = ctx_alloc_bytes(c, n * vs);
    E.vzero = ctx_alloc_bytes(c, n * vs);
    E.w = ctx_alloc<double>(c, n);
    E.y = ctx_alloc<double>(c, n);
    if (c->method == 1) {
        E.hbar = ctx_alloc<double>(c, n);
        if (!E.hbar) return fail(c, LSQR_E_OOM, "device allocation failed");
    }
    E.P1 = ctx_alloc<double>(c, E.g_fwd);
    E.P2 = ctx_alloc<double>(c, E.g_adj);
    E.P3 = ctx_alloc<double>(c, E.g_upd);
    E.ctl = ctx_alloc<int>(c, C_WORDS);
    if (!E.T[0] || !E.T[1] || (R.sigma && !E.Ts) || !E.q || !E.v || !E.z || !E.vzero || !E.w ||
        !E.y || !E.P1 || !E.P2 || !E.P3 || !E.ctl)
        return fail(nullptr, LSQR_E_OOM, "device allocation failed");
    return LSQR_OK;
}

lsqr_status ensure_state(lsqr_ctx *c, Engine &E, int iters)
{
    const int64_t need = (int64_t)iters + 2;
    if (E.s_rows >= need) return LSQR_OK;
    if (E.S) ctx_release(c, E.S);
    const int64_t rows = std::max<int64_t>(need, 512);
    E.S = ctx_alloc<double>(c, (size_t)rows * kStateWords);
    if (!E.S) return fail(c, LSQR_E_OOM, "state allocation failed");
    E.s_rows = rows;
    if (E.gexec) { (void)hipGraphExecDestroy(E.gexec); E.gexec = nullptr; }
    return LSQR_OK;
}

// One LSQR iteration of parity p (0: odd k, 1: even k).
void launch_iteration(lsqr_ctx *c, Engine &E, hipStream_t st, int p, double tol, bool timing,
                      int slot)
{
    const Problem &P = c->P;
    void *Tprev = E.T[p], *Tcur = E.T[1 - p];
    if (timing) (void)hipEventRecord(c->ev[4 * slot + 0], st);
    launch_fwd(st, P, E.g_fwd, E.vec, E.R, E.z, Tprev, Tcur, E.Ts, E.P1, E.P3, E.g_upd, E.S,
               E.ctl, p, tol, MODE_ITER);
    if (timing) (void)hipEventRecord(c->ev[4 * slot + 1], st);
    if (timing) (void)hipEventRecord(c->ev[4 * slot + 2], st);
    launch_adj(st, P, E.g_adj, E.vec, E.C, c->d, Tcur, E.Ts ? E.Ts : Tcur, E.v, E.q, E.P2, E.P1,
               E.g_fwd, E.S, E.ctl, p, MODE_ITER, 0);
    if (timing) (void)hipEventRecord(c->ev[4 * slot + 3], st);
    launch_update(st, P, E.g_upd, E.vec, c->d, E.q, E.v, E.w, E.y, E.z, E.P3, E.P2, E.g_adj, E.S,
                  E.ctl, p, MODE_ITER, E.hbar);
}

lsqr_status build_graph(lsqr_ctx *c, Engine &E, int iters, double tol)
{
    if (E.gexec && E.graph_iters == iters && E.graph_tol == tol) return LSQR_OK;
    if (E.gexec) { (void)hipGraphExecDestroy(E.gexec); E.gexec = nullptr; }
    if (!c->cap_st) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIP_TRY(c, hipStreamBeginCapture(c->cap_st, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < iters; ++i) launch_iteration(c, E, c->cap_st, i & 1, tol, false, 0);
    HIP_TRY(c, hipStreamEndCapture(c->cap_st, &graph));
    hipError_t e = hipGraphInstantiate(&E.gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        E.gexec = nullptr;
        return fail(c, LSQR_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    E.graph_iters = iters;
    E.graph_tol = tol;
    return LSQR_OK;
}

// Run LSQR on engine E from x0 = 0 with right-hand side rhs ([dt; 0; 0] when
// full == 0, else a full FP64 [m+2n] vector); writes D y into out (or adds it
// when accumulate != 0).  Leaves the stop state in E.ctl and E.S; returns after
// enqueuing (polls the device only when tol > 0).
lsqr_status engine_solve(lsqr_ctx *c, Engine &E, const double *rhs, int full, int iters,
                         double tol, double *out, int accumulate, bool timing)
{
    hipStream_t st = c->st;
    const Problem &P = c->P;
    lsqr_status s = ensure_state(c, E, iters);
    if (s != LSQR_OK) return s;
    if (timing && (int)c->ev.size() < 4 * iters) {
        while ((int)c->ev.size() < 4 * iters) {
            hipEvent_t e;
            HIP_TRY(c, hipEventCreate(&e));
            c->ev.push_back(e);
        }
    }
    const bool use_graph = !timing && !(c->flags & LSQR_FLAG_NO_GRAPH);
    // start: beta_1 u_1 = rhs, alpha_1 v_1 = A_D^T u_1
    launch_init(st, P, E.g_fwd, E.vec, rhs, full, E.T[0], E.R.sigma, E.Ts, E.y, E.vzero, E.P1,
                E.ctl, iters);
    launch_adj(st, P, E.g_adj, E.vec, E.C, c->d, E.T[0], E.Ts ? E.Ts : E.T[0], E.vzero, E.q, E.P2,
               E.P1, E.g_fwd, E.S, E.ctl, 0, MODE_INIT, 0);
    launch_update(st, P, E.g_upd, E.vec, c->d, E.q, E.v, E.w, E.y, E.z, E.P3, E.P2, E.g_adj, E.S,
                  E.ctl, 0, MODE_INIT, E.hbar);
    HIP_TRY(c, hipGetLastError());
    // iterations: blocks of an even number of iterations replayed as one graph
    // (parity returns to 0 after each block); with tol > 0 the host reads the
    // device stop flag after every block of check_every iterations
    const int block = tol > 0.0 ? c->check_every : iters;
    int done = 0;
    bool stopped = false;
    auto poll = [&]() -> lsqr_status {
        HIP_TRY(c, hipMemcpyAsync(c->hctl, E.ctl, C_WORDS * sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
        stopped = c->hctl[C_STOP] != 0;
        return LSQR_OK;
    };
    if (use_graph && block >= 2) {
        const int gb = std::min(block, 64) & ~1;
        s = build_graph(c, E, gb, tol);
        if (s != LSQR_OK) return s;
        while (!stopped && iters - done >= gb) {
            HIP_TRY(c, hipGraphLaunch(E.gexec, st));
            done += gb;
            if (tol > 0.0 && done < iters && (s = poll()) != LSQR_OK) return s;
        }
    }
    while (!stopped && done < iters) {
        launch_iteration(c, E, st, done & 1, tol, timing, done);
        ++done;
        if (tol > 0.0 && done % c->check_every == 0 && done < iters && (s = poll()) != LSQR_OK)
            return s;
    }
    launch_finalize(st, P, E.g_upd, c->d, E.y, out, E.P3, E.g_upd, E.S, E.ctl, tol, accumulate);
    HIP_TRY(c, hipGetLastError());
    if (timing) {
        HIP_TRY(c, hipStreamSynchronize(st));
        const int nt = std::min(done, iters);
        for (int i = 0; i < nt; ++i) {
            float a = 0.f, b = 0.f;
            if (hipEventElapsedTime(&a, c->ev[4 * i + 0], c->ev[4 * i + 1]) == hipSuccess) {
                c->ks.fwd_ms += a; c->ks.fwd_launches++;
            }
            if (hipEventElapsedTime(&b, c->ev[4 * i + 2], c->ev[4 * i + 3]) == hipSuccess) {
                c->ks.adj_ms += b; c->ks.adj_launches++;
            }
        }
    }
    return LSQR_OK;
}

// Reads the engine's stop state and history after a solve.
lsqr_status read_state(lsqr_ctx *c, Engine &E, int iters, std::vector<double> &hs)
{
    hipStream_t st = c->st;
    HIP_TRY(c, hipMemcpyAsync(c->hctl, E.ctl, C_WORDS * sizeof(int), hipMemcpyDeviceToHost, st));
    hs.resize((size_t)(iters + 1) * kStateWords);
    HIP_TRY(c, hipMemcpyAsync(hs.data(), E.S, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (c->hctl[C_ERR]) return fail(c, LSQR_E_NONFINITE, "a solver scalar became non-finite");
    return LSQR_OK;
}

void write_history(const std::vector<double> &hs, int iters, int kdone, int istop, double *res_hist)
{
    for (int k = 0; k <= iters; ++k) {
        for (int f = 0; f < 3; ++f) res_hist[3 * k + f] = NAN;
        if (k > kdone || (istop == 0 && k > 0)) continue;
        const double *Sk = hs.data() + (size_t)k * kStateWords;
        if (istop == 0) {  // bbar = 0 or Abar^T bbar = 0
            res_hist[0] = Sk[S_BETA]; res_hist[1] = 0.0; res_hist[2] = 0.0;
            continue;
        }
        res_hist[3 * k + 0] = Sk[S_PHIBAR];
        res_hist[3 * k + 1] = Sk[S_PSI];
        res_hist[3 * k + 2] = Sk[S_ETA];
    }
}

}  // namespace

extern "C" {

const char *lsqr_status_string(lsqr_status s)
{
    switch (s) {
    case LSQR_OK: return "ok";
    case LSQR_E_INVALID_ARG: return "invalid argument";
    case LSQR_E_BAD_CSR: return "malformed CSR matrix";
    case LSQR_E_NONFINITE: return "non-finite value";
    case LSQR_E_DEVICE: return "device error";
    case LSQR_E_OOM: return "out of memory";
    case LSQR_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *lsqr_last_error(const lsqr_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_err.c_str();
}

void lsqr_destroy(lsqr_ctx *c)
{
    if (!c) return;
    DeviceGuard dg(c->device);
    if (c->st) (void)hipStreamSynchronize(c->st);
    if (c->eng.gexec) (void)hipGraphExecDestroy(c->eng.gexec);
    if (c->eng32.gexec) (void)hipGraphExecDestroy(c->eng32.gexec);
    if (c->cap_st) (void)hipStreamDestroy(c->cap_st);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    for (auto &pr : c->owned) c->al.put(pr.first, pr.second);
    if (c->hctl) (void)hipHostFree(c->hctl);
    if (c->hsum) (void)hipHostFree(c->hsum);
    delete c;
}

lsqr_status lsqr_create(const lsqr_csr *G, double damp, double smooth_weight,
                        const lsqr_opts *opts, lsqr_ctx **out)
{
    if (!out) return fail(nullptr, LSQR_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!G) return fail(nullptr, LSQR_E_INVALID_ARG, "G is NULL");
    if (G->m < 0 || G->n <= 0 || G->nnz < 0 || G->nx <= 0 || G->ny <= 0 || G->nz <= 0)
        return fail(nullptr, LSQR_E_INVALID_ARG, "sizes must be positive (m, nnz may be 0)");
    if ((int64_t)G->nx * G->ny * G->nz != G->n)
        return fail(nullptr, LSQR_E_INVALID_ARG, "n must equal nx*ny*nz");
    if (G->n >= ((int64_t)1 << 31) || G->m >= ((int64_t)1 << 31))
        return fail(nullptr, LSQR_E_UNSUPPORTED, "m and n must be below 2^31");
    if (!G->row_ptr || (G->nnz > 0 && (!G->col_idx || !G->val)))
        return fail(nullptr, LSQR_E_INVALID_ARG, "CSR arrays are NULL");
    if (!(damp >= 0.0) || !isfinite(damp) || !(smooth_weight >= 0.0) || !isfinite(smooth_weight))
        return fail(nullptr, LSQR_E_INVALID_ARG, "damp and smooth_weight must be finite and >= 0");
    lsqr_opts o{};
    if (opts) o = *opts;
    if (o.precision < LSQR_FP64 || o.precision > LSQR_FP16)
        return fail(nullptr, LSQR_E_INVALID_ARG, "unknown precision");
    const bool mixed = o.precision == LSQR_BF16 || o.precision == LSQR_FP16;
    if (mixed && !(damp > 0.0))
        return fail(nullptr, LSQR_E_UNSUPPORTED,
                    "the BF16/FP16 forms need damp > 0 (the refinement corrects through the damping block)");
    if (o.precond < LSQR_PRECOND_NONE || o.precond > LSQR_PRECOND_USER)
        return fail(nullptr, LSQR_E_INVALID_ARG, "unknown precond");
    if (o.precond == LSQR_PRECOND_USER && !o.col_scale)
        return fail(nullptr, LSQR_E_INVALID_ARG, "precond USER needs col_scale");
    if ((o.lanes_per_row && !valid_lanes(o.lanes_per_row)) ||
        (o.lanes_per_col && !valid_lanes(o.lanes_per_col)))
        return fail(nullptr, LSQR_E_INVALID_ARG, "lanes must be 0, 4, 8, 16, 32 or 64");
    if (o.row_format != 0 && o.row_format != 1 && o.row_format != 4)
        return fail(nullptr, LSQR_E_INVALID_ARG, "row_format must be 0, 1 or 4");
    if (o.col_format != 0 && o.col_format != 1 && o.col_format != 2 && o.col_format != 4)
        return fail(nullptr, LSQR_E_INVALID_ARG, "col_format must be 0, 1, 2 or 4");
    if (o.flags & ~(LSQR_FLAG_TIMING | LSQR_FLAG_NO_GRAPH))
        return fail(nullptr, LSQR_E_INVALID_ARG, "unknown flag");
    if (o.method < 0 || o.method > 1)
        return fail(nullptr, LSQR_E_INVALID_ARG, "method must be 0 (LSQR) or 1 (LSMR)");
    if (o.check_every < 0) return fail(nullptr, LSQR_E_INVALID_ARG, "check_every must be >= 0");
    if (o.refine_sweeps < 0) return fail(nullptr, LSQR_E_INVALID_ARG, "refine_sweeps must be >= 0");
    if (o.fallback_iters < 0) return fail(nullptr, LSQR_E_INVALID_ARG, "fallback_iters must be >= 0");
    if (!(o.refine_inner_tol >= 0.0 && o.refine_inner_tol < 1.0))
        return fail(nullptr, LSQR_E_INVALID_ARG, "refine_inner_tol must be in [0, 1)");
    if (!(o.refine_stall_ratio >= 0.0 && o.refine_stall_ratio <= 1.0))
        return fail(nullptr, LSQR_E_INVALID_ARG, "refine_stall_ratio must be in [0, 1]");
    if (G->mem == LSQR_MEM_HOST) {
        lsqr_status s = validate_host_csr(G);
        if (s != LSQR_OK) return s;
    } else if (G->mem != LSQR_MEM_DEVICE) {
        return fail(nullptr, LSQR_E_INVALID_ARG, "unknown memory kind");
    }

    lsqr_ctx *c = new lsqr_ctx();
    c->P.m = G->m; c->P.n = G->n; c->P.nnz = G->nnz;
    c->P.nx = G->nx; c->P.ny = G->ny; c->P.nz = G->nz;
    c->P.w = smooth_weight; c->P.damp = damp;
    c->al.alloc = o.alloc; c->al.dealloc = o.dealloc; c->al.user = o.alloc_user;
    c->st = (hipStream_t)o.stream;
    c->prec = o.precision; c->precond = o.precond; c->flags = o.flags;
    c->method = o.method;
    c->fallback_iters = o.fallback_iters;
    c->check_every = o.check_every > 0 ? o.check_every : 32;
    c->check_every += c->check_every & 1;
    c->refine_sweeps = o.refine_sweeps > 0 ? o.refine_sweeps : 5;
    // an inner solve need not go far below the per-sweep gain the quantisation
    // allows (~1e-2 for BF16, ~1e-3 for FP16 on the tomography systems)
    c->refine_inner_tol = o.refine_inner_tol > 0.0 ? o.refine_inner_tol : 1e-2;
    c->stall_ratio = o.refine_stall_ratio > 0.0 ? o.refine_stall_ratio : 0.5;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(nullptr, LSQR_E_DEVICE, "no HIP device available");
    }
    const int64_t m = G->m, n = G->n, nnz = G->nnz, mb = m + 2 * n;
    auto bail = [&](lsqr_status s, const std::string &msg) {
        lsqr_destroy(c);
        return fail(nullptr, s, msg);
    };
#define CR_TRY(expr)                                                                        \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess) return bail(LSQR_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

    c->rp = ctx_alloc<int64_t>(c, m + 1);
    c->ci = ctx_alloc<int32_t>(c, nnz);
    c->va = ctx_alloc<double>(c, nnz + 8);       // zeros past the end (entries in groups of 2-8)
    c->cp = ctx_alloc<int64_t>(c, n + 1);
    c->ri = ctx_alloc<int32_t>(c, nnz);
    c->cv = ctx_alloc<double>(c, nnz);
    c->d = ctx_alloc<double>(c, n);
    c->ones = ctx_alloc<double>(c, n);
    c->dtbuf = ctx_alloc<double>(c, std::max<int64_t>(m, 1));
    c->dmbuf = ctx_alloc<double>(c, n);
    c->flag = ctx_alloc<int>(c, 4);
    c->g_ref = cap_blocks(mb, kBlock, 1024);
    c->ybuf = ctx_alloc<double>(c, mb);
    c->Pr = ctx_alloc<double>(c, c->g_ref);
    c->Pa = ctx_alloc<double>(c, 2048);   // partials of operator launches (<= 2048 workgroups)
    c->Pf = ctx_alloc<double>(c, 2048);
    c->sums = ctx_alloc<double>(c, 4);
    if (!c->rp || !c->ci || !c->va || !c->cp || !c->ri || !c->cv || !c->d || !c->ones ||
        !c->dtbuf || !c->dmbuf || !c->flag || !c->ybuf || !c->Pr || !c->Pa || !c->Pf || !c->sums)
        return bail(LSQR_E_OOM, "device allocation failed");
    CR_TRY(hipHostMalloc((void **)&c->hctl, C_WORDS * sizeof(int), hipHostMallocDefault));
    CR_TRY(hipHostMalloc((void **)&c->hsum, 4 * sizeof(double), hipHostMallocDefault));

    hipStream_t st = c->st;
    const hipMemcpyKind kind = G->mem == LSQR_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    CR_TRY(hipMemcpyAsync(c->rp, G->row_ptr, (m + 1) * sizeof(int64_t), kind, st));
    if (nnz > 0) {
        CR_TRY(hipMemcpyAsync(c->ci, G->col_idx, nnz * sizeof(int32_t), kind, st));
        CR_TRY(hipMemcpyAsync(c->va, G->val, nnz * sizeof(double), kind, st));
    }
    CR_TRY(hipMemsetAsync(c->va + nnz, 0, 8 * sizeof(double), st));
    std::vector<int64_t> hrp;
    std::vector<int32_t> hci;
    const int64_t *hrow = G->row_ptr;
    const int32_t *hcol = G->col_idx;
    if (G->mem == LSQR_MEM_DEVICE) {
        int64_t ends[2] = {0, 0};
        CR_TRY(hipMemcpyAsync(&ends[0], c->rp, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        CR_TRY(hipMemcpyAsync(&ends[1], c->rp + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        CR_TRY(hipStreamSynchronize(st));
        if (ends[0] != 0 || ends[1] != nnz)
            return bail(LSQR_E_BAD_CSR, "row_ptr[0] must be 0 and row_ptr[m] must equal nnz");
        CR_TRY(hipMemsetAsync(c->flag, 0, sizeof(int), st));
        launch_check_csr(st, m, n, c->rp, c->ci, c->va, c->flag);
        int f = 0;
        CR_TRY(hipMemcpyAsync(&f, c->flag, sizeof(int), hipMemcpyDeviceToHost, st));
        CR_TRY(hipStreamSynchronize(st));
        if (f & 1) return bail(LSQR_E_BAD_CSR, "row_ptr is not non-decreasing");
        if (f & 2) return bail(LSQR_E_BAD_CSR, "column index out of range");
        if (f & 4) return bail(LSQR_E_BAD_CSR, "columns not strictly increasing within a row");
        if (f & 8) return bail(LSQR_E_NONFINITE, "non-finite value in G");
        hrp.resize((size_t)m + 1);
        hci.resize((size_t)nnz);
        CR_TRY(hipMemcpy(hrp.data(), c->rp, (m + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
        if (nnz) CR_TRY(hipMemcpy(hci.data(), c->ci, nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
        hrow = hrp.data();
        hcol = hci.data();
    }
    {
        std::string terr;
        hipError_t e = build_transpose(st, c->al, m, n, nnz, c->rp, c->ci, c->va, c->cp, c->ri,
                                       c->cv, terr);
        if (e != hipSuccess)
            return bail(e == hipErrorOutOfMemory ? LSQR_E_OOM : LSQR_E_DEVICE,
                        terr + ": " + hipGetErrorString(e));
    }
    const double avg_row = m > 0 ? (double)nnz / (double)m : 0.0;
    const double avg_col = (double)nnz / (double)n;
    // node runs of the data block for the transposed product
    // (auto: node runs whenever the format can hold the matrix; the faster
    // transposed product measured on gfx950)
    bool use_nruns = false;
    NodeRuns NR;
    const bool nruns_ok = (o.col_format == 2 || o.col_format == 0 || o.col_format == 4) && nnz > 0 &&
                          build_node_runs_host(m, n, G->nz, hrow, hcol, NR);
    if ((o.col_format == 2 || o.col_format == 4) && nnz > 0 && !nruns_ok)
        return bail(LSQR_E_UNSUPPORTED, "node runs need nz <= 64, m < 2^32 and nnz < 2^32");
    if (nruns_ok) {
        const int64_t nr = NR.nrp.back(), nn = n / G->nz;
        c->nnruns = nr;
        c->nrp = ctx_alloc<int64_t>(c, nn + 1);
        c->nvq = ctx_alloc<int64_t>(c, 4 * nn + 1);
        c->nrow = ctx_alloc<uint32_t>(c, nr);
        c->ndesc = ctx_alloc<uint16_t>(c, nr);
        c->norder = ctx_alloc<int32_t>(c, nn);
        c->nsrc = ctx_alloc<uint32_t>(c, nr);
        c->ndst = ctx_alloc<uint32_t>(c, nr);
        c->nval = ctx_alloc<double>(c, nnz);
        if (!c->nrp || !c->nvq || !c->nrow || !c->ndesc || !c->norder || !c->nsrc || !c->ndst || !c->nval)
            return bail(LSQR_E_OOM, "device allocation failed");
        CR_TRY(hipMemcpy(c->nrp, NR.nrp.data(), (nn + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
        CR_TRY(hipMemcpy(c->nvq, NR.nvq.data(), (4 * nn + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
        CR_TRY(hipMemcpy(c->nrow, NR.row.data(), nr * sizeof(uint32_t), hipMemcpyHostToDevice));
        CR_TRY(hipMemcpy(c->ndesc, NR.desc.data(), nr * sizeof(uint16_t), hipMemcpyHostToDevice));
        CR_TRY(hipMemcpy(c->norder, NR.order.data(), nn * sizeof(int32_t), hipMemcpyHostToDevice));
        CR_TRY(hipMemcpy(c->nsrc, NR.src.data(), nr * sizeof(uint32_t), hipMemcpyHostToDevice));
        CR_TRY(hipMemcpy(c->ndst, NR.dst.data(), nr * sizeof(uint32_t), hipMemcpyHostToDevice));
        launch_gather_runs(st, nr, c->nsrc, c->ndst, c->ndesc, c->va, c->nval, 8);
        // depth-pair layout (auto and col_format 4): runs padded to aligned
        // pairs of depths, the faster transposed product measured on gfx950
        std::vector<uint32_t> dstp;
        std::vector<int64_t> nvqp;
        const bool pairs_ok = (o.col_format == 4 || o.col_format == 0) &&
                              pair_layout_host(NR, nn, dstp, nvqp, c->npad);
        if (o.col_format == 4 && !pairs_ok)
            return bail(LSQR_E_UNSUPPORTED, "the depth-pair layout needs fewer than 2^32 padded values");
        if (pairs_ok) {
            c->nvqp = ctx_alloc<int64_t>(c, 4 * nn + 1);
            c->ndstp = ctx_alloc<uint32_t>(c, nr);
            c->nvalp = ctx_alloc<double>(c, c->npad + 2);
            if (!c->nvqp || !c->ndstp || !c->nvalp) return bail(LSQR_E_OOM, "device allocation failed");
            CR_TRY(hipMemcpy(c->nvqp, nvqp.data(), (4 * nn + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
            CR_TRY(hipMemcpy(c->ndstp, dstp.data(), nr * sizeof(uint32_t), hipMemcpyHostToDevice));
            CR_TRY(hipMemsetAsync(c->nvalp, 0, (c->npad + 2) * sizeof(double), st));
            launch_gather_runs(st, nr, c->nsrc, c->ndstp, c->ndesc, c->va, c->nvalp, 8);
        }
        if (G->nz <= 32) {        // row order of the runs, for the batched forward product
            std::vector<int64_t> rrp;
            std::vector<uint32_t> rrid;
            row_order_of_runs(NR, m, rrp, rrid);
            c->rrp = ctx_alloc<int64_t>(c, m + 1);
            c->rrid = ctx_alloc<uint32_t>(c, nr);
            if (!c->rrp || !c->rrid) return bail(LSQR_E_OOM, "device allocation failed");
            CR_TRY(hipMemcpy(c->rrp, rrp.data(), (m + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
            CR_TRY(hipMemcpy(c->rrid, rrid.data(), nr * sizeof(uint32_t), hipMemcpyHostToDevice));
        }
        use_nruns = true;
    }
    // row groups with local columns (index the CSR values directly).  auto:
    // for rows of the pipelined length (64 lanes) when the groups' column
    // lists hold at most half as many columns as there are stored entries
    // (the staging pass then costs well under the per-entry gathers it
    // replaces; measured faster on gfx950 for the tomography rows)
    const bool groups_auto = o.row_format == 0 && !o.lanes_per_row && pick_lanes(avg_row) == 64;
    if ((o.row_format == 4 || groups_auto) && nnz > 0) {
        // the group size: the longest row rounded up to a multiple of 1024
        int64_t longest = 0;
        for (int64_t i = 0; i < m; ++i) longest = std::max<int64_t>(longest, hrow[i + 1] - hrow[i]);
        const int64_t cap = std::max<int64_t>(1024, (longest + 1023) / 1024 * 1024);
        RowGroups RG;
        const bool built = cap <= kLcolMaxCap && build_row_groups_host(m, n, hrow, hcol, (int)cap, RG);
        if (!built && o.row_format == 4)
            return bail(LSQR_E_UNSUPPORTED, "row groups need rows of at most 7168 entries and m < 2^31");
        if (built && (o.row_format == 4 || 2 * RG.gcp.back() <= nnz)) {
            c->gcap = (int)cap;
            c->ngroups = (int)(RG.gp.size() - 1);
            c->ngcols = RG.gcp.back();
            c->gp = ctx_alloc<int32_t>(c, c->ngroups + 1);
            c->gcp = ctx_alloc<int64_t>(c, c->ngroups + 1);
            c->gcol = ctx_alloc<int32_t>(c, std::max<int64_t>(c->ngcols, 1));
            c->slot = ctx_alloc<uint16_t>(c, nnz + 8);
            if (!c->gp || !c->gcp || !c->gcol || !c->slot) return bail(LSQR_E_OOM, "device allocation failed");
            CR_TRY(hipMemcpy(c->gp, RG.gp.data(), (c->ngroups + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
            CR_TRY(hipMemcpy(c->gcp, RG.gcp.data(), (c->ngroups + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
            if (c->ngcols)
                CR_TRY(hipMemcpy(c->gcol, RG.gcol.data(), c->ngcols * sizeof(int32_t), hipMemcpyHostToDevice));
            CR_TRY(hipMemcpy(c->slot, RG.slot.data(), nnz * sizeof(uint16_t), hipMemcpyHostToDevice));
            CR_TRY(hipMemset(c->slot + nnz, 0, 8 * sizeof(uint16_t)));
        }
    }
    // FP64 formats
    c->R64.vt = VT_F64; c->R64.rp = c->rp; c->R64.ci = c->ci; c->R64.val = c->va;
    c->R64.lpr = o.lanes_per_row ? o.lanes_per_row : pick_lanes(avg_row);
    if (c->slot) {
        c->R64.gp = c->gp; c->R64.gcp = c->gcp; c->R64.gcol = c->gcol; c->R64.slot = c->slot;
        c->R64.ngroups = c->ngroups; c->R64.gcap = c->gcap; c->R64.padded = 8;
    }
    c->C64.vt = VT_F64; c->C64.cp = c->cp; c->C64.ri = c->ri; c->C64.val = c->cv;
    c->C64.lpc = o.lanes_per_col ? o.lanes_per_col : pick_lanes(avg_col);
    // column scaling
    launch_fill(st, n, 1.0, c->ones);
    if (o.precond == LSQR_PRECOND_NONE) {
        launch_fill(st, n, 1.0, c->d);
    } else {
        bool use_jacobi = o.precond == LSQR_PRECOND_JACOBI;
        if (!use_jacobi) {
            bool ok = true;
            for (int64_t j = 0; j < n && ok; ++j) ok = isfinite(o.col_scale[j]) && o.col_scale[j] > 0.0;
            if (ok) {
                CR_TRY(hipMemcpyAsync(c->d, o.col_scale, n * sizeof(double), hipMemcpyHostToDevice, st));
                c->user_scale = true;
            } else {
                use_jacobi = true;
                c->fallback_used = 1;
            }
        }
        if (use_jacobi) launch_jacobi(st, c->P, c->C64, c->d);
    }
    // the solver's formats
    RowFmt R = c->R64;
    ColFmt C = c->C64;
    if (use_nruns) {
        C.nrp = c->nrp; C.nvq = c->nvq; C.nrow = c->nrow; C.ndesc = c->ndesc;
        C.norder = c->norder; C.val = c->nval;
        if (c->nvalp) { C.nvq = c->nvqp; C.val = c->nvalp; C.pairs = 2; }
    }
    int vec = VT_F64;
    if (o.precision == LSQR_FP32) {
        c->va32 = ctx_alloc<float>(c, nnz + 8);     // with va's padding elements
        c->cv32 = ctx_alloc<float>(c, nnz);
        if (!c->va32 || !c->cv32) return bail(LSQR_E_OOM, "device allocation failed");
        launch_convert_f32(st, nnz + 8, c->va, c->va32);
        launch_convert_f32(st, nnz, c->cv, c->cv32);
        R.vt = VT_F32; R.val = c->va32;
        C.vt = VT_F32; C.val = c->cv32;
        if (use_nruns) {
            c->nval32 = ctx_alloc<float>(c, nnz);
            if (!c->nval32) return bail(LSQR_E_OOM, "device allocation failed");
            launch_convert_f32(st, nnz, c->nval, c->nval32);
            C.val = c->nval32;
            if (c->nvalp && kF32FourDepths) {   // four depths to a word (one 16-byte load)
                lsqr_status q4 = build_four_depth(c, NR, G->nz, c->va32, 4, 4, (void **)&c->nvalp4f);
                if (q4 != LSQR_OK) { const std::string m = c->err; return bail(q4, m); }
                C.val = c->nvalp4f;
                C.nvq = c->nvqp4;
                C.pairs = 4;
            } else if (c->nvalp) {
                c->nvalp32 = ctx_alloc<float>(c, c->npad + 2);
                if (!c->nvalp32) return bail(LSQR_E_OOM, "device allocation failed");
                launch_convert_f32(st, c->npad + 2, c->nvalp, c->nvalp32);
                C.val = c->nvalp32;
            }
        }
        vec = VT_F32;
    } else if (mixed) {
        const int vt = o.precision == LSQR_BF16 ? VT_BF16 : VT_F16;
        c->sigma = ctx_alloc<float>(c, std::max<int64_t>(m, 1));
        c->qrow = ctx_alloc<uint16_t>(c, nnz + 8);  // zero codes past the end
        c->qcol = ctx_alloc<uint16_t>(c, nnz);
        c->xbuf = ctx_alloc<double>(c, n);
        c->rbar = ctx_alloc<double>(c, mb);
        c->gbuf = ctx_alloc<double>(c, n);
        c->fbuf = ctx_alloc<double>(c, mb);
        if (!c->sigma || !c->qrow || !c->qcol || !c->xbuf || !c->rbar || !c->gbuf || !c->fbuf)
            return bail(LSQR_E_OOM, "device allocation failed");
        launch_row_scales(st, m, c->rp, c->va, vt, c->sigma);
        CR_TRY(hipMemsetAsync(c->qrow + nnz, 0, 8 * sizeof(uint16_t), st));
        launch_quantise_rows(st, m, c->rp, c->va, c->sigma, vt, c->qrow);
        launch_quantise_cols(st, nnz, c->ri, c->cv, c->sigma, vt, c->qcol);
        R.vt = vt; R.val = c->qrow; R.sigma = c->sigma;
        C.vt = vt; C.val = c->qcol;
        if (use_nruns) {      // the same codes, node-major
            c->nvalq = ctx_alloc<uint16_t>(c, nnz);
            if (!c->nvalq) return bail(LSQR_E_OOM, "device allocation failed");
            launch_gather_runs(st, c->nnruns, c->nsrc, c->ndst, c->ndesc, c->qrow, c->nvalq, 2);
            C.val = c->nvalq;
            if (c->nvalp) {   // the codes kQDepths depths to a word (one 8- or 16-byte load)
                lsqr_status q4 = build_four_depth(c, NR, G->nz, c->qrow, 2, kQDepths, (void **)&c->nvalpq);
                if (q4 != LSQR_OK) { const std::string m = c->err; return bail(q4, m); }
                C.val = c->nvalpq;
                C.nvq = c->nvqp4;
                C.pairs = kQDepths;
            }
        }
        vec = VT_F32;
    }
    lsqr_status s = setup_engine(c, c->eng, vec, R, C);
    if (s != LSQR_OK) return bail(s, g_err);
    CR_TRY(hipGetLastError());
    CR_TRY(hipStreamSynchronize(st));
    if (use_nruns) {          // the run map is only needed for the value gathers
        ctx_release(c, c->nsrc);
        ctx_release(c, c->ndst);
        c->nsrc = c->ndst = nullptr;
    }
    *out = c;
    return LSQR_OK;
#undef CR_TRY
}

// eta of dm in the original variables, recomputed with the FP64 operator:
// |Abar^T (bbar - Abar dm)| / |Abar^T bbar| (the stopping ratio of the
// solver section's normal-equation residual, checked outside the
// recurrence).  0 when Abar^T bbar = 0 and dm satisfies the normal equations.
static lsqr_status verify_eta(lsqr_ctx *c, const double *ddt, const double *ddm, double *eta)
{
    hipStream_t st = c->st;
    const Problem &P = c->P;
    const int64_t n = P.n, mb = P.m + 2 * n;
    const int gadj = std::min(2048, c->eng.g_adj);
    if (!c->wr) c->wr = ctx_alloc<double>(c, mb);
    if (!c->wg) c->wg = ctx_alloc<double>(c, n);
    if (!c->wr || !c->wg) return fail(c, LSQR_E_OOM, "device allocation failed");
    launch_fwd(st, P, c->eng.g_fwd, VT_F64, c->R64, ddm, nullptr, c->ybuf, nullptr, c->Pf, nullptr,
               0, nullptr, nullptr, 0, 0.0, MODE_OPERATOR);
    launch_residual(st, P, c->g_ref, ddt, c->ybuf, c->wr, c->Pr);
    launch_adj(st, P, gadj, VT_F64, c->C64, c->ones, c->wr, c->wr, nullptr, c->wg, c->Pa, nullptr,
               0, nullptr, nullptr, 0, MODE_OPERATOR, 0);
    launch_sum_partials(st, c->Pa, gadj, c->sums + 0);
    launch_residual(st, P, c->g_ref, ddt, nullptr, c->wr, c->Pr);
    launch_adj(st, P, gadj, VT_F64, c->C64, c->ones, c->wr, c->wr, nullptr, c->wg, c->Pa, nullptr,
               0, nullptr, nullptr, 0, MODE_OPERATOR, 0);
    launch_sum_partials(st, c->Pa, gadj, c->sums + 1);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipMemcpyAsync(c->hsum, c->sums, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    const double num = sqrt(c->hsum[0]), den = sqrt(c->hsum[1]);
    *eta = den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0);
    return LSQR_OK;
}

// Learned-scale fallback: swap the Jacobi scale in (keeping the caller's
// scale to restore afterwards), and back.
static lsqr_status fallback_to_jacobi(lsqr_ctx *c)
{
    const int64_t n = c->P.n;
    if (!c->d_user) c->d_user = ctx_alloc<double>(c, n);
    if (!c->d_user) return fail(c, LSQR_E_OOM, "device allocation failed");
    HIP_TRY(c, hipMemcpyAsync(c->d_user, c->d, n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
    launch_jacobi(c->st, c->P, c->C64, c->d);
    HIP_TRY(c, hipGetLastError());
    return LSQR_OK;
}

static lsqr_status restore_user_scale(lsqr_ctx *c)
{
    HIP_TRY(c, hipMemcpyAsync(c->d, c->d_user, c->P.n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return LSQR_OK;
}

static lsqr_status solve_mixed(lsqr_ctx *c, const double *ddt, const double *dx0, int iters,
                               double tol, double *ddm, double *res_hist, lsqr_info *info);

// The inner solves of a quantised context after its refinement stalled: FP32
// copies of the FP64 values in the forward product's stored rows (row groups
// or CSR) and in the CSC, FP32 vectors; built once, on first use (the node-run
// layouts are not rebuilt: their value map is released after create).
static lsqr_status ensure_fp32_engine(lsqr_ctx *c)
{
    if (c->have_eng32) return LSQR_OK;
    const int64_t nnz = c->P.nnz;
    if (!c->va32) c->va32 = ctx_alloc<float>(c, nnz + 8);   // with va's padding elements
    if (!c->cv32) c->cv32 = ctx_alloc<float>(c, nnz);
    if (!c->va32 || !c->cv32) return fail(c, LSQR_E_OOM, "device allocation failed");
    launch_convert_f32(c->st, nnz + 8, c->va, c->va32);
    launch_convert_f32(c->st, nnz, c->cv, c->cv32);
    RowFmt R = c->R64;
    R.vt = VT_F32;
    R.val = c->va32;
    ColFmt C = c->C64;
    C.vt = VT_F32;
    C.val = c->cv32;
    lsqr_status s = setup_engine(c, c->eng32, VT_F32, R, C);
    if (s != LSQR_OK) return fail(c, s, g_err);
    HIP_TRY(c, hipGetLastError());
    c->have_eng32 = true;
    return LSQR_OK;
}
static lsqr_status solve_warm(lsqr_ctx *c, const double *ddt, int iters, double tol, double *ddm,
                              double *res_hist, lsqr_info *info);

// Cold start of the plain (FP64 / FP32) forms on the device right-hand side.
static lsqr_status solve_plain(lsqr_ctx *c, const double *ddt, int iters, double tol, double *ddm,
                               double *res_hist, lsqr_info *info)
{
    const bool timing = (c->flags & LSQR_FLAG_TIMING) != 0;
    if (timing) c->ks = lsqr_kstats{};
    lsqr_status s = engine_solve(c, c->eng, ddt, 0, iters, tol, ddm, 0, timing);
    if (s != LSQR_OK) return s;
    std::vector<double> hs;
    s = read_state(c, c->eng, iters, hs);
    if (s != LSQR_OK) return s;
    const int kdone = c->hctl[C_ITERS], istop = c->hctl[C_ISTOP];
    if (res_hist) write_history(hs, iters, kdone, istop, res_hist);
    info->istop = istop;
    info->iters = kdone;
    info->sweeps = 0;
    info->fallback_used = c->fallback_used;
    info->inner_fp32 = 0;
    const double *Sk = hs.data() + (size_t)kdone * kStateWords;
    info->eta = istop == 0 ? 0.0 : Sk[S_ETA];
    info->phibar = istop == 0 ? hs[S_BETA] : Sk[S_PHIBAR];
    return LSQR_OK;
}

static lsqr_status solve_common(lsqr_ctx *c, const double *dt, const double *x0, lsqr_mem vec_mem,
                                int iters, double tol, double *dm, double *res_hist,
                                lsqr_info *info)
{
    if (!c) return fail(nullptr, LSQR_E_INVALID_ARG, "ctx is NULL");
    if (!dt || !dm) return fail(c, LSQR_E_INVALID_ARG, "dt and dm must not be NULL");
    if (iters < 0) return fail(c, LSQR_E_INVALID_ARG, "iters must be >= 0");
    if (!(tol >= 0.0) || !isfinite(tol)) return fail(c, LSQR_E_INVALID_ARG, "tol must be finite and >= 0");
    if (vec_mem != LSQR_MEM_HOST && vec_mem != LSQR_MEM_DEVICE)
        return fail(c, LSQR_E_INVALID_ARG, "unknown memory kind");
    const bool mixed = c->prec == LSQR_BF16 || c->prec == LSQR_FP16;
    if (mixed && !(tol > 0.0))
        return fail(c, LSQR_E_INVALID_ARG, "the BF16/FP16 forms refine to a tolerance: tol must be > 0");
    DeviceGuard dg(c->device);
    hipStream_t st = c->st;
    const int64_t m = c->P.m, n = c->P.n;

    // right-hand side in, checked for NaN/Inf
    const double *ddt = dt;
    if (vec_mem == LSQR_MEM_HOST) {
        for (int64_t i = 0; i < m; ++i)
            if (!isfinite(dt[i])) return fail(c, LSQR_E_NONFINITE, "non-finite value in dt");
        if (m > 0) HIP_TRY(c, hipMemcpyAsync(c->dtbuf, dt, m * sizeof(double), hipMemcpyHostToDevice, st));
        ddt = c->dtbuf;
    } else {
        HIP_TRY(c, hipMemsetAsync(c->flag, 0, sizeof(int), st));
        launch_check_vec(st, m, dt, 0, c->flag);
        HIP_TRY(c, hipMemcpyAsync(c->hctl, c->flag, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
        if (c->hctl[0]) return fail(c, LSQR_E_NONFINITE, "non-finite value in dt");
    }
    double *ddm = vec_mem == LSQR_MEM_HOST ? c->dmbuf : dm;
    // initial solution in: checked, then held in ddm (the mixed forms copy it)
    if (x0) {
        if (vec_mem == LSQR_MEM_HOST) {
            for (int64_t j = 0; j < n; ++j)
                if (!isfinite(x0[j])) return fail(c, LSQR_E_NONFINITE, "non-finite value in x0");
            HIP_TRY(c, hipMemcpyAsync(ddm, x0, n * sizeof(double), hipMemcpyHostToDevice, st));
        } else {
            HIP_TRY(c, hipMemsetAsync(c->flag, 0, sizeof(int), st));
            launch_check_vec(st, n, x0, 0, c->flag);
            HIP_TRY(c, hipMemcpyAsync(c->hctl, c->flag, sizeof(int), hipMemcpyDeviceToHost, st));
            HIP_TRY(c, hipStreamSynchronize(st));
            if (c->hctl[0]) return fail(c, LSQR_E_NONFINITE, "non-finite value in x0");
            if (x0 != ddm)
                HIP_TRY(c, hipMemcpyAsync(ddm, x0, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        }
    }
    lsqr_status s;
    lsqr_info loc{};
    if (!info) info = &loc;
    // the learned-scale fallback: a first attempt capped at fallback_iters
    const bool fb = !mixed && c->user_scale && c->fallback_iters > 0 && tol > 0.0 &&
                    iters > c->fallback_iters;
    if (mixed) {
        s = solve_mixed(c, ddt, x0 ? ddm : nullptr, iters, tol, ddm, res_hist, info);
        if (s != LSQR_OK) return s;
    } else if (x0 || fb) {
        const int first = fb ? c->fallback_iters : iters;
        s = x0 ? solve_warm(c, ddt, first, tol, ddm, res_hist, info)
               : solve_plain(c, ddt, first, tol, ddm, res_hist, info);
        if (s != LSQR_OK) return s;
        if (fb && info->istop == 2) {
            // not converged within the budget: Jacobi from the current dm
            const int used = info->iters;
            if ((s = fallback_to_jacobi(c)) != LSQR_OK) return s;
            s = solve_warm(c, ddt, iters - used, tol, ddm, res_hist, info);
            lsqr_status r = restore_user_scale(c);
            if (s != LSQR_OK) return s;
            if (r != LSQR_OK) return r;
            info->iters += used;
            info->fallback_used = 1;
        }
    } else {
        s = solve_plain(c, ddt, iters, tol, ddm, res_hist, info);
        if (s != LSQR_OK) return s;
    }
    info->eta_final_fp64 = NAN;
    if (tol > 0.0) {
        if (mixed) {
            // every exit of the refinement follows its FP64 eta of the final dm
            info->eta_final_fp64 = info->eta;
        } else {
            s = verify_eta(c, ddt, ddm, &info->eta_final_fp64);
            if (s != LSQR_OK) return s;
        }
    }
    if (vec_mem == LSQR_MEM_HOST) {
        HIP_TRY(c, hipMemcpyAsync(dm, c->dmbuf, n * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
    }
    return LSQR_OK;
}

lsqr_status lsqr_solve(lsqr_ctx *c, const double *dt, lsqr_mem vec_mem, int iters, double tol,
                       double *dm, double *res_hist, lsqr_info *info)
{
    return solve_common(c, dt, nullptr, vec_mem, iters, tol, dm, res_hist, info);
}

lsqr_status lsqr_solve_x0(lsqr_ctx *c, const double *dt, const double *x0, lsqr_mem vec_mem,
                          int iters, double tol, double *dm, double *res_hist, lsqr_info *info)
{
    if (c && !x0) return fail(c, LSQR_E_INVALID_ARG, "x0 must not be NULL");
    return solve_common(c, dt, x0, vec_mem, iters, tol, dm, res_hist, info);
}

// Iterative refinement of the quantised forms.  Each sweep: rbar = bbar -
// Abar x with the FP64 operator; g = G^T r_G (FP64 values); the exact eta =
// |Abar^T rbar| / |Abar^T bbar|; then an inner LSQR on the quantised
// operator with right-hand side f = [0; 0; (Abar^T rbar)/lambda], for which
// Ahat^T f = Abar^T rbar, so the refinement's fixed point is the FP64
// solution (and f, unlike rbar, vanishes there: see refine.hip); x += D y_inner.
static lsqr_status solve_mixed(lsqr_ctx *c, const double *ddt, const double *dx0, int iters,
                               double tol, double *ddm, double *res_hist, lsqr_info *info)
{
    hipStream_t st = c->st;
    const Problem &P = c->P;
    const int64_t n = P.n;
    Engine &E = c->eng;
    const double inner_tol = c->refine_inner_tol;
    const int gadj = std::min(2048, E.g_adj);
    const bool timing = (c->flags & LSQR_FLAG_TIMING) != 0;   // inner products, all sweeps
    if (timing) c->ks = lsqr_kstats{};
    auto fetch = [&]() -> lsqr_status {
        HIP_TRY(c, hipMemcpyAsync(c->hsum, c->sums, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
        return LSQR_OK;
    };
    if (dx0) HIP_TRY(c, hipMemcpyAsync(c->xbuf, dx0, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    else launch_fill(st, n, 0.0, c->xbuf);
    // |Abar^T bbar| = |G^T dt|
    launch_adj(st, P, gadj, VT_F64, c->C64, c->ones, nullptr, ddt, nullptr, c->gbuf, c->Pa,
               nullptr, 0, nullptr, nullptr, 0, MODE_OPERATOR, 1);
    launch_sum_partials(st, c->Pa, gadj, c->sums + 0);
    lsqr_status s = fetch();
    if (s != LSQR_OK) return s;
    const double arnorm = sqrt(c->hsum[0]);
    int istop = 2, total = 0, sweeps = 0, last_iters = 0, last_istop = 2;
    double eta = 0.0, rnorm = 0.0, eta_prev = INFINITY;
    // learned-scale fallback: Jacobi once the inner iterations pass the budget
    const bool fb = c->user_scale && c->fallback_iters > 0;
    bool switched = false;
    // the inner solves' kernels: the quantised ones, FP32 values after a stall
    Engine *EI = &E;
    int inner32 = 0;
    std::vector<double> hs;
    if (!(arnorm > 0.0)) {
        istop = 0;
    } else {
        for (int sw = 0;; ++sw) {
            // FP64 residual and its normal-equation residual
            const bool from_x = sw > 0 || dx0;              // x != 0
            if (from_x)
                launch_fwd(st, P, E.g_fwd, VT_F64, c->R64, c->xbuf, nullptr, c->ybuf, nullptr,
                           c->Pf, nullptr, 0, nullptr, nullptr, 0, 0.0, MODE_OPERATOR);
            launch_residual(st, P, c->g_ref, ddt, from_x ? c->ybuf : nullptr, c->rbar, c->Pr);
            launch_sum_partials(st, c->Pr, c->g_ref, c->sums + 1);
            launch_adj(st, P, gadj, VT_F64, c->C64, c->ones, nullptr, c->rbar, nullptr, c->gbuf,
                       c->Pa, nullptr, 0, nullptr, nullptr, 0, MODE_OPERATOR, 1);
            launch_normal_rhs(st, P, c->g_ref, c->rbar, c->gbuf, c->fbuf, c->Pr);
            launch_sum_partials(st, c->Pr, c->g_ref, c->sums + 2);
            HIP_TRY(c, hipGetLastError());
            if ((s = fetch()) != LSQR_OK) return s;
            rnorm = sqrt(c->hsum[1]);
            eta = sqrt(c->hsum[2]) / arnorm;
            if (!isfinite(eta)) return fail(c, LSQR_E_NONFINITE, "refinement residual became non-finite");
            if (eta <= tol) { istop = 1; break; }
            if (sw >= c->refine_sweeps) { istop = 2; break; }
            if (sw > 0 && eta > c->stall_ratio * eta_prev) {
                if (fb && !switched) {
                    // a user scale that stalls the refinement: Jacobi from here
                    if ((s = fallback_to_jacobi(c)) != LSQR_OK) return s;
                    switched = true;
                } else if (!inner32) {
                    // the quantised operator is too far from the FP64 one for
                    // the sweeps to contract: FP32 values from here
                    if ((s = ensure_fp32_engine(c)) != LSQR_OK) return s;
                    EI = &c->eng32;
                    inner32 = 1;
                } else {
                    istop = 4;
                    break;
                }
            }
            eta_prev = eta;
            // inner solve on the quantised (or FP32) operator, x += D y
            s = engine_solve(c, *EI, c->fbuf, 1, iters, inner_tol, c->xbuf, 1, timing);
            if (s != LSQR_OK) return s;
            if ((s = read_state(c, *EI, iters, hs)) != LSQR_OK) return s;
            last_iters = c->hctl[C_ITERS];
            last_istop = c->hctl[C_ISTOP];
            total += last_iters;
            ++sweeps;
            if (fb && !switched && total >= c->fallback_iters) {
                if ((s = fallback_to_jacobi(c)) != LSQR_OK) return s;
                switched = true;
                eta_prev = INFINITY;      // the stall test restarts with the new scale
            }
        }
    }
    if (switched && (s = restore_user_scale(c)) != LSQR_OK) return s;
    HIP_TRY(c, hipMemcpyAsync(ddm, c->xbuf, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (res_hist) {
        if (sweeps > 0) write_history(hs, iters, last_iters, last_istop, res_hist);
        else for (int k = 0; k <= iters; ++k) for (int f = 0; f < 3; ++f) res_hist[3 * k + f] = NAN;
    }
    if (info) {
        info->istop = istop;
        info->iters = total;
        info->sweeps = sweeps;
        info->fallback_used = c->fallback_used | (switched ? 1 : 0);
        info->inner_fp32 = inner32;
        info->eta = eta;
        info->phibar = rnorm;
    }
    return LSQR_OK;
}

// Warm start of the plain (FP64 / FP32) forms: x = x0 + D y with y the
// solver's iterate on the correction problem A_D y ~ r0 = bbar - Abar x0 (a
// full right-hand side).  The correction solve measures its stopping ratio
// against |Abar^T r0| (LSQR; LSMR: |D Abar^T r0|), so its tolerance is the
// caller's times |Abar^T bbar| / |Abar^T r0|, and its history's eta column is
// rescaled by the inverse: eta keeps its meaning for the original problem.
// x0 is in ddm already; the correction is added to it.
static lsqr_status solve_warm(lsqr_ctx *c, const double *ddt, int iters, double tol, double *ddm,
                              double *res_hist, lsqr_info *info)
{
    hipStream_t st = c->st;
    const Problem &P = c->P;
    const int64_t n = P.n, mb = P.m + 2 * n;
    Engine &E = c->eng;
    const int gadj = std::min(2048, E.g_adj);
    if (!c->wr) c->wr = ctx_alloc<double>(c, mb);
    if (!c->wg) c->wg = ctx_alloc<double>(c, n);
    if (!c->wr || !c->wg) return fail(c, LSQR_E_OOM, "device allocation failed");
    const double *dv = c->method == 1 ? c->d : c->ones;
    // r0 = bbar - Abar x0 and |Abar^T r0|; then bbar and |Abar^T bbar|
    launch_fwd(st, P, E.g_fwd, VT_F64, c->R64, ddm, nullptr, c->ybuf, nullptr, c->Pf, nullptr, 0,
               nullptr, nullptr, 0, 0.0, MODE_OPERATOR);
    launch_residual(st, P, c->g_ref, ddt, c->ybuf, c->wr, c->Pr);
    launch_adj(st, P, gadj, VT_F64, c->C64, dv, c->wr, c->wr, nullptr, c->wg, c->Pa, nullptr, 0,
               nullptr, nullptr, 0, MODE_OPERATOR, 0);
    launch_sum_partials(st, c->Pa, gadj, c->sums + 0);
    launch_residual(st, P, c->g_ref, ddt, nullptr, c->ybuf, c->Pr);
    launch_adj(st, P, gadj, VT_F64, c->C64, dv, c->ybuf, c->ybuf, nullptr, c->wg, c->Pa, nullptr, 0,
               nullptr, nullptr, 0, MODE_OPERATOR, 0);
    launch_sum_partials(st, c->Pa, gadj, c->sums + 1);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipMemcpyAsync(c->hsum, c->sums, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    const double nr = sqrt(c->hsum[0]), nb = sqrt(c->hsum[1]);
    if (!isfinite(nr)) return fail(c, LSQR_E_NONFINITE, "non-finite residual at x0");
    // with Abar^T bbar = 0, eta is measured against |Abar^T r0| instead
    const double ratio = nb > 0.0 ? nr / nb : 1.0;
    if (!(nr > 0.0)) {                     // x0 satisfies the normal equations
        if (res_hist)
            for (int k = 0; k <= iters; ++k)
                for (int f = 0; f < 3; ++f) res_hist[3 * k + f] = k == 0 ? 0.0 : NAN;
        if (info) {
            info->istop = 1;
            info->iters = 0;
            info->sweeps = 0;
            info->fallback_used = c->fallback_used;
            info->inner_fp32 = 0;
            info->eta = 0.0;
            info->phibar = 0.0;
        }
        return LSQR_OK;
    }
    const bool timing = (c->flags & LSQR_FLAG_TIMING) != 0;
    if (timing) c->ks = lsqr_kstats{};
    lsqr_status s = engine_solve(c, E, c->wr, 1, iters, tol > 0.0 ? tol / ratio : 0.0, ddm, 1, timing);
    if (s != LSQR_OK) return s;
    std::vector<double> hs;
    if ((s = read_state(c, E, iters, hs)) != LSQR_OK) return s;
    const int kdone = c->hctl[C_ITERS], istop = c->hctl[C_ISTOP];
    if (res_hist) {
        write_history(hs, iters, kdone, istop, res_hist);
        for (int k = 0; k <= iters; ++k) res_hist[3 * k + 2] *= ratio;
    }
    if (info) {
        info->istop = istop;
        info->iters = kdone;
        info->sweeps = 0;
        info->fallback_used = c->fallback_used;
        info->inner_fp32 = 0;
        const double *Sk = hs.data() + (size_t)kdone * kStateWords;
        info->eta = istop == 0 ? 0.0 : Sk[S_ETA] * ratio;
        info->phibar = istop == 0 ? hs[S_BETA] : Sk[S_PHIBAR];
    }
    return LSQR_OK;
}

lsqr_status lsqr_apply(lsqr_ctx *c, const double *x, double *y)
{
    if (!c) return fail(nullptr, LSQR_E_INVALID_ARG, "ctx is NULL");
    if (!x || !y) return fail(c, LSQR_E_INVALID_ARG, "x and y must not be NULL");
    DeviceGuard dg(c->device);
    launch_scale_vec(c->st, c->P.n, c->d, x, c->dmbuf);
    launch_fwd(c->st, c->P, c->eng.g_fwd, VT_F64, c->R64, c->dmbuf, nullptr, y, nullptr,
               c->Pf, nullptr, 0, nullptr, nullptr, 0, 0.0, MODE_OPERATOR);
    HIP_TRY(c, hipGetLastError());
    return LSQR_OK;
}

lsqr_status lsqr_apply_t(lsqr_ctx *c, const double *y, double *x)
{
    if (!c) return fail(nullptr, LSQR_E_INVALID_ARG, "ctx is NULL");
    if (!x || !y) return fail(c, LSQR_E_INVALID_ARG, "x and y must not be NULL");
    DeviceGuard dg(c->device);
    // the FP64 transposed format the solver reads (node runs when built)
    ColFmt C = c->C64;
    if (c->nrp) {
        C.nrp = c->nrp; C.nvq = c->nvq; C.nrow = c->nrow; C.ndesc = c->ndesc;
        C.norder = c->norder; C.val = c->nval;
        if (c->nvalp) { C.nvq = c->nvqp; C.val = c->nvalp; C.pairs = 2; }
    }
    launch_adj(c->st, c->P, std::min(2048, c->eng.g_adj), VT_F64, C, c->d, y, y, nullptr, x,
               c->Pa, nullptr, 0, nullptr, nullptr, 0, MODE_OPERATOR, 0);
    HIP_TRY(c, hipGetLastError());
    return LSQR_OK;
}

lsqr_status lsqr_apply_stored(lsqr_ctx *c, const void *z, void *y)
{
    if (!c) return fail(nullptr, LSQR_E_INVALID_ARG, "ctx is NULL");
    if (!z || !y) return fail(c, LSQR_E_INVALID_ARG, "z and y must not be NULL");
    DeviceGuard dg(c->device);
    Engine &E = c->eng;
    launch_fwd(c->st, c->P, E.g_fwd, E.vec, E.R, z, nullptr, y, nullptr, E.P1, nullptr, 0,
               nullptr, nullptr, 0, 0.0, MODE_OPERATOR);
    HIP_TRY(c, hipGetLastError());
    return LSQR_OK;
}

lsqr_status lsqr_apply_t_stored(lsqr_ctx *c, const void *y, const void *tg, void *q)
{
    if (!c) return fail(nullptr, LSQR_E_INVALID_ARG, "ctx is NULL");
    if (!y || !q) return fail(c, LSQR_E_INVALID_ARG, "y and q must not be NULL");
    DeviceGuard dg(c->device);
    Engine &E = c->eng;
    launch_adj(c->st, c->P, E.g_adj, E.vec, E.C, c->ones, y, tg ? tg : y, nullptr, q, E.P2,
               nullptr, 0, nullptr, nullptr, 0, MODE_OPERATOR, 0);
    HIP_TRY(c, hipGetLastError());
    return LSQR_OK;
}

lsqr_status lsqr_set_scale(lsqr_ctx *c, const double *d)
{
    if (!c) return fail(nullptr, LSQR_E_INVALID_ARG, "ctx is NULL");
    if (!d) return fail(c, LSQR_E_INVALID_ARG, "d is NULL");
    for (int64_t j = 0; j < c->P.n; ++j)
        if (!(isfinite(d[j]) && d[j] > 0.0))
            return fail(c, LSQR_E_INVALID_ARG, "column scale must be finite and > 0");
    DeviceGuard dg(c->device);
    HIP_TRY(c, hipMemcpyAsync(c->d, d, c->P.n * sizeof(double), hipMemcpyHostToDevice, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    c->fallback_used = 0;
    c->user_scale = true;
    return LSQR_OK;
}

lsqr_status lsqr_get_scale(const lsqr_ctx *cc, double *d)
{
    lsqr_ctx *c = const_cast<lsqr_ctx *>(cc);
    if (!c) return fail(nullptr, LSQR_E_INVALID_ARG, "ctx is NULL");
    if (!d) return fail(c, LSQR_E_INVALID_ARG, "d is NULL");
    DeviceGuard dg(c->device);
    HIP_TRY(c, hipMemcpyAsync(d, c->d, c->P.n * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return LSQR_OK;
}

lsqr_status lsqr_get_transpose(const lsqr_ctx *cc, int64_t *col_ptr, int32_t *row_idx, double *val)
{
    lsqr_ctx *c = const_cast<lsqr_ctx *>(cc);
    if (!c) return fail(nullptr, LSQR_E_INVALID_ARG, "ctx is NULL");
    DeviceGuard dg(c->device);
    const hipMemcpyKind k = hipMemcpyDeviceToHost;
    if (col_ptr) HIP_TRY(c, hipMemcpyAsync(col_ptr, c->cp, (c->P.n + 1) * sizeof(int64_t), k, c->st));
    if (row_idx && c->P.nnz) HIP_TRY(c, hipMemcpyAsync(row_idx, c->ri, c->P.nnz * sizeof(int32_t), k, c->st));
    if (val && c->P.nnz) HIP_TRY(c, hipMemcpyAsync(val, c->cv, c->P.nnz * sizeof(double), k, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return LSQR_OK;
}

lsqr_status lsqr_get_quantised(const lsqr_ctx *cc, float *row_scale, uint16_t *q_rows,
                               uint16_t *q_cols)
{
    lsqr_ctx *c = const_cast<lsqr_ctx *>(cc);
    if (!c) return fail(nullptr, LSQR_E_INVALID_ARG, "ctx is NULL");
    if (!c->qrow) return fail(c, LSQR_E_UNSUPPORTED, "the context holds no quantised values");
    DeviceGuard dg(c->device);
    const hipMemcpyKind k = hipMemcpyDeviceToHost;
    if (row_scale && c->P.m) HIP_TRY(c, hipMemcpyAsync(row_scale, c->sigma, c->P.m * sizeof(float), k, c->st));
    if (q_rows && c->P.nnz) HIP_TRY(c, hipMemcpyAsync(q_rows, c->qrow, c->P.nnz * 2, k, c->st));
    if (q_cols && c->P.nnz) HIP_TRY(c, hipMemcpyAsync(q_cols, c->qcol, c->P.nnz * 2, k, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return LSQR_OK;
}

lsqr_status lsqr_kernel_stats(const lsqr_ctx *c, lsqr_kstats *out)
{
    if (!c || !out) return fail(nullptr, LSQR_E_INVALID_ARG, "ctx and out must not be NULL");
    *out = c->ks;
    // algorithmic bytes of one launch of the solver's kernels: every stored
    // value and index once, the row/column pointers, one pass over each vector
    const Engine &E = c->eng;
    const double nnz = (double)c->P.nnz, m = (double)c->P.m, n = (double)c->P.n;
    const double mb = m + 2 * n;
    const double sv = (double)vt_size(E.R.vt), sx = (double)vt_size(E.vec);
    double fwd = nnz * sv + (m + 1) * 8.0 + n * sx + 2.0 * mb * sx;
    if (E.R.slot) fwd += nnz * 2.0 + (double)c->ngcols * 4.0 + (double)(c->ngroups + 1) * 12.0;
    else fwd += nnz * 4.0;
    if (E.R.sigma) fwd += m * 4.0 + m * sx;
    out->fwd_bytes = fwd;
    out->row_format = E.R.slot ? 4 : 1;
    out->col_format = E.C.nrp ? (E.C.pairs ? 4 : 2) : 1;
    out->fwd_entries_per_load = !E.R.slot            ? 0
                                : lcol_octs_ok(E.R)  ? 8
                                : lcol_quads_ok(E.R) ? 4
                                : lcol_pairs_ok(E.R) ? 2
                                                     : 1;
    out->adj_depths_per_word = E.C.nrp ? (E.C.pairs ? E.C.pairs : 1) : 0;
    out->groups = E.R.slot ? c->ngroups : 0;
    out->staged_cols = E.R.slot ? c->ngcols : 0;
    out->padded_values = (E.C.nrp && E.C.pairs == 2) ? c->npad - c->P.nnz
                         : (E.C.nrp && E.C.pairs >= 4) ? c->npad4 - c->P.nnz : 0;
    if (E.C.nrp) {
        // the method's values only: the zeros a layout pads runs with are
        // format overhead, not algorithmic bytes (they show in the counters)
        const double nn = n / (double)c->P.nz;
        out->adj_bytes = nnz * (double)vt_size(E.C.vt) + (double)c->nnruns * 6.0 +
                         (nn + 1) * 8.0 + (4 * nn + 1) * 8.0 + nn * 4.0 + mb * sx +
                         n * (8.0 + 2.0 * sx);
    } else {
        out->adj_bytes = nnz * ((double)vt_size(E.C.vt) + 4.0) + (n + 1) * 8.0 + mb * sx +
                         n * (8.0 + 2.0 * sx);
    }
    return LSQR_OK;
}

}  // extern "C"
