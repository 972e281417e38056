// Host runtime of the C ABI declared in lsqr_mi355x.h.
//
// Owns validation, device buffers (through the caller's allocator), the
// transpose and scale set-up, the iteration schedule on the caller's stream,
// optional hipGraph replay of blocks of iterations, and read-back of the stop
// state and residual history.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace lsqr;

struct lsqr_ctx {
    Problem P;
    Geometry g;
    Allocator al;
    hipStream_t st = nullptr;
    hipStream_t cap_st = nullptr;   // private stream used only for graph capture
    int device = 0;
    lsqr_precision prec = LSQR_FP64;
    lsqr_precond precond = LSQR_PRECOND_NONE;
    uint32_t flags = 0;
    int check_every = 32;
    int fallback_used = 0;
    std::vector<std::pair<void *, size_t>> owned;
    // operator
    int64_t *rp = nullptr; int32_t *ci = nullptr; double *va = nullptr;
    int64_t *cp = nullptr; int32_t *ri = nullptr; double *cv = nullptr;
    double *d = nullptr;
    // work
    double *T[2] = {nullptr, nullptr};
    double *q = nullptr, *v = nullptr, *w = nullptr, *y = nullptr, *z = nullptr;
    double *vzero = nullptr, *dtbuf = nullptr, *dmbuf = nullptr;
    double *P1 = nullptr, *P2 = nullptr, *P3 = nullptr;
    double *S = nullptr;
    int64_t s_rows = 0;
    int *ctl = nullptr;
    int *flag = nullptr;
    int *hctl = nullptr;            // pinned host mirror of the control words
    // graph of `graph_iters` iterations (even), rebuilt when S moves
    hipGraphExec_t gexec = nullptr;
    int graph_iters = 0;
    double graph_tol = -1.0;
    // timing
    std::vector<hipEvent_t> ev;
    lsqr_kstats ks{};
    std::string err;
};

static thread_local std::string g_err;

static lsqr_status fail(lsqr_ctx *c, lsqr_status s, const std::string &msg)
{
    if (c) c->err = msg;
    else g_err = msg;
    return s;
}

#define HIP_TRY(ctx, expr)                                                                  \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess)                                                               \
            return fail(ctx, LSQR_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

template <class T>
T *ctx_alloc(lsqr_ctx *c, size_t count)
{
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = sizeof(T);
    void *p = c->al.get(bytes);
    if (p) c->owned.push_back({p, bytes});
    return (T *)p;
}

void ctx_release(lsqr_ctx *c, void *p)
{
    for (size_t i = 0; i < c->owned.size(); ++i)
        if (c->owned[i].first == p) {
            c->al.put(p, c->owned[i].second);
            c->owned.erase(c->owned.begin() + (long)i);
            return;
        }
}

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
                    const int32_t c = G->col_idx[p];
                    if (c < 0 || c >= n) b |= 2;
                    if (p > G->row_ptr[i] && c <= G->col_idx[p - 1]) b |= 4;
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

lsqr_status ensure_state(lsqr_ctx *c, int iters)
{
    const int64_t need = (int64_t)iters + 2;
    if (c->s_rows >= need) return LSQR_OK;
    if (c->S) ctx_release(c, c->S);
    const int64_t rows = std::max<int64_t>(need, 512);
    c->S = ctx_alloc<double>(c, (size_t)rows * kStateWords);
    if (!c->S) return fail(c, LSQR_E_OOM, "state allocation failed");
    c->s_rows = rows;
    if (c->gexec) { (void)hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
    return LSQR_OK;
}

// One LSQR iteration of parity p (0: odd k, 1: even k).
void launch_iteration(lsqr_ctx *c, hipStream_t st, int p, double tol, bool timing, int slot)
{
    const DevCSR A{c->rp, c->ci, c->va}, At{c->cp, c->ri, c->cv};
    double *Tprev = c->T[p], *Tcur = c->T[1 - p];
    if (timing) (void)hipEventRecord(c->ev[4 * slot + 0], st);
    launch_fwd(st, c->P, c->g, A, c->z, Tprev, Tcur, c->P1, c->P3, c->S, c->ctl, p, tol, MODE_ITER);
    if (timing) (void)hipEventRecord(c->ev[4 * slot + 1], st);
    if (timing) (void)hipEventRecord(c->ev[4 * slot + 2], st);
    launch_adj(st, c->P, c->g, At, c->d, Tcur, c->v, c->q, c->P2, c->P1, c->S, c->ctl, p, MODE_ITER);
    if (timing) (void)hipEventRecord(c->ev[4 * slot + 3], st);
    launch_update(st, c->P, c->g, c->d, c->q, c->v, c->w, c->y, c->z, c->P3, c->P2, c->S, c->ctl,
                  p, MODE_ITER);
}

lsqr_status build_graph(lsqr_ctx *c, int iters, double tol)
{
    if (c->gexec && c->graph_iters == iters && c->graph_tol == tol) return LSQR_OK;
    if (c->gexec) { (void)hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
    if (!c->cap_st) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIP_TRY(c, hipStreamBeginCapture(c->cap_st, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < iters; ++i) launch_iteration(c, c->cap_st, i & 1, tol, false, 0);
    HIP_TRY(c, hipStreamEndCapture(c->cap_st, &graph));
    hipError_t e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        c->gexec = nullptr;
        return fail(c, LSQR_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    c->graph_iters = iters;
    c->graph_tol = tol;
    return LSQR_OK;
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
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->cap_st) (void)hipStreamDestroy(c->cap_st);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    for (auto &pr : c->owned) c->al.put(pr.first, pr.second);
    if (c->hctl) (void)hipHostFree(c->hctl);
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
    if (o.precision != LSQR_FP64)
        return fail(nullptr, LSQR_E_UNSUPPORTED, "only LSQR_FP64 is provided by this build");
    if (o.precond < LSQR_PRECOND_NONE || o.precond > LSQR_PRECOND_USER)
        return fail(nullptr, LSQR_E_INVALID_ARG, "unknown precond");
    if (o.precond == LSQR_PRECOND_USER && !o.col_scale)
        return fail(nullptr, LSQR_E_INVALID_ARG, "precond USER needs col_scale");
    if ((o.lanes_per_row && !valid_lanes(o.lanes_per_row)) ||
        (o.lanes_per_col && !valid_lanes(o.lanes_per_col)))
        return fail(nullptr, LSQR_E_INVALID_ARG, "lanes must be 0, 4, 8, 16, 32 or 64");
    if (o.check_every < 0) return fail(nullptr, LSQR_E_INVALID_ARG, "check_every must be >= 0");
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
    c->check_every = o.check_every > 0 ? o.check_every : 32;
    c->check_every += c->check_every & 1;
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
    c->va = ctx_alloc<double>(c, nnz);
    c->cp = ctx_alloc<int64_t>(c, n + 1);
    c->ri = ctx_alloc<int32_t>(c, nnz);
    c->cv = ctx_alloc<double>(c, nnz);
    c->d = ctx_alloc<double>(c, n);
    c->T[0] = ctx_alloc<double>(c, mb);
    c->T[1] = ctx_alloc<double>(c, mb);
    c->q = ctx_alloc<double>(c, n); c->v = ctx_alloc<double>(c, n); c->w = ctx_alloc<double>(c, n);
    c->y = ctx_alloc<double>(c, n); c->z = ctx_alloc<double>(c, n);
    c->vzero = ctx_alloc<double>(c, n); c->dtbuf = ctx_alloc<double>(c, std::max<int64_t>(m, 1));
    c->dmbuf = ctx_alloc<double>(c, n);
    c->ctl = ctx_alloc<int>(c, C_WORDS);
    c->flag = ctx_alloc<int>(c, 4);
    if (!c->rp || !c->ci || !c->va || !c->cp || !c->ri || !c->cv || !c->d || !c->T[0] || !c->T[1] ||
        !c->q || !c->v || !c->w || !c->y || !c->z || !c->vzero || !c->dtbuf || !c->dmbuf ||
        !c->ctl || !c->flag)
        return bail(LSQR_E_OOM, "device allocation failed");
    CR_TRY(hipHostMalloc((void **)&c->hctl, C_WORDS * sizeof(int), hipHostMallocDefault));

    // launch geometry: enough resident workgroups to fill 256 CUs
    const double avg_row = m > 0 ? (double)nnz / (double)m : 0.0;
    const double avg_col = (double)nnz / (double)n;
    c->g.lpr = o.lanes_per_row ? o.lanes_per_row : pick_lanes(avg_row);
    c->g.lpc = o.lanes_per_col ? o.lanes_per_col : pick_lanes(avg_col);
    auto cap_blocks = [](int64_t work, int per, int cap) {
        int64_t b = (work + per - 1) / per;
        return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
    };
    c->g.g_fwd = cap_blocks(std::max<int64_t>(m * c->g.lpr, 2 * n), kBlock, 2048);
    c->g.g_adj = cap_blocks(n * c->g.lpc, kBlock, 2048);
    c->g.g_upd = cap_blocks(n, kBlock, 1024);
    c->P1 = ctx_alloc<double>(c, c->g.g_fwd);
    c->P2 = ctx_alloc<double>(c, c->g.g_adj);
    c->P3 = ctx_alloc<double>(c, c->g.g_upd);
    if (!c->P1 || !c->P2 || !c->P3) return bail(LSQR_E_OOM, "device allocation failed");

    hipStream_t st = c->st;
    const hipMemcpyKind kind = G->mem == LSQR_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    CR_TRY(hipMemcpyAsync(c->rp, G->row_ptr, (m + 1) * sizeof(int64_t), kind, st));
    if (nnz > 0) {
        CR_TRY(hipMemcpyAsync(c->ci, G->col_idx, nnz * sizeof(int32_t), kind, st));
        CR_TRY(hipMemcpyAsync(c->va, G->val, nnz * sizeof(double), kind, st));
    }
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
    }
    {
        std::string terr;
        hipError_t e = build_transpose(st, c->al, m, n, nnz, DevCSR{c->rp, c->ci, c->va}, c->cp,
                                       c->ri, c->cv, terr);
        if (e != hipSuccess)
            return bail(e == hipErrorOutOfMemory ? LSQR_E_OOM : LSQR_E_DEVICE,
                        terr + ": " + hipGetErrorString(e));
    }
    // column scaling
    if (o.precond == LSQR_PRECOND_NONE) {
        launch_fill(st, n, 1.0, c->d);
    } else {
        bool use_jacobi = o.precond == LSQR_PRECOND_JACOBI;
        if (!use_jacobi) {
            bool ok = true;
            for (int64_t j = 0; j < n && ok; ++j) ok = isfinite(o.col_scale[j]) && o.col_scale[j] > 0.0;
            if (ok) CR_TRY(hipMemcpyAsync(c->d, o.col_scale, n * sizeof(double), hipMemcpyHostToDevice, st));
            else { use_jacobi = true; c->fallback_used = 1; }
        }
        if (use_jacobi) launch_jacobi(st, c->P, DevCSR{c->cp, c->ri, c->cv}, c->d);
    }
    CR_TRY(hipGetLastError());
    CR_TRY(hipStreamSynchronize(st));
    *out = c;
    return LSQR_OK;
#undef CR_TRY
}

lsqr_status lsqr_solve(lsqr_ctx *c, const double *dt, lsqr_mem vec_mem, int iters, double tol,
                       double *dm, double *res_hist, lsqr_info *info)
{
    if (!c) return fail(nullptr, LSQR_E_INVALID_ARG, "ctx is NULL");
    if (!dt || !dm) return fail(c, LSQR_E_INVALID_ARG, "dt and dm must not be NULL");
    if (iters < 0) return fail(c, LSQR_E_INVALID_ARG, "iters must be >= 0");
    if (!(tol >= 0.0) || !isfinite(tol)) return fail(c, LSQR_E_INVALID_ARG, "tol must be finite and >= 0");
    if (vec_mem != LSQR_MEM_HOST && vec_mem != LSQR_MEM_DEVICE)
        return fail(c, LSQR_E_INVALID_ARG, "unknown memory kind");
    DeviceGuard dg(c->device);
    hipStream_t st = c->st;
    const Problem &P = c->P;
    const int64_t m = P.m, n = P.n;
    lsqr_status s = ensure_state(c, iters);
    if (s != LSQR_OK) return s;

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

    const bool timing = (c->flags & LSQR_FLAG_TIMING) != 0;
    const bool use_graph = !timing && !(c->flags & LSQR_FLAG_NO_GRAPH);
    if (timing && (int)c->ev.size() < 4 * iters) {
        while ((int)c->ev.size() < 4 * iters) {
            hipEvent_t e;
            HIP_TRY(c, hipEventCreate(&e));
            c->ev.push_back(e);
        }
    }
    const DevCSR At{c->cp, c->ri, c->cv};
    // start: beta_1 u_1 = bbar, alpha_1 v_1 = A_D^T u_1
    launch_init_rhs(st, P, c->g, ddt, c->T[0], c->y, c->vzero, c->P1, c->ctl, iters);
    launch_adj(st, P, c->g, At, c->d, c->T[0], c->vzero, c->q, c->P2, c->P1, c->S, c->ctl, 0, MODE_INIT);
    launch_update(st, P, c->g, c->d, c->q, c->v, c->w, c->y, c->z, c->P3, c->P2, c->S, c->ctl, 0,
                  MODE_INIT);
    HIP_TRY(c, hipGetLastError());

    // iterations: blocks of an even number of iterations replayed as one graph
    // (parity returns to 0 after each block); with tol > 0 the host reads the
    // device stop flag after every block of check_every iterations
    const int block = tol > 0.0 ? c->check_every : iters;
    int done = 0;
    bool stopped = false;
    auto poll = [&]() -> lsqr_status {
        HIP_TRY(c, hipMemcpyAsync(c->hctl, c->ctl, C_WORDS * sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
        stopped = c->hctl[C_STOP] != 0;
        return LSQR_OK;
    };
    if (use_graph && block >= 2) {
        const int gb = std::min(block, 64) & ~1;
        s = build_graph(c, gb, tol);
        if (s != LSQR_OK) return s;
        while (!stopped && iters - done >= gb) {
            HIP_TRY(c, hipGraphLaunch(c->gexec, st));
            done += gb;
            if (tol > 0.0 && done < iters && (s = poll()) != LSQR_OK) return s;
        }
    }
    while (!stopped && done < iters) {
        launch_iteration(c, st, done & 1, tol, timing, done);
        ++done;
        if (tol > 0.0 && done % c->check_every == 0 && done < iters && (s = poll()) != LSQR_OK)
            return s;
    }
    launch_finalize(st, P, c->g, c->d, c->y, ddm, c->P3, c->S, c->ctl, 0, tol);
    HIP_TRY(c, hipGetLastError());
    if (vec_mem == LSQR_MEM_HOST)
        HIP_TRY(c, hipMemcpyAsync(dm, c->dmbuf, n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipMemcpyAsync(c->hctl, c->ctl, C_WORDS * sizeof(int), hipMemcpyDeviceToHost, st));
    std::vector<double> hs;
    if (res_hist || info) {
        hs.resize((size_t)(iters + 1) * kStateWords);
        HIP_TRY(c, hipMemcpyAsync(hs.data(), c->S, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(c, hipStreamSynchronize(st));
    if (timing) {
        c->ks = lsqr_kstats{};
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
    const int kdone = c->hctl[C_ITERS];
    const int istop = c->hctl[C_ISTOP];
    if (c->hctl[C_ERR]) return fail(c, LSQR_E_NONFINITE, "a solver scalar became non-finite");
    if (res_hist) {
        for (int k = 0; k <= iters; ++k) {
            const bool ok = k <= kdone && !(istop == 0 && k > 0);
            for (int f = 0; f < 3; ++f) res_hist[3 * k + f] = NAN;
            if (!ok) continue;
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
    if (info) {
        info->istop = istop;
        info->iters = kdone;
        info->sweeps = 0;
        info->fallback_used = c->fallback_used;
        const double *Sk = hs.data() + (size_t)kdone * kStateWords;
        info->eta = istop == 0 ? 0.0 : Sk[S_ETA];
        info->phibar = istop == 0 ? hs[S_BETA] : Sk[S_PHIBAR];
    }
    return LSQR_OK;
}

lsqr_status lsqr_apply(lsqr_ctx *c, const double *x, double *y)
{
    if (!c) return fail(nullptr, LSQR_E_INVALID_ARG, "ctx is NULL");
    if (!x || !y) return fail(c, LSQR_E_INVALID_ARG, "x and y must not be NULL");
    DeviceGuard dg(c->device);
    launch_scale_vec(c->st, c->P.n, c->d, x, c->z);
    launch_fwd(c->st, c->P, c->g, DevCSR{c->rp, c->ci, c->va}, c->z, nullptr, y, c->P1, c->P3,
               c->S, c->ctl, 0, 0.0, MODE_OPERATOR);
    HIP_TRY(c, hipGetLastError());
    return LSQR_OK;
}

lsqr_status lsqr_apply_t(lsqr_ctx *c, const double *y, double *x)
{
    if (!c) return fail(nullptr, LSQR_E_INVALID_ARG, "ctx is NULL");
    if (!x || !y) return fail(c, LSQR_E_INVALID_ARG, "x and y must not be NULL");
    DeviceGuard dg(c->device);
    launch_adj(c->st, c->P, c->g, DevCSR{c->cp, c->ri, c->cv}, c->d, y, nullptr, x, c->P2, c->P1,
               c->S, c->ctl, 0, MODE_OPERATOR);
    HIP_TRY(c, hipGetLastError());
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

lsqr_status lsqr_kernel_stats(const lsqr_ctx *c, lsqr_kstats *out)
{
    if (!c || !out) return fail(nullptr, LSQR_E_INVALID_ARG, "ctx and out must not be NULL");
    *out = c->ks;
    const double nnz = (double)c->P.nnz, m = (double)c->P.m, n = (double)c->P.n;
    // algorithmic bytes of one launch: matrix stream + pointers + one read of
    // each gathered vector + vector writes
    out->fwd_bytes = nnz * 12.0 + (m + 1) * 8.0 + n * 8.0 + (m + 2 * n) * 16.0;
    out->adj_bytes = nnz * 12.0 + (n + 1) * 8.0 + (m + 2 * n) * 8.0 + n * 8.0 * 3.0;
    return LSQR_OK;
}

}  // extern "C"
