// Private host-side context of the library (shared by api.hip and batched.hip).
#pragma once

#include <math.h>

#include <string>
#include <vector>

#include "internal.h"

namespace lsqr {

// One LSQR kernel set: the stored formats it reads, its vector type and its
// work buffers, loop state and captured graph.
struct Engine {
    int vec = VT_F64;
    RowFmt R;
    ColFmt C;
    int g_fwd = 1, g_adj = 1, g_upd = 1;
    void *T[2] = {nullptr, nullptr};
    void *Ts = nullptr;            // sigma * t for the quantised forms
    void *q = nullptr, *v = nullptr, *z = nullptr, *vzero = nullptr;
    double *w = nullptr, *y = nullptr;
    double *hbar = nullptr;        // LSMR only (w then holds h)
    int32_t *wrow = nullptr;       // balanced wave partition of the CSR rows (or nullptr)
    double *P1 = nullptr, *P2 = nullptr, *P3 = nullptr;
    double *S = nullptr;
    int64_t s_rows = 0;
    int *ctl = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_iters = 0;
    double graph_tol = -1.0;
};

// Buffers of the batched (multi right-hand side) solver for one system.
struct BatchEngine {
    int R = 0;                     // padded right-hand sides (power of two <= 32)
    int rt = 32;                   // right-hand side tile of the sparse kernels
    int grid = 1024;               // workgroups of the sparse kernels (cap)
    int g_fwd = 1, g_adj = 1, g_upd = 1;
    float *T[2] = {nullptr, nullptr};
    float *V = nullptr, *Q = nullptr, *Z = nullptr;
    double *W = nullptr, *Y = nullptr, *rhs = nullptr, *dm = nullptr;
    double *P1 = nullptr, *P2 = nullptr, *P3 = nullptr;
    float *Pr = nullptr;           // [node runs][R] per-run partial sums of the forward product
    double *S = nullptr;
    int64_t s_rows = 0;
    int *act = nullptr, *why = nullptr, *ctl = nullptr;
    int tuned = 0;                 // 1 once rt/grid were chosen by the autotuner or the caller
    // refinement (lsqr_solve_batched_refined): the solution, the inner
    // right-hand sides, per-RHS reductions
    double *X = nullptr;           // [n][R]
    double *F = nullptr;           // [m+2n][R]
    double *rsum = nullptr;        // [R][4]
};

// f = [0; 0; (Abar^T rbar) / damp] and the partials of |Abar^T rbar|^2: the
// inner right-hand side of a refinement sweep (refine.hip).
void launch_normal_rhs(hipStream_t st, const Problem &P, int grid, const double *rbar,
                       const double *g, double *f, double *part);

}  // namespace lsqr

struct lsqr_ctx {
    lsqr::Problem P;
    lsqr::Allocator al;
    hipStream_t st = nullptr;
    hipStream_t cap_st = nullptr;   // private stream used only for graph capture
    int device = 0;
    lsqr_precision prec = LSQR_FP64;
    lsqr_precond precond = LSQR_PRECOND_NONE;
    uint32_t flags = 0;
    int check_every = 32;
    int method = 0;                 // 0 LSQR, 1 LSMR
    int refine_sweeps = 5;
    double refine_inner_tol = 1e-3;
    int fallback_used = 0;          // set at creation when user scales were rejected
    int fallback_iters = 0;         // opts.fallback_iters
    double *d_user = nullptr;       // the accepted user scale (restored after a fallback)
    bool user_scale = false;        // D is a caller's scale (create USER or lsqr_set_scale)
    std::vector<std::pair<void *, size_t>> owned;
    // FP64 operator: CSR, CSC, column scale
    int64_t *rp = nullptr; int32_t *ci = nullptr; double *va = nullptr;
    int64_t *cp = nullptr; int32_t *ri = nullptr; double *cv = nullptr;
    // node runs of the data block (transposed product), values in node-major order
    int64_t *nrp = nullptr, *nvq = nullptr; uint32_t *nrow = nullptr; uint16_t *ndesc = nullptr;
    int32_t *norder = nullptr; double *nval = nullptr; float *nval32 = nullptr;
    int64_t *rrp = nullptr; uint32_t *rrid = nullptr;   // row order of the node runs (batched forward)
    uint16_t *nvalq = nullptr; uint32_t *nsrc = nullptr, *ndst = nullptr;
    int64_t nnruns = 0;
    // depth-pair layout of the node-run values (k_adj_npair)
    int64_t *nvqp = nullptr; uint32_t *ndstp = nullptr; int64_t npad = 0;
    double *nvalp = nullptr; float *nvalp32 = nullptr; uint16_t *nvalpq = nullptr;
    // the 16-bit codes in the four-depth layout (mixed forms)
    int64_t *nvqp4 = nullptr; uint32_t *ndstp4 = nullptr; int64_t npad4 = 0;
    float *nvalp4f = nullptr;     // FP32 node-run values in the four-depth layout
    // row groups with local columns (forward product over va)
    int32_t *gp = nullptr, *gcol = nullptr; int64_t *gcp = nullptr; uint16_t *slot = nullptr;
    int ngroups = 0, gcap = 0;
    int64_t ngcols = 0;
    double *d = nullptr, *ones = nullptr;
    lsqr::RowFmt R64;
    lsqr::ColFmt C64;
    // reduced-precision copies
    float *va32 = nullptr, *cv32 = nullptr;
    float *sigma = nullptr;
    uint16_t *qrow = nullptr, *qcol = nullptr;
    lsqr::Engine eng;               // the solver's kernel set
    lsqr::Engine eng32;             // quantised forms: FP32 inner solves after a stall
    bool have_eng32 = false;
    double stall_ratio = 0.5;       // refinement: a sweep must bring eta below this x the last
    lsqr::BatchEngine beng;         // the batched solver's buffers
    // refinement and operator scratch (FP64)
    double *xbuf = nullptr, *ybuf = nullptr, *rbar = nullptr, *gbuf = nullptr;
    double *fbuf = nullptr, *Pr = nullptr, *Pa = nullptr, *Pf = nullptr;
    double *sums = nullptr;
    int g_ref = 1;
    double *dtbuf = nullptr, *dmbuf = nullptr;
    double *wr = nullptr, *wg = nullptr;   // warm start: residual at x0 [m+2n], transposed product [n]
    int *flag = nullptr;
    int *hctl = nullptr;            // pinned host mirror of control words
    double *hsum = nullptr;         // pinned host mirror of reductions
    std::vector<hipEvent_t> ev;
    lsqr_kstats ks{};
    std::string err;
};

namespace lsqr {

lsqr_status fail(lsqr_ctx *c, lsqr_status s, const std::string &msg);

#define HIP_TRY(ctx, expr)                                                                  \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess)                                                               \
            return lsqr::fail(ctx, LSQR_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

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

inline void *ctx_alloc_bytes(lsqr_ctx *c, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    void *p = c->al.get(bytes);
    if (p) c->owned.push_back({p, bytes});
    return p;
}

template <class T>
inline T *ctx_alloc(lsqr_ctx *c, size_t count)
{
    return (T *)ctx_alloc_bytes(c, count * sizeof(T));
}

inline void ctx_release(lsqr_ctx *c, void *p)
{
    for (size_t i = 0; i < c->owned.size(); ++i)
        if (c->owned[i].first == p) {
            c->al.put(p, c->owned[i].second);
            c->owned.erase(c->owned.begin() + (long)i);
            return;
        }
}

}  // namespace lsqr
