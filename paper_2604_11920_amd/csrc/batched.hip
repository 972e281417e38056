// Batched multi right-hand-side LSQR: host runtime of lsqr_solve_batched,
// the block operator entry points and the schedule autotuner.
//
// All systems' iterations are captured into one hipGraph (a block of up to 32
// iterations x every system x three kernel stages) and replayed; each
// system's right-hand sides carry their own FP64 scalars on the device.
#include <math.h>

#include <algorithm>
#include <vector>

#include "ctx.h"
#include "lsqr_batched.cuh"

using namespace lsqr;

namespace {

int pow2_at_least(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

BArgs base_args(lsqr_ctx *c, BatchEngine &B)
{
    BArgs a{};
    a.rp = c->rp; a.ci = c->ci; a.va = c->va32;
    a.cp = c->cp; a.ri = c->ri; a.cv = c->cv32;
    if (c->nval32 && c->P.nz <= kMaxNzBatched) {   // transposed product over node runs
        a.nrp = c->nrp; a.nvq = c->nvq; a.nrow = c->nrow; a.ndesc = c->ndesc;
        a.norder = c->norder; a.nval = c->nval32;
        if (B.Pr) { a.rrp = c->rrp; a.rrid = c->rrid; a.Pr = B.Pr; a.g_pr = B.g_adj; }
    }
    a.d = c->d;
    a.m = c->P.m; a.n = (int)c->P.n; a.nx = c->P.nx; a.ny = c->P.ny; a.nz = c->P.nz;
    a.w = c->P.w; a.damp = c->P.damp;
    a.R = B.R;
    a.act = B.act; a.why = B.why; a.ctl = B.ctl; a.S = B.S;
    return a;
}

template <int RT>
void launch_tile(hipStream_t st, int kind, int grid, const BArgs &a)
{
    switch (kind) {
    case 0: hipLaunchKernelGGL((k_binit<RT>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 1:
        if (a.Pr && RT == 32) {       // two-phase product over the node runs
            hipLaunchKernelGGL(k_bfwd_pr32, dim3(a.g_pr), dim3(kBlock), 0, st, a);
            hipLaunchKernelGGL((k_bfwd<RT>), dim3(grid), dim3(kBlock), 0, st, a);
        } else {                      // entry-wise over the CSR rows
            BArgs b = a;
            b.Pr = nullptr;
            hipLaunchKernelGGL((k_bfwd<RT>), dim3(grid), dim3(kBlock), 0, st, b);
        }
        break;
    default:
        if (a.nrp && RT == 32) hipLaunchKernelGGL(k_badj_mfma32, dim3(grid), dim3(kBlock), 0, st, a);
        else if (a.nrp) hipLaunchKernelGGL((k_badj_nruns<RT>), dim3(grid), dim3(kBlock), 0, st, a);
        else hipLaunchKernelGGL((k_badj<RT>), dim3(grid), dim3(kBlock), 0, st, a);
        break;
    }
}

void launch_tiled(hipStream_t st, int kind, int grid, BArgs a, int R, int rt)
{
    for (int r0 = 0; r0 < R; r0 += rt) {
        a.r0 = r0;
        switch (rt) {
        case 1: launch_tile<1>(st, kind, grid, a); break;
        case 2: launch_tile<2>(st, kind, grid, a); break;
        case 4: launch_tile<4>(st, kind, grid, a); break;
        case 8: launch_tile<8>(st, kind, grid, a); break;
        case 16: launch_tile<16>(st, kind, grid, a); break;
        default: launch_tile<32>(st, kind, grid, a); break;
        }
    }
}

// FP32 copies of the values (the batched kernels read FP32).
lsqr_status ensure_fp32(lsqr_ctx *c, hipStream_t st)
{
    const int64_t nnz = c->P.nnz;
    if (!c->va32 || !c->cv32) {
        c->va32 = ctx_alloc<float>(c, nnz);
        c->cv32 = ctx_alloc<float>(c, nnz);
        if (!c->va32 || !c->cv32) return fail(c, LSQR_E_OOM, "device allocation failed");
        launch_convert_f32(st, nnz, c->va, c->va32);
        launch_convert_f32(st, nnz, c->cv, c->cv32);
    }
    if (c->nval && !c->nval32) {     // node-run values for the transposed block product
        c->nval32 = ctx_alloc<float>(c, nnz);
        if (!c->nval32) return fail(c, LSQR_E_OOM, "device allocation failed");
        launch_convert_f32(st, nnz, c->nval, c->nval32);
    }
    HIP_TRY(c, hipGetLastError());
    return LSQR_OK;
}

int cap(int64_t work, int per, int lim)
{
    int64_t b = (work + per - 1) / per;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, lim));
}

// Buffers for R right-hand sides and `iters` iterations.
lsqr_status ensure_batch(lsqr_ctx *c, hipStream_t st, int R, int iters)
{
    BatchEngine &B = c->beng;
    const int64_t m = c->P.m, n = c->P.n, mb = m + 2 * n;
    lsqr_status s = ensure_fp32(c, st);
    if (s != LSQR_OK) return s;
    if (B.R != R) {
        for (void *p : {(void *)B.T[0], (void *)B.T[1], (void *)B.V, (void *)B.Q, (void *)B.Z,
                        (void *)B.W, (void *)B.Y, (void *)B.rhs, (void *)B.dm, (void *)B.P1,
                        (void *)B.P2, (void *)B.P3, (void *)B.act, (void *)B.why, (void *)B.ctl,
                        (void *)B.Pr, (void *)B.X, (void *)B.F, (void *)B.rsum})
            if (p) ctx_release(c, p);
        const int keep_rt = B.tuned ? B.rt : 0, keep_grid = B.tuned ? B.grid : 0;
        B = BatchEngine{};
        B.R = R;
        B.rt = keep_rt && keep_rt <= R ? keep_rt : std::min(R, 32);
        B.grid = keep_grid ? keep_grid : 1024;
        B.T[0] = ctx_alloc<float>(c, mb * R);
        B.T[1] = ctx_alloc<float>(c, mb * R);
        B.V = ctx_alloc<float>(c, n * R);
        B.Q = ctx_alloc<float>(c, n * R);
        B.Z = ctx_alloc<float>(c, n * R);
        B.W = ctx_alloc<double>(c, n * R);
        B.Y = ctx_alloc<double>(c, n * R);
        B.rhs = ctx_alloc<double>(c, std::max<int64_t>(m, 1) * R);
        B.dm = ctx_alloc<double>(c, n * R);
        B.P1 = ctx_alloc<double>(c, (size_t)2048 * R);
        B.P2 = ctx_alloc<double>(c, (size_t)2048 * R);
        B.P3 = ctx_alloc<double>(c, (size_t)2048 * R);
        B.act = ctx_alloc<int>(c, R);
        B.why = ctx_alloc<int>(c, R);
        B.ctl = ctx_alloc<int>(c, C_WORDS);
        if (!B.T[0] || !B.T[1] || !B.V || !B.Q || !B.Z || !B.W || !B.Y || !B.rhs || !B.dm ||
            !B.P1 || !B.P2 || !B.P3 || !B.act || !B.why || !B.ctl)
            return fail(c, LSQR_E_OOM, "device allocation failed");
        // per-run partial rows of the two-phase forward product (node runs)
        if (c->rrid && c->nval32 && c->P.nz <= kMaxNzBatched) {
            B.Pr = ctx_alloc<float>(c, std::max<int64_t>(c->nnruns, 1) * R);
            if (!B.Pr) return fail(c, LSQR_E_OOM, "device allocation failed");
        }
    }
    const int64_t need = (int64_t)iters + 2;
    if (B.s_rows < need) {
        if (B.S) ctx_release(c, B.S);
        B.s_rows = std::max<int64_t>(need, 512);
        B.S = ctx_alloc<double>(c, (size_t)B.s_rows * R * kStateWords);
        if (!B.S) return fail(c, LSQR_E_OOM, "state allocation failed");
    }
    B.g_fwd = cap(m * 64, kBlock, B.grid);
    if (c->nval32 && c->P.nz <= kMaxNzBatched)      // a workgroup per lateral node
        B.g_adj = (int)std::max<int64_t>(1, std::min<int64_t>(n / c->P.nz, B.grid));
    else
        B.g_adj = cap(n * 64, kBlock, B.grid);
    B.g_upd = cap(n * R, kBlock, 512);
    return LSQR_OK;
}

void batch_init(lsqr_ctx *c, hipStream_t st, double tol, bool full = false)
{
    BatchEngine &B = c->beng;
    BArgs a = base_args(c, B);
    a.rhs = full ? B.F : B.rhs; a.rhs_full = full ? 1 : 0;
    a.Tcur = B.T[0]; a.V = B.V; a.Y = B.Y; a.W = B.W; a.Zout = B.Z; a.Q = B.Q;
    a.tol = tol;
    a.part_out = B.P1;
    launch_tiled(st, 0, B.g_fwd, a, B.R, B.rt);
    a.mode = MODE_INIT;
    a.part_in = B.P1; a.np_in = B.g_fwd; a.part_out = B.P2;
    launch_tiled(st, 2, B.g_adj, a, B.R, B.rt);
    a.part_in = B.P2; a.np_in = B.g_adj; a.part_out = B.P3;
    hipLaunchKernelGGL(k_bupdate, dim3(B.g_upd), dim3(kBlock), 0, st, a);
}

void batch_iter(lsqr_ctx *c, hipStream_t st, int p, double tol)
{
    BatchEngine &B = c->beng;
    BArgs a = base_args(c, B);
    a.parity = p; a.mode = MODE_ITER; a.tol = tol;
    a.V = B.V; a.Q = B.Q; a.W = B.W; a.Y = B.Y;
    // forward: T[1-p] = A_D Z - alpha U
    a.Z = B.Z; a.Tprev = B.T[p]; a.Tcur = B.T[1 - p];
    a.part_in = B.P3; a.np_in = B.g_upd; a.part_out = B.P1;
    launch_tiled(st, 1, B.g_fwd, a, B.R, B.rt);
    // transposed: Q = D A^T T / beta - beta V
    a.part_in = B.P1; a.np_in = B.g_fwd; a.part_out = B.P2;
    launch_tiled(st, 2, B.g_adj, a, B.R, B.rt);
    // update
    a.part_in = B.P2; a.np_in = B.g_adj; a.part_out = B.P3; a.Zout = B.Z;
    hipLaunchKernelGGL(k_bupdate, dim3(B.g_upd), dim3(kBlock), 0, st, a);
}

__global__ void k_set_kmax(int *ctl, int kmax) { ctl[C_KMAX] = kmax; }

// Column r of a row-major [rows][R] FP64 block: read into v, write from v
// (v == nullptr: zeros), or add the whole block src to dst.
__global__ void k_col_get(int64_t rows, int R, int r, const double *blk, double *v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x)
        v[i] = blk[i * R + r];
}

__global__ void k_col_put(int64_t rows, int R, int r, const double *v, double *blk)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x)
        blk[i * R + r] = v ? v[i] : 0.0;
}

__global__ void k_blk_add(int64_t count, const double *src, double *dst)
{
#pragma clang fp contract(off)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = dst[i] + src[i];
}

int grid_for(int64_t work) { return cap(work, 256, 4096); }

// Checks shared by the batched entry points.
lsqr_status batch_args(lsqr_ctx *const *ctxs, int nsys, int nrhs, const double *const *dt,
                       lsqr_mem vec_mem, int iters, double tol, double *const *dm)
{
    if (!ctxs || nsys < 1) return fail(nullptr, LSQR_E_INVALID_ARG, "need at least one context");
    for (int s = 0; s < nsys; ++s)
        if (!ctxs[s]) return fail(nullptr, LSQR_E_INVALID_ARG, "context is NULL");
    lsqr_ctx *c0 = ctxs[0];
    if (nrhs < 1 || nrhs > kMaxRhs) return fail(c0, LSQR_E_INVALID_ARG, "nrhs must be in 1..32");
    if (!dt || !dm) return fail(c0, LSQR_E_INVALID_ARG, "dt and dm must not be NULL");
    if (iters < 0) return fail(c0, LSQR_E_INVALID_ARG, "iters must be >= 0");
    if (!(tol >= 0.0) || !isfinite(tol)) return fail(c0, LSQR_E_INVALID_ARG, "tol must be finite and >= 0");
    if (vec_mem != LSQR_MEM_HOST && vec_mem != LSQR_MEM_DEVICE)
        return fail(c0, LSQR_E_INVALID_ARG, "unknown memory kind");
    for (int s = 0; s < nsys; ++s) {
        if (!dt[s] || !dm[s]) return fail(c0, LSQR_E_INVALID_ARG, "dt[s] and dm[s] must not be NULL");
        if (ctxs[s]->device != c0->device) return fail(c0, LSQR_E_INVALID_ARG, "contexts on different devices");
        if (vec_mem == LSQR_MEM_HOST)
            for (int64_t i = 0; i < ctxs[s]->P.m * (int64_t)nrhs; ++i)
                if (!isfinite(dt[s][i])) return fail(c0, LSQR_E_NONFINITE, "non-finite value in dt");
    }
    return LSQR_OK;
}

// Copies every system's [m][nrhs] right-hand sides into its padded [m][R]
// block B.rhs (buffers for `iters` iterations made ready first).
lsqr_status batch_load_rhs(lsqr_ctx *const *ctxs, int nsys, int nrhs, int R, const double *const *dt,
                           lsqr_mem vec_mem, int iters)
{
    lsqr_ctx *c0 = ctxs[0];
    hipStream_t st = c0->st;
    const hipMemcpyKind kin = vec_mem == LSQR_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    for (int s = 0; s < nsys; ++s) {
        lsqr_ctx *c = ctxs[s];
        lsqr_status e = ensure_batch(c, st, R, iters);
        if (e != LSQR_OK) return fail(c0, e, c->err);
        BatchEngine &B = c->beng;
        if (R != nrhs) launch_fill(st, std::max<int64_t>(c->P.m, 1) * R, 0.0, B.rhs);
        if (c->P.m > 0)
            HIP_TRY(c0, hipMemcpy2DAsync(B.rhs, R * sizeof(double), dt[s], nrhs * sizeof(double),
                                         nrhs * sizeof(double), c->P.m, kin, st));
    }
    HIP_TRY(c0, hipGetLastError());
    return LSQR_OK;
}

// Runs every system's batch from its start (B.rhs, or B.F when full) for up
// to `iters` iterations: a captured graph of a block of iterations of all
// systems, replayed while any right-hand side is active, then single
// iterations; leaves dm = D y of every system in its B.dm.
lsqr_status batch_run(lsqr_ctx *const *ctxs, int nsys, int nrhs, int R, int iters, double tol,
                      bool full)
{
    lsqr_ctx *c0 = ctxs[0];
    hipStream_t st = c0->st;
    for (int s = 0; s < nsys; ++s) {
        batch_init(ctxs[s], st, tol, full);
        hipLaunchKernelGGL(k_set_kmax, dim3(1), dim3(1), 0, st, ctxs[s]->beng.ctl, iters);
    }
    HIP_TRY(c0, hipGetLastError());
    int done = 0;
    bool stopped = false;
    std::vector<int> hact((size_t)R);
    auto poll = [&]() -> lsqr_status {
        int live = 0;
        for (int s = 0; s < nsys; ++s) {
            HIP_TRY(c0, hipMemcpyAsync(hact.data(), ctxs[s]->beng.act, R * sizeof(int),
                                       hipMemcpyDeviceToHost, st));
            HIP_TRY(c0, hipStreamSynchronize(st));
            for (int r = 0; r < nrhs; ++r) live += hact[r];
        }
        stopped = live == 0;
        return LSQR_OK;
    };
    const int gb = std::min(iters, tol > 0.0 ? c0->check_every : 32) & ~1;
    lsqr_status e;
    if (gb >= 2 && !(c0->flags & LSQR_FLAG_NO_GRAPH)) {
        if (!c0->cap_st) HIP_TRY(c0, hipStreamCreateWithFlags(&c0->cap_st, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        HIP_TRY(c0, hipStreamBeginCapture(c0->cap_st, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < gb; ++i)
            for (int s = 0; s < nsys; ++s) batch_iter(ctxs[s], c0->cap_st, i & 1, tol);
        HIP_TRY(c0, hipStreamEndCapture(c0->cap_st, &graph));
        hipError_t ge = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ge != hipSuccess) return fail(c0, LSQR_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ge));
        while (!stopped && iters - done >= gb) {
            hipError_t le = hipGraphLaunch(exec, st);
            if (le != hipSuccess) {
                (void)hipGraphExecDestroy(exec);
                return fail(c0, LSQR_E_DEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(le));
            }
            done += gb;
            if (tol > 0.0 && done < iters && (e = poll()) != LSQR_OK) { (void)hipGraphExecDestroy(exec); return e; }
        }
        (void)hipStreamSynchronize(st);
        (void)hipGraphExecDestroy(exec);
    }
    while (!stopped && done < iters) {
        for (int s = 0; s < nsys; ++s) batch_iter(ctxs[s], st, done & 1, tol);
        ++done;
        if (tol > 0.0 && done % c0->check_every == 0 && done < iters && (e = poll()) != LSQR_OK) return e;
    }
    for (int s = 0; s < nsys; ++s) {
        lsqr_ctx *c = ctxs[s];
        BatchEngine &B = c->beng;
        BArgs a = base_args(c, B);
        a.Y = B.Y; a.tol = tol; a.part_in = B.P3; a.np_in = B.g_upd;
        hipLaunchKernelGGL(k_bfinal, dim3(cap(c->P.n * R, kBlock, 1024)), dim3(kBlock), 0, st, a, B.dm);
    }
    HIP_TRY(c0, hipGetLastError());
    return LSQR_OK;
}

// The state rows of system c's last batch run: per right-hand side r <
// nrhs its stop reason, the last iteration it advanced (klast) and the rows
// hs [(kdone + 1)][R][kStateWords]; err |= the device error flag.
lsqr_status batch_state(lsqr_ctx *c0, lsqr_ctx *c, int nrhs, int &err, std::vector<int> &why,
                        std::vector<int> &klast, std::vector<double> &hs, int &kdone)
{
    BatchEngine &B = c->beng;
    const int R = B.R;
    int ctl[C_WORDS];
    why.assign((size_t)R, 0);
    klast.assign((size_t)nrhs, 0);
    HIP_TRY(c0, hipMemcpy(ctl, B.ctl, sizeof(ctl), hipMemcpyDeviceToHost));
    HIP_TRY(c0, hipMemcpy(why.data(), B.why, R * sizeof(int), hipMemcpyDeviceToHost));
    kdone = ctl[C_ITERS];
    err |= ctl[C_ERR];
    hs.assign((size_t)(kdone + 1) * R * kStateWords, 0.0);
    HIP_TRY(c0, hipMemcpy(hs.data(), B.S, hs.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int r = 0; r < nrhs; ++r) {
        int kl = 0;
        for (int k = 1; k <= kdone; ++k) {
            const double *Sk = hs.data() + ((size_t)k * R + r) * kStateWords;
            const double *Sp = hs.data() + ((size_t)(k - 1) * R + r) * kStateWords;
            if (Sk[S_PHIBAR] != Sp[S_PHIBAR] || Sk[S_PSI] != Sp[S_PSI]) kl = k;
        }
        if (why[r] == 0) kl = 0;
        if (why[r] == 2) kl = kdone;
        klast[(size_t)r] = kl;
    }
    return LSQR_OK;
}

// FP64 refinement scratch of a context (allocated on first use).
lsqr_status ensure_refine_buffers(lsqr_ctx *c)
{
    const int64_t m = c->P.m, n = c->P.n, mb = m + 2 * n;
    if (!c->xbuf) c->xbuf = ctx_alloc<double>(c, n);
    if (!c->rbar) c->rbar = ctx_alloc<double>(c, mb);
    if (!c->gbuf) c->gbuf = ctx_alloc<double>(c, n);
    if (!c->fbuf) c->fbuf = ctx_alloc<double>(c, mb);
    BatchEngine &B = c->beng;
    if (!B.X) B.X = ctx_alloc<double>(c, n * B.R);
    if (!B.F) B.F = ctx_alloc<double>(c, mb * B.R);
    if (!B.rsum) B.rsum = ctx_alloc<double>(c, (size_t)4 * B.R);
    if (!c->xbuf || !c->rbar || !c->gbuf || !c->fbuf || !B.X || !B.F || !B.rsum)
        return fail(c, LSQR_E_OOM, "device allocation failed");
    return LSQR_OK;
}

}  // namespace

extern "C" {

lsqr_status lsqr_solve_batched(lsqr_ctx *const *ctxs, int nsys, int nrhs, const double *const *dt,
                               lsqr_mem vec_mem, int iters, double tol, double *const *dm,
                               double *const *res_hist, lsqr_info *info)
{
    lsqr_status e = batch_args(ctxs, nsys, nrhs, dt, vec_mem, iters, tol, dm);
    if (e != LSQR_OK) return e;
    lsqr_ctx *c0 = ctxs[0];
    DeviceGuard dg(c0->device);
    hipStream_t st = c0->st;
    const int R = pow2_at_least(nrhs);
    const hipMemcpyKind kout = vec_mem == LSQR_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    // the batch runs on the first context's stream, after each context's own work
    for (int s = 1; s < nsys; ++s)
        if (ctxs[s]->st != st) HIP_TRY(c0, hipStreamSynchronize(ctxs[s]->st));
    if ((e = batch_load_rhs(ctxs, nsys, nrhs, R, dt, vec_mem, iters)) != LSQR_OK) return e;
    if ((e = batch_run(ctxs, nsys, nrhs, R, iters, tol, false)) != LSQR_OK) return e;
    for (int s = 0; s < nsys; ++s) {
        lsqr_ctx *c = ctxs[s];
        HIP_TRY(c0, hipMemcpy2DAsync(dm[s], nrhs * sizeof(double), c->beng.dm, R * sizeof(double),
                                     nrhs * sizeof(double), c->P.n, kout, st));
    }
    HIP_TRY(c0, hipGetLastError());
    HIP_TRY(c0, hipStreamSynchronize(st));
    int err = 0;
    for (int s = 0; s < nsys; ++s) {
        lsqr_ctx *c = ctxs[s];
        std::vector<int> why, klast;
        std::vector<double> hs;
        int kdone = 0;
        if ((e = batch_state(c0, c, nrhs, err, why, klast, hs, kdone)) != LSQR_OK) return e;
        for (int r = 0; r < nrhs; ++r) {
            const int kl = klast[(size_t)r];
            if (res_hist && res_hist[s]) {
                double *h = res_hist[s];
                for (int k = 0; k <= iters; ++k)
                    for (int f = 0; f < 3; ++f) h[((size_t)k * nrhs + r) * 3 + f] = NAN;
                for (int k = 0; k <= kl; ++k) {
                    const double *Sk = hs.data() + ((size_t)k * R + r) * kStateWords;
                    double *o = h + ((size_t)k * nrhs + r) * 3;
                    if (why[r] == 0) { o[0] = Sk[S_BETA]; o[1] = 0.0; o[2] = 0.0; break; }
                    o[0] = Sk[S_PHIBAR]; o[1] = Sk[S_PSI]; o[2] = Sk[S_ETA];
                }
            }
            if (info) {
                lsqr_info &I = info[(size_t)s * nrhs + r];
                const double *Sk = hs.data() + ((size_t)kl * R + r) * kStateWords;
                I.istop = why[r];
                I.iters = kl;
                I.sweeps = 0;
                I.fallback_used = c->fallback_used;
                I.inner_fp32 = 0;
                I.eta = why[r] == 0 ? 0.0 : Sk[S_ETA];
                I.phibar = why[r] == 0 ? Sk[S_BETA] : Sk[S_PHIBAR];
                I.eta_final_fp64 = NAN;
            }
        }
    }
    if (err) return fail(c0, LSQR_E_NONFINITE, "a solver scalar became non-finite");
    return LSQR_OK;
}

lsqr_status lsqr_solve_batched_refined(lsqr_ctx *const *ctxs, int nsys, int nrhs,
                                       const double *const *dt, lsqr_mem vec_mem, int iters,
                                       double tol, double inner_tol, int sweeps,
                                       double *const *dm, lsqr_info *info)
{
    lsqr_status e = batch_args(ctxs, nsys, nrhs, dt, vec_mem, iters, tol, dm);
    if (e != LSQR_OK) return e;
    lsqr_ctx *c0 = ctxs[0];
    if (!(tol > 0.0)) return fail(c0, LSQR_E_INVALID_ARG, "the refined batch needs tol > 0");
    if (!(inner_tol >= 0.0 && inner_tol < 1.0))
        return fail(c0, LSQR_E_INVALID_ARG, "inner_tol must be in [0, 1)");
    if (sweeps < 1) return fail(c0, LSQR_E_INVALID_ARG, "sweeps must be >= 1");
    for (int s = 0; s < nsys; ++s)
        if (!(ctxs[s]->P.damp > 0.0))
            return fail(c0, LSQR_E_UNSUPPORTED, "the refinement needs damp > 0 (its correction goes into the damping block)");
    DeviceGuard dg(c0->device);
    hipStream_t st = c0->st;
    const int R = pow2_at_least(nrhs);
    const hipMemcpyKind kout = vec_mem == LSQR_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    for (int s = 1; s < nsys; ++s)
        if (ctxs[s]->st != st) HIP_TRY(c0, hipStreamSynchronize(ctxs[s]->st));
    if ((e = batch_load_rhs(ctxs, nsys, nrhs, R, dt, vec_mem, iters)) != LSQR_OK) return e;
    // per system and right-hand side: |Abar^T bbar|, eta, stop reason, work
    const size_t NR = (size_t)nsys * nrhs;
    std::vector<double> arnorm(NR, 0.0), eta(NR, INFINITY), eta_prev(NR, INFINITY), rn(NR, 0.0);
    std::vector<int> istop(NR, 2), total(NR, 0), nsw(NR, 0), live(NR, 1);
    std::vector<double> hsum((size_t)4 * R);
    for (int s = 0; s < nsys; ++s) {
        lsqr_ctx *c = ctxs[s];
        if ((e = ensure_refine_buffers(c)) != LSQR_OK) return fail(c0, e, c->err);
        BatchEngine &B = c->beng;
        const Problem &P = c->P;
        const int gadj = std::min(2048, c->eng.g_adj);
        launch_fill(st, P.n * R, 0.0, B.X);
        launch_fill(st, (P.m + 2 * P.n) * R, 0.0, B.F);
        for (int r = 0; r < nrhs; ++r) {
            if (P.m > 0)
                hipLaunchKernelGGL(k_col_get, dim3(grid_for(P.m)), dim3(256), 0, st, P.m, R, r, B.rhs, c->dtbuf);
            launch_adj(st, P, gadj, VT_F64, c->C64, c->ones, nullptr, c->dtbuf, nullptr, c->gbuf, c->Pa,
                       nullptr, 0, nullptr, nullptr, 0, MODE_OPERATOR, 1);
            launch_sum_partials(st, c->Pa, gadj, B.rsum + 4 * r);
        }
        HIP_TRY(c0, hipMemcpyAsync(hsum.data(), B.rsum, 4 * R * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(c0, hipStreamSynchronize(st));
        for (int r = 0; r < nrhs; ++r) {
            const size_t k = (size_t)s * nrhs + r;
            arnorm[k] = sqrt(hsum[4 * (size_t)r]);
            if (!(arnorm[k] > 0.0)) { istop[k] = 0; live[k] = 0; eta[k] = 0.0; }
        }
    }
    for (int sw = 0;; ++sw) {
        // FP64 residual of every live right-hand side and the next inner
        // right-hand side f = [0; 0; (Abar^T rbar) / damp] (refine.hip)
        for (int s = 0; s < nsys; ++s) {
            lsqr_ctx *c = ctxs[s];
            BatchEngine &B = c->beng;
            const Problem &P = c->P;
            const int64_t mb = P.m + 2 * P.n;
            const int gadj = std::min(2048, c->eng.g_adj);
            for (int r = 0; r < nrhs; ++r) {
                const size_t k = (size_t)s * nrhs + r;
                if (!live[k]) {
                    hipLaunchKernelGGL(k_col_put, dim3(grid_for(mb)), dim3(256), 0, st, mb, R, r,
                                       (const double *)nullptr, B.F);
                    continue;
                }
                if (P.m > 0)
                    hipLaunchKernelGGL(k_col_get, dim3(grid_for(P.m)), dim3(256), 0, st, P.m, R, r, B.rhs, c->dtbuf);
                if (sw > 0) {
                    hipLaunchKernelGGL(k_col_get, dim3(grid_for(P.n)), dim3(256), 0, st, P.n, R, r, B.X, c->xbuf);
                    launch_fwd(st, P, c->eng.g_fwd, VT_F64, c->R64, c->xbuf, nullptr, c->ybuf, nullptr,
                               c->Pf, nullptr, 0, nullptr, nullptr, 0, 0.0, MODE_OPERATOR);
                }
                launch_residual(st, P, c->g_ref, c->dtbuf, sw > 0 ? c->ybuf : nullptr, c->rbar, c->Pr);
                launch_sum_partials(st, c->Pr, c->g_ref, B.rsum + 4 * r + 1);
                launch_adj(st, P, gadj, VT_F64, c->C64, c->ones, nullptr, c->rbar, nullptr, c->gbuf,
                           c->Pa, nullptr, 0, nullptr, nullptr, 0, MODE_OPERATOR, 1);
                launch_normal_rhs(st, P, c->g_ref, c->rbar, c->gbuf, c->fbuf, c->Pr);
                launch_sum_partials(st, c->Pr, c->g_ref, B.rsum + 4 * r + 2);
                hipLaunchKernelGGL(k_col_put, dim3(grid_for(mb)), dim3(256), 0, st, mb, R, r,
                                   (const double *)c->fbuf, B.F);
            }
            HIP_TRY(c0, hipGetLastError());
            HIP_TRY(c0, hipMemcpyAsync(hsum.data(), B.rsum, 4 * R * sizeof(double), hipMemcpyDeviceToHost, st));
            HIP_TRY(c0, hipStreamSynchronize(st));
            for (int r = 0; r < nrhs; ++r) {
                const size_t k = (size_t)s * nrhs + r;
                if (!live[k]) continue;
                rn[k] = sqrt(hsum[4 * (size_t)r + 1]);
                eta[k] = sqrt(hsum[4 * (size_t)r + 2]) / arnorm[k];
                if (!isfinite(eta[k])) return fail(c0, LSQR_E_NONFINITE, "refinement residual became non-finite");
                if (eta[k] <= tol) { istop[k] = 1; live[k] = 0; }
                else if (sw >= sweeps) { istop[k] = 2; live[k] = 0; }
                else if (sw > 0 && eta[k] > 0.5 * eta_prev[k]) { istop[k] = 4; live[k] = 0; }
                if (!live[k])          // no further correction for it
                    hipLaunchKernelGGL(k_col_put, dim3(grid_for(mb)), dim3(256), 0, st, mb, R, r,
                                       (const double *)nullptr, B.F);
                eta_prev[k] = eta[k];
            }
        }
        int any = 0;
        for (size_t k = 0; k < NR; ++k) any |= live[k];
        if (!any) break;
        // inner batched LSQR on (Ahat D, f) for every right-hand side; x += D y
        if ((e = batch_run(ctxs, nsys, nrhs, R, iters, inner_tol, true)) != LSQR_OK) return e;
        int err = 0;
        for (int s = 0; s < nsys; ++s) {
            lsqr_ctx *c = ctxs[s];
            BatchEngine &B = c->beng;
            hipLaunchKernelGGL(k_blk_add, dim3(grid_for(c->P.n * R)), dim3(256), 0, st,
                               c->P.n * (int64_t)R, (const double *)B.dm, B.X);
            std::vector<int> why, klast;
            std::vector<double> hs;
            int kdone = 0;
            if ((e = batch_state(c0, c, nrhs, err, why, klast, hs, kdone)) != LSQR_OK) return e;
            for (int r = 0; r < nrhs; ++r) {
                const size_t k = (size_t)s * nrhs + r;
                if (!live[k]) continue;
                total[k] += klast[(size_t)r];
                nsw[k] += 1;
            }
        }
        if (err) return fail(c0, LSQR_E_NONFINITE, "a solver scalar became non-finite");
    }
    for (int s = 0; s < nsys; ++s) {
        lsqr_ctx *c = ctxs[s];
        HIP_TRY(c0, hipMemcpy2DAsync(dm[s], nrhs * sizeof(double), c->beng.X, R * sizeof(double),
                                     nrhs * sizeof(double), c->P.n, kout, st));
    }
    HIP_TRY(c0, hipGetLastError());
    HIP_TRY(c0, hipStreamSynchronize(st));
    if (info)
        for (size_t k = 0; k < NR; ++k) {
            lsqr_info &I = info[k];
            I.istop = istop[k];
            I.iters = total[k];
            I.sweeps = nsw[k];
            I.fallback_used = ctxs[k / nrhs]->fallback_used;
            I.inner_fp32 = 0;
            I.eta = eta[k];
            I.phibar = rn[k];
            I.eta_final_fp64 = eta[k];
        }
    return LSQR_OK;
}

lsqr_status lsqr_apply_block(lsqr_ctx *c, int nrhs, const float *x, float *y)
{
    if (!c) return fail(nullptr, LSQR_E_INVALID_ARG, "ctx is NULL");
    if (!x || !y) return fail(c, LSQR_E_INVALID_ARG, "x and y must not be NULL");
    if (nrhs < 1 || nrhs > kMaxRhs || (nrhs & (nrhs - 1)))
        return fail(c, LSQR_E_INVALID_ARG, "nrhs must be a power of two <= 32");
    DeviceGuard dg(c->device);
    lsqr_status e = ensure_batch(c, c->st, nrhs, 1);
    if (e != LSQR_OK) return e;
    BatchEngine &B = c->beng;
    BArgs a = base_args(c, B);
    a.mode = MODE_OPERATOR; a.Z = x; a.Tcur = y; a.part_out = B.P1;
    launch_tiled(c->st, 1, B.g_fwd, a, B.R, B.rt);
    HIP_TRY(c, hipGetLastError());
    return LSQR_OK;
}

lsqr_status lsqr_apply_t_block(lsqr_ctx *c, int nrhs, const float *y, float *x)
{
    if (!c) return fail(nullptr, LSQR_E_INVALID_ARG, "ctx is NULL");
    if (!x || !y) return fail(c, LSQR_E_INVALID_ARG, "x and y must not be NULL");
    if (nrhs < 1 || nrhs > kMaxRhs || (nrhs & (nrhs - 1)))
        return fail(c, LSQR_E_INVALID_ARG, "nrhs must be a power of two <= 32");
    if (nrhs >= 4 && ((uintptr_t)y & 15u))                // rows of y are read as 16-byte vectors
        return fail(c, LSQR_E_INVALID_ARG, "y must be 16-byte aligned when nrhs >= 4");
    DeviceGuard dg(c->device);
    lsqr_status e = ensure_batch(c, c->st, nrhs, 1);
    if (e != LSQR_OK) return e;
    BatchEngine &B = c->beng;
    BArgs a = base_args(c, B);
    a.mode = MODE_OPERATOR; a.Tcur = const_cast<float *>(y); a.Q = x; a.part_out = B.P2;
    launch_tiled(c->st, 2, B.g_adj, a, B.R, B.rt);
    HIP_TRY(c, hipGetLastError());
    return LSQR_OK;
}

lsqr_status lsqr_set_batch_config(lsqr_ctx *c, const lsqr_batch_cfg *cfg)
{
    if (!c || !cfg) return fail(c, LSQR_E_INVALID_ARG, "ctx and cfg must not be NULL");
    const int rt = cfg->rhs_tile, g = cfg->grid;
    if (rt < 1 || rt > kMaxRhs || (rt & (rt - 1)) || g < 1 || g > 2048)
        return fail(c, LSQR_E_INVALID_ARG, "rhs_tile must be a power of two <= 32, grid in 1..2048");
    c->beng.rt = rt;
    c->beng.grid = g;
    c->beng.tuned = 1;
    return LSQR_OK;
}

lsqr_status lsqr_autotune_batched(lsqr_ctx *c, int nrhs, int probe_iters, lsqr_batch_cfg *best)
{
    if (!c || !best) return fail(c, LSQR_E_INVALID_ARG, "ctx and best must not be NULL");
    if (nrhs < 1 || nrhs > kMaxRhs) return fail(c, LSQR_E_INVALID_ARG, "nrhs must be in 1..32");
    if (probe_iters < 2) probe_iters = 2;
    DeviceGuard dg(c->device);
    const int R = pow2_at_least(nrhs);
    hipStream_t st = c->st;
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    lsqr_batch_cfg top{0, 0, INFINITY};
    const int tiles[] = {8, 16, 32};
    const int grids[] = {256, 512, 1024, 2048};
    for (int rt : tiles) {
        if (rt > R) continue;
        for (int g : grids) {
            BatchEngine &B = c->beng;
            B.rt = rt;
            B.grid = g;
            B.tuned = 1;
            lsqr_status e = ensure_batch(c, st, R, probe_iters);
            if (e != LSQR_OK) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); return e; }
            launch_fill(st, std::max<int64_t>(c->P.m, 1) * R, 1.0, B.rhs);
            std::vector<float> ms;
            for (int rep = 0; rep < 5; ++rep) {
                batch_init(c, st, 0.0);
                hipLaunchKernelGGL(k_set_kmax, dim3(1), dim3(1), 0, st, B.ctl, probe_iters);
                (void)hipEventRecord(e0, st);
                for (int i = 0; i < probe_iters; ++i) batch_iter(c, st, i & 1, 0.0);
                (void)hipEventRecord(e1, st);
                HIP_TRY(c, hipEventSynchronize(e1));
                float t = 0.f;
                HIP_TRY(c, hipEventElapsedTime(&t, e0, e1));
                ms.push_back(t / (float)probe_iters);
            }
            std::sort(ms.begin(), ms.end());
            const double med = ms[ms.size() / 2];
            if (med < top.ms_per_iter) top = lsqr_batch_cfg{rt, g, med};
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->beng.rt = top.rhs_tile;
    c->beng.grid = top.grid;
    c->beng.tuned = 1;
    lsqr_status e = ensure_batch(c, st, R, 1);
    if (e != LSQR_OK) return e;
    *best = top;
    return LSQR_OK;
}

}  // extern "C"
