// Batched LSQR kernels: R right-hand sides of one system advance together.
//
// Vectors are row-major blocks [rows][R] (FP32), so the R values one stored
// entry multiplies are one contiguous segment: a wave covers 64/RT entries x
// RT right-hand sides per step (RT = RHS tile: 8, 16 or 32) and reads the
// matrix once per tile instead of once per right-hand side.  Every right-hand
// side keeps its own FP64 LSQR scalars in a state row S[k][r]; per-RHS partial
// sums [workgroup][R] are reduced in a fixed order by every consumer
// workgroup, as in the single-RHS kernels (no atomics).  A right-hand side
// whose eta reaches the tolerance (or that breaks down) is frozen: its
// products are still formed but its x, w, v no longer change.
//
// R is a power of two <= 32 (the host pads with zero right-hand sides), so R
// divides the workgroup size and thread t always owns right-hand side t % R
// in every grid-stride loop over (row, rhs) pairs.
#pragma once

#include "lsqr_kernels.cuh"

namespace lsqr {

constexpr int kMaxRhs = 32;
constexpr int kMaxNzBatched = 32;      // node-run block products: depths per node

// Stored entries per lane in flight in the batched products.
#ifndef LSQR_BATCH_UNROLL
#define LSQR_BATCH_UNROLL 8
#endif
constexpr int kBatchUnroll = LSQR_BATCH_UNROLL;



struct BArgs {
    // operator (FP32 values)
    const int64_t *rp;
    const int32_t *ci;
    const float *va;
    const int64_t *cp;
    const int32_t *ri;
    const float *cv;
    // node runs of the data block (k_badj_nruns; nval in node-major run order)
    const int64_t *nrp;
    const int64_t *nvq;
    const uint32_t *nrow;
    const uint16_t *ndesc;
    const int32_t *norder;
    const float *nval;
    // two-phase forward product over the node runs: per-run partial rows Pr
    // (k_bfwd_pr, a workgroup per node), then per-row sums over the row's runs
    // rrid[rrp[i] .. rrp[i+1]) (k_bfwd); Pr == nullptr: entry-wise CSR
    const int64_t *rrp;
    const uint32_t *rrid;
    float *Pr;              // [node runs][R]
    int g_pr;               // workgroups of k_bfwd_pr
    const double *d;
    int64_t m;
    int n, nx, ny, nz;
    double w, damp;
    int R;                  // right-hand sides (power of two <= 32)
    // vectors (row-major [rows][R])
    const float *Z;         // D v   [n][R]
    const float *Tprev;     // [m+2n][R]
    float *Tcur;            // [m+2n][R]
    float *V;               // [n][R]
    float *Q;               // [n][R]
    double *W, *Y;          // [n][R]
    float *Zout;            // [n][R]
    const double *rhs;      // [m][R] FP64 (init); [m+2n][R] with rhs_full
    int rhs_full;           // 1: rhs holds every block of the right-hand side
    // partials [workgroup][R]
    double *part_out;
    const double *part_in;
    int np_in;
    double *S;              // [(K+2)][R][kStateWords]
    int *act;               // [R] 1 active, 0 frozen
    int *why;               // [R] stop reason
    int *ctl;               // counters, kmax, error flag
    int parity;
    int mode;
    double tol;
    int r0;                 // first right-hand side of this launch's tile
};

__device__ __forceinline__ double *srow(const BArgs &a, int k, int r)
{
    return a.S + ((int64_t)k * a.R + r) * kStateWords;
}

// out[r] = sum over b < np of p[b][r], for every r < R, in a fixed order; all
// threads take part.  accs has kBlock entries.
__device__ __forceinline__ void sum_rhs_all(const double *p, int np, int R, double *accs,
                                            double *out)
{
    const int r = threadIdx.x % R, slot = threadIdx.x / R, per = kBlock / R;
    double acc = 0.0;
    for (int b = slot; b < np; b += per) acc += p[(int64_t)b * R + r];
    accs[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < R) {
        double s = 0.0;
        for (int q = 0; q < per; ++q) s += accs[q * R + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// Per-RHS sum of one value per thread (thread t holds right-hand side
// t % RR, RR divides 64); result in out[0..RR), fixed order.
template <int RR>
__device__ __forceinline__ void block_sum_rhs(double v, double *accs, double *out)
{
#pragma unroll
    for (int off = RR; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane < RR) accs[wid * RR + lane] = v;
    __syncthreads();
    if (threadIdx.x < RR) {
        const int r = threadIdx.x;
        out[r] = ((accs[r] + accs[RR + r]) + accs[2 * RR + r]) + accs[3 * RR + r];
    }
    __syncthreads();
}

// ----------------------------------------------------------------- init --
// T0 = [rhs; 0; 0] (or the full rhs) for the tile's right-hand sides, y = v =
// 0, partials of |b|^2.
template <int RT>
__global__ __launch_bounds__(kBlock) void k_binit(BArgs a)
{
    __shared__ double accs[kBlock];
    __shared__ double res[kMaxRhs];
    const int64_t mb = a.m + 2 * (int64_t)a.n;
    const int rr = threadIdx.x % RT, c = a.r0 + rr;
    double sq = 0.0;
    for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < mb * RT;
         idx += (int64_t)gridDim.x * kBlock) {
        const int64_t i = idx / RT;
        const double b = (a.rhs_full || i < a.m) ? a.rhs[i * a.R + c] : 0.0;
        a.Tcur[i * a.R + c] = (float)b;
        sq += b * b;
        if (i < a.n) { a.Y[i * a.R + c] = 0.0; a.V[i * a.R + c] = 0.0f; }
    }
    block_sum_rhs<RT>(sq, accs, res);
    if (threadIdx.x < RT) a.part_out[(int64_t)blockIdx.x * a.R + a.r0 + threadIdx.x] = res[threadIdx.x];
    if (blockIdx.x == 0 && threadIdx.x < RT) {
        a.act[a.r0 + threadIdx.x] = 1;
        a.why[a.r0 + threadIdx.x] = 2;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.r0 == 0) {
        a.ctl[C_STOP] = 0; a.ctl[C_ISTOP] = 2; a.ctl[C_ITERS] = 0; a.ctl[C_ERR] = 0;
        a.ctl[C_CNT0] = 1; a.ctl[C_CNT1] = 0;
    }
}

// --------------------------------------------------------------- forward --
// T = A_D V - U diag(alpha) with U = Tprev diag(1/beta), for the tile.
template <int RT>
__global__ __launch_bounds__(kBlock) void k_bfwd(BArgs a)
{
#pragma clang fp contract(off)
    __shared__ double accs[kBlock];
    __shared__ double res[kMaxRhs];
    __shared__ double vns[kMaxRhs];
    __shared__ double sal[kMaxRhs], sbe[kMaxRhs];
    const bool op = a.mode == MODE_OPERATOR;       // plain product: alpha = 0, no state
    const int k = op ? 0 : a.ctl[C_CNT0 + a.parity];
    if (!op && k > a.ctl[C_KMAX]) return;
    if (op) {
        if (threadIdx.x < RT) { sal[threadIdx.x] = 0.0; sbe[threadIdx.x] = 1.0; }
    } else {
        sum_rhs_all(a.part_in, a.np_in, a.R, accs, vns);
    }
    if (!op && threadIdx.x < RT) {
        const int r = a.r0 + threadIdx.x;
        const double *Sp = srow(a, k - 1, r);
        sal[threadIdx.x] = Sp[S_ALPHA];
        sbe[threadIdx.x] = Sp[S_BETA];
        if (blockIdx.x == 0) {
            // eta of the previous step and the per-RHS stop rules
            const double vn = sqrt(vns[r]);
            double *S0 = srow(a, 0, r);
            if (k == 1) {
                S0[S_ARNORM0] = (S0[S_ALPHA] * S0[S_BETA]) * vn;
                S0[S_VNORM] = vn;
            } else {
                double *Sw = srow(a, k - 1, r);
                const double eta = Sp[S_PSI] * vn / S0[S_ARNORM0];
                Sw[S_ETA] = eta;
                Sw[S_VNORM] = vn;
                if (a.act[r]) {
                    if (a.tol > 0.0 && eta <= a.tol) { a.act[r] = 0; a.why[r] = 1; }
                    else if (Sp[S_ALPHA] == 0.0 || Sp[S_BETA] == 0.0) { a.act[r] = 0; a.why[r] = 3; }
                }
            }
        }
    }
    __syncthreads();
    constexpr int EPW = 64 / RT;
    const int lane = threadIdx.x & 63, er = lane / RT, rr = lane % RT;
    const double alpha = sal[rr], beta = sbe[rr] > 0.0 ? sbe[rr] : 1.0;
    const int R = a.R, cofs = a.r0 + rr;
    double sq = 0.0;
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t row = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); row < a.m;
         row += nwaves) {
        float ac[kBatchUnroll];
#pragma unroll
        for (int u = 0; u < kBatchUnroll; ++u) ac[u] = 0.f;
        if (a.Pr) {
            // sums of the row's per-run partials, in the order of its entries
            const int64_t s = a.rrp[row], e = a.rrp[row + 1];
            int64_t p = s + er;
            for (; p + (kBatchUnroll - 1) * EPW < e; p += kBatchUnroll * EPW) {
                uint32_t q[kBatchUnroll];
#pragma unroll
                for (int u = 0; u < kBatchUnroll; ++u) q[u] = __builtin_nontemporal_load(a.rrid + p + u * EPW);
#pragma unroll
                for (int u = 0; u < kBatchUnroll; ++u)
                    ac[u] += __builtin_nontemporal_load(a.Pr + (int64_t)q[u] * R + cofs);
            }
            for (; p < e; p += EPW)
                ac[0] += __builtin_nontemporal_load(
                    a.Pr + (int64_t)__builtin_nontemporal_load(a.rrid + p) * R + cofs);
        } else {
            const int64_t s = a.rp[row], e = a.rp[row + 1];
            int64_t p = s + er;
            for (; p + (kBatchUnroll - 1) * EPW < e; p += kBatchUnroll * EPW) {
                float g[kBatchUnroll];
                int c[kBatchUnroll];
#pragma unroll
                for (int u = 0; u < kBatchUnroll; ++u) {
                    g[u] = __builtin_nontemporal_load(a.va + p + u * EPW);
                    c[u] = __builtin_nontemporal_load(a.ci + p + u * EPW);
                }
#pragma unroll
                for (int u = 0; u < kBatchUnroll; ++u)
                    ac[u] = fmaf(g[u], a.Z[(int64_t)c[u] * R + cofs], ac[u]);
            }
            for (; p < e; p += EPW)
                ac[0] = fmaf(__builtin_nontemporal_load(a.va + p),
                             a.Z[(int64_t)__builtin_nontemporal_load(a.ci + p) * R + cofs], ac[0]);
        }
        float acc = tree_sum<kBatchUnroll>(ac);
#pragma unroll
        for (int off = RT; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
        if (er == 0) {
            const double u = op ? 0.0 : (double)a.Tprev[row * R + cofs] / beta;
            const float t = (float)((double)acc - alpha * u);
            a.Tcur[row * R + cofs] = t;
            sq += (double)t * (double)t;
        }
    }
    // smoothing and damping rows: one thread per (row, rhs)
    const int64_t nreg = 2 * (int64_t)a.n;
    for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < nreg * RT;
         idx += (int64_t)gridDim.x * kBlock) {
        const int64_t r = idx / RT;
        float yv;
        if (r < a.n) {
            const int pp = (int)r;
            const int iz = pp % a.nz, ixy = pp / a.nz, ix = ixy % a.nx, iy = ixy / a.nx;
            const int sxy = a.nx * a.nz;
            float acc = 0.f;
            int deg = 0;
            if (ix > 0) { acc += a.Z[(int64_t)(pp - a.nz) * R + cofs]; ++deg; }
            if (ix < a.nx - 1) { acc += a.Z[(int64_t)(pp + a.nz) * R + cofs]; ++deg; }
            if (iy > 0) { acc += a.Z[(int64_t)(pp - sxy) * R + cofs]; ++deg; }
            if (iy < a.ny - 1) { acc += a.Z[(int64_t)(pp + sxy) * R + cofs]; ++deg; }
            if (iz > 0) { acc += a.Z[(int64_t)(pp - 1) * R + cofs]; ++deg; }
            if (iz < a.nz - 1) { acc += a.Z[(int64_t)(pp + 1) * R + cofs]; ++deg; }
            yv = (acc - (float)deg * a.Z[(int64_t)pp * R + cofs]) * (float)a.w;
        } else {
            yv = (float)a.damp * a.Z[(r - a.n) * R + cofs];
        }
        const int64_t row = a.m + r;
        const double u = op ? 0.0 : (double)a.Tprev[row * R + cofs] / beta;
        const float t = (float)((double)yv - alpha * u);
        a.Tcur[row * R + cofs] = t;
        sq += (double)t * (double)t;
    }
    block_sum_rhs<RT>(sq, accs, res);
    if (threadIdx.x < RT) a.part_out[(int64_t)blockIdx.x * a.R + a.r0 + threadIdx.x] = res[threadIdx.x];
}

// First phase of the two-phase forward block product (32-wide tiles): for
// every node run (row i, depths iz0 .. iz0+len-1 of lateral node k) the
// partial row Pr[run, c] = sum_e val_e Z[k nz + iz0 + e, c] over the tile's
// 32 right-hand sides.  Per node this is a dense product: the node's runs as
// rows of a [runs x 32] matrix (run r holds its values at depths iz0 ..
// iz0+len-1, zeros elsewhere; nz <= 32) times the node's [32 x 32] block of
// Z, done on the matrix cores with v_mfma_f32_32x32x2f32, 32 runs by 32
// right-hand sides per product, 16 products over the depth pairs.  A
// workgroup per node (decreasing work, boustrophedon, as the transposed
// product); its 4 waves take fixed quarters of the node's runs, stage the
// values of 64 runs at a time in their own LDS area (all loads in flight
// together) and keep the node's Z block as the B operand in registers.  The
// Z gathers fall from one per stored entry to one per (node, depth).
typedef float floatx16 __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(kBlock) void k_bfwd_pr32(BArgs a)
{
    if (a.mode == MODE_ITER) {
        const int k = a.ctl[C_CNT0 + a.parity];
        if (k > a.ctl[C_KMAX]) return;
    }
    constexpr int kStage = 16;                     // value loads per lane in flight
    __shared__ float vs[kBlock / 64][64 * kMaxNzBatched];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int hi = lane >> 5, j = lane & 31;       // MFMA operand row/column roles
    const int R = a.R, nz = a.nz, nnodes = a.n / nz, G = gridDim.x;
    float *my = vs[wid];
    for (int s = 0; s * G < nnodes; ++s) {
        const int idx = s * G + ((s & 1) ? G - 1 - (int)blockIdx.x : (int)blockIdx.x);
        if (idx >= nnodes) continue;                        // uniform over the workgroup
        const int node = a.norder[idx];
        // B operand of product t: Z[node nz + 2t + hi][r0 + j] (zero past nz)
        float zb[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int k = 2 * t + hi;
            zb[t] = k < nz ? a.Z[((int64_t)node * nz + k) * R + a.r0 + j] : 0.f;
        }
        const int64_t rs0 = a.nrp[node], cnt = a.nrp[node + 1] - rs0;
        const int64_t rs = rs0 + cnt * wid / 4, re = rs0 + cnt * (wid + 1) / 4;
        int64_t vb = a.nvq[4 * (int64_t)node + wid];
        for (int64_t base = rs; base < re; base += 64) {
            const int nr = (int)(re - base < 64 ? re - base : 64);
            // every lane loads (lanes past the chunk its last run, masked
            // here), so the load does not sit under a divergent branch
            uint32_t dsc = __builtin_nontemporal_load(a.ndesc + base + (lane < nr ? lane : nr - 1));
            dsc = lane < nr ? dsc : 0u;
            const int len = (int)(dsc & 255u);
            int incl = len;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o);
                if (lane >= o) incl += y;
            }
            // (value offset in the chunk << 16) | (iz0 << 8) | len; offsets < 64 * 64
            const uint32_t pk = ((uint32_t)(incl - len) << 16) | dsc;
            const int tot = __shfl(incl, 63);               // >= 1: runs are not empty
            // the chunk's values into the wave's LDS area, kStage loads per
            // lane in flight (slots past the end read the last value, in
            // bounds, and are not stored); the previous chunk's reads first
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int i0 = 0; i0 < tot; i0 += 64 * kStage) {
                float t[kStage];
#pragma unroll
                for (int k = 0; k < kStage; ++k) {
                    const int i = i0 + 64 * k + lane;
                    t[k] = __builtin_nontemporal_load(a.nval + vb + (i < tot ? i : tot - 1));
                }
                // slots past the end store the last value again (same value,
                // same slot): no branch for the compiler to sink the loads into
#pragma unroll
                for (int k = 0; k < kStage; ++k) {
                    const int i = i0 + 64 * k + lane;
                    my[i < tot ? i : tot - 1] = t[k];
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int blk = 0; blk < nr; blk += 32) {
                // A operand of product t: row j = run blk + j, column 2t + hi
                const int r = blk + j;
                const uint32_t p = __shfl(pk, r & 63);
                const int rlen = r < nr ? (int)(p & 255u) : 0;
                const int iz0 = (int)((p >> 8) & 255u);
                const int voff = (int)(p >> 16);
                floatx16 acc = {};
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const int e = 2 * t + hi - iz0;
                    const bool in = (unsigned)e < (unsigned)rlen;
                    const float v = my[in ? voff + e : 0];
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(in ? v : 0.f, zb[t], acc, 0, 0, 0);
                }
                // D[row][col]: col = lane mod 32, row = 8 (q / 4) + 4 hi + q mod 4
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int row = 8 * (q >> 2) + 4 * hi + (q & 3);
                    if (blk + row < nr) a.Pr[(base + blk + row) * R + a.r0 + j] = acc[q];
                }
            }
            vb += tot;
        }
    }
}

// ------------------------------------------------------------- transposed --
// Q = D A^T T diag(1/beta) - V diag(beta) for the tile (INIT: no V term).
// Column j, right-hand side c of Q from g = (G^T T)_{j,c}: smoothing and
// damping blocks, scale, the -beta v term; stores Q and returns Q^2.
__device__ __forceinline__ double badj_col_out(const BArgs &a, int64_t j, int c, float g,
                                               double beta, double ib)
{
#pragma clang fp contract(off)
    const int R = a.R;
    const int64_t tL = a.m, tD = a.m + a.n;
    const int pp = (int)j;
    const int iz = pp % a.nz, ixy = pp / a.nz, ix = ixy % a.nx, iy = ixy / a.nx;
    const int sxy = a.nx * a.nz;
    const float *TL = a.Tcur + tL * R;
    float acc = 0.f;
    int deg = 0;
    if (ix > 0) { acc += TL[(int64_t)(pp - a.nz) * R + c]; ++deg; }
    if (ix < a.nx - 1) { acc += TL[(int64_t)(pp + a.nz) * R + c]; ++deg; }
    if (iy > 0) { acc += TL[(int64_t)(pp - sxy) * R + c]; ++deg; }
    if (iy < a.ny - 1) { acc += TL[(int64_t)(pp + sxy) * R + c]; ++deg; }
    if (iz > 0) { acc += TL[(int64_t)(pp - 1) * R + c]; ++deg; }
    if (iz < a.nz - 1) { acc += TL[(int64_t)(pp + 1) * R + c]; ++deg; }
    const float lap = acc - (float)deg * TL[(int64_t)pp * R + c];
    const float sj = g + (float)a.w * lap + (float)a.damp * a.Tcur[(tD + j) * R + c];
    const double xj = a.d[j] * (double)sj;
    const double vj = a.mode == MODE_ITER ? (double)a.V[j * R + c] : 0.0;
    const float qv = (float)(xj / ib - beta * vj);
    a.Q[j * R + c] = qv;
    return (double)qv * (double)qv;
}

template <int RT>
__global__ __launch_bounds__(kBlock) void k_badj(BArgs a)
{
#pragma clang fp contract(off)
    __shared__ double accs[kBlock];
    __shared__ double res[kMaxRhs];
    __shared__ double b2[kMaxRhs];
    const bool op = a.mode == MODE_OPERATOR;       // plain product: beta = 1, no v
    int k = 0;
    if (a.mode == MODE_ITER) {
        k = a.ctl[C_CNT0 + a.parity];
        if (k > a.ctl[C_KMAX]) return;
    }
    if (op) {
        if (threadIdx.x < a.R) b2[threadIdx.x] = 1.0;
        __syncthreads();
    } else {
        sum_rhs_all(a.part_in, a.np_in, a.R, accs, b2);
    }
    if (!op && blockIdx.x == 0 && threadIdx.x < RT) {
        const int r = a.r0 + threadIdx.x;
        srow(a, k, r)[S_BETA] = sqrt(b2[r]);
    }
    constexpr int EPW = 64 / RT;
    const int lane = threadIdx.x & 63, er = lane / RT, rr = lane % RT;
    const int R = a.R, cofs = a.r0 + rr;
    const double beta = sqrt(b2[cofs]);
    const double ib = beta > 0.0 ? beta : 1.0;
    const int64_t tL = a.m, tD = a.m + a.n;
    double sq = 0.0;
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t j = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); j < a.n; j += nwaves) {
        const int64_t s = a.cp[j], e = a.cp[j + 1];
        // kBatchUnroll entries (each a row segment of RT right-hand sides) in flight
        float ac[kBatchUnroll];
#pragma unroll
        for (int u = 0; u < kBatchUnroll; ++u) ac[u] = 0.f;
        int64_t p = s + er;
        for (; p + (kBatchUnroll - 1) * EPW < e; p += kBatchUnroll * EPW) {
            float g[kBatchUnroll];
            int i[kBatchUnroll];
#pragma unroll
            for (int u = 0; u < kBatchUnroll; ++u) {
                g[u] = __builtin_nontemporal_load(a.cv + p + u * EPW);
                i[u] = __builtin_nontemporal_load(a.ri + p + u * EPW);
            }
#pragma unroll
            for (int u = 0; u < kBatchUnroll; ++u)
                ac[u] = fmaf(g[u], a.Tcur[(int64_t)i[u] * R + cofs], ac[u]);
        }
        for (; p < e; p += EPW)
            ac[0] = fmaf(__builtin_nontemporal_load(a.cv + p),
                         a.Tcur[(int64_t)__builtin_nontemporal_load(a.ri + p) * R + cofs], ac[0]);
        float g = tree_sum<kBatchUnroll>(ac);
#pragma unroll
        for (int off = RT; off < 64; off <<= 1) g += __shfl_xor(g, off, 64);
        if (er == 0) sq += badj_col_out(a, j, cofs, g, beta, ib);
    }
    block_sum_rhs<RT>(sq, accs, res);
    if (threadIdx.x < RT) a.part_out[(int64_t)blockIdx.x * a.R + a.r0 + threadIdx.x] = res[threadIdx.x];
}

// Transposed block product over node runs on the matrix cores (32-wide
// tiles): per lateral node, Q_node[depth, c] = sum over the node's runs r of
// V[r, depth] T[row_r, c], a product [32 depths x runs] x [runs x 32
// right-hand sides] reduced over the runs by v_mfma_f32_32x32x2f32, two runs
// per product (A: the runs' values at the 32 depths, zero outside their depth
// windows, from the chunk staged in the wave's LDS area; B: the runs' rows of
// T).  A workgroup per node (decreasing work, boustrophedon); its 4 waves
// take fixed quarters of the node's runs, each accumulating in its own
// matrix-core registers; the column sums add the waves in order.
__global__ __launch_bounds__(kBlock) void k_badj_mfma32(BArgs a)
{
#pragma clang fp contract(off)
    constexpr int RT = 32;
    constexpr int kStage = 16;                     // value loads per lane in flight
    constexpr int kPairs = 8;                      // products (run pairs) per batch
    __shared__ double accs[kBlock];
    __shared__ double res[kMaxRhs];
    __shared__ double b2[kMaxRhs];
    __shared__ float vs[kBlock / 64][64 * kMaxNzBatched];
    __shared__ float wsum[kBlock / 64][kMaxNzBatched][RT];
    const bool op = a.mode == MODE_OPERATOR;
    int k = 0;
    if (a.mode == MODE_ITER) {
        k = a.ctl[C_CNT0 + a.parity];
        if (k > a.ctl[C_KMAX]) return;
    }
    if (op) {
        if (threadIdx.x < a.R) b2[threadIdx.x] = 1.0;
        __syncthreads();
    } else {
        sum_rhs_all(a.part_in, a.np_in, a.R, accs, b2);
    }
    if (!op && blockIdx.x == 0 && threadIdx.x < RT) {
        const int r = a.r0 + threadIdx.x;
        srow(a, k, r)[S_BETA] = sqrt(b2[r]);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int hi = lane >> 5, j = lane & 31;       // MFMA operand roles
    const int R = a.R, nz = a.nz, nnodes = a.n / nz, G = gridDim.x;
    float *my = vs[wid];
    double sq = 0.0;
    for (int s = 0; s * G < nnodes; ++s) {
        const int idx = s * G + ((s & 1) ? G - 1 - (int)blockIdx.x : (int)blockIdx.x);
        if (idx >= nnodes) continue;                        // uniform over the workgroup
        const int node = a.norder[idx];
        const int64_t rs0 = a.nrp[node], cnt = a.nrp[node + 1] - rs0;
        const int64_t rs = rs0 + cnt * wid / 4, re = rs0 + cnt * (wid + 1) / 4;
        int64_t vb = a.nvq[4 * (int64_t)node + wid];
        floatx16 acc = {};
        for (int64_t base = rs; base < re; base += 64) {
            const int nr = (int)(re - base < 64 ? re - base : 64);
            // every lane loads (lanes past the chunk its last run: a valid
            // row whose values are zero; the descriptor masked here)
            const int64_t li = base + (lane < nr ? lane : nr - 1);
            uint32_t dsc = __builtin_nontemporal_load(a.ndesc + li);
            const uint32_t row = __builtin_nontemporal_load(a.nrow + li);
            dsc = lane < nr ? dsc : 0u;
            const int len = (int)(dsc & 255u);
            int incl = len;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o);
                if (lane >= o) incl += y;
            }
            // (value offset in the chunk << 16) | (iz0 << 8) | len; offsets < 64 * 64
            const uint32_t pk = ((uint32_t)(incl - len) << 16) | dsc;
            const int tot = __shfl(incl, 63);               // >= 1: runs are not empty
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int i0 = 0; i0 < tot; i0 += 64 * kStage) {
                float t[kStage];
#pragma unroll
                for (int q = 0; q < kStage; ++q) {
                    const int i = i0 + 64 * q + lane;
                    t[q] = __builtin_nontemporal_load(a.nval + vb + (i < tot ? i : tot - 1));
                }
#pragma unroll
                for (int q = 0; q < kStage; ++q) {
                    const int i = i0 + 64 * q + lane;
                    my[i < tot ? i : tot - 1] = t[q];    // past the end: the last value again
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // products over run pairs: A[depth j][run hi], B[run hi][rhs j]
            for (int p0 = 0; p0 < nr; p0 += 2 * kPairs) {
                float av[kPairs], bv[kPairs];
#pragma unroll
                for (int u = 0; u < kPairs; ++u) {
                    const int r = p0 + 2 * u + hi;          // past nr: row 0, zero values
                    const uint32_t pp = __shfl(pk, r & 63);
                    const uint32_t rw = __shfl(row, r & 63);
                    const int rlen = r < nr ? (int)(pp & 255u) : 0;
                    const int e = j - (int)((pp >> 8) & 255u);
                    const bool in = (unsigned)e < (unsigned)rlen;
                    const float v = my[in ? (int)(pp >> 16) + e : 0];
                    av[u] = in ? v : 0.f;
                    bv[u] = a.Tcur[(int64_t)(r < nr ? rw : 0u) * R + a.r0 + j];
                }
#pragma unroll
                for (int u = 0; u < kPairs; ++u)
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[u], bv[u], acc, 0, 0, 0);
            }
            vb += tot;
        }
        // D[depth][rhs]: rhs = lane mod 32, depth = 8 (q / 4) + 4 hi + q mod 4
#pragma unroll
        for (int q = 0; q < 16; ++q) wsum[wid][8 * (q >> 2) + 4 * hi + (q & 3)][j] = acc[q];
        __syncthreads();
        for (int cell = threadIdx.x; cell < nz * RT; cell += kBlock) {
            const int cz = cell / RT, cr = cell % RT;
            const float g = ((wsum[0][cz][cr] + wsum[1][cz][cr]) + wsum[2][cz][cr]) + wsum[3][cz][cr];
            const int c = a.r0 + cr;
            const double bc = sqrt(b2[c]);
            sq += badj_col_out(a, (int64_t)node * nz + cz, c, g, bc, bc > 0.0 ? bc : 1.0);
        }
        __syncthreads();
    }
    // per-RHS partial sums: thread t's squares belong to rhs lane t % RT
    block_sum_rhs<RT>(sq, accs, res);
    if (threadIdx.x < RT) a.part_out[(int64_t)blockIdx.x * a.R + a.r0 + threadIdx.x] = res[threadIdx.x];
}

// Transposed block product over node runs (see k_adj_nruns): a workgroup per
// lateral node, its 4 waves on fixed quarters of the node's runs, lanes in
// 64/nz groups of nz lanes, lane iz of a group owning depth iz and keeping the
// RT right-hand sides of its column in registers.  Per run, a group reads the
// run's values (consecutive lanes, one value each) and the run's row of T
// once (RT floats, the same address for the whole group), and every lane adds
// val * T[row, :] to its RT accumulators.  The t gathers fall from one per
// stored entry to one per run and no LDS is touched in the run loop.  Column
// sums: groups in order (shuffles), then waves in order (LDS).

template <int RT>
__device__ __forceinline__ void ld_trow(const float *p, float *t)
{
    if constexpr (RT >= 4) {
#pragma unroll
        for (int q = 0; q < RT / 4; ++q) {
            const float4 x = *(const float4 *)(p + 4 * q);
            t[4 * q] = x.x; t[4 * q + 1] = x.y; t[4 * q + 2] = x.z; t[4 * q + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < RT; ++q) t[q] = p[q];
    }
}

template <int RT>
__global__ __launch_bounds__(kBlock) void k_badj_nruns(BArgs a)
{
#pragma clang fp contract(off)
    constexpr int K = RT >= 32 ? 2 : 4;            // runs per group in flight
    __shared__ double accs[kBlock];
    __shared__ double res[kMaxRhs];
    __shared__ double b2[kMaxRhs];
    __shared__ float wsum[kBlock / 64][kMaxNzBatched][RT];
    const bool op = a.mode == MODE_OPERATOR;
    int k = 0;
    if (a.mode == MODE_ITER) {
        k = a.ctl[C_CNT0 + a.parity];
        if (k > a.ctl[C_KMAX]) return;
    }
    if (op) {
        if (threadIdx.x < a.R) b2[threadIdx.x] = 1.0;
        __syncthreads();
    } else {
        sum_rhs_all(a.part_in, a.np_in, a.R, accs, b2);
    }
    if (!op && blockIdx.x == 0 && threadIdx.x < RT) {
        const int r = a.r0 + threadIdx.x;
        srow(a, k, r)[S_BETA] = sqrt(b2[r]);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int R = a.R, nz = a.nz, ngr = 64 / nz, nnodes = a.n / nz;
    const int grp = lane / nz, iz = lane - grp * nz;
    const bool live = grp < ngr;
    const int G = gridDim.x;
    double sq = 0.0;
    for (int s = 0; s * G < nnodes; ++s) {
        const int idx = s * G + ((s & 1) ? G - 1 - (int)blockIdx.x : (int)blockIdx.x);
        if (idx >= nnodes) continue;                        // uniform over the workgroup
        const int node = a.norder[idx];
        const int64_t rs0 = a.nrp[node], cnt = a.nrp[node + 1] - rs0;
        const int64_t rs = rs0 + cnt * wid / 4, re = rs0 + cnt * (wid + 1) / 4;
        int64_t vb = a.nvq[4 * (int64_t)node + wid];
        float acc[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[r] = 0.f;
        for (int64_t base = rs; base < re; base += 64) {
            const int nr = (int)(re - base < 64 ? re - base : 64);
            // every lane loads (lanes past the chunk its last run: a valid
            // row whose values are zero; the descriptor masked here)
            const int64_t li = base + (lane < nr ? lane : nr - 1);
            uint32_t dsc = __builtin_nontemporal_load(a.ndesc + li);
            const uint32_t row = __builtin_nontemporal_load(a.nrow + li);
            dsc = lane < nr ? dsc : 0u;
            const int len = (int)(dsc & 255u);
            int incl = len;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o);
                if (lane >= o) incl += y;
            }
            const uint32_t pk = ((uint32_t)(incl - len) << 16) | dsc;
            const int tot = __shfl(incl, 63);
            for (int s0 = 0; s0 < nr; s0 += K * ngr) {
                float v[K];
                uint32_t rw[K];
#pragma unroll
                for (int u = 0; u < K; ++u) {
                    const int r = s0 + grp + u * ngr;
                    const uint32_t p = __shfl(pk, r & 63);
                    rw[u] = __shfl(row, r & 63);               // rows past nr: a valid row, zero values
                    const int e = iz - (int)((p >> 8) & 255u);
                    const bool in = live && r < nr && (unsigned)e < (p & 255u);
                    const float x = __builtin_nontemporal_load(
                        a.nval + (in ? vb + (int64_t)(p >> 16) + e : vb));
                    v[u] = in ? x : 0.f;
                }
#pragma unroll
                for (int u = 0; u < K; ++u) {
                    float t[RT];
                    ld_trow<RT>(a.Tcur + (int64_t)rw[u] * R + a.r0, t);
#pragma unroll
                    for (int r = 0; r < RT; ++r) acc[r] = fmaf(v[u], t[r], acc[r]);
                }
            }
            vb += tot;
        }
        // groups in order (shuffles), then waves in order (LDS)
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            float col = 0.f;
            for (int g = 0; g < ngr; ++g) col += __shfl(acc[r], (g * nz + iz) & 63);
            if (lane < nz) wsum[wid][lane][r] = col;
        }
        __syncthreads();
        for (int cell = threadIdx.x; cell < nz * RT; cell += kBlock) {
            const int cz = cell / RT, cr = cell % RT;
            const float g = ((wsum[0][cz][cr] + wsum[1][cz][cr]) + wsum[2][cz][cr]) + wsum[3][cz][cr];
            const int c = a.r0 + cr;
            const double bc = sqrt(b2[c]);
            sq += badj_col_out(a, (int64_t)node * nz + cz, c, g, bc, bc > 0.0 ? bc : 1.0);
        }
        __syncthreads();
    }
    // per-RHS partial sums: thread t's squares belong to rhs lane t % RT
    block_sum_rhs<RT>(sq, accs, res);
    if (threadIdx.x < RT) a.part_out[(int64_t)blockIdx.x * a.R + a.r0 + threadIdx.x] = res[threadIdx.x];
}

// ----------------------------------------------------------------- update --
// All R right-hand sides: alpha_r, the Givens step per r (FP64) and the
// x/w/v sweep over [n][R]; frozen right-hand sides keep x, w, v.  Writes the
// per-RHS partials of |D^-1 v|^2.
__global__ __launch_bounds__(kBlock) void k_bupdate(BArgs a)
{
#pragma clang fp contract(off)
    __shared__ double accs[kBlock];
    __shared__ double a2[kMaxRhs], res[kMaxRhs];
    __shared__ double t1s[kMaxRhs], t2s[kMaxRhs], als[kMaxRhs];
    __shared__ int live[kMaxRhs];
    const int R = a.R;
    int k = 0;
    if (a.mode == MODE_ITER) {
        k = a.ctl[C_CNT0 + a.parity];
        if (k > a.ctl[C_KMAX]) return;
    }
    sum_rhs_all(a.part_in, a.np_in, R, accs, a2);
    if (threadIdx.x < R) {
        const int r = threadIdx.x;
        double *Sk = srow(a, k, r);
        const double beta = Sk[S_BETA];
        const double alpha = beta > 0.0 ? sqrt(a2[r]) : 0.0;
        int on = a.act[r];
        if (a.mode == MODE_INIT) {
            on = alpha > 0.0 && beta > 0.0;
            if (blockIdx.x == 0) {
                Sk[S_ALPHA] = alpha; Sk[S_RHOBAR] = alpha; Sk[S_PHIBAR] = beta;
                Sk[S_PSI] = alpha * beta; Sk[S_ETA] = on ? 1.0 : 0.0;
                if (!on) { a.act[r] = 0; a.why[r] = 0; }
                if (!isfinite(alpha) || !isfinite(beta)) { a.act[r] = 0; a.why[r] = -3; a.ctl[C_ERR] = 1; }
            }
            als[r] = alpha; t1s[r] = 0.0; t2s[r] = 0.0;
        } else {
            const double *Sp = srow(a, k - 1, r);
            const double rhobar = Sp[S_RHOBAR], phibar = Sp[S_PHIBAR];
            const double rho = sqrt(rhobar * rhobar + beta * beta);
            const double c = rhobar / rho, s = beta / rho;
            const double theta = s * alpha, rhobar_n = -c * alpha;
            const double phi = c * phibar, phibar_n = s * phibar;
            const double psi = phibar_n * alpha * fabs(c);
            if (blockIdx.x == 0) {
                if (on) {
                    Sk[S_ALPHA] = alpha; Sk[S_RHOBAR] = rhobar_n; Sk[S_PHIBAR] = phibar_n;
                    Sk[S_RHO] = rho; Sk[S_C] = c; Sk[S_S] = s; Sk[S_THETA] = theta;
                    Sk[S_PHI] = phi; Sk[S_PSI] = psi;
                    if (!isfinite(alpha) || !isfinite(rho) || !isfinite(phi)) {
                        a.act[r] = 0; a.why[r] = -3; a.ctl[C_ERR] = 1;
                    }
                } else {
                    // frozen: carry the last state forward
                    for (int f = 0; f < kStateWords; ++f) Sk[f] = Sp[f];
                }
            }
            als[r] = alpha;
            t1s[r] = on ? phi / rho : 0.0;
            t2s[r] = on ? theta / rho : 0.0;
        }
        live[r] = on;
    }
    __syncthreads();
    double sq = 0.0;
    const int64_t tot = (int64_t)a.n * R;
    for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < tot;
         idx += (int64_t)gridDim.x * kBlock) {
        const int r = (int)(idx % R);           // == threadIdx.x % R
        const int64_t j = idx / R;
        double vj;
        if (live[r] && als[r] > 0.0) {
            const float vv = (float)((double)a.Q[idx] / als[r]);
            a.V[idx] = vv;
            vj = (double)vv;
        } else {
            vj = (double)a.V[idx];
        }
        if (a.mode == MODE_INIT) {
            a.W[idx] = vj;
        } else if (live[r]) {
            const double wj = a.W[idx];
            a.Y[idx] = a.Y[idx] + t1s[r] * wj;
            a.W[idx] = vj - t2s[r] * wj;
        }
        a.Zout[idx] = (float)(a.d[j] * vj);
        const double dv = vj / a.d[j];
        sq += dv * dv;
    }
    // per-RHS sum over the workgroup in a fixed order
    accs[threadIdx.x] = sq;
    __syncthreads();
    if (threadIdx.x < R) {
        double s2 = 0.0;
        for (int q = 0; q < kBlock / R; ++q) s2 += accs[q * R + threadIdx.x];
        a.part_out[(int64_t)blockIdx.x * R + threadIdx.x] = s2;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.mode == MODE_ITER) {
        a.ctl[C_ITERS] = k;
        a.ctl[C_CNT0 + (1 - a.parity)] = k + 1;
    }
}

// dm[j][r] = d_j y[j][r]; eta of the last step for right-hand sides still active.
__global__ __launch_bounds__(kBlock) void k_bfinal(BArgs a, double *dm)
{
#pragma clang fp contract(off)
    __shared__ double accs[kBlock];
    __shared__ double v2[kMaxRhs];
    const int R = a.R;
    const int kk = a.ctl[C_ITERS];
    if (blockIdx.x == 0 && kk >= 1) {
        sum_rhs_all(a.part_in, a.np_in, R, accs, v2);
        if (threadIdx.x < R) {
            const int r = threadIdx.x;
            double *Sk = srow(a, kk, r);
            if (a.act[r]) {
                const double vn = sqrt(v2[r]);
                const double eta = Sk[S_PSI] * vn / srow(a, 0, r)[S_ARNORM0];
                Sk[S_ETA] = eta;
                Sk[S_VNORM] = vn;
                if (a.tol > 0.0 && eta <= a.tol) a.why[r] = 1;
                else if (Sk[S_ALPHA] == 0.0 || Sk[S_BETA] == 0.0) a.why[r] = 3;
            }
        }
    }
    const int64_t tot = (int64_t)a.n * R;
    for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < tot;
         idx += (int64_t)gridDim.x * kBlock)
        dm[idx] = a.d[idx / R] * a.Y[idx];
}

}  // namespace lsqr
