// Templated LSQR kernels for gfx950 (wave64), shared by the per-precision
// translation units.
//
// One LSQR iteration k is three launches on one stream:
//   fwd    t = Abar D v_k - alpha_k u_k over the data rows (plain CSR or
//          depth-run rows), the 7-point smoothing rows and the damping rows;
//          per-workgroup partial sums of t^2 (FP64)
//   adj    beta_{k+1} from those partials; q = D Abar^T t / beta - beta v_k
//          over the stored transpose (CSC, no atomics); partial sums of q^2
//   update alpha_{k+1}, the Givens step (Paige & Saunders) in FP64 and the
//          x/w/v sweep (x, w in FP64)
// Every workgroup of a consumer kernel reduces the producer's partials in the
// same fixed order, so all workgroups hold bitwise-identical scalars without a
// separate reduction launch or atomics.  The iteration index, stop flag and
// per-iteration scalars live in device memory, so a block of iterations can be
// captured once as a hipGraph and replayed.
//
// Type parameters: M = stored matrix value (double, float, bf16_t, fp16_t),
// V = vector element (double, float).  Products accumulate in double when V
// is double and in float otherwise; norms and LSQR scalars are always FP64.
#pragma once

#include <math.h>

#include "internal.h"

namespace lsqr {

struct bf16_t { uint16_t b; };
struct fp16_t { uint16_t b; };

template <class V> struct AccOf { using type = float; };
template <> struct AccOf<double> { using type = double; };

template <class A> __device__ __forceinline__ A ld(const double *p) { return (A)*p; }
template <class A> __device__ __forceinline__ A ld(const float *p) { return (A)*p; }
template <class A> __device__ __forceinline__ A ld(const bf16_t *p)
{
    return (A)__uint_as_float((uint32_t)p->b << 16);
}
template <class A> __device__ __forceinline__ A ld(const fp16_t *p)
{
    _Float16 h;
    __builtin_memcpy(&h, &p->b, 2);
    return (A)(float)h;
}
template <class A> __device__ __forceinline__ A ld_nt(const double *p)
{
    return (A)__builtin_nontemporal_load(p);
}
template <class A> __device__ __forceinline__ A ld_nt(const float *p)
{
    return (A)__builtin_nontemporal_load(p);
}
template <class A> __device__ __forceinline__ A ld_nt(const bf16_t *p)
{
    const uint16_t b = __builtin_nontemporal_load(&p->b);
    return (A)__uint_as_float((uint32_t)b << 16);
}
template <class A> __device__ __forceinline__ A ld_nt(const fp16_t *p)
{
    const uint16_t b = __builtin_nontemporal_load(&p->b);
    _Float16 h;
    __builtin_memcpy(&h, &b, 2);
    return (A)(float)h;
}

// Raw stored bits of a value (loaded under a lane mask, converted after it, so
// that no conversion waits on a load inside the masked region); raw 0 is +0
// in every format.
template <class M> struct RawOf { using type = M; };
template <> struct RawOf<bf16_t> { using type = uint16_t; };
template <> struct RawOf<fp16_t> { using type = uint16_t; };
__device__ __forceinline__ double raw_nt(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float raw_nt(const float *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ uint16_t raw_nt(const bf16_t *p) { return __builtin_nontemporal_load(&p->b); }
__device__ __forceinline__ uint16_t raw_nt(const fp16_t *p) { return __builtin_nontemporal_load(&p->b); }
template <class A, class M> __device__ __forceinline__ A from_raw(typename RawOf<M>::type r)
{
    if constexpr (sizeof(M) >= 4) {
        return (A)r;
    } else if constexpr (sizeof(M) == 2 && __is_same(M, bf16_t)) {
        return (A)__uint_as_float((uint32_t)r << 16);
    } else {
        _Float16 h;
        __builtin_memcpy(&h, &r, 2);
        return (A)(float)h;
    }
}

// 1: the CSR / CSC products load the next row's (column's) bounds and the
// current row's u term before the current row's entries.
#ifndef LSQR_ROW_PREFETCH
#define LSQR_ROW_PREFETCH 1
#endif

// ------------------------------------------------------------ reductions --
// Pairwise sum of U values in a fixed tree order.
template <int U, class T>
__device__ __forceinline__ T tree_sum(const T *v)
{
    if constexpr (U == 1) {
        return v[0];
    } else {
        return tree_sum<U / 2>(v) + tree_sum<U - U / 2>(v + U / 2);
    }
}

// One DPP move of a 32- or 64-bit value (64-bit: both halves); lanes whose
// source is outside the row, and rows masked off, receive zero.
template <int ctrl, int rmask, bool bound_zero, class T>
__device__ __forceinline__ T dpp_move(T v)
{
    if constexpr (sizeof(T) == 8) {
        int2 h;
        __builtin_memcpy(&h, &v, 8);
        h.x = __builtin_amdgcn_update_dpp(0, h.x, ctrl, rmask, 0xf, bound_zero);
        h.y = __builtin_amdgcn_update_dpp(0, h.y, ctrl, rmask, 0xf, bound_zero);
        __builtin_memcpy(&v, &h, 8);
        return v;
    } else {
        int x;
        __builtin_memcpy(&x, &v, 4);
        x = __builtin_amdgcn_update_dpp(0, x, ctrl, rmask, 0xf, bound_zero);
        __builtin_memcpy(&v, &x, 4);
        return v;
    }
}
template <class T>
__device__ __forceinline__ T lane_value(T v, int lane)
{
    if constexpr (sizeof(T) == 8) {
        int2 h;
        __builtin_memcpy(&h, &v, 8);
        h.x = __builtin_amdgcn_readlane(h.x, lane);
        h.y = __builtin_amdgcn_readlane(h.y, lane);
        __builtin_memcpy(&v, &h, 8);
        return v;
    } else {
        int x;
        __builtin_memcpy(&x, &v, 4);
        x = __builtin_amdgcn_readlane(x, lane);
        __builtin_memcpy(&v, &x, 4);
        return v;
    }
}

template <int W, class T>
__device__ __forceinline__ T group_sum(T v)
{
    if constexpr (W == 64) {
        // prefix sums within rows of 16 lanes, then the row sums into lane
        // 63: ((row 3 + row 2) + (row 1 + row 0)), returned to every lane.
        // On the VALU in place of six shuffles through the LDS crossbar: the
        // per-row sums of the forward products, BF16 471 -> 457 us, FP32
        // 650 -> 642 us, FP64 984 -> 980 us on the config-1 system
        v += dpp_move<0x111, 0xf, true>(v);
        v += dpp_move<0x112, 0xf, true>(v);
        v += dpp_move<0x114, 0xf, true>(v);
        v += dpp_move<0x118, 0xf, true>(v);
        v += dpp_move<0x142, 0xa, false>(v);
        v += dpp_move<0x143, 0xc, false>(v);
        return lane_value(v, 63);
    }
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
    return v;
}

// Sum over the workgroup (kBlock threads) in a fixed order; every thread
// receives the same value.
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    v = group_sum<64>(v);
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[wid] = v;
    __syncthreads();
    double r = ((lds[0] + lds[1]) + lds[2]) + lds[3];
    __syncthreads();
    return r;
}

// Total of a producer's per-workgroup partials, identical in every workgroup.
__device__ __forceinline__ double reduce_partials(const double *p, int np, double *lds)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += kBlock) acc += p[i];
    return block_sum(acc, lds);
}

// (L x)_p for the 7-point Laplacian, neighbours in the order -x +x -y +y -z +z,
// centre -(number of in-grid neighbours).
template <class V>
__device__ __forceinline__ typename AccOf<V>::type stencil(const V *x, int p, int nx, int ny, int nz)
{
#pragma clang fp contract(off)
    using A = typename AccOf<V>::type;
    const int iz = p % nz, ixy = p / nz, ix = ixy % nx, iy = ixy / nx;
    const int sxy = nx * nz;
    A acc = 0;
    int deg = 0;
    if (ix > 0) { acc += (A)x[p - nz]; ++deg; }
    if (ix < nx - 1) { acc += (A)x[p + nz]; ++deg; }
    if (iy > 0) { acc += (A)x[p - sxy]; ++deg; }
    if (iy < ny - 1) { acc += (A)x[p + sxy]; ++deg; }
    if (iz > 0) { acc += (A)x[p - 1]; ++deg; }
    if (iz < nz - 1) { acc += (A)x[p + 1]; ++deg; }
    return acc - (A)deg * (A)x[p];
}

// ----------------------------------------------------------------- init --
// T0 = rhs (bbar = [dt; 0; 0] when full == 0, else a full [m+2n] vector),
// y = 0, vzero = 0, partial sums of rhs^2 (FP64), control words.
template <class V>
__global__ __launch_bounds__(kBlock) void k_init_rhs(int64_t m, int64_t n, const double *rhs,
                                                     int full, V *T0, const float *sigma, V *Ts0,
                                                     double *y, V *vzero, double *part, int *ctl,
                                                     int kmax)
{
    __shared__ double lds[4];
    const int64_t mb = m + 2 * n;
    double sq = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < mb;
         i += (int64_t)gridDim.x * kBlock) {
        const double b = (full || i < m) ? rhs[i] : 0.0;
        T0[i] = (V)b;
        if (Ts0 && i < m) Ts0[i] = (V)((double)sigma[i] * b);
        sq += b * b;
        if (i < n) { y[i] = 0.0; vzero[i] = (V)0; }
    }
    const double tot = block_sum(sq, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl[C_STOP] = 0; ctl[C_ISTOP] = 2; ctl[C_ITERS] = 0; ctl[C_ERR] = 0;
        ctl[C_CNT0] = 1; ctl[C_CNT1] = 0; ctl[C_KMAX] = kmax;
    }
}

// --------------------------------------------------------------- forward --
struct FwdArgs {
    // data rows
    const int64_t *rp;        // [m+1] value offsets
    const int32_t *ci;        // [nnz] columns (plain CSR) or nullptr
    const void *va;           // [nnz] values of type M
    const float *sigma;       // [m] row scales or nullptr
    int64_t m;
    int n, nx, ny, nz;
    double w, damp;
    const void *z;            // D v   [n] (V)
    const void *Tprev;        // previous t (u = Tprev / beta_k) [m+2n] (V)
    void *Tcur;               // [m+2n] (V)
    void *Ts;                 // [m] sigma * t (V) or nullptr
    double *part_out;         // [gridDim.x]
    const double *part_v;     // partials of |D^-1 v_k|^2
    int np_v;
    double *S;
    int *ctl;
    int parity;
    int mode;
    double tol;
    const int32_t *wrow;      // balanced wave partition (see RowFmt) or nullptr
    int wgrid;
    // row groups with local columns (see RowFmt) or nullptr
    const int32_t *gp;
    const int64_t *gcp;
    const int32_t *gcol;
    const uint16_t *slot;
    int ngroups;
    int gcap;
};

// Prologue of an LSQR forward step: the scalars of the previous step, the
// convergence check on eta_{k-1} and the stop flag.  Returns false when this
// launch has nothing to do.
__device__ __forceinline__ bool fwd_prologue(const FwdArgs &a, double &alpha, double &beta,
                                             double *lds)
{
#pragma clang fp contract(off)
    alpha = 0.0;
    beta = 1.0;
    if (a.mode != MODE_ITER) return true;
    if (a.ctl[C_STOP]) return false;
    const int k = a.ctl[C_CNT0 + a.parity];
    if (k > a.ctl[C_KMAX]) return false;
    double *Sp = a.S + (int64_t)(k - 1) * kStateWords;
    alpha = Sp[S_ALPHA];
    beta = Sp[S_BETA];
    const double vn = sqrt(reduce_partials(a.part_v, a.np_v, lds));
    double arnorm0, eta = 1.0;
    bool stop = false;
    int istop = 2;
    // LSMR keeps |A_D^T r_k| = |zetabar_{k+1}| itself: eta in the scaled
    // variables, against alpha_1 beta_1 (set by its start step)
    const bool lsmr = a.S[S_METHOD] != 0.0;
    if (k == 1) {
        arnorm0 = lsmr ? a.S[S_ARNORM0] : (a.S[S_ALPHA] * a.S[S_BETA]) * vn;
    } else {
        arnorm0 = a.S[S_ARNORM0];
        eta = lsmr ? Sp[S_PSI] / arnorm0 : Sp[S_PSI] * vn / arnorm0;
        if (a.tol > 0.0 && eta <= a.tol) { stop = true; istop = 1; }
        else if (alpha == 0.0 || beta == 0.0) { stop = true; istop = 3; }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (k == 1) { a.S[S_ARNORM0] = arnorm0; a.S[S_VNORM] = vn; }
        else { Sp[S_ETA] = eta; Sp[S_VNORM] = vn; }
        if (stop) { a.ctl[C_ISTOP] = istop; a.ctl[C_STOP] = 1; }
    }
    return !stop;
}

// Row epilogue: t_i = sigma_i acc - alpha u_i with u_i = Tprev_i / beta.
template <class V>
__device__ __forceinline__ double fwd_row_out(const FwdArgs &a, int64_t row, double acc,
                                              double alpha, double beta)
{
#pragma clang fp contract(off)
    const double sacc = a.sigma ? (double)a.sigma[row] * acc : acc;
    const double u = a.mode == MODE_ITER ? (double)((const V *)a.Tprev)[row] / beta : 0.0;
    const V t = (V)(sacc - alpha * u);
    ((V *)a.Tcur)[row] = t;
    if (a.Ts) ((V *)a.Ts)[row] = (V)((double)a.sigma[row] * (double)t);
    return (double)t * (double)t;
}

// As fwd_row_out, with t_prev[row] already loaded.
template <class V>
__device__ __forceinline__ double fwd_row_out_u(const FwdArgs &a, int64_t row, double acc,
                                                double alpha, double beta, double tprev)
{
#pragma clang fp contract(off)
    const double sacc = a.sigma ? (double)a.sigma[row] * acc : acc;
    const double u = a.mode == MODE_ITER ? tprev / beta : 0.0;
    const V t = (V)(sacc - alpha * u);
    ((V *)a.Tcur)[row] = t;
    if (a.Ts) ((V *)a.Ts)[row] = (V)((double)a.sigma[row] * (double)t);
    return (double)t * (double)t;
}

// Smoothing rows (m .. m+n) and damping rows (m+n .. m+2n): one thread each.
template <class V>
__device__ __forceinline__ double fwd_reg_rows(const FwdArgs &a, double alpha, double beta)
{
#pragma clang fp contract(off)
    using A = typename AccOf<V>::type;
    const V *z = (const V *)a.z;
    double sq = 0.0;
    const int64_t nreg = 2 * (int64_t)a.n;
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < nreg;
         r += (int64_t)gridDim.x * kBlock) {
        A yv;
        if (r < a.n) yv = stencil<V>(z, (int)r, a.nx, a.ny, a.nz) * (A)a.w;
        else yv = (A)a.damp * (A)z[r - a.n];
        const double u = a.mode == MODE_ITER ? (double)((const V *)a.Tprev)[a.m + r] / beta : 0.0;
        const V t = (V)((double)yv - alpha * u);
        ((V *)a.Tcur)[a.m + r] = t;
        sq += (double)t * (double)t;
    }
    return sq;
}

// Plain CSR rows, LPR lanes per row.
template <class M, class V, int LPR>
__global__ __launch_bounds__(kBlock) void k_fwd_csr(FwdArgs a)
{
    using A = typename AccOf<V>::type;
    __shared__ double lds[4];
    double alpha, beta;
    if (!fwd_prologue(a, alpha, beta, lds)) return;
    const M *va = (const M *)a.va;
    const V *z = (const V *)a.z;
    double sq = 0.0;
    constexpr int RPB = kBlock / LPR;
    const int lane = threadIdx.x % LPR;
    const int64_t gstride = (int64_t)gridDim.x * RPB;
#if LSQR_ROW_PREFETCH
    int64_t row = (int64_t)blockIdx.x * RPB + threadIdx.x / LPR;
    int64_t s = 0, e = 0;
    if (row < a.m) { s = a.rp[row]; e = a.rp[row + 1]; }
    for (; row < a.m; row += gstride) {
        const int64_t nrow = row + gstride;
        int64_t ns = 0, ne = 0;
        if (nrow < a.m) { ns = a.rp[nrow]; ne = a.rp[nrow + 1]; }
        double up = 0.0;
        if (lane == 0 && a.mode == MODE_ITER) up = (double)((const V *)a.Tprev)[row];
#else
    for (int64_t row = (int64_t)blockIdx.x * RPB + threadIdx.x / LPR; row < a.m; row += gstride) {
        const int64_t s = a.rp[row], e = a.rp[row + 1];
#endif
        A a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        int64_t j = s + lane;
        for (; j + 3 * LPR < e; j += 4 * LPR) {
            const int c0 = __builtin_nontemporal_load(a.ci + j);
            const int c1 = __builtin_nontemporal_load(a.ci + j + LPR);
            const int c2 = __builtin_nontemporal_load(a.ci + j + 2 * LPR);
            const int c3 = __builtin_nontemporal_load(a.ci + j + 3 * LPR);
            const A v0 = ld_nt<A>(va + j), v1 = ld_nt<A>(va + j + LPR);
            const A v2 = ld_nt<A>(va + j + 2 * LPR), v3 = ld_nt<A>(va + j + 3 * LPR);
            a0 = fma(v0, (A)z[c0], a0);
            a1 = fma(v1, (A)z[c1], a1);
            a2 = fma(v2, (A)z[c2], a2);
            a3 = fma(v3, (A)z[c3], a3);
        }
        for (; j < e; j += LPR) a0 = fma(ld_nt<A>(va + j), (A)z[__builtin_nontemporal_load(a.ci + j)], a0);
        const A acc = group_sum<LPR>((a0 + a1) + (a2 + a3));
#if LSQR_ROW_PREFETCH
        if (lane == 0) sq += fwd_row_out_u<V>(a, row, (double)acc, alpha, beta, up);
        s = ns;
        e = ne;
#else
        if (lane == 0) sq += fwd_row_out<V>(a, row, (double)acc, alpha, beta);
#endif
    }
    sq += fwd_reg_rows<V>(a, alpha, beta);
    const double tot = block_sum(sq, lds);
    if (threadIdx.x == 0) a.part_out[blockIdx.x] = tot;
}

// Plain CSR rows, one wave per row, software-pipelined.  A wave walks its
// rows as one stream of batches of U entries per lane (64 U per batch): the
// columns and values of the next batch (the rest of this row, else the start
// of the wave's next row) are loaded before the current batch's v gathers and
// products, so HBM loads stay in flight while the gathers wait on L2 and
// while a finished row is reduced.  Lanes past a row's end load nothing and
// add zero.
#ifndef LSQR_FWD_PIPE
#define LSQR_FWD_PIPE 1
#endif
// Entries per lane and batch: 6 for 8-byte values, 8 for 4- and 2-byte
// values (measured on config 1).
#ifdef LSQR_FWD_PIPE_U
template <class M> struct PipeU { static constexpr int value = LSQR_FWD_PIPE_U; };
#else
template <class M> struct PipeU { static constexpr int value = sizeof(M) >= 8 ? 6 : 8; };
#endif
// 1: the balanced row ranges belong to workgroups and the workgroup's 4 waves
// take its rows in turn (neighbouring rows share columns, so their v gathers
// meet in L1); 0: each wave has its own range.
#ifndef LSQR_FWD_WG_ROWS
#define LSQR_FWD_WG_ROWS 1
#endif

// A load through the constant address space: with a wave-uniform index it
// becomes a scalar load, whose wait does not hold up the vector loads in
// flight.  Only for memory that no kernel of the launch writes.
template <class T>
__device__ __forceinline__ T ld_uniform(const T *p, int64_t i)
{
    return ((const __attribute__((address_space(4))) T *)p)[i];
}

// One batch of a CSR row walk: U entries per lane (entry jb + lane + 64 u).
// Entries past eb load a clamped in-range address (the row's last entry, else
// entry 0) and are left out of the products (u >= the lane's valid count):
// every batch issues the same loads with no branch, and the raw values are
// converted only where they are used, so no wait is placed before the use.
template <class M, int U>
struct CsrBatch {
    int c[U];
    typename RawOf<M>::type r[U];
    int nv;                              // entries u < nv of this lane are in the row
};

template <class M, int U>
__device__ __forceinline__ void csr_batch(const FwdArgs &a, const M *va, int64_t jb, int64_t eb,
                                          int lane, CsrBatch<M, U> &b)
{
    const int64_t safe = jb < eb ? eb - 1 : 0;
    const int64_t left = eb - jb - lane;                 // entries from this lane's first on
    b.nv = left <= 0 ? 0 : (left >= 64 * (int64_t)U ? U : (int)((left + 63) >> 6));
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t j = jb + lane + 64 * u;
        const int64_t jj = j < eb ? j : safe;
        b.c[u] = __builtin_nontemporal_load(a.ci + jj);
        b.r[u] = raw_nt(va + jj);
    }
}

// As csr_batch, reading the entries' local column slots (row groups).
template <class M, int U>
__device__ __forceinline__ void slot_batch(const FwdArgs &a, const M *va, int64_t jb, int64_t eb,
                                           int lane, CsrBatch<M, U> &b)
{
    const int64_t safe = jb < eb ? eb - 1 : 0;
    const int64_t left = eb - jb - lane;
    b.nv = left <= 0 ? 0 : (left >= 64 * (int64_t)U ? U : (int)((left + 63) >> 6));
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t j = jb + lane + 64 * u;
        const int64_t jj = j < eb ? j : safe;
        b.c[u] = (int)__builtin_nontemporal_load(a.slot + jj);
        b.r[u] = raw_nt(va + jj);
    }
}

template <class M, class V>
__global__ __launch_bounds__(kBlock) void k_fwd_pipe(FwdArgs a)
{
    using A = typename AccOf<V>::type;
    constexpr int U = PipeU<M>::value;
    constexpr int64_t B = 64 * U;
    __shared__ double lds[4];
    double alpha, beta;
    if (!fwd_prologue(a, alpha, beta, lds)) return;
    const M *va = (const M *)a.va;
    const V *z = (const V *)a.z;
    const V *tp = (const V *)a.Tprev;
    const bool iter = a.mode == MODE_ITER;
    double sq = 0.0;
    const int lane = threadIdx.x & 63;
    // the wave's rows: a contiguous balanced range, else every wstride-th row.
    // Row indexes are uniform over the wave: row bounds and the u term come
    // through scalar loads.
    const int wave = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)));
    int row = wave, rend = (int)a.m, wstride = gridDim.x * (kBlock / 64);
    if (a.wrow && a.wgrid == (int)gridDim.x) {
        if (LSQR_FWD_WG_ROWS) {
            row = ld_uniform(a.wrow, (int)blockIdx.x) + (wave & 3);
            rend = ld_uniform(a.wrow, (int)blockIdx.x + 1);
            wstride = kBlock / 64;
        } else {
            row = ld_uniform(a.wrow, wave);
            rend = ld_uniform(a.wrow, wave + 1);
            wstride = 1;
        }
    }
    if (a.m > 0 && a.rp[a.m] == 0) {                      // no stored entries: rows of zeros
        for (; row < rend; row += wstride)
            if (lane == 0) sq += fwd_row_out<V>(a, row, 0.0, alpha, beta);
    }
    if (row < rend) {
        int64_t j = ld_uniform(a.rp, row), e = ld_uniform(a.rp, row + 1);
        int nrow = row + wstride;
        int64_t ns = 0, ne = 0;
        if (nrow < rend) { ns = ld_uniform(a.rp, nrow); ne = ld_uniform(a.rp, nrow + 1); }
        double up = iter ? (double)ld_uniform(tp, row) : 0.0;
        double sg = a.sigma ? (double)ld_uniform(a.sigma, row) : 1.0;
        CsrBatch<M, U> b0, b1;
        A acc[U];
        csr_batch<M, U>(a, va, j, e, lane, b0);
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = 0;
        // one batch: gathers of the current batch, loads of the next one (the
        // current batch's gathers go first: loads complete in issue order, so
        // the products wait for the gathers only), products, and the row's end
        auto step = [&](const CsrBatch<M, U> &cur, CsrBatch<M, U> &nxt) -> bool {
            const bool last = j + B >= e;
            const int64_t jn = last ? ns : j + B, en = last ? ne : e;
            A zg[U];
#pragma unroll
            for (int u = 0; u < U; ++u) zg[u] = (A)z[cur.c[u]];
            csr_batch<M, U>(a, va, jn, en, lane, nxt);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const A p = fma(from_raw<A, M>(cur.r[u]), zg[u], acc[u]);
                acc[u] = u < cur.nv ? p : acc[u];
            }
            j = jn;
            if (last) {
                const A t = group_sum<64>(tree_sum<U>(acc));
                if (lane == 0) {                          // as fwd_row_out, sigma preloaded
#pragma clang fp contract(off)
                    const double sacc = a.sigma ? sg * (double)t : (double)t;
                    const double u = iter ? up / beta : 0.0;
                    const V tv = (V)(sacc - alpha * u);
                    ((V *)a.Tcur)[row] = tv;
                    if (a.Ts) ((V *)a.Ts)[row] = (V)(sg * (double)tv);
                    sq += (double)tv * (double)tv;
                }
                if (nrow >= rend) return true;
                row = nrow;
                e = ne;
                nrow = row + wstride;
                ns = ne = 0;
                if (nrow < rend) { ns = ld_uniform(a.rp, nrow); ne = ld_uniform(a.rp, nrow + 1); }
                up = iter ? (double)ld_uniform(tp, row) : 0.0;
                if (a.sigma) sg = (double)ld_uniform(a.sigma, row);
#pragma unroll
                for (int u = 0; u < U; ++u) acc[u] = 0;
            }
            return false;
        };
        // two register sets in turn, so no batch is copied
        for (;;) {
            if (step(b0, b1)) break;
            if (step(b1, b0)) break;
        }
    }
    sq += fwd_reg_rows<V>(a, alpha, beta);
    const double tot = block_sum(sq, lds);
    if (threadIdx.x == 0) a.part_out[blockIdx.x] = tot;
}

// Row groups with local columns: a workgroup takes its groups in turn (a
// contiguous range balanced in entries, wrow[b] .. wrow[b+1]-1, when the
// launch has wgrid workgroups; else groups b, b + grid, ...).  Per group the
// 256 threads gather D v at the group's columns into LDS (one coalesced pass
// over the column list, whose stretches of consecutive depths share cache
// lines), then the four waves take the group's rows in turn and walk them as
// k_fwd_pipe does (U entries per lane per batch, the next batch's slots and
// values loaded while the current batch is multiplied), reading D v from LDS
// through the entries' 16-bit slots.  Per row the sum order is that of
// k_fwd_pipe, so t is the same to the bit.  The launch gives gcap entries of
// A of dynamic LDS; slots of entries outside the current group (the clamped
// loads of an empty row) are below gcap too, so every LDS read stays inside
// the array; such entries are not summed.

// Row groups, E entries per lane and load (E = 2: pairs; E = 4: quads, for
// 4- and 2-byte values; E = 8: octets, for 16-bit codes): a row's entries
// are taken in aligned groups of E (positions p .. p + E - 1, p a multiple
// of E; the first group of a row that starts inside one holds entries of
// the previous row, the last may hold the next row's first or, at the end of
// the arrays, padding elements), so one load brings E values (pairs: 16
// bytes for FP64, 8 for FP32, 4 for 16-bit codes; quads: 16 bytes for FP32,
// 8 for 16-bit codes; octets: 16 bytes of 16-bit codes) and one load their
// E 16-bit slots.  Entries outside the row are left out of the sums.  Pairs
// halve the load instructions per entry of k_fwd_lcol, quads halve them
// again, and octets once more.
typedef double f64x2p __attribute__((ext_vector_type(2)));
typedef float f32x2p __attribute__((ext_vector_type(2)));
typedef float f32x4p __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4p __attribute__((ext_vector_type(4)));
// E raw stored values in one word
template <class M, int E> struct EntRaw { using type = uint32_t; };          // 2 x 16-bit
template <> struct EntRaw<double, 2> { using type = f64x2p; };
template <> struct EntRaw<float, 2> { using type = f32x2p; };
template <> struct EntRaw<float, 4> { using type = f32x4p; };
template <> struct EntRaw<bf16_t, 4> { using type = uint64_t; };
template <> struct EntRaw<fp16_t, 4> { using type = uint64_t; };
template <> struct EntRaw<bf16_t, 8> { using type = u32x4p; };
template <> struct EntRaw<fp16_t, 8> { using type = u32x4p; };
// E 16-bit slots in one word
template <int E> struct SlotRaw { using type = uint32_t; };
template <> struct SlotRaw<4> { using type = uint64_t; };
template <> struct SlotRaw<8> { using type = u32x4p; };
// 16-bit field k of a word of E of them
template <int E, class T>
__device__ __forceinline__ uint32_t half_at(T w, int k)
{
    if constexpr (E == 8) return (w[k >> 1] >> (16 * (k & 1))) & 0xffffu;
    else return (uint32_t)(w >> (16 * k)) & 0xffffu;
}
template <class A, class M, int E>
__device__ __forceinline__ void ent_values(typename EntRaw<M, E>::type r, A (&x)[E])
{
    if constexpr (sizeof(M) >= 4) {
#pragma unroll
        for (int k = 0; k < E; ++k) x[k] = (A)r[k];
    } else {
#pragma unroll
        for (int k = 0; k < E; ++k) x[k] = from_raw<A, M>((uint16_t)half_at<E>(r, k));
    }
}
template <class M, int U, int E>
struct EntBatch {
    typename SlotRaw<E>::type c[U];      // E slots
    typename EntRaw<M, E>::type r[U];    // E values
    int64_t e0[U];                       // position of the group's first entry
};
template <class M, int U, int E>
__device__ __forceinline__ void ent_batch(const FwdArgs &a, const M *va, int64_t jb, int64_t eb,
                                          int lane, EntBatch<M, U, E> &b)
{
    // groups p = jb + E lane + 64 E u (jb a multiple of E); a group at or
    // past eb loads the group holding entry eb - 1 (else group 0): in
    // bounds, not summed
    const int64_t safe = eb > 0 ? ((eb - 1) & ~(int64_t)(E - 1)) : 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t p = jb + E * lane + 64 * E * u;
        const int64_t pp = p < eb ? p : safe;
        b.e0[u] = p;
        b.c[u] = __builtin_nontemporal_load((const typename SlotRaw<E>::type *)(a.slot + pp));
        b.r[u] = __builtin_nontemporal_load((const typename EntRaw<M, E>::type *)(va + pp));
    }
}

template <class M, class V>
__global__ __launch_bounds__(kBlock) void k_fwd_lcol(FwdArgs a)
{
    using A = typename AccOf<V>::type;
    constexpr int U = PipeU<M>::value;
    constexpr int64_t B = 64 * U;
    constexpr int SU = 8;                                 // staging loads in flight per thread
    __shared__ double lds[4];
    extern __shared__ double zdyn[];
    A *zl = (A *)zdyn;                                    // [gcap]
    double alpha, beta;
    if (!fwd_prologue(a, alpha, beta, lds)) return;
    const M *va = (const M *)a.va;
    const V *z = (const V *)a.z;
    const V *tp = (const V *)a.Tprev;
    const bool iter = a.mode == MODE_ITER;
    double sq = 0.0;
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    int g = blockIdx.x, gend = a.ngroups, gstep = gridDim.x;
    if (a.wrow && a.wgrid == (int)gridDim.x) {
        g = ld_uniform(a.wrow, (int)blockIdx.x);
        gend = ld_uniform(a.wrow, (int)blockIdx.x + 1);
        gstep = 1;
    }
    for (; g < gend; g += gstep) {
        const int r0 = ld_uniform(a.gp, g), r1 = ld_uniform(a.gp, g + 1);
        const int64_t c0 = ld_uniform(a.gcp, g);
        const int nc = (int)(ld_uniform(a.gcp, g + 1) - c0);
        __syncthreads();                                  // the previous group's reads are done
        for (int j0 = 0; j0 < nc; j0 += kBlock * SU) {
            A zs[SU];
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const int j = j0 + (int)threadIdx.x + kBlock * u;
                zs[u] = (A)z[a.gcol[c0 + (j < nc ? j : nc - 1)]];
            }
            // lanes past the list store the last column's value again (the
            // same value to the same slot): an unconditional store keeps the
            // compiler from sinking a lane's loads into a branch of their own
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const int j = j0 + (int)threadIdx.x + kBlock * u;
                zl[j < nc ? j : nc - 1] = zs[u];
            }
        }
        __syncthreads();
        int row = r0 + wid;
        if (row >= r1) continue;
        int64_t j = ld_uniform(a.rp, row), e = ld_uniform(a.rp, row + 1);
        int nrow = row + 4;
        int64_t ns = 0, ne = 0;
        if (nrow < r1) { ns = ld_uniform(a.rp, nrow); ne = ld_uniform(a.rp, nrow + 1); }
        double up = iter ? (double)ld_uniform(tp, row) : 0.0;
        double sg = a.sigma ? (double)ld_uniform(a.sigma, row) : 1.0;
        CsrBatch<M, U> b0, b1;
        A acc[U];
        slot_batch<M, U>(a, va, j, e, lane, b0);
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = 0;
        auto step = [&](const CsrBatch<M, U> &cur, CsrBatch<M, U> &nxt) -> bool {
            const bool last = j + B >= e;
            const int64_t jn = last ? ns : j + B, en = last ? ne : e;
            A zg[U];
#pragma unroll
            for (int u = 0; u < U; ++u) zg[u] = zl[cur.c[u]];
            slot_batch<M, U>(a, va, jn, en, lane, nxt);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const A p = fma(from_raw<A, M>(cur.r[u]), zg[u], acc[u]);
                acc[u] = u < cur.nv ? p : acc[u];
            }
            j = jn;
            if (last) {
                const A t = group_sum<64>(tree_sum<U>(acc));
                if (lane == 0) {
#pragma clang fp contract(off)
                    const double sacc = a.sigma ? sg * (double)t : (double)t;
                    const double u = iter ? up / beta : 0.0;
                    const V tv = (V)(sacc - alpha * u);
                    ((V *)a.Tcur)[row] = tv;
                    if (a.Ts) ((V *)a.Ts)[row] = (V)(sg * (double)tv);
                    sq += (double)tv * (double)tv;
                }
                if (nrow >= r1) return true;
                row = nrow;
                e = ne;
                nrow = row + 4;
                ns = ne = 0;
                if (nrow < r1) { ns = ld_uniform(a.rp, nrow); ne = ld_uniform(a.rp, nrow + 1); }
                up = iter ? (double)ld_uniform(tp, row) : 0.0;
                if (a.sigma) sg = (double)ld_uniform(a.sigma, row);
#pragma unroll
                for (int u = 0; u < U; ++u) acc[u] = 0;
            }
            return false;
        };
        for (;;) {
            if (step(b0, b1)) break;
            if (step(b1, b0)) break;
        }
    }
    sq += fwd_reg_rows<V>(a, alpha, beta);
    const double tot = block_sum(sq, lds);
    if (threadIdx.x == 0) a.part_out[blockIdx.x] = tot;
}

// Groups of E entries per lane and batch of k_fwd_lcol_pair.
#ifdef LSQR_FWD_PAIR_U
template <class M, int E> struct PairU { static constexpr int value = LSQR_FWD_PAIR_U; };
#else
template <class M, int E> struct PairU { static constexpr int value = E == 2 ? 3 : E == 4 ? 2 : 1; };
#endif

// See ent_batch.
template <class M, class V, int E>
__global__ __launch_bounds__(kBlock) void k_fwd_lcol_pair(FwdArgs a)
{
    using A = typename AccOf<V>::type;
    constexpr int SU = 8;                                 // staging loads in flight per thread
    __shared__ double lds[4];
    extern __shared__ double zdyn[];
    A *zl = (A *)zdyn;                                    // [gcap]
    double alpha, beta;
    if (!fwd_prologue(a, alpha, beta, lds)) return;
    const M *va = (const M *)a.va;
    const V *z = (const V *)a.z;
    const V *tp = (const V *)a.Tprev;
    const bool iter = a.mode == MODE_ITER;
    double sq = 0.0;
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    int g = blockIdx.x, gend = a.ngroups, gstep = gridDim.x;
    if (a.wrow && a.wgrid == (int)gridDim.x) {
        g = ld_uniform(a.wrow, (int)blockIdx.x);
        gend = ld_uniform(a.wrow, (int)blockIdx.x + 1);
        gstep = 1;
    }
    for (; g < gend; g += gstep) {
        const int r0 = ld_uniform(a.gp, g), r1 = ld_uniform(a.gp, g + 1);
        const int64_t c0 = ld_uniform(a.gcp, g);
        const int nc = (int)(ld_uniform(a.gcp, g + 1) - c0);
        __syncthreads();                                  // the previous group's reads are done
        for (int j0 = 0; j0 < nc; j0 += kBlock * SU) {
            A zs[SU];
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const int j = j0 + (int)threadIdx.x + kBlock * u;
                zs[u] = (A)z[a.gcol[c0 + (j < nc ? j : nc - 1)]];
            }
            // lanes past the list store the last column's value again (the
            // same value to the same slot): an unconditional store keeps the
            // compiler from sinking a lane's loads into a branch of their own
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const int j = j0 + (int)threadIdx.x + kBlock * u;
                zl[j < nc ? j : nc - 1] = zs[u];
            }
        }
        __syncthreads();
        int row = r0 + wid;
        if (row >= r1) continue;
        int64_t jr = ld_uniform(a.rp, row), e = ld_uniform(a.rp, row + 1);
        int nrow = row + 4;
        int64_t ns = 0, ne = 0;
        if (nrow < r1) { ns = ld_uniform(a.rp, nrow); ne = ld_uniform(a.rp, nrow + 1); }
        double up = iter ? (double)ld_uniform(tp, row) : 0.0;
        double sg = a.sigma ? (double)ld_uniform(a.sigma, row) : 1.0;
        constexpr int UP = PairU<M, E>::value;
        constexpr int64_t BP = 64 * E * UP;
        constexpr int64_t AL = ~(int64_t)(E - 1);
        int64_t jb = jr & AL;
        EntBatch<M, UP, E> b0, b1;
        A acc[UP];
        ent_batch<M, UP, E>(a, va, jb, e, lane, b0);
#pragma unroll
        for (int u = 0; u < UP; ++u) acc[u] = 0;
        auto step = [&](const EntBatch<M, UP, E> &cur, EntBatch<M, UP, E> &nxt) -> bool {
            const bool last = jb + BP >= e;
            const int64_t jn = last ? (ns & AL) : jb + BP, en = last ? ne : e;
            A zg[UP][E];
#pragma unroll
            for (int u = 0; u < UP; ++u)
#pragma unroll
                for (int k = 0; k < E; ++k) zg[u][k] = zl[half_at<E>(cur.c[u], k)];
            ent_batch<M, UP, E>(a, va, jn, en, lane, nxt);
            // entry p + k is in the row when 0 <= p + k - jr < e - jr: one
            // unsigned 32-bit compare (p - jr lies in [1 - E, e - jr + BP),
            // rows of row groups hold fewer than 2^31 entries), which keeps
            // the sum a select rather than a branch per entry
            const uint32_t len = (uint32_t)(e - jr);
#pragma unroll
            for (int u = 0; u < UP; ++u) {
                const int32_t d = (int32_t)(cur.e0[u] - jr);
                A x[E];
                ent_values<A, M, E>(cur.r[u], x);
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const A q = fma(x[k], zg[u][k], acc[u]);
                    acc[u] = (uint32_t)(d + k) < len ? q : acc[u];
                }
            }
            jb = jn;
            if (last) {
                const A t = group_sum<64>(tree_sum<UP>(acc));
                if (lane == 0) {
#pragma clang fp contract(off)
                    const double sacc = a.sigma ? sg * (double)t : (double)t;
                    const double u = iter ? up / beta : 0.0;
                    const V tv = (V)(sacc - alpha * u);
                    ((V *)a.Tcur)[row] = tv;
                    if (a.Ts) ((V *)a.Ts)[row] = (V)(sg * (double)tv);
                    sq += (double)tv * (double)tv;
                }
                if (nrow >= r1) return true;
                row = nrow;
                jr = ns;
                e = ne;
                nrow = row + 4;
                ns = ne = 0;
                if (nrow < r1) { ns = ld_uniform(a.rp, nrow); ne = ld_uniform(a.rp, nrow + 1); }
                up = iter ? (double)ld_uniform(tp, row) : 0.0;
                if (a.sigma) sg = (double)ld_uniform(a.sigma, row);
#pragma unroll
                for (int u = 0; u < UP; ++u) acc[u] = 0;
            }
            return false;
        };
        for (;;) {
            if (step(b0, b1)) break;
            if (step(b1, b0)) break;
        }
    }
    sq += fwd_reg_rows<V>(a, alpha, beta);
    const double tot = block_sum(sq, lds);
    if (threadIdx.x == 0) a.part_out[blockIdx.x] = tot;
}

// ------------------------------------------------------------- transposed --
struct AdjArgs {
    const int64_t *cp;
    const int32_t *ri;
    const void *cv;          // [nnz] values of type M
    int64_t m;
    int n, nx, ny, nz;
    double w, damp;
    const double *d;         // column scale [n]
    const void *T;           // t [m+2n] (V): smoothing/damping blocks
    const void *Tg;          // data block gathered by rows (sigma * t when scaled) (V)
    const void *v;           // v_k [n] (V) or nullptr
    void *q;                 // out [n] (V)
    double *part_out;
    const double *part_t;    // partials of |t|^2
    int np_t;
    double *S;
    int *ctl;
    int parity;
    int mode;
    int data_only;           // 1: G^T part only (no smoothing/damping, no scale)
    // node runs (k_adj_nruns): see ColFmt
    const int64_t *nrp;
    const int64_t *nvq;
    const uint32_t *nrow;
    const uint16_t *ndesc;
    const int32_t *norder;
};

// beta_{k+1} from the forward partials (FP64, fixed order); false when the
// workgroup has nothing to do (stopped, past the last iteration, breakdown).
__device__ __forceinline__ bool adj_prologue(const AdjArgs &a, double &beta, double *lds)
{
    beta = 1.0;
    if (a.mode == MODE_OPERATOR) return true;
    if (a.ctl[C_STOP]) return false;
    int k = 0;
    if (a.mode == MODE_ITER) {
        k = a.ctl[C_CNT0 + a.parity];
        if (k > a.ctl[C_KMAX]) return false;
    }
    beta = sqrt(reduce_partials(a.part_t, a.np_t, lds));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.S[(int64_t)k * kStateWords + S_BETA] = beta;
        if (a.mode == MODE_INIT && beta == 0.0) { a.ctl[C_ISTOP] = 0; a.ctl[C_STOP] = 1; }
    }
    return beta != 0.0;      // breakdown: the update kernel sets alpha = 0
}

// Column j of q from g = (G^T t)_j: adds the smoothing and damping blocks,
// applies the scale and the -beta v term, stores q_j and returns q_j^2.
template <class V>
__device__ __forceinline__ double adj_col_out(const AdjArgs &a, int j,
                                              typename AccOf<V>::type g, double beta)
{
#pragma clang fp contract(off)
    using A = typename AccOf<V>::type;
    const V *T = (const V *)a.T;
    const V *vv = (const V *)a.v;
    double qj;
    if (a.data_only) {
        qj = (double)g;
    } else {
        const A lap = stencil<V>(T + a.m, j, a.nx, a.ny, a.nz);
        const A sj = g + (A)a.w * lap + (A)a.damp * (A)T[a.m + a.n + j];
        const double xj = a.d[j] * (double)sj;
        qj = vv ? xj / beta - beta * (double)vv[j] : xj / beta;
    }
    const V qv = (V)qj;
    ((V *)a.q)[j] = qv;
    return (double)qv * (double)qv;
}

template <class M, class V, int LPC>
__global__ __launch_bounds__(kBlock) void k_adj(AdjArgs a)
{
#pragma clang fp contract(off)
    using A = typename AccOf<V>::type;
    __shared__ double lds[4];
    double beta;
    if (!adj_prologue(a, beta, lds)) return;
    const M *cv = (const M *)a.cv;
    const V *Tg = (const V *)a.Tg;
    double sq = 0.0;
    constexpr int CPB = kBlock / LPC;
    const int lane = threadIdx.x % LPC;
    const int jhi = a.n, jstart = blockIdx.x * CPB, jstep = gridDim.x * CPB;
#if LSQR_ROW_PREFETCH
    int j = jstart + threadIdx.x / LPC;
    int64_t s = 0, e = 0;
    if (j < jhi) { s = a.cp[j]; e = a.cp[j + 1]; }
    for (; j < jhi; j += jstep) {
        const int jn = j + jstep;
        int64_t ns = 0, ne = 0;
        if (jn < jhi) { ns = a.cp[jn]; ne = a.cp[jn + 1]; }
#else
    for (int j = jstart + threadIdx.x / LPC; j < jhi; j += jstep) {
        const int64_t s = a.cp[j], e = a.cp[j + 1];
#endif
        A a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        int64_t p = s + lane;
        for (; p + 3 * LPC < e; p += 4 * LPC) {
            const int r0 = __builtin_nontemporal_load(a.ri + p);
            const int r1 = __builtin_nontemporal_load(a.ri + p + LPC);
            const int r2 = __builtin_nontemporal_load(a.ri + p + 2 * LPC);
            const int r3 = __builtin_nontemporal_load(a.ri + p + 3 * LPC);
            const A v0 = ld_nt<A>(cv + p), v1 = ld_nt<A>(cv + p + LPC);
            const A v2 = ld_nt<A>(cv + p + 2 * LPC), v3 = ld_nt<A>(cv + p + 3 * LPC);
            a0 = fma(v0, (A)Tg[r0], a0);
            a1 = fma(v1, (A)Tg[r1], a1);
            a2 = fma(v2, (A)Tg[r2], a2);
            a3 = fma(v3, (A)Tg[r3], a3);
        }
        for (; p < e; p += LPC)
            a0 = fma(ld_nt<A>(cv + p), (A)Tg[__builtin_nontemporal_load(a.ri + p)], a0);
        const A g = group_sum<LPC>((a0 + a1) + (a2 + a3));
        if (lane == 0) sq += adj_col_out<V>(a, j, g, beta);
#if LSQR_ROW_PREFETCH
        s = ns;
        e = ne;
#endif
    }
    const double tot = block_sum(sq, lds);
    if (threadIdx.x == 0) a.part_out[blockIdx.x] = tot;
}

// Transposed product over node runs.  The data block is stored per lateral
// node (the nz consecutive columns of one (ix, iy), eq. 7) as runs: for each
// data row reaching the node, in ascending row order, its stretch of
// consecutive depths [iz0, iz0 + len) and their values.  Row indices and the
// gathers of t are paid once per run instead of once per entry.
//
// One workgroup per node; nodes are visited in decreasing order of run count,
// dealt to workgroups boustrophedon-wise so every workgroup gets a similar
// load.  The 4 waves of a workgroup take fixed contiguous quarters of the
// node's runs (value offsets of the quarters are stored).  Inside a wave the
// lanes form 64/nz groups of nz lanes, lane iz of a group owning depth iz.
// The wave walks its runs in chunks of kRunsPerGroup runs per group: the
// chunk's descriptors and t values sit one per lane, a wave prefix sum gives
// each run's value offset, and every lane issues all of its chunk's value
// loads before the first multiply-add, while the next chunk's descriptors and
// t gathers are already in flight.  Per column, the sum runs over the chunks
// in order, then over the groups in order, then over the waves in order:
// fixed, no atomics.
// Runs per group per chunk (value loads in flight per lane): 12 for 8-byte
// values, 16 for 4- and 2-byte values (measured on config 1).
#ifdef LSQR_RUNS_PER_GROUP
template <class M> struct RunsPerGroup { static constexpr int value = LSQR_RUNS_PER_GROUP; };
#else
template <class M> struct RunsPerGroup { static constexpr int value = sizeof(M) >= 8 ? 12 : 16; };
#endif

template <class M, class V>
__global__ __launch_bounds__(kBlock) void k_adj_nruns(AdjArgs a)
{
#pragma clang fp contract(off)
    using A = typename AccOf<V>::type;
    __shared__ double lds[4];
    __shared__ A wsum[kBlock / 64][64];
    double beta;
    if (!adj_prologue(a, beta, lds)) return;
    const M *nv = (const M *)a.cv;
    const V *Tg = (const V *)a.Tg;
    constexpr int kRunsPerGroup = RunsPerGroup<M>::value;
    const int nz = a.nz, ngr = 64 / nz;
    const int ch = ngr * kRunsPerGroup < 64 ? ngr * kRunsPerGroup : 64;   // runs per chunk
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int grp = lane / nz, iz = lane - grp * nz;
    const bool live = grp < ngr;
    // nodes: serpentine over norder
    const int G = gridDim.x, slot = blockIdx.x, nnodes = a.n / nz;
    double sq = 0.0;
    for (int s = 0; s * G < nnodes; ++s) {
        const int idx = s * G + ((s & 1) ? G - 1 - slot : slot);
        if (idx >= nnodes) continue;         // uniform over the workgroup
        const int node = a.norder[idx];
        const int64_t rs0 = a.nrp[node], cnt = a.nrp[node + 1] - rs0;
        const int64_t rs = rs0 + cnt * wid / 4, re = rs0 + cnt * (wid + 1) / 4;
        int64_t vb = a.nvq[4 * (int64_t)node + wid];
        A acc = 0;
        // first chunk's descriptors and t
        int64_t base = rs;
        int nr = (int)(re - base < ch ? re - base : ch);
        uint32_t dsc = 0u;
        A tr = 0;
        if (lane < nr) {
            dsc = __builtin_nontemporal_load(a.ndesc + base + lane);
            tr = (A)Tg[__builtin_nontemporal_load(a.nrow + base + lane)];
        }
        while (base < re) {
            const int len = (int)(dsc & 255u);
            int incl = len;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o);
                if (lane >= o) incl += y;
            }
            // (value offset in the chunk << 16) | (iz0 << 8) | len; offsets < 64 * 64
            const uint32_t pk = ((uint32_t)(incl - len) << 16) | dsc;
            const int tot = __shfl(incl, 63);
            // next chunk's descriptors (issued before this chunk's values)
            const int64_t nb = base + nr;
            const int nn = nb < re ? (int)(re - nb < ch ? re - nb : ch) : 0;
            uint32_t dsc_n = 0u, row_n = 0u;
            if (lane < nn) {
                dsc_n = __builtin_nontemporal_load(a.ndesc + nb + lane);
                row_n = __builtin_nontemporal_load(a.nrow + nb + lane);
            }
            // this chunk's values: run grp + u ngr of the chunk for lane (grp, iz)
            // loads are unconditional (an idle slot reads the chunk's first
            // value, always in bounds) and masked afterwards, so no branch
            // separates them and all are in flight before the first use
            A v[kRunsPerGroup];
#pragma unroll
            for (int u = 0; u < kRunsPerGroup; ++u) {
                const int r = grp + u * ngr;
                const uint32_t p = __shfl(pk, r & 63);
                const int e = iz - (int)((p >> 8) & 255u);
                const bool in = live && r < nr && (unsigned)e < (p & 255u);
                const A x = ld_nt<A>(nv + (in ? vb + (int64_t)(p >> 16) + e : vb));
                v[u] = in ? x : (A)0;
            }
            A tr_n = 0;
            if (lane < nn) tr_n = (A)Tg[row_n];
#pragma unroll
            for (int u = 0; u < kRunsPerGroup; ++u)
                acc = fma(v[u], __shfl(tr, (grp + u * ngr) & 63), acc);
            vb += tot;
            base = nb;
            nr = nn;
            dsc = dsc_n;
            tr = tr_n;
        }
        A col = 0;
        for (int g = 0; g < ngr; ++g) col += __shfl(acc, (g * nz + iz) & 63);
        if (lane < nz) wsum[wid][lane] = col;
        __syncthreads();
        if (wid == 0 && lane < nz) {
            const A g = ((wsum[0][lane] + wsum[1][lane]) + wsum[2][lane]) + wsum[3][lane];
            sq += adj_col_out<V>(a, node * nz + lane, g, beta);
        }
        __syncthreads();
    }
    const double tot = block_sum(sq, lds);
    if (threadIdx.x == 0) a.part_out[blockIdx.x] = tot;
}

// W consecutive stored values from a position aligned to W elements (W = 2;
// W = 4 for 16-bit codes).
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <class A, class M, int W>
__device__ __forceinline__ void ld_word(const M *p, A (&x)[W])
{
    if constexpr (sizeof(M) == 8) {
        static_assert(W == 2, "FP64 values: pairs");
        const f64x2 v = __builtin_nontemporal_load((const f64x2 *)p);
        x[0] = (A)v.x; x[1] = (A)v.y;
    } else if constexpr (sizeof(M) == 4 && W == 4) {       // FP32: four depths, 16 bytes
        const f32x4 v = __builtin_nontemporal_load((const f32x4 *)p);
        x[0] = (A)v.x; x[1] = (A)v.y; x[2] = (A)v.z; x[3] = (A)v.w;
    } else if constexpr (sizeof(M) == 4) {
        static_assert(W == 2, "FP32 values: pairs or quads");
        const f32x2 v = __builtin_nontemporal_load((const f32x2 *)p);
        x[0] = (A)v.x; x[1] = (A)v.y;
    } else if constexpr (W == 2) {
        const uint32_t w = __builtin_nontemporal_load((const uint32_t *)p);
        x[0] = from_raw<A, M>((uint16_t)(w & 0xffffu));
        x[1] = from_raw<A, M>((uint16_t)(w >> 16));
    } else if constexpr (W == 4) {
        const uint64_t w = __builtin_nontemporal_load((const uint64_t *)p);
#pragma unroll
        for (int h = 0; h < 4; ++h) x[h] = from_raw<A, M>((uint16_t)(w >> (16 * h)));
    } else {
        static_assert(W == 8, "16-bit codes: two, four or eight depths");
        const u32x4 w = __builtin_nontemporal_load((const u32x4 *)p);
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            x[2 * h] = from_raw<A, M>((uint16_t)(w[h] & 0xffffu));
            x[2 * h + 1] = from_raw<A, M>((uint16_t)(w[h] >> 16));
        }
    }
}

// Transposed product over node runs in the depth-pair layout (see
// pair_layout_host): as k_adj_nruns, but a lane owns two depths, 2k and
// 2k+1, so a group of ceil(nz/2) lanes covers a node's depths and a wave
// holds twice as many groups.  Runs start at even positions with zeros
// before an odd first depth and after an odd end, so a lane reads both of
// its depths of a run with one aligned two-element load and no per-element
// mask: a pair outside the run's window is skipped (its load reads the
// quarter's first word, always in bounds, and is multiplied as zero).  Half
// the load, shuffle and multiply-add instructions per value of k_adj_nruns,
// for about one padding element per run.  Per column the sum order is fixed
// (chunks, runs of a group, groups, waves): no atomics.
// Runs per group and chunk.  A chunk holds at most 64 runs (one descriptor
// per lane), so with W = 4 (12 groups per wave at nz = 20) 6 runs per group
// already cover it and more only issue masked loads; with the wave-uniform
// wave index 5 measured best (FP32 571 -> 545 us on the paper-shaped system;
// 4: 736 us), and 3 at W = 8 (21 groups per wave).
#ifndef LSQR_PAIR_RPG2
#define LSQR_PAIR_RPG2 10
#endif
#ifndef LSQR_PAIR_RPG4
#define LSQR_PAIR_RPG4 5
#endif
#ifndef LSQR_PAIR_RPG8
#define LSQR_PAIR_RPG8 3
#endif
// Inclusive prefix sum over the 64 lanes of a wave, on the VALU with DPP:
// row shifts by 1, 2, 4 and 8 within rows of 16 lanes (a lane shifted in
// from outside its row adds zero), then the broadcast of lane 15 into rows 1
// and 3 and of lane 31 into rows 2 and 3.  In place of six dependent
// shuffles through the LDS crossbar: BF16 codes 398 -> 385 us on the
// transposed product of the config-1 system.
__device__ __forceinline__ int wave_incl_scan(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
    return x;
}

template <int W> struct PairRPG {
    static constexpr int value = W == 2 ? LSQR_PAIR_RPG2 : W == 4 ? LSQR_PAIR_RPG4 : LSQR_PAIR_RPG8;
};

template <class M, class V, int W>
__global__ __launch_bounds__(kBlock) void k_adj_npair(AdjArgs a)
{
#pragma clang fp contract(off)
    using A = typename AccOf<V>::type;
    constexpr int RPG = PairRPG<W>::value;
    __shared__ double lds[4];
    __shared__ A wsum[kBlock / 64][64];
    double beta;
    if (!adj_prologue(a, beta, lds)) return;
    const M *nv = (const M *)a.cv;
    const V *Tg = (const V *)a.Tg;
    const int nz = a.nz, hz = (nz + W - 1) / W, ngr = 64 / hz;
    const int ch = ngr * RPG < 64 ? ngr * RPG : 64;       // runs per chunk
    // the wave index as a wave-uniform value: the quarter bounds, the value
    // offset and the chunk loop are then scalar (BF16 codes: 459 -> 416 us on
    // the paper-shaped system; FP64 and FP32 unchanged)
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int grp = lane / hz, k2 = W * (lane - grp * hz);  // the lane's depths k2 .. k2 + W - 1
    const bool live = grp < ngr;
    const int G = gridDim.x, slot = blockIdx.x, nnodes = a.n / nz;
    double sq = 0.0;
    for (int s = 0; s * G < nnodes; ++s) {
        const int idx = s * G + ((s & 1) ? G - 1 - slot : slot);
        if (idx >= nnodes) continue;         // uniform over the workgroup
        const int node = a.norder[idx];
        const int64_t rs0 = a.nrp[node], cnt = a.nrp[node + 1] - rs0;
        const int64_t rs = rs0 + cnt * wid / 4, re = rs0 + cnt * (wid + 1) / 4;
        int64_t vb = a.nvq[4 * (int64_t)node + wid];        // a multiple of W
        A acc[W];
#pragma unroll
        for (int h = 0; h < W; ++h) acc[h] = 0;
        if (re > rs) {
            // a chunk's descriptors and T values, loaded one chunk ahead
            struct Pre {
                uint32_t dsc;
                A tr;
            };
            Pre s0, s1;
            int64_t base = rs;
            int nr = (int)(re - base < ch ? re - base : ch);
            {
                // every lane loads (lanes past the chunk reload its first
                // run), so no load sits under a divergent branch; lanes past
                // the chunk are masked where the descriptors are used
                const int64_t li = lane < nr ? base + lane : base;
                s0.dsc = __builtin_nontemporal_load(a.ndesc + li);
                s0.tr = (A)Tg[__builtin_nontemporal_load(a.nrow + li)];
            }
            auto step = [&](const Pre &cur, Pre &nxt) -> bool {
                const uint32_t dsc = lane < nr ? cur.dsc : 0u;
                // padded length: iz0 mod W zeros before, and up to a multiple of W
                const int iz0l = (int)((dsc >> 8) & 255u);
                const int plen = ((int)(dsc & 255u) + (iz0l & (W - 1)) + W - 1) & ~(W - 1);
                const int incl = wave_incl_scan(plen);
                // (padded offset in the chunk << 16) | (iz0 << 8) | len; offsets < 64 * 68
                const uint32_t pk = ((uint32_t)(incl - plen) << 16) | dsc;
                const int tot = __builtin_amdgcn_readlane(incl, 63);
                const int64_t nb = base + nr;
                const int nn = nb < re ? (int)(re - nb < ch ? re - nb : ch) : 0;
                // the next chunk's runs; with none left, this chunk's last
                // run again (in bounds, never used)
                const int64_t li = lane < nn ? nb + lane : nb - 1;
                nxt.dsc = __builtin_nontemporal_load(a.ndesc + li);
                const uint32_t row_n = __builtin_nontemporal_load(a.nrow + li);
                A v[RPG][W];
#pragma unroll
                for (int u = 0; u < RPG; ++u) {
                    const int r = grp + u * ngr;
                    const uint32_t p = __shfl(pk, r & 63);
                    const int iz0 = (int)((p >> 8) & 255u), lo = iz0 & ~(W - 1);
                    const bool in = live & (r < nr) & (k2 >= lo) & (k2 < iz0 + (int)(p & 255u));
                    // a lane outside the run's window reads the quarter's first
                    // word (a line the wave streams anyway) and drops it
                    ld_word<A, M, W>(nv + (in ? vb + (int64_t)(p >> 16) + (k2 - lo) : vb), v[u]);
#pragma unroll
                    for (int h = 0; h < W; ++h) v[u][h] = in ? v[u][h] : (A)0;
                }
                nxt.tr = (A)Tg[row_n];
                // runs past the chunk carry a finite T value and zero values
#pragma unroll
                for (int u = 0; u < RPG; ++u) {
                    const A t = __shfl(cur.tr, (grp + u * ngr) & 63);
#pragma unroll
                    for (int h = 0; h < W; ++h) acc[h] = fma(v[u][h], t, acc[h]);
                }
                vb += tot;
                base = nb;
                nr = nn;
                return nn == 0;
            };
            for (;;) {
                if (step(s0, s1)) break;
                if (step(s1, s0)) break;
            }
        }
        // lane l < nz: depth l = word l / W, element l mod W, summed over groups
        const int kk = lane / W, hh = lane % W;
        A col = 0;
        for (int g = 0; g < ngr; ++g) {
            A c = 0;
#pragma unroll
            for (int h = 0; h < W; ++h) {
                const A ch_ = __shfl(acc[h], (g * hz + kk) & 63);
                c = h == hh ? ch_ : c;
            }
            col += c;
        }
        if (lane < nz) wsum[wid][lane] = col;
        __syncthreads();
        if (wid == 0 && lane < nz) {
            const A g = ((wsum[0][lane] + wsum[1][lane]) + wsum[2][lane]) + wsum[3][lane];
            sq += adj_col_out<V>(a, node * nz + lane, g, beta);
        }
        __syncthreads();
    }
    const double tot = block_sum(sq, lds);
    if (threadIdx.x == 0) a.part_out[blockIdx.x] = tot;
}

// ----------------------------------------------------------------- update --
struct UpdArgs {
    int n;
    const double *d;
    const void *q;           // (V)
    void *v;                 // (V)
    double *w, *y;
    void *z;                 // D v (V)
    double *part_out;        // partials of |D^-1 v_{k+1}|^2
    const double *part_q;    // partials of |q|^2
    int np_q;
    double *S;
    int *ctl;
    int parity;
    int mode;
    double *hbar;            // LSMR only: hbar [n] (w holds h)
};

template <class V>
__global__ __launch_bounds__(kBlock) void k_update(UpdArgs a)
{
#pragma clang fp contract(off)
    __shared__ double lds[4];
    if (a.ctl[C_STOP]) return;
    const V *q = (const V *)a.q;
    V *v = (V *)a.v;
    V *z = (V *)a.z;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (a.mode == MODE_INIT) {
        const double beta = a.S[S_BETA];
        const double alpha = sqrt(reduce_partials(a.part_q, a.np_q, lds));
        if (!isfinite(alpha) || !isfinite(beta)) {
            if (lead) { a.ctl[C_ERR] = 1; a.ctl[C_ISTOP] = -3; a.ctl[C_STOP] = 1; }
            return;
        }
        if (alpha == 0.0) {
            if (lead) { a.S[S_ALPHA] = 0.0; a.ctl[C_ISTOP] = 0; a.ctl[C_STOP] = 1; }
            return;
        }
        double sq = 0.0;
        for (int j = blockIdx.x * kBlock + threadIdx.x; j < a.n; j += gridDim.x * kBlock) {
            const double vj = (double)q[j] / alpha;
            const V vv = (V)vj;
            v[j] = vv;
            a.w[j] = (double)vv;
            z[j] = (V)(a.d[j] * (double)vv);
            const double dv = (double)vv / a.d[j];
            sq += dv * dv;
        }
        const double tot = block_sum(sq, lds);
        if (threadIdx.x == 0) a.part_out[blockIdx.x] = tot;
        if (lead) {
            double *S0 = a.S;
            S0[S_ALPHA] = alpha; S0[S_RHOBAR] = alpha; S0[S_PHIBAR] = beta;
            S0[S_PSI] = alpha * beta; S0[S_ETA] = 1.0; S0[S_METHOD] = 0.0;
        }
        return;
    }
    const int k = a.ctl[C_CNT0 + a.parity];
    if (k > a.ctl[C_KMAX]) return;
    const double *Sp = a.S + (int64_t)(k - 1) * kStateWords;
    double *Sk = a.S + (int64_t)k * kStateWords;
    const double beta = Sk[S_BETA];
    const double alpha = beta > 0.0 ? sqrt(reduce_partials(a.part_q, a.np_q, lds)) : 0.0;
    const double rhobar = Sp[S_RHOBAR], phibar = Sp[S_PHIBAR];
    const double rho = sqrt(rhobar * rhobar + beta * beta);
    const double c = rhobar / rho;
    const double s = beta / rho;
    const double theta = s * alpha;
    const double rhobar_n = -c * alpha;
    const double phi = c * phibar;
    const double phibar_n = s * phibar;
    const double t1 = phi / rho;
    const double t2 = theta / rho;
    const double psi = phibar_n * alpha * fabs(c);
    if (!isfinite(alpha) || !isfinite(beta) || !isfinite(rho) || !isfinite(phi)) {
        if (lead) { a.ctl[C_ERR] = 1; a.ctl[C_ISTOP] = -3; a.ctl[C_STOP] = 1; }
        return;
    }
    double sq = 0.0;
    const bool newv = alpha > 0.0;
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < a.n; j += gridDim.x * kBlock) {
        double vj;
        if (newv) {
            const V vv = (V)((double)q[j] / alpha);
            v[j] = vv;
            vj = (double)vv;
        } else {
            vj = (double)v[j];
        }
        const double wj = a.w[j];
        a.y[j] = a.y[j] + t1 * wj;
        a.w[j] = vj - t2 * wj;
        z[j] = (V)(a.d[j] * vj);
        const double dv = vj / a.d[j];
        sq += dv * dv;
    }
    const double tot = block_sum(sq, lds);
    if (threadIdx.x == 0) a.part_out[blockIdx.x] = tot;
    if (lead) {
        Sk[S_ALPHA] = alpha; Sk[S_RHOBAR] = rhobar_n; Sk[S_PHIBAR] = phibar_n; Sk[S_RHO] = rho;
        Sk[S_C] = c; Sk[S_S] = s; Sk[S_THETA] = theta; Sk[S_PHI] = phi; Sk[S_PSI] = psi;
        a.ctl[C_ITERS] = k;
        a.ctl[C_CNT0 + (1 - a.parity)] = k + 1;
    }
}

// LSMR step (Fong & Saunders 2011): after the bidiagonalisation shared with
// LSQR (forward and transposed kernels), the rotation P_k on
// [alphabar_k; beta_{k+1}], the rotation Pbar_k on [cbar_{k-1} rho_k;
// theta_{k+1}], the h / hbar / y sweep, and the third rotation chain that
// carries |r_k|.  Every workgroup computes the scalars identically (FP64, no
// contraction) from the previous state row; w holds h.
template <class V>
__global__ __launch_bounds__(kBlock) void k_update_lsmr(UpdArgs a)
{
#pragma clang fp contract(off)
    __shared__ double lds[4];
    if (a.ctl[C_STOP]) return;
    const V *q = (const V *)a.q;
    V *v = (V *)a.v;
    V *z = (V *)a.z;
    double *h = a.w, *hbar = a.hbar;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (a.mode == MODE_INIT) {
        const double beta = a.S[S_BETA];
        const double alpha = sqrt(reduce_partials(a.part_q, a.np_q, lds));
        if (!isfinite(alpha) || !isfinite(beta)) {
            if (lead) { a.ctl[C_ERR] = 1; a.ctl[C_ISTOP] = -3; a.ctl[C_STOP] = 1; }
            return;
        }
        if (alpha == 0.0) {
            if (lead) { a.S[S_ALPHA] = 0.0; a.ctl[C_ISTOP] = 0; a.ctl[C_STOP] = 1; }
            return;
        }
        double sq = 0.0;
        for (int j = blockIdx.x * kBlock + threadIdx.x; j < a.n; j += gridDim.x * kBlock) {
            const V vv = (V)((double)q[j] / alpha);
            v[j] = vv;
            h[j] = (double)vv;
            hbar[j] = 0.0;
            z[j] = (V)(a.d[j] * (double)vv);
            const double dv = (double)vv / a.d[j];
            sq += dv * dv;
        }
        const double tot = block_sum(sq, lds);
        if (threadIdx.x == 0) a.part_out[blockIdx.x] = tot;
        if (lead) {
            double *S0 = a.S;
            S0[S_ALPHA] = alpha; S0[S_ALPHABAR] = alpha; S0[S_ZETABAR] = alpha * beta;
            S0[S_RHO] = 1.0; S0[S_RHOBAR] = 1.0; S0[S_CBAR] = 1.0; S0[S_SBAR] = 0.0;
            S0[S_ZETA] = 0.0; S0[S_BETADD] = beta; S0[S_BETAD] = 0.0; S0[S_RHODOLD] = 1.0;
            S0[S_TAUTILDE] = 0.0; S0[S_THETATILDE] = 0.0;
            S0[S_PHIBAR] = beta; S0[S_PSI] = alpha * beta; S0[S_ETA] = 1.0;
            S0[S_ARNORM0] = alpha * beta; S0[S_METHOD] = 1.0;
        }
        return;
    }
    const int k = a.ctl[C_CNT0 + a.parity];
    if (k > a.ctl[C_KMAX]) return;
    const double *Sp = a.S + (int64_t)(k - 1) * kStateWords;
    double *Sk = a.S + (int64_t)k * kStateWords;
    const double beta = Sk[S_BETA];
    const double alpha = beta > 0.0 ? sqrt(reduce_partials(a.part_q, a.np_q, lds)) : 0.0;
    // rotation P_k
    const double rhoold = Sp[S_RHO], alphabar = Sp[S_ALPHABAR];
    const double rho = sqrt(alphabar * alphabar + beta * beta);
    const double c = alphabar / rho, s = beta / rho;
    const double thetanew = s * alpha, alphabar_n = c * alpha;
    // rotation Pbar_k
    const double rhobarold = Sp[S_RHOBAR], zetaold = Sp[S_ZETA], zetabar = Sp[S_ZETABAR];
    const double thetabar = Sp[S_SBAR] * rho, rhotemp = Sp[S_CBAR] * rho;
    const double rhobar = sqrt(rhotemp * rhotemp + thetanew * thetanew);
    const double cbar = rhotemp / rhobar, sbar = thetanew / rhobar;
    const double zeta = cbar * zetabar, zetabar_n = -sbar * zetabar;
    const double c1 = thetabar * rho / (rhoold * rhobarold);
    const double c2 = zeta / (rho * rhobar);
    const double c3 = thetanew / rho;
    // |r_k| chain
    const double betahat = c * Sp[S_BETADD], betadd = -s * Sp[S_BETADD];
    const double thetatildeold = Sp[S_THETATILDE], rhodoldp = Sp[S_RHODOLD];
    const double rhotildeold = sqrt(rhodoldp * rhodoldp + thetabar * thetabar);
    const double ctildeold = rhodoldp / rhotildeold, stildeold = thetabar / rhotildeold;
    const double thetatilde = stildeold * rhobar, rhodold = ctildeold * rhobar;
    const double betad = -stildeold * Sp[S_BETAD] + ctildeold * betahat;
    const double tautilde = (zetaold - thetatildeold * Sp[S_TAUTILDE]) / rhotildeold;
    const double taud = (zeta - thetatilde * tautilde) / rhodold;
    const double normr = sqrt((betad - taud) * (betad - taud) + betadd * betadd);
    const double normar = fabs(zetabar_n);
    if (!isfinite(alpha) || !isfinite(rho) || !isfinite(rhobar) || !isfinite(zeta) ||
        !isfinite(normr)) {
        if (lead) { a.ctl[C_ERR] = 1; a.ctl[C_ISTOP] = -3; a.ctl[C_STOP] = 1; }
        return;
    }
    double sq = 0.0;
    const bool newv = alpha > 0.0;
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < a.n; j += gridDim.x * kBlock) {
        double vj;
        if (newv) {
            const V vv = (V)((double)q[j] / alpha);
            v[j] = vv;
            vj = (double)vv;
        } else {
            vj = (double)v[j];
        }
        const double hb = h[j] - c1 * hbar[j];
        hbar[j] = hb;
        a.y[j] = a.y[j] + c2 * hb;
        h[j] = vj - c3 * h[j];
        z[j] = (V)(a.d[j] * vj);
        const double dv = vj / a.d[j];
        sq += dv * dv;
    }
    const double tot = block_sum(sq, lds);
    if (threadIdx.x == 0) a.part_out[blockIdx.x] = tot;
    if (lead) {
        Sk[S_ALPHA] = alpha; Sk[S_ALPHABAR] = alphabar_n; Sk[S_RHO] = rho; Sk[S_RHOBAR] = rhobar;
        Sk[S_CBAR] = cbar; Sk[S_SBAR] = sbar; Sk[S_ZETA] = zeta; Sk[S_ZETABAR] = zetabar_n;
        Sk[S_BETADD] = betadd; Sk[S_BETAD] = betad; Sk[S_RHODOLD] = rhodold;
        Sk[S_TAUTILDE] = tautilde; Sk[S_THETATILDE] = thetatilde;
        Sk[S_C] = c; Sk[S_S] = s; Sk[S_THETA] = thetanew;
        Sk[S_PHIBAR] = normr; Sk[S_PSI] = normar;
        a.ctl[C_ITERS] = k;
        a.ctl[C_CNT0 + (1 - a.parity)] = k + 1;
    }
}

}  // namespace lsqr

// ---------------------------------------------------------------- launchers --
// Instantiated once per vector type V in kernels_f64.hip / kernels_f32.hip.
namespace lsqr {

template <class M, class V>
static void fwd_launch_m(hipStream_t st, int grid, const RowFmt &R, const FwdArgs &a)
{
    if (R.slot) {
        const size_t sh = (size_t)R.gcap * sizeof(typename AccOf<V>::type);
        if constexpr (sizeof(M) == 2) {
            if (lcol_octs_ok(R)) {
                hipLaunchKernelGGL((k_fwd_lcol_pair<M, V, 8>), dim3(grid), dim3(kBlock), sh, st, a);
                return;
            }
        }
        if constexpr (sizeof(M) <= 4) {
            if (lcol_quads_ok(R)) {
                hipLaunchKernelGGL((k_fwd_lcol_pair<M, V, 4>), dim3(grid), dim3(kBlock), sh, st, a);
                return;
            }
        }
        if (lcol_pairs_ok(R)) {
            hipLaunchKernelGGL((k_fwd_lcol_pair<M, V, 2>), dim3(grid), dim3(kBlock), sh, st, a);
            return;
        }
        hipLaunchKernelGGL((k_fwd_lcol<M, V>), dim3(grid), dim3(kBlock), sh, st, a);
        return;
    }
    switch (R.lpr) {
    case 4: hipLaunchKernelGGL((k_fwd_csr<M, V, 4>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_fwd_csr<M, V, 8>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_fwd_csr<M, V, 16>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 32: hipLaunchKernelGGL((k_fwd_csr<M, V, 32>), dim3(grid), dim3(kBlock), 0, st, a); break;
    default:
        if (LSQR_FWD_PIPE) hipLaunchKernelGGL((k_fwd_pipe<M, V>), dim3(grid), dim3(kBlock), 0, st, a);
        else hipLaunchKernelGGL((k_fwd_csr<M, V, 64>), dim3(grid), dim3(kBlock), 0, st, a);
        break;
    }
}

template <class M, class V>
static void adj_launch_m(hipStream_t st, int grid, const ColFmt &C, const AdjArgs &a)
{
    if (C.nrp) {
        if (C.pairs) {
            if constexpr (sizeof(M) == 2) {
                if (C.pairs == 8) hipLaunchKernelGGL((k_adj_npair<M, V, 8>), dim3(grid), dim3(kBlock), 0, st, a);
                else if (C.pairs == 4) hipLaunchKernelGGL((k_adj_npair<M, V, 4>), dim3(grid), dim3(kBlock), 0, st, a);
                else hipLaunchKernelGGL((k_adj_npair<M, V, 2>), dim3(grid), dim3(kBlock), 0, st, a);
            } else if constexpr (sizeof(M) == 4) {
                if (C.pairs == 4) hipLaunchKernelGGL((k_adj_npair<M, V, 4>), dim3(grid), dim3(kBlock), 0, st, a);
                else hipLaunchKernelGGL((k_adj_npair<M, V, 2>), dim3(grid), dim3(kBlock), 0, st, a);
            } else {
                hipLaunchKernelGGL((k_adj_npair<M, V, 2>), dim3(grid), dim3(kBlock), 0, st, a);
            }
        }
        else hipLaunchKernelGGL((k_adj_nruns<M, V>), dim3(grid), dim3(kBlock), 0, st, a);
        return;
    }
    switch (C.lpc) {
    case 4: hipLaunchKernelGGL((k_adj<M, V, 4>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_adj<M, V, 8>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_adj<M, V, 16>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 32: hipLaunchKernelGGL((k_adj<M, V, 32>), dim3(grid), dim3(kBlock), 0, st, a); break;
    default: hipLaunchKernelGGL((k_adj<M, V, 64>), dim3(grid), dim3(kBlock), 0, st, a); break;
    }
}

// The stored value types a vector type supports: FP64 vectors take FP64
// values (and, in the transposed product of the refinements, FP32 and
// quantised values); FP32 vectors take FP32 and quantised values.
template <class V> struct Wide { static constexpr bool value = false; };
template <> struct Wide<double> { static constexpr bool value = true; };

template <class V>
hipError_t fwd_launch(hipStream_t st, const Problem &P, int grid, const RowFmt &R,
                      const void *z, const void *Tprev, void *Tcur, void *Ts, double *part_out,
                      const double *part_v, int np_v, double *S, int *ctl, int parity,
                      double tol, int mode)
{
    FwdArgs a{R.rp, R.ci, R.val, R.sigma, P.m, (int)P.n, P.nx, P.ny,
              P.nz, P.w, P.damp, z, Tprev, Tcur, Ts, part_out, part_v, np_v, S, ctl, parity,
              mode, tol, R.wrow, R.wgrid, R.gp, R.gcp, R.gcol, R.slot, R.ngroups, R.gcap};
    if constexpr (Wide<V>::value) {
        if (R.vt != VT_F64) return hipErrorInvalidValue;
        fwd_launch_m<double, V>(st, grid, R, a);
    } else {
        switch (R.vt) {
        case VT_F32: fwd_launch_m<float, V>(st, grid, R, a); break;
        case VT_BF16: fwd_launch_m<bf16_t, V>(st, grid, R, a); break;
        case VT_F16: fwd_launch_m<fp16_t, V>(st, grid, R, a); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

// Workgroups of k_fwd_pipe per compute unit for R's value type.
template <class V>
int fwd_pipe_blocks_per_cu(const RowFmt &R)
{
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    if constexpr (Wide<V>::value) {
        if (R.vt == VT_F64)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_pipe<double, V>, kBlock, 0);
    } else {
        switch (R.vt) {
        case VT_F32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_pipe<float, V>, kBlock, 0); break;
        case VT_BF16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_pipe<bf16_t, V>, kBlock, 0); break;
        case VT_F16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_pipe<fp16_t, V>, kBlock, 0); break;
        default: break;
        }
    }
    return e == hipSuccess ? nb : 0;
}

// Workgroups of k_fwd_lcol per compute unit for R's value type and group size.
template <class V>
int fwd_lcol_blocks_per_cu(const RowFmt &R)
{
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    const size_t sh = (size_t)R.gcap * sizeof(typename AccOf<V>::type);
    if constexpr (Wide<V>::value) {
        if (R.vt == VT_F64)
            e = lcol_pairs_ok(R)
                    ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_lcol_pair<double, V, 2>, kBlock, sh)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_lcol<double, V>, kBlock, sh);
    } else {
#define LSQR_LCOL_OCC(M_)                                                                                   \
    (sizeof(M_) == 2 && lcol_octs_ok(R) ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_lcol_pair<M_, V, (sizeof(M_) == 2 ? 8 : 4)>, kBlock, sh) \
     : lcol_quads_ok(R) ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_lcol_pair<M_, V, 4>, kBlock, sh) \
     : lcol_pairs_ok(R) ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_lcol_pair<M_, V, 2>, kBlock, sh) \
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_lcol<M_, V>, kBlock, sh))
        switch (R.vt) {
        case VT_F32: e = LSQR_LCOL_OCC(float); break;
        case VT_BF16: e = LSQR_LCOL_OCC(bf16_t); break;
        case VT_F16: e = LSQR_LCOL_OCC(fp16_t); break;
        default: break;
        }
#undef LSQR_LCOL_OCC
    }
    return e == hipSuccess ? nb : 0;
}

// Workgroups of the node-run transposed product per compute unit for C's
// value type (0 when C does not use it).
template <class V>
int adj_nruns_blocks_per_cu(const ColFmt &C)
{
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    if (!C.nrp) return 0;
#define LSQR_ADJ_OCC(M_) (C.pairs == 8 && sizeof(M_) == 2                                                              \
                              ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adj_npair<M_, V, (sizeof(M_) == 2 ? 8 : 2)>, kBlock, 0) \
                          : C.pairs == 4 && sizeof(M_) <= 4                                                              \
                              ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adj_npair<M_, V, (sizeof(M_) <= 4 ? 4 : 2)>, kBlock, 0) \
                          : C.pairs ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adj_npair<M_, V, 2>, kBlock, 0) \
                              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adj_nruns<M_, V>, kBlock, 0))
    switch (C.vt) {
    case VT_F64:
        if constexpr (Wide<V>::value) e = LSQR_ADJ_OCC(double);
        break;
    case VT_F32:
        if constexpr (!Wide<V>::value) e = LSQR_ADJ_OCC(float);
        break;
    case VT_BF16: e = LSQR_ADJ_OCC(bf16_t); break;
    case VT_F16: e = LSQR_ADJ_OCC(fp16_t); break;
    default: break;
    }
#undef LSQR_ADJ_OCC
    // at most 4 workgroups per compute unit for depth pairs, 6 for words of
    // 4 or 8 depths: with the registers the scan frees, one more resident
    // workgroup per compute unit (a larger single-round grid) measured
    // FP64 918 -> 940 us and BF16 385 -> 496 us on the config-1 system,
    // and fewer than these caps were slower too
    const int cap = C.pairs == 2 ? 4 : C.pairs ? 6 : nb;
    if (nb > cap) nb = cap;
    return e == hipSuccess ? nb : 0;
}

template <class V>
hipError_t adj_launch(hipStream_t st, const Problem &P, int grid, const ColFmt &C,
                      const double *d, const void *T, const void *Tg, const void *v, void *q,
                      double *part_out, const double *part_t, int np_t, double *S, int *ctl,
                      int parity, int mode, int data_only)
{
    AdjArgs a{C.cp, C.ri, C.val, P.m, (int)P.n, P.nx, P.ny, P.nz, P.w, P.damp, d, T, Tg, v, q,
              part_out, part_t, np_t, S, ctl, parity, mode, data_only,
              C.nrp, C.nvq, C.nrow, C.ndesc, C.norder};
    switch (C.vt) {
    case VT_F64:
        if constexpr (Wide<V>::value) adj_launch_m<double, V>(st, grid, C, a);
        else return hipErrorInvalidValue;
        break;
    case VT_F32: adj_launch_m<float, V>(st, grid, C, a); break;
    case VT_BF16: adj_launch_m<bf16_t, V>(st, grid, C, a); break;
    case VT_F16: adj_launch_m<fp16_t, V>(st, grid, C, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class V>
hipError_t init_launch(hipStream_t st, const Problem &P, int grid, const double *rhs, int full,
                       void *T0, const float *sigma, void *Ts0, double *y, void *vzero,
                       double *part, int *ctl, int kmax)
{
    hipLaunchKernelGGL((k_init_rhs<V>), dim3(grid), dim3(kBlock), 0, st, P.m, P.n, rhs, full,
                       (V *)T0, sigma, (V *)Ts0, y, (V *)vzero, part, ctl, kmax);
    return hipGetLastError();
}

template <class V>
hipError_t update_launch(hipStream_t st, const Problem &P, int grid, const double *d,
                         const void *q, void *v, double *w, double *y, void *z, double *part_out,
                         const double *part_q, int np_q, double *S, int *ctl, int parity, int mode,
                         double *hbar)
{
    UpdArgs a{(int)P.n, d, q, v, w, y, z, part_out, part_q, np_q, S, ctl, parity, mode, hbar};
    if (hbar) hipLaunchKernelGGL((k_update_lsmr<V>), dim3(grid), dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL((k_update<V>), dim3(grid), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

#define LSQR_INSTANTIATE_LAUNCHERS(V)                                                            \
    template int fwd_pipe_blocks_per_cu<V>(const RowFmt &);                                      \
    template int fwd_lcol_blocks_per_cu<V>(const RowFmt &);                                      \
    template int adj_nruns_blocks_per_cu<V>(const ColFmt &);                                     \
    template hipError_t fwd_launch<V>(hipStream_t, const Problem &, int, const RowFmt &,         \
                                      const void *, const void *, void *, void *, double *,      \
                                      const double *, int, double *, int *, int, double, int);   \
    template hipError_t adj_launch<V>(hipStream_t, const Problem &, int, const ColFmt &,         \
                                      const double *, const void *, const void *, const void *,  \
                                      void *, double *, const double *, int, double *, int *,    \
                                      int, int, int);                                            \
    template hipError_t init_launch<V>(hipStream_t, const Problem &, int, const double *, int,   \
                                       void *, const float *, void *, double *, void *,          \
                                       double *, int *, int);                                    \
    template hipError_t update_launch<V>(hipStream_t, const Problem &, int, const double *,      \
                                         const void *, void *, double *, double *, void *,       \
                                         double *, const double *, int, double *, int *, int,    \
                                         int, double *);

}  // namespace lsqr
