// Type-independent kernels: finalisation, scaling, Jacobi norms, validation,
// value conversion and quantisation, and the element-wise steps of the FP64
// iterative refinement.  Also the vector-type dispatch of the LSQR launchers.
#include <math.h>

#include <algorithm>

#include "lsqr_kernels.cuh"

namespace lsqr {

template <class V>
hipError_t fwd_launch(hipStream_t, const Problem &, int, const RowFmt &, const void *, const void *,
                      void *, void *, double *, const double *, int, double *, int *, int, double,
                      int);
template <class V>
hipError_t adj_launch(hipStream_t, const Problem &, int, const ColFmt &, const double *,
                      const void *, const void *, const void *, void *, double *, const double *,
                      int, double *, int *, int, int, int);
template <class V>
hipError_t init_launch(hipStream_t, const Problem &, int, const double *, int, void *,
                       const float *, void *, double *, void *, double *, int *, int);
template <class V>
hipError_t update_launch(hipStream_t, const Problem &, int, const double *, const void *, void *,
                         double *, double *, void *, double *, const double *, int, double *,
                         int *, int, int, double *);

template <class V>
int fwd_pipe_blocks_per_cu(const RowFmt &);
template <class V>
int fwd_lcol_blocks_per_cu(const RowFmt &);

// Workgroups the device holds at once at per_cu per compute unit (0 when unknown).
static int resident(int per_cu)
{
    int dev = 0, cus = 0;
    if (per_cu < 1 || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return 0;
    return per_cu * cus;
}

// Balanced partition of the CSR rows into `waves` contiguous ranges: boundary
// w is the first row r with rp[r] + kRowCost r >= w (nnz + kRowCost m) / waves
// (each row also costs a reduction and a store, counted as kRowCost entries).
// One thread per boundary, binary search; boundaries are non-decreasing,
// wrow[0] = 0, wrow[waves] = m.
constexpr int64_t kRowCost = 64;

__global__ void k_wave_rows(const int64_t *rp, int64_t m, int waves, int32_t *wrow)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w > waves) return;
    const int64_t total = rp[m] + kRowCost * m;
    const int64_t target = (int64_t)(((__int128)total * w) / waves);
    int64_t lo = 0, hi = m;                          // first r in [0, m] with cost(r) >= target
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (rp[mid] + kRowCost * mid >= target) hi = mid;
        else lo = mid + 1;
    }
    wrow[w] = (int32_t)(w == waves ? m : lo);
}

void launch_wave_rows(hipStream_t st, const int64_t *rp, int64_t m, int waves, int32_t *wrow)
{
    hipLaunchKernelGGL(k_wave_rows, dim3((waves + 1 + 255) / 256), dim3(256), 0, st, rp, m, waves,
                       wrow);
}

// Balanced partition of row groups into `parts` contiguous ranges: boundary w
// is the first group g with cost(g) >= w cost(ng) / parts, cost(g) = rp[gp[g]]
// + kRowCost gp[g] (entries and rows before group g).  cost is strictly
// increasing (every group has a row), so boundaries are non-decreasing,
// wgrp[0] = 0 and wgrp[parts] = ng.
__global__ void k_group_parts(const int64_t *rp, const int32_t *gp, int ng, int parts, int32_t *wgrp)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w > parts) return;
    const int64_t total = rp[gp[ng]] + kRowCost * (int64_t)gp[ng];
    const int64_t target = (int64_t)(((__int128)total * w) / parts);
    int lo = 0, hi = ng;
    while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if (rp[gp[mid]] + kRowCost * (int64_t)gp[mid] >= target) hi = mid;
        else lo = mid + 1;
    }
    wgrp[w] = w == parts ? ng : lo;
}

void launch_group_parts(hipStream_t st, const int64_t *rp, const int32_t *gp, int ng, int parts,
                        int32_t *wgrp)
{
    hipLaunchKernelGGL(k_group_parts, dim3((parts + 1 + 255) / 256), dim3(256), 0, st, rp, gp, ng,
                       parts, wgrp);
}

int fwd_lcol_grid(int vec, const RowFmt &R)
{
    if (!R.slot) return 0;
    const int g = resident(vec == VT_F64 ? fwd_lcol_blocks_per_cu<double>(R) : fwd_lcol_blocks_per_cu<float>(R));
    return std::min(g, 2048);
}

template <class V>
int adj_nruns_blocks_per_cu(const ColFmt &);


int adj_nruns_grid(int vec, const ColFmt &C)
{
    return resident(vec == VT_F64 ? adj_nruns_blocks_per_cu<double>(C) : adj_nruns_blocks_per_cu<float>(C));
}

int fwd_pipe_parts(int grid) { return LSQR_FWD_WG_ROWS ? grid : grid * (kBlock / 64); }

int fwd_pipe_grid(int vec, const RowFmt &R)
{
    if (!LSQR_FWD_PIPE || R.slot || R.lpr != 64) return 0;
    const int per_cu = vec == VT_F64 ? fwd_pipe_blocks_per_cu<double>(R) : fwd_pipe_blocks_per_cu<float>(R);
    int dev = 0, cus = 0;
    if (per_cu < 1 || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return 0;
    return std::min(per_cu * cus, 2048);
}

size_t vt_size(int vt)
{
    switch (vt) {
    case VT_F64: return 8;
    case VT_F32: return 4;
    default: return 2;
    }
}

void launch_init(hipStream_t st, const Problem &P, int grid, int vec, const double *rhs, int full,
                 void *T0, const float *sigma, void *Ts0, double *y, void *vzero, double *part,
                 int *ctl, int kmax)
{
    if (vec == VT_F64) init_launch<double>(st, P, grid, rhs, full, T0, sigma, Ts0, y, vzero, part, ctl, kmax);
    else init_launch<float>(st, P, grid, rhs, full, T0, sigma, Ts0, y, vzero, part, ctl, kmax);
}

void launch_fwd(hipStream_t st, const Problem &P, int grid, int vec, const RowFmt &R,
                const void *z, const void *Tprev, void *Tcur, void *Ts, double *part_out,
                const double *part_v, int np_v, double *S, int *ctl, int parity, double tol,
                int mode)
{
    if (vec == VT_F64)
        fwd_launch<double>(st, P, grid, R, z, Tprev, Tcur, Ts, part_out, part_v, np_v, S, ctl, parity, tol, mode);
    else
        fwd_launch<float>(st, P, grid, R, z, Tprev, Tcur, Ts, part_out, part_v, np_v, S, ctl, parity, tol, mode);
}

void launch_adj(hipStream_t st, const Problem &P, int grid, int vec, const ColFmt &C,
                const double *d, const void *T, const void *Tg, const void *v, void *q,
                double *part_out, const double *part_t, int np_t, double *S, int *ctl,
                int parity, int mode, int data_only)
{
    if (vec == VT_F64)
        adj_launch<double>(st, P, grid, C, d, T, Tg, v, q, part_out, part_t, np_t, S, ctl, parity, mode, data_only);
    else
        adj_launch<float>(st, P, grid, C, d, T, Tg, v, q, part_out, part_t, np_t, S, ctl, parity, mode, data_only);
}

void launch_update(hipStream_t st, const Problem &P, int grid, int vec, const double *d,
                   const void *q, void *v, double *w, double *y, void *z, double *part_out,
                   const double *part_q, int np_q, double *S, int *ctl, int parity, int mode,
                   double *hbar)
{
    if (vec == VT_F64)
        update_launch<double>(st, P, grid, d, q, v, w, y, z, part_out, part_q, np_q, S, ctl, parity,
                              mode, hbar);
    else
        update_launch<float>(st, P, grid, d, q, v, w, y, z, part_out, part_q, np_q, S, ctl, parity,
                             mode, hbar);
}

// --------------------------------------------------------------- finalize --
// eta of the last iteration (unless a stop rule already fired), the stop
// reason, and dm = D y (or dm += D y).
__global__ __launch_bounds__(kBlock) void k_finalize(int n, const double *d, const double *y,
                                                     double *dm, const double *part_v, int np_v,
                                                     double *S, int *ctl, double tol, int accumulate)
{
#pragma clang fp contract(off)
    __shared__ double lds[4];
    const int kk = ctl[C_ITERS];
    const bool stopped = ctl[C_STOP] != 0;
    if (!stopped && kk >= 1) {
        const double vn = sqrt(reduce_partials(part_v, np_v, lds));
        double *Sk = S + (int64_t)kk * kStateWords;
        // |Abar^T bbar| was stored by the forward kernel of iteration 1 (from
        // |D^-1 v_1|); LSMR: the scaled normal residual |zetabar| / (alpha_1 beta_1)
        const double arnorm0 = S[S_ARNORM0];
        const double eta = S[S_METHOD] != 0.0 ? Sk[S_PSI] / arnorm0 : Sk[S_PSI] * vn / arnorm0;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            Sk[S_ETA] = eta;
            Sk[S_VNORM] = vn;
            int istop = 2;
            if (tol > 0.0 && eta <= tol) istop = 1;
            else if (Sk[S_ALPHA] == 0.0 || Sk[S_BETA] == 0.0) istop = 3;
            ctl[C_ISTOP] = istop;
        }
    }
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock) {
        const double v = d[j] * y[j];
        dm[j] = accumulate ? dm[j] + v : v;
    }
}

void launch_finalize(hipStream_t st, const Problem &P, int grid, const double *d,
                     const double *y, double *dm, const double *part_v, int np_v, double *S,
                     int *ctl, double tol, int accumulate)
{
    hipLaunchKernelGGL(k_finalize, dim3(grid), dim3(kBlock), 0, st, (int)P.n, d, y, dm, part_v,
                       np_v, S, ctl, tol, accumulate);
}

// ---------------------------------------------------------------- helpers --
static inline int blocks_for(int64_t work, int per_block, int cap)
{
    int64_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    return (int)(b < cap ? b : cap);
}

__global__ void k_scale_vec(int64_t n, const double *d, const double *x, double *z)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        z[j] = d[j] * x[j];
}

void launch_scale_vec(hipStream_t st, int64_t n, const double *d, const double *x, double *z)
{
    hipLaunchKernelGGL(k_scale_vec, dim3(blocks_for(n, kBlock, 4096)), dim3(kBlock), 0, st, n, d,
                       x, z);
}

__global__ void k_fill(int64_t n, double value, double *x)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        x[j] = value;
}

void launch_fill(hipStream_t st, int64_t n, double value, double *x)
{
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, kBlock, 4096)), dim3(kBlock), 0, st, n, value,
                       x);
}

// d_j = 1 / |column j of Abar|: data entries from the CSC, the Laplacian column
// (centre -deg, deg ones) times w, and lambda.  One wave per column.
__global__ __launch_bounds__(kBlock) void k_jacobi(int n, int nx, int ny, int nz, double w,
                                                   double damp, const int64_t *cp,
                                                   const double *cv, double *d)
{
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    for (int j = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); j < n;
         j += gridDim.x * (kBlock / 64)) {
        double acc = 0.0;
        for (int64_t p = cp[j] + lane; p < cp[j + 1]; p += 64) acc += cv[p] * cv[p];
        acc = group_sum<64>(acc);
        if (lane == 0) {
            const int iz = j % nz, ixy = j / nz, ix = ixy % nx, iy = ixy / nx;
            const int deg = (ix > 0) + (ix < nx - 1) + (iy > 0) + (iy < ny - 1) + (iz > 0) +
                            (iz < nz - 1);
            const double lsq = (double)deg * (double)deg + (double)deg;
            const double s = acc + w * w * lsq + damp * damp;
            d[j] = 1.0 / sqrt(s);
        }
    }
}

void launch_jacobi(hipStream_t st, const Problem &P, const ColFmt &C, double *d)
{
    hipLaunchKernelGGL(k_jacobi, dim3(blocks_for(P.n, kBlock / 64, 8192)), dim3(kBlock), 0, st,
                       (int)P.n, P.nx, P.ny, P.nz, P.w, P.damp, C.cp, (const double *)C.val, d);
}

// Validation of a device-resident CSR: bit 1 row_ptr decreasing, bit 2 column
// out of range, bit 4 columns not strictly increasing, bit 8 non-finite value.
__global__ void k_check_csr(int64_t m, int64_t n, const int64_t *rp, const int32_t *ci,
                            const double *va, int *flag)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = rp[i], e = rp[i + 1];
        int f = 0;
        if (e < s) f |= 1;
        for (int64_t p = s; p < e && !(f & 1); ++p) {
            const int c = ci[p];
            if (c < 0 || c >= n) f |= 2;
            if (p > s && c <= ci[p - 1]) f |= 4;
            if (!isfinite(va[p])) f |= 8;
        }
        if (f) atomicOr(flag, f);
    }
}

void launch_check_csr(hipStream_t st, int64_t m, int64_t n, const int64_t *row_ptr,
                      const int32_t *col, const double *val, int *flag)
{
    hipLaunchKernelGGL(k_check_csr, dim3(blocks_for(m, kBlock, 8192)), dim3(kBlock), 0, st, m, n,
                       row_ptr, col, val, flag);
}

// bit 1 non-finite, bit 2 not positive (when positive != 0).
__global__ void k_check_vec(int64_t n, const double *x, int positive, int *flag)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        int f = 0;
        if (!isfinite(x[j])) f |= 1;
        else if (positive && !(x[j] > 0.0)) f |= 2;
        if (f) atomicOr(flag, f);
    }
}

void launch_check_vec(hipStream_t st, int64_t n, const double *x, int positive, int *flag)
{
    hipLaunchKernelGGL(k_check_vec, dim3(blocks_for(n, kBlock, 4096)), dim3(kBlock), 0, st, n, x,
                       positive, flag);
}

// ------------------------------------------------------ value conversion --
__global__ void k_convert_f32(int64_t nnz, const double *src, float *dst)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = (float)src[e];
}

void launch_convert_f32(hipStream_t st, int64_t nnz, const double *src, float *dst)
{
    hipLaunchKernelGGL(k_convert_f32, dim3(blocks_for(nnz, kBlock, 65536)), dim3(kBlock), 0, st,
                       nnz, src, dst);
}

// Round an FP64 value to the nearest value of a binary format with p
// significand bits (implicit bit included), minimum normal exponent emin and
// exponent bias `bias`, ties to even, directly from the FP64 bits (one
// rounding).  Returns the 16-bit encoding.
__device__ uint16_t round_rne16(double x, int p, int emin, int ebits, int bias)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint16_t sign = (uint16_t)((b >> 63) << 15);
    const int ex = (int)((b >> 52) & 0x7ff);
    const uint64_t man = b & 0xFFFFFFFFFFFFFull;
    if (ex == 0 && man == 0) return sign;
    uint64_t M;
    int E;                                   // |x| = M * 2^E
    if (ex == 0) { M = man; E = -1074; }
    else { M = man | (1ull << 52); E = ex - 1075; }
    const int lead = E + (63 - __clzll(M));  // floor(log2 |x|)
    int qe = lead - (p - 1);
    if (qe < emin - (p - 1)) qe = emin - (p - 1);
    const int shift = qe - E;
    uint64_t N;
    if (shift <= 0) {
        N = M << (-shift);
    } else if (shift >= 64) {
        N = 0;
    } else {
        N = M >> shift;
        const uint64_t rem = M & ((1ull << shift) - 1);
        const uint64_t half = 1ull << (shift - 1);
        if (rem > half || (rem == half && (N & 1))) N += 1;
    }
    if (N == 0) return sign;
    if (N >= (1ull << p)) { N >>= 1; qe += 1; }
    if (N < (1ull << (p - 1))) return (uint16_t)(sign | (uint16_t)N);   // subnormal
    const int ef = qe + (p - 1) + bias;
    if (ef >= (1 << ebits) - 1) return (uint16_t)(sign | (uint16_t)(((1 << ebits) - 1) << (p - 1)));
    return (uint16_t)(sign | (uint16_t)(ef << (p - 1)) | (uint16_t)(N - (1ull << (p - 1))));
}

__device__ __forceinline__ uint16_t quantise(double x, int vt)
{
    return vt == VT_BF16 ? round_rne16(x, 8, -126, 8, 127) : round_rne16(x, 11, -14, 5, 15);
}

// Row scale: the power of two 2^ceil(log2 max_j |g_ij|) (BF16), or that
// power times 2^-14 (FP16, so the largest entry sits near 2^14 and small
// entries stay out of the subnormal range).  Empty or zero rows get 1.
__global__ void k_row_scales(int64_t m, const int64_t *rp, const double *val, int vt, float *sigma)
{
    const int lane = threadIdx.x & 63;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < m;
         i += ((int64_t)gridDim.x * blockDim.x) >> 6) {
        double mx = 0.0;
        for (int64_t e = rp[i] + lane; e < rp[i + 1]; e += 64) mx = fmax(mx, fabs(val[e]));
        for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
        if (lane == 0) {
            float s = 1.0f;
            if (mx > 0.0) {
                int e2;
                const double f = frexp(mx, &e2);           // mx = f 2^e2, f in [0.5, 1)
                const int E = f == 0.5 ? e2 - 1 : e2;      // ceil(log2 mx)
                s = ldexpf(1.0f, vt == VT_BF16 ? E : E - 14);
            }
            sigma[i] = s;
        }
    }
}

void launch_row_scales(hipStream_t st, int64_t m, const int64_t *rp, const double *val, int vt,
                       float *sigma)
{
    hipLaunchKernelGGL(k_row_scales, dim3(blocks_for(m * 64, kBlock, 65536)), dim3(kBlock), 0, st,
                       m, rp, val, vt, sigma);
}

__global__ void k_quantise_rows(int64_t m, const int64_t *rp, const double *val,
                                const float *sigma, int vt, uint16_t *q)
{
    const int lane = threadIdx.x & 63;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < m;
         i += ((int64_t)gridDim.x * blockDim.x) >> 6) {
        const double s = (double)sigma[i];
        for (int64_t e = rp[i] + lane; e < rp[i + 1]; e += 64) q[e] = quantise(val[e] / s, vt);
    }
}

void launch_quantise_rows(hipStream_t st, int64_t m, const int64_t *rp, const double *val,
                          const float *sigma, int vt, uint16_t *q)
{
    hipLaunchKernelGGL(k_quantise_rows, dim3(blocks_for(m * 64, kBlock, 65536)), dim3(kBlock), 0,
                       st, m, rp, val, sigma, vt, q);
}

// The transpose's values quantised with the scale of their row: bitwise the
// same codes as the row-major copy, so the two products are exact transposes.
__global__ void k_quantise_cols(int64_t nnz, const int32_t *ri, const double *cv,
                                const float *sigma, int vt, uint16_t *q)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x)
        q[p] = quantise(cv[p] / (double)sigma[ri[p]], vt);
}

void launch_quantise_cols(hipStream_t st, int64_t nnz, const int32_t *ri, const double *cv,
                          const float *sigma, int vt, uint16_t *q)
{
    hipLaunchKernelGGL(k_quantise_cols, dim3(blocks_for(nnz, kBlock, 65536)), dim3(kBlock), 0, st,
                       nnz, ri, cv, sigma, vt, q);
}

// ------------------------------------------------------------ refinement --
__global__ __launch_bounds__(kBlock) void k_residual(int64_t m, int64_t n, const double *dt,
                                                     const double *y, double *rbar, double *part)
{
#pragma clang fp contract(off)
    __shared__ double lds[4];
    const int64_t mb = m + 2 * n;
    double sq = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < mb;
         i += (int64_t)gridDim.x * kBlock) {
        const double b = i < m ? dt[i] : 0.0;
        const double r = y ? b - y[i] : b;
        rbar[i] = r;
        sq += r * r;
    }
    const double tot = block_sum(sq, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

void launch_residual(hipStream_t st, const Problem &P, int grid, const double *dt,
                     const double *y, double *rbar, double *part)
{
    hipLaunchKernelGGL(k_residual, dim3(grid), dim3(kBlock), 0, st, P.m, P.n, dt, y, rbar, part);
}

__global__ __launch_bounds__(kBlock) void k_sum_partials(const double *part, int np, double *out)
{
    __shared__ double lds[4];
    const double s = reduce_partials(part, np, lds);
    if (threadIdx.x == 0) out[0] = s;
}

void launch_sum_partials(hipStream_t st, const double *part, int np, double *out)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, st, part, np, out);
}

}  // namespace lsqr

namespace lsqr {

template <class T>
__global__ void k_gather_runs(int64_t nr, const uint32_t *src, const uint32_t *dst,
                              const uint16_t *desc, const T *in, T *out)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nr;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int len = desc[r] & 255;
        const int64_t s = src[r], d = dst[r];
        for (int e = 0; e < len; ++e) out[d + e] = in[s + e];
    }
}

void launch_gather_runs(hipStream_t st, int64_t nr, const uint32_t *src, const uint32_t *dst,
                        const uint16_t *desc, const void *in, void *out, int elem_bytes)
{
    if (nr <= 0) return;
    const int grid = (int)std::min<int64_t>((nr + 255) / 256, 65536);
    switch (elem_bytes) {
    case 8:
        hipLaunchKernelGGL(k_gather_runs<uint64_t>, dim3(grid), dim3(256), 0, st, nr, src, dst,
                           desc, (const uint64_t *)in, (uint64_t *)out);
        break;
    case 4:
        hipLaunchKernelGGL(k_gather_runs<uint32_t>, dim3(grid), dim3(256), 0, st, nr, src, dst,
                           desc, (const uint32_t *)in, (uint32_t *)out);
        break;
    default:
        hipLaunchKernelGGL(k_gather_runs<uint16_t>, dim3(grid), dim3(256), 0, st, nr, src, dst,
                           desc, (const uint16_t *)in, (uint16_t *)out);
        break;
    }
}

}  // namespace lsqr
