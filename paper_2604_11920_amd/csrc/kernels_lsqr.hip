// FP64 LSQR kernels for gfx950 (wave64).
//
// One LSQR iteration k is three launches on one stream:
//   fwd    t = Abar D v_k - alpha_k u_k over the CSR data rows, the 7-point
//          smoothing rows and the damping rows; per-workgroup partial sums of t^2
//   adj    beta_{k+1} from those partials; q = D Abar^T t / beta - beta v_k over
//          the stored CSC (no atomics); partial sums of q^2
//   update alpha_{k+1}, the Givens step (Paige & Saunders) and the x/w/v sweep
// Every workgroup of a consumer kernel reduces the producer's partials in the
// same fixed order, so all workgroups hold bitwise-identical scalars without a
// separate reduction launch or atomics.  The iteration index, stop flag and
// per-iteration scalars live in device memory, so a block of iterations can be
// captured once as a hipGraph and replayed.
#include <math.h>

#include "internal.h"

namespace lsqr {

// ------------------------------------------------------------ reductions --
template <int W>
__device__ __forceinline__ double group_sum(double v)
{
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
__device__ __forceinline__ double stencil(const double *x, int p, int nx, int ny, int nz)
{
#pragma clang fp contract(off)
    const int iz = p % nz, ixy = p / nz, ix = ixy % nx, iy = ixy / nx;
    const int sxy = nx * nz;
    double acc = 0.0;
    int deg = 0;
    if (ix > 0) { acc += x[p - nz]; ++deg; }
    if (ix < nx - 1) { acc += x[p + nz]; ++deg; }
    if (iy > 0) { acc += x[p - sxy]; ++deg; }
    if (iy < ny - 1) { acc += x[p + sxy]; ++deg; }
    if (iz > 0) { acc += x[p - 1]; ++deg; }
    if (iz < nz - 1) { acc += x[p + 1]; ++deg; }
    return acc - (double)deg * x[p];
}

// ------------------------------------------------------------------ init --
// T0 = bbar = [dt; 0; 0]; y = 0; vzero = 0; partial sums of dt^2; control words.
__global__ __launch_bounds__(kBlock) void k_init_rhs(int64_t m, int64_t n, const double *dt,
                                                     double *T0, double *y, double *vzero,
                                                     double *part, int *ctl, int kmax)
{
    __shared__ double lds[4];
    const int64_t mb = m + 2 * n;
    double sq = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < mb;
         i += (int64_t)gridDim.x * kBlock) {
        double b = i < m ? dt[i] : 0.0;
        T0[i] = b;
        sq += b * b;
        if (i < n) { y[i] = 0.0; vzero[i] = 0.0; }
    }
    double tot = block_sum(sq, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl[C_STOP] = 0; ctl[C_ISTOP] = 2; ctl[C_ITERS] = 0; ctl[C_ERR] = 0;
        ctl[C_CNT0] = 1; ctl[C_CNT1] = 0; ctl[C_KMAX] = kmax;
    }
}

// --------------------------------------------------------------- forward --
struct FwdArgs {
    const int64_t *rp;
    const int32_t *ci;
    const double *va;
    int64_t m;
    int n, nx, ny, nz;
    double w, damp;
    const double *z;        // D v   [n]
    const double *Tprev;    // t of the previous step (u = Tprev / beta_k) [m+2n]
    double *Tcur;           // [m+2n]
    double *part_out;       // [gridDim.x]
    const double *part_v;   // partials of |D^-1 v_k|^2
    int np_v;
    double *S;
    int *ctl;
    int parity;
    int mode;
    double tol;
};

template <int LPR>
__global__ __launch_bounds__(kBlock) void k_fwd(FwdArgs a)
{
#pragma clang fp contract(off)
    __shared__ double lds[4];
    double alpha = 0.0, beta = 1.0;
    if (a.mode == MODE_ITER) {
        if (a.ctl[C_STOP]) return;
        const int k = a.ctl[C_CNT0 + a.parity];
        if (k > a.ctl[C_KMAX]) return;
        double *Sp = a.S + (int64_t)(k - 1) * kStateWords;
        alpha = Sp[S_ALPHA];
        beta = Sp[S_BETA];
        const double vn = sqrt(reduce_partials(a.part_v, a.np_v, lds));
        double arnorm0, eta = 1.0;
        bool stop = false;
        int istop = 2;
        if (k == 1) {
            arnorm0 = (a.S[S_ALPHA] * a.S[S_BETA]) * vn;
        } else {
            arnorm0 = a.S[S_ARNORM0];
            eta = Sp[S_PSI] * vn / arnorm0;
            if (a.tol > 0.0 && eta <= a.tol) { stop = true; istop = 1; }
            else if (alpha == 0.0 || beta == 0.0) { stop = true; istop = 3; }
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (k == 1) { a.S[S_ARNORM0] = arnorm0; a.S[S_VNORM] = vn; }
            else { Sp[S_ETA] = eta; Sp[S_VNORM] = vn; }
            if (stop) { a.ctl[C_ISTOP] = istop; a.ctl[C_STOP] = 1; }
        }
        if (stop) return;
    }
    const bool has_prev = a.mode == MODE_ITER;
    double sq = 0.0;

    // data rows: LPR lanes per row, grid-stride over rows
    constexpr int RPB = kBlock / LPR;
    const int lane = threadIdx.x % LPR;
    const int64_t gstride = (int64_t)gridDim.x * RPB;
    for (int64_t row = (int64_t)blockIdx.x * RPB + threadIdx.x / LPR; row < a.m; row += gstride) {
        const int64_t s = a.rp[row], e = a.rp[row + 1];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int64_t j = s + lane;
        for (; j + 3 * LPR < e; j += 4 * LPR) {
            const int c0 = __builtin_nontemporal_load(a.ci + j);
            const int c1 = __builtin_nontemporal_load(a.ci + j + LPR);
            const int c2 = __builtin_nontemporal_load(a.ci + j + 2 * LPR);
            const int c3 = __builtin_nontemporal_load(a.ci + j + 3 * LPR);
            const double v0 = __builtin_nontemporal_load(a.va + j);
            const double v1 = __builtin_nontemporal_load(a.va + j + LPR);
            const double v2 = __builtin_nontemporal_load(a.va + j + 2 * LPR);
            const double v3 = __builtin_nontemporal_load(a.va + j + 3 * LPR);
            a0 = fma(v0, a.z[c0], a0);
            a1 = fma(v1, a.z[c1], a1);
            a2 = fma(v2, a.z[c2], a2);
            a3 = fma(v3, a.z[c3], a3);
        }
        for (; j < e; j += LPR)
            a0 = fma(__builtin_nontemporal_load(a.va + j), a.z[__builtin_nontemporal_load(a.ci + j)], a0);
        double acc = group_sum<LPR>((a0 + a1) + (a2 + a3));
        if (lane == 0) {
            const double u = has_prev ? a.Tprev[row] / beta : 0.0;
            const double t = acc - alpha * u;
            a.Tcur[row] = t;
            sq += t * t;
        }
    }
    // smoothing rows (m .. m+n) and damping rows (m+n .. m+2n): one thread each
    const int64_t nreg = 2 * (int64_t)a.n;
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < nreg;
         r += (int64_t)gridDim.x * kBlock) {
        double yv;
        if (r < a.n) yv = stencil(a.z, (int)r, a.nx, a.ny, a.nz) * a.w;
        else yv = a.damp * a.z[r - a.n];
        const double u = has_prev ? a.Tprev[a.m + r] / beta : 0.0;
        const double t = yv - alpha * u;
        a.Tcur[a.m + r] = t;
        sq += t * t;
    }
    const double tot = block_sum(sq, lds);
    if (threadIdx.x == 0) a.part_out[blockIdx.x] = tot;
}

// ------------------------------------------------------------- transposed --
struct AdjArgs {
    const int64_t *cp;
    const int32_t *ri;
    const double *cv;
    int64_t m;
    int n, nx, ny, nz;
    double w, damp;
    const double *d;        // column scale [n]
    const double *T;        // t [m+2n] (u = t / beta)
    const double *v;        // v_k [n] (nullptr in operator mode)
    double *q;              // out [n]
    double *part_out;
    const double *part_t;   // partials of |t|^2
    int np_t;
    double *S;
    int *ctl;
    int parity;
    int mode;
};

template <int LPC>
__global__ __launch_bounds__(kBlock) void k_adj(AdjArgs a)
{
#pragma clang fp contract(off)
    __shared__ double lds[4];
    double beta = 1.0;
    if (a.mode != MODE_OPERATOR) {
        if (a.ctl[C_STOP]) return;
        int k = 0;
        if (a.mode == MODE_ITER) {
            k = a.ctl[C_CNT0 + a.parity];
            if (k > a.ctl[C_KMAX]) return;
        }
        beta = sqrt(reduce_partials(a.part_t, a.np_t, lds));
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            a.S[(int64_t)k * kStateWords + S_BETA] = beta;
            if (a.mode == MODE_INIT && beta == 0.0) { a.ctl[C_ISTOP] = 0; a.ctl[C_STOP] = 1; }
        }
        if (beta == 0.0) return;   // breakdown: the update kernel sets alpha = 0
    }
    double sq = 0.0;
    constexpr int CPB = kBlock / LPC;
    const int lane = threadIdx.x % LPC;
    const int64_t tL = a.m, tD = a.m + a.n;
    for (int j = blockIdx.x * CPB + threadIdx.x / LPC; j < a.n; j += gridDim.x * CPB) {
        const int64_t s = a.cp[j], e = a.cp[j + 1];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int64_t p = s + lane;
        for (; p + 3 * LPC < e; p += 4 * LPC) {
            const int r0 = __builtin_nontemporal_load(a.ri + p);
            const int r1 = __builtin_nontemporal_load(a.ri + p + LPC);
            const int r2 = __builtin_nontemporal_load(a.ri + p + 2 * LPC);
            const int r3 = __builtin_nontemporal_load(a.ri + p + 3 * LPC);
            const double v0 = __builtin_nontemporal_load(a.cv + p);
            const double v1 = __builtin_nontemporal_load(a.cv + p + LPC);
            const double v2 = __builtin_nontemporal_load(a.cv + p + 2 * LPC);
            const double v3 = __builtin_nontemporal_load(a.cv + p + 3 * LPC);
            a0 = fma(v0, a.T[r0], a0);
            a1 = fma(v1, a.T[r1], a1);
            a2 = fma(v2, a.T[r2], a2);
            a3 = fma(v3, a.T[r3], a3);
        }
        for (; p < e; p += LPC)
            a0 = fma(__builtin_nontemporal_load(a.cv + p), a.T[__builtin_nontemporal_load(a.ri + p)], a0);
        const double g = group_sum<LPC>((a0 + a1) + (a2 + a3));
        if (lane == 0) {
            const double lap = stencil(a.T + tL, j, a.nx, a.ny, a.nz);
            const double sj = g + a.w * lap + a.damp * a.T[tD + j];
            const double xj = a.d[j] * sj;
            const double qj = a.v ? xj / beta - beta * a.v[j] : xj / beta;
            a.q[j] = qj;
            sq += qj * qj;
        }
    }
    const double tot = block_sum(sq, lds);
    if (threadIdx.x == 0) a.part_out[blockIdx.x] = tot;
}

// ----------------------------------------------------------------- update --
struct UpdArgs {
    int n;
    const double *d;
    const double *q;
    double *v, *w, *y, *z;
    double *part_out;       // partials of |D^-1 v_{k+1}|^2
    const double *part_q;   // partials of |q|^2
    int np_q;
    double *S;
    int *ctl;
    int parity;
    int mode;
};

__global__ __launch_bounds__(kBlock) void k_update(UpdArgs a)
{
#pragma clang fp contract(off)
    __shared__ double lds[4];
    if (a.ctl[C_STOP]) return;
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
            const double vj = a.q[j] / alpha;
            a.v[j] = vj;
            a.w[j] = vj;
            a.z[j] = a.d[j] * vj;
            const double dv = vj / a.d[j];
            sq += dv * dv;
        }
        const double tot = block_sum(sq, lds);
        if (threadIdx.x == 0) a.part_out[blockIdx.x] = tot;
        if (lead) {
            double *S0 = a.S;
            S0[S_ALPHA] = alpha; S0[S_RHOBAR] = alpha; S0[S_PHIBAR] = beta;
            S0[S_PSI] = alpha * beta; S0[S_ETA] = 1.0;
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
        const double vj = newv ? a.q[j] / alpha : a.v[j];
        if (newv) a.v[j] = vj;
        const double wj = a.w[j];
        a.y[j] = a.y[j] + t1 * wj;
        a.w[j] = vj - t2 * wj;
        a.z[j] = a.d[j] * vj;
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

// --------------------------------------------------------------- finalize --
// eta of the last iteration (unless a stop rule already fired), the stop
// reason, and dm = D y.
__global__ __launch_bounds__(kBlock) void k_finalize(int n, const double *d, const double *y,
                                                     double *dm, const double *part_v, int np_v,
                                                     double *S, int *ctl, double tol)
{
#pragma clang fp contract(off)
    __shared__ double lds[4];
    const int kk = ctl[C_ITERS];
    const bool stopped = ctl[C_STOP] != 0;
    if (!stopped && kk >= 1) {
        const double vn = sqrt(reduce_partials(part_v, np_v, lds));
        double *Sk = S + (int64_t)kk * kStateWords;
        // |Abar^T bbar| was stored by the forward kernel of iteration 1 (from |D^-1 v_1|)
        const double arnorm0 = S[S_ARNORM0];
        const double eta = Sk[S_PSI] * vn / arnorm0;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            Sk[S_ETA] = eta;
            Sk[S_VNORM] = vn;
            int istop = 2;
            if (tol > 0.0 && eta <= tol) istop = 1;
            else if (Sk[S_ALPHA] == 0.0 || Sk[S_BETA] == 0.0) istop = 3;
            ctl[C_ISTOP] = istop;
        }
    }
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock)
        dm[j] = d[j] * y[j];
}

// ---------------------------------------------------------------- helpers --
__global__ void k_scale_vec(int64_t n, const double *d, const double *x, double *z)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        z[j] = d[j] * x[j];
}

__global__ void k_fill(int64_t n, double value, double *x)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        x[j] = value;
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

// -------------------------------------------------------------- launchers --
static inline int blocks_for(int64_t work, int per_block, int cap)
{
    int64_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    return (int)(b < cap ? b : cap);
}

void launch_init_rhs(hipStream_t st, const Problem &P, const Geometry &g, const double *dt,
                     double *T0, double *y, double *vzero, double *part, int *ctl, int kmax)
{
    hipLaunchKernelGGL(k_init_rhs, dim3(g.g_fwd), dim3(kBlock), 0, st, P.m, P.n, dt, T0, y, vzero,
                       part, ctl, kmax);
}

template <int L>
static void fwd_t(hipStream_t st, int grid, const FwdArgs &a)
{
    hipLaunchKernelGGL(k_fwd<L>, dim3(grid), dim3(kBlock), 0, st, a);
}

void launch_fwd(hipStream_t st, const Problem &P, const Geometry &g, DevCSR A, const double *z,
                const double *Tprev, double *Tcur, double *part_out, const double *part_v,
                double *S, int *ctl, int parity, double tol, int mode)
{
    FwdArgs a{A.ptr, A.idx, A.val, P.m, (int)P.n, P.nx, P.ny, P.nz, P.w, P.damp, z, Tprev, Tcur,
              part_out, part_v, g.g_upd, S, ctl, parity, mode, tol};
    switch (g.lpr) {
    case 4: fwd_t<4>(st, g.g_fwd, a); break;
    case 8: fwd_t<8>(st, g.g_fwd, a); break;
    case 16: fwd_t<16>(st, g.g_fwd, a); break;
    case 32: fwd_t<32>(st, g.g_fwd, a); break;
    default: fwd_t<64>(st, g.g_fwd, a); break;
    }
}

template <int L>
static void adj_t(hipStream_t st, int grid, const AdjArgs &a)
{
    hipLaunchKernelGGL(k_adj<L>, dim3(grid), dim3(kBlock), 0, st, a);
}

void launch_adj(hipStream_t st, const Problem &P, const Geometry &g, DevCSR At, const double *d,
                const double *T, const double *v, double *q, double *part_out,
                const double *part_t, double *S, int *ctl, int parity, int mode)
{
    AdjArgs a{At.ptr, At.idx, At.val, P.m, (int)P.n, P.nx, P.ny, P.nz, P.w, P.damp, d, T, v, q,
              part_out, part_t, g.g_fwd, S, ctl, parity, mode};
    switch (g.lpc) {
    case 4: adj_t<4>(st, g.g_adj, a); break;
    case 8: adj_t<8>(st, g.g_adj, a); break;
    case 16: adj_t<16>(st, g.g_adj, a); break;
    case 32: adj_t<32>(st, g.g_adj, a); break;
    default: adj_t<64>(st, g.g_adj, a); break;
    }
}

void launch_update(hipStream_t st, const Problem &P, const Geometry &g, const double *d,
                   const double *q, double *v, double *w, double *y, double *z,
                   double *part_out, const double *part_q, double *S, int *ctl, int parity,
                   int mode)
{
    UpdArgs a{(int)P.n, d, q, v, w, y, z, part_out, part_q, g.g_adj, S, ctl, parity, mode};
    hipLaunchKernelGGL(k_update, dim3(g.g_upd), dim3(kBlock), 0, st, a);
}

void launch_finalize(hipStream_t st, const Problem &P, const Geometry &g, const double *d,
                     const double *y, double *dm, const double *part_v, double *S, int *ctl,
                     int parity, double tol)
{
    (void)parity;
    hipLaunchKernelGGL(k_finalize, dim3(g.g_upd), dim3(kBlock), 0, st, (int)P.n, d, y, dm, part_v,
                       g.g_upd, S, ctl, tol);
}

void launch_scale_vec(hipStream_t st, int64_t n, const double *d, const double *x, double *z)
{
    hipLaunchKernelGGL(k_scale_vec, dim3(blocks_for(n, kBlock, 4096)), dim3(kBlock), 0, st, n, d,
                       x, z);
}

void launch_fill(hipStream_t st, int64_t n, double value, double *x)
{
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, kBlock, 4096)), dim3(kBlock), 0, st, n, value,
                       x);
}

void launch_jacobi(hipStream_t st, const Problem &P, DevCSR At, double *d)
{
    hipLaunchKernelGGL(k_jacobi, dim3(blocks_for(P.n, kBlock / 64, 8192)), dim3(kBlock), 0, st,
                       (int)P.n, P.nx, P.ny, P.nz, P.w, P.damp, At.ptr, At.val, d);
}

void launch_check_csr(hipStream_t st, int64_t m, int64_t n, const int64_t *row_ptr,
                      const int32_t *col, const double *val, int *flag)
{
    hipLaunchKernelGGL(k_check_csr, dim3(blocks_for(m, kBlock, 8192)), dim3(kBlock), 0, st, m, n,
                       row_ptr, col, val, flag);
}

void launch_check_vec(hipStream_t st, int64_t n, const double *x, int positive, int *flag)
{
    hipLaunchKernelGGL(k_check_vec, dim3(blocks_for(n, kBlock, 4096)), dim3(kBlock), 0, st, n, x,
                       positive, flag);
}

}  // namespace lsqr
