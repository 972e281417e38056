// The right-hand side of the FP64 iterative refinement's inner solves (the
// single-system mixed forms and the batched solve).
//
// A sweep needs an inner right-hand side f whose normal-equation image under
// the inner operator Ahat = [Ghat; w L; lambda I] equals the true one,
// Ahat^T f = Abar^T rbar (rbar = bbar - Abar x in FP64, Abar with the FP64
// G): then the inner LSQR's iterates, which depend on f only through
// Ahat^T f, converge to the correction of the FP64 problem.  The damping
// block makes one such f free of the residual itself:
//     f = [0; 0; (Abar^T rbar) / lambda],   Ahat^T f = lambda f_D.
// The residual rbar tends to the least-squares residual r*, which does not
// vanish; an f that carries it (e.g. [r_G; r_L; r_D + (G - Ghat)^T r_G /
// lambda]) is rounded to FP32 in the inner vectors with an error of u32 |r*|
// whose image under Ahat^T bounds the attainable eta (about 3e-7 on a
// config-1-shaped system).  This f shrinks with eta, so that floor goes
// with it.
#include <math.h>

#include "ctx.h"
#include "lsqr_kernels.cuh"

namespace lsqr {

// f = [0; 0; at / damp] with at = Abar^T rbar = g + w L^T r_L + damp r_D
// (g = G^T r_G in FP64); partials of |at|^2 (the refinement's eta).
__global__ __launch_bounds__(kBlock) void k_normal_rhs(int64_t m, int n, int nx, int ny, int nz,
                                                       double w, double damp, const double *rbar,
                                                       const double *g, double *f, double *part)
{
#pragma clang fp contract(off)
    __shared__ double lds[4];
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m + n;
         i += (int64_t)gridDim.x * kBlock)
        f[i] = 0.0;
    double sq = 0.0;
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock) {
        const double lap = stencil<double>(rbar + m, j, nx, ny, nz);
        const double at = g[j] + w * lap + damp * rbar[m + n + j];
        f[m + n + j] = at / damp;
        sq += at * at;
    }
    const double tot = block_sum(sq, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

void launch_normal_rhs(hipStream_t st, const Problem &P, int grid, const double *rbar,
                       const double *g, double *f, double *part)
{
    hipLaunchKernelGGL(k_normal_rhs, dim3(grid), dim3(kBlock), 0, st, P.m, (int)P.n, P.nx, P.ny,
                       P.nz, P.w, P.damp, rbar, g, f, part);
}

}  // namespace lsqr
