// Internal declarations shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lsqr_mi355x.h"

namespace lsqr {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kStateWords = 16;      // doubles per per-iteration state row

// Per-iteration state row S[k] (doubles), written by the update kernel of
// iteration k (k = 0 is the start) and read by the next iteration.
enum StateField {
    S_ALPHA = 0,    // alpha_{k+1}
    S_BETA = 1,     // beta_{k+1}
    S_RHOBAR = 2,   // rhobar_{k+1}
    S_PHIBAR = 3,   // phibar_{k+1} = |rbar_k| estimate
    S_RHO = 4,
    S_C = 5,
    S_S = 6,
    S_THETA = 7,
    S_PHI = 8,
    S_PSI = 9,      // |A_D^T rbar_k| estimate
    S_ETA = 10,     // psi_k |D^-1 v_{k+1}| / |Abar^T bbar|
    S_VNORM = 11,   // |D^-1 v_{k+1}|
    S_ARNORM0 = 12, // |Abar^T bbar| (row 0 only)
};

// Control words (int32) on the device.
enum CtlField {
    C_STOP = 0,     // 1 once the solve has stopped
    C_ISTOP = 1,    // stop reason
    C_ITERS = 2,    // iterations completed
    C_ERR = 3,      // 1 if a scalar became non-finite
    C_CNT0 = 4,     // iteration counter read by iterations of parity 0
    C_CNT1 = 5,     // ... parity 1
    C_KMAX = 6,     // iteration limit of the current solve
    C_WORDS = 8,
};

struct DevCSR {
    const int64_t *ptr = nullptr;   // [rows+1]
    const int32_t *idx = nullptr;   // [nnz]
    const double *val = nullptr;    // [nnz]
};

// Launch geometry of the solver kernels.
struct Geometry {
    int lpr = 64;      // lanes per data row (forward)
    int lpc = 64;      // lanes per column (transposed)
    int g_fwd = 1;     // workgroups of the forward kernel
    int g_adj = 1;     // workgroups of the transposed kernel
    int g_upd = 1;     // workgroups of the update kernel
};

struct Problem {
    int64_t m = 0, n = 0, nnz = 0;
    int32_t nx = 0, ny = 0, nz = 0;
    double w = 0.0, damp = 0.0;
};

// Kernel launchers (kernels_lsqr.hip).
void launch_init_rhs(hipStream_t st, const Problem &P, const Geometry &g, const double *dt,
                     double *T0, double *y, double *vzero, double *part, int *ctl, int kmax);
void launch_fwd(hipStream_t st, const Problem &P, const Geometry &g, DevCSR A, const double *z,
                const double *Tprev, double *Tcur, double *part_out, const double *part_v,
                double *S, int *ctl, int parity, double tol, int mode);
void launch_adj(hipStream_t st, const Problem &P, const Geometry &g, DevCSR At, const double *d,
                const double *T, const double *v, double *q, double *part_out,
                const double *part_t, double *S, int *ctl, int parity, int mode);
void launch_update(hipStream_t st, const Problem &P, const Geometry &g, const double *d,
                   const double *q, double *v, double *w, double *y, double *z,
                   double *part_out, const double *part_q, double *S, int *ctl, int parity,
                   int mode);
void launch_finalize(hipStream_t st, const Problem &P, const Geometry &g, const double *d,
                     const double *y, double *dm, const double *part_v, double *S, int *ctl,
                     int parity, double tol);
void launch_scale_vec(hipStream_t st, int64_t n, const double *d, const double *x, double *z);
void launch_jacobi(hipStream_t st, const Problem &P, DevCSR At, double *d);
void launch_fill(hipStream_t st, int64_t n, double value, double *x);
void launch_check_csr(hipStream_t st, int64_t m, int64_t n, const int64_t *row_ptr,
                      const int32_t *col, const double *val, int *flag);
void launch_check_vec(hipStream_t st, int64_t n, const double *x, int positive, int *flag);

// Modes of the generic kernels.
enum { MODE_ITER = 0, MODE_INIT = 1, MODE_OPERATOR = 2 };

// Transpose (transpose.hip): CSC of the m x n CSR, rows ascending within a
// column.  Scratch is obtained from the allocator callbacks.
struct Allocator {
    lsqr_alloc_fn alloc = nullptr;
    lsqr_free_fn dealloc = nullptr;
    void *user = nullptr;
    void *get(size_t bytes);
    void put(void *p, size_t bytes);
};
hipError_t build_transpose(hipStream_t st, Allocator &al, int64_t m, int64_t n, int64_t nnz,
                           DevCSR A, int64_t *col_ptr, int32_t *row_idx, double *cval,
                           std::string &err);

}  // namespace lsqr
