// Internal declarations shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lsqr_mi355x.h"

namespace lsqr {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kStateWords = 32;      // doubles per per-iteration state row

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
    S_ARNORM0 = 12, // |Abar^T bbar| (row 0 only; LSMR: alpha_1 beta_1)
    // LSMR (Fong & Saunders): the second rotation chain and the |r| chain;
    // S_PHIBAR holds |r_k|, S_PSI |A_D^T r_k| = |zetabar_{k+1}|
    S_ALPHABAR = 13,
    S_ZETABAR = 14,
    S_CBAR = 15,
    S_SBAR = 16,
    S_ZETA = 17,
    S_BETADD = 18,
    S_BETAD = 19,
    S_RHODOLD = 20,
    S_TAUTILDE = 21,
    S_THETATILDE = 22,
    S_METHOD = 23,  // row 0: 0 LSQR, 1 LSMR (written by the start step)
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

enum { MODE_ITER = 0, MODE_INIT = 1, MODE_OPERATOR = 2 };

// Element types of stored matrix values and of vectors.
enum ValType { VT_F64 = 0, VT_F32 = 1, VT_BF16 = 2, VT_F16 = 3 };
size_t vt_size(int vt);

struct Problem {
    int64_t m = 0, n = 0, nnz = 0;
    int32_t nx = 0, ny = 0, nz = 0;
    double w = 0.0, damp = 0.0;
};

// Data rows of the forward product.
// Most columns a row group may hold (its part of D v is staged in LDS: 56 KB
// at FP64, within the 64 KB a workgroup may take on any CDNA part).
constexpr int kLcolMaxCap = 7168;

struct RowFmt {
    int vt = VT_F64;
    const int64_t *rp = nullptr;       // [m+1] value offsets
    const int32_t *ci = nullptr;       // [nnz] columns (plain CSR)
    const void *val = nullptr;
    const float *sigma = nullptr;      // [m] row scales (quantised values) or nullptr
    int lpr = 64;                      // lanes per row (plain CSR)
    // plain CSR with 64 lanes per row: a launch of wgrid workgroups takes
    // contiguous row ranges balanced in entries, wrow[p] .. wrow[p+1]-1, one
    // per workgroup (its waves interleaved) or per wave (fwd_pipe_parts);
    // other launch sizes take rows w, w + waves, ...
    const int32_t *wrow = nullptr;     // [fwd_pipe_parts(wgrid) + 1]
    int wgrid = 0;
    // row groups with local columns (used instead of ci when slot is set):
    // group g = rows gp[g] .. gp[g+1]-1, its sorted columns gcol[gcp[g] ..
    // gcp[g+1]-1] (at most gcap), slot[p] = position of entry p's column
    // in its group's list.  With slot set, wrow holds the launch's group
    // ranges (wrow[b] .. wrow[b+1]-1 for workgroup b of wgrid).
    const int32_t *gp = nullptr;       // [ngroups + 1]
    const int64_t *gcp = nullptr;      // [ngroups + 1]
    const int32_t *gcol = nullptr;
    const uint16_t *slot = nullptr;    // [nnz]
    int ngroups = 0;
    int gcap = 0;                      // columns per group at most (<= kLcolMaxCap)
    int padded = 0;                    // zero elements val and slot hold past the last entry
};

// The row-group kernel with entries in pairs reads two values and two slots
// at a time from even positions, and one element past the last entry
// (RowFmt::padded).
static inline bool lcol_pairs_ok(const RowFmt &R)
{
    const uintptr_t w = 2 * (uintptr_t)vt_size(R.vt);
    return R.padded >= 1 && ((uintptr_t)R.val & (w - 1)) == 0 && ((uintptr_t)R.slot & 3u) == 0;
}

// Entries in quads (4- and 2-byte values): four values and four slots from
// positions that are multiples of four, and up to three elements past the
// last entry.  Measured on the paper-shaped system against pairs: FP32
// 699 -> 655 us, FP16 569 -> 527 us, BF16 585 -> 566 us.
#ifndef LSQR_FWD_QUADS
#define LSQR_FWD_QUADS 1
#endif
static inline bool lcol_quads_ok(const RowFmt &R)
{
    const uintptr_t w = 4 * (uintptr_t)vt_size(R.vt);
    return LSQR_FWD_QUADS && vt_size(R.vt) <= 4 && R.padded >= 3 && ((uintptr_t)R.val & (w - 1)) == 0 &&
           ((uintptr_t)R.slot & 7u) == 0;
}

// Entries in octets (16-bit codes): eight codes and eight slots, one 16-byte
// load each, from positions that are multiples of eight, and up to seven
// elements past the last entry.  Measured on the config-1 system against
// quads: BF16 532 -> 507 us, FP16 506 -> 467 us.
#ifndef LSQR_FWD_OCTS
#define LSQR_FWD_OCTS 1
#endif
static inline bool lcol_octs_ok(const RowFmt &R)
{
    return LSQR_FWD_OCTS && vt_size(R.vt) == 2 && R.padded >= 7 && ((uintptr_t)R.val & 15u) == 0 &&
           ((uintptr_t)R.slot & 15u) == 0;
}

// Stored transpose (CSC) for the transposed product.
struct ColFmt {
    int vt = VT_F64;
    const int64_t *cp = nullptr;       // [n+1]
    const int32_t *ri = nullptr;       // [nnz] rows, ascending within a column
    const void *val = nullptr;
    int lpc = 64;
    // Node runs (used instead of the CSC when nrp is set; val then holds the
    // values in node-major run order).  Node k = columns [k nz, (k+1) nz).
    const int64_t *nrp = nullptr;      // [nnodes+1] runs of node k: [nrp[k], nrp[k+1])
    const int64_t *nvq = nullptr;      // [4 nnodes+1] value offset of each quarter of a node's runs
    const uint32_t *nrow = nullptr;    // [nruns] data row of the run
    const uint16_t *ndesc = nullptr;   // [nruns] (iz0 << 8) | len
    const int32_t *norder = nullptr;   // [nnodes] nodes by decreasing work
    int pairs = 0;                     // W = 2, 4 or 8: val / nvq in the layout of W
                                       // depths to a word (k_adj_npair<W>)
};

// Type-dispatched launchers (kernels_f64.hip, kernels_f32.hip).
void launch_init(hipStream_t st, const Problem &P, int grid, int vec, const double *rhs, int full,
                 void *T0, const float *sigma, void *Ts0, double *y, void *vzero, double *part,
                 int *ctl, int kmax);
// Workgroups of the pipelined CSR forward product that the device holds at
// once (0 when R does not use it), and its balanced wave partition.
int fwd_pipe_grid(int vec, const RowFmt &R);
int fwd_pipe_parts(int grid);          // row ranges of the balanced partition for a grid
// Workgroups of the node-run transposed product the device holds at once (0
// when C does not use it).
int adj_nruns_grid(int vec, const ColFmt &C);
void launch_wave_rows(hipStream_t st, const int64_t *rp, int64_t m, int waves, int32_t *wrow);
// Row groups (RowFmt::slot): workgroups of k_fwd_lcol the device holds at once
// (0 without groups) and the balanced group ranges of a launch of `parts`.
int fwd_lcol_grid(int vec, const RowFmt &R);
void launch_group_parts(hipStream_t st, const int64_t *rp, const int32_t *gp, int ng, int parts,
                        int32_t *wgrp);
void launch_fwd(hipStream_t st, const Problem &P, int grid, int vec, const RowFmt &R,
                const void *z, const void *Tprev, void *Tcur, void *Ts, double *part_out,
                const double *part_v, int np_v, double *S, int *ctl, int parity, double tol,
                int mode);
void launch_adj(hipStream_t st, const Problem &P, int grid, int vec, const ColFmt &C,
                const double *d, const void *T, const void *Tg, const void *v, void *q,
                double *part_out, const double *part_t, int np_t, double *S, int *ctl,
                int parity, int mode, int data_only);
// hbar != nullptr selects the LSMR step (w then holds LSMR's h).
void launch_update(hipStream_t st, const Problem &P, int grid, int vec, const double *d,
                   const void *q, void *v, double *w, double *y, void *z, double *part_out,
                   const double *part_q, int np_q, double *S, int *ctl, int parity, int mode,
                   double *hbar);

// Helpers (kernels_common.hip).
void launch_finalize(hipStream_t st, const Problem &P, int grid, const double *d,
                     const double *y, double *dm, const double *part_v, int np_v, double *S,
                     int *ctl, double tol, int accumulate);
void launch_scale_vec(hipStream_t st, int64_t n, const double *d, const double *x, double *z);
void launch_fill(hipStream_t st, int64_t n, double value, double *x);
void launch_jacobi(hipStream_t st, const Problem &P, const ColFmt &C, double *d);
void launch_check_csr(hipStream_t st, int64_t m, int64_t n, const int64_t *row_ptr,
                      const int32_t *col, const double *val, int *flag);
void launch_check_vec(hipStream_t st, int64_t n, const double *x, int positive, int *flag);
// out[dst[r] + e] = in[src[r] + e] for e < len(desc[r]) (elements of elem_bytes = 2, 4 or 8)
void launch_gather_runs(hipStream_t st, int64_t nr, const uint32_t *src, const uint32_t *dst,
                        const uint16_t *desc, const void *in, void *out, int elem_bytes);
void launch_convert_f32(hipStream_t st, int64_t nnz, const double *src, float *dst);
void launch_row_scales(hipStream_t st, int64_t m, const int64_t *rp, const double *val, int vt,
                       float *sigma);
void launch_quantise_rows(hipStream_t st, int64_t m, const int64_t *rp, const double *val,
                          const float *sigma, int vt, uint16_t *q);
void launch_quantise_cols(hipStream_t st, int64_t nnz, const int32_t *ri, const double *cv,
                          const float *sigma, int vt, uint16_t *q);
// rbar = bbar - y in FP64 (y = NULL: rbar = bbar); partials of |rbar|^2
void launch_residual(hipStream_t st, const Problem &P, int grid, const double *dt,
                     const double *y, double *rbar, double *part);
void launch_sum_partials(hipStream_t st, const double *part, int np, double *out);

// Transpose (transpose.hip).
struct Allocator {
    lsqr_alloc_fn alloc = nullptr;
    lsqr_free_fn dealloc = nullptr;
    void *user = nullptr;
    void *get(size_t bytes);
    void put(void *p, size_t bytes);
};
hipError_t build_transpose(hipStream_t st, Allocator &al, int64_t m, int64_t n, int64_t nnz,
                           const int64_t *rp, const int32_t *ci, const double *val,
                           int64_t *col_ptr, int32_t *row_idx, double *cval, std::string &err);

}  // namespace lsqr
