/*
 * Row assembler for the synthetic sensitivity matrix G (input generation only).
 *
 * One data row per kept (path, period) pair, pair-major and period-minor.  A row
 * is the outer product of the path's lateral segment lengths (one entry per
 * lateral grid node the ray touches, nodes ascending) with the period's depth
 * weights (a contiguous run of depth nodes), scaled by -1/c(T): the linearised
 * traveltime of eq. (1) written in relative velocity perturbations, with the
 * depth integral of eq. (2)/(5) replaced by a normalised Gaussian depth kernel.
 * Columns follow the unknown ordering of eq. (7): column = node * nz + depth.
 *
 * Built with gcc as a small shared library and driven from synth/__init__.py.
 */
#include <stdint.h>
#include <string.h>

/* Pass 1: row pointer and (pair, period) of every kept row.  Returns m. */
int64_t synth_count(int64_t npairs, int32_t nper, const uint8_t *keep,
                    const int64_t *node_ptr, const int32_t *nj,
                    int64_t *row_ptr, int32_t *row_pair, int32_t *row_period)
{
    int64_t r = 0, nnz = 0;
    if (row_ptr) row_ptr[0] = 0;
    for (int64_t p = 0; p < npairs; ++p) {
        int64_t nk = node_ptr[p + 1] - node_ptr[p];
        for (int32_t t = 0; t < nper; ++t) {
            if (!keep[p * nper + t]) continue;
            nnz += nk * (int64_t)nj[t];
            if (row_pair) row_pair[r] = (int32_t)p;
            if (row_period) row_period[r] = t;
            ++r;
            if (row_ptr) row_ptr[r] = nnz;
        }
    }
    return r;
}

/* Pass 2: fill columns and values of every row; also y = G * m_true per row
 * (summed in storage order).  Rows are independent, so threads split them. */
void synth_fill(int64_t m, int32_t nz, const int64_t *row_ptr,
                const int32_t *row_pair, const int32_t *row_period,
                const int64_t *node_ptr, const int32_t *node_k, const double *node_len,
                const double *cvel, const int32_t *j0, const int32_t *nj,
                const int64_t *w_ptr, const double *wflat,
                const double *m_true, int32_t *col, double *val, double *gm)
{
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < m; ++r) {
        int64_t p = row_pair[r];
        int32_t t = row_period[r];
        int64_t e = row_ptr[r];
        const double *w = wflat + w_ptr[t];
        double acc = 0.0;
        for (int64_t a = node_ptr[p]; a < node_ptr[p + 1]; ++a) {
            double s = -node_len[a] / cvel[t];
            int64_t base = (int64_t)node_k[a] * nz + j0[t];
            for (int32_t b = 0; b < nj[t]; ++b, ++e) {
                double g = s * w[b];
                col[e] = (int32_t)(base + b);
                val[e] = g;
                if (m_true) acc += g * m_true[base + b];
            }
        }
        if (gm) gm[r] = acc;
    }
}
