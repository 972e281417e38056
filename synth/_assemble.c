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

/*
 * The generator's variant closer to the paper's G: every kept row (path,
 * period) has its own ray (node list of path q = pair * nper + period) and
 * every lateral node its own depth kernel per period (eq. (5): the depth
 * sensitivity depends on the local model), table entry k * nper + t:
 * depths dj0[..] .. dj0[..] + dnj[..] - 1 with weights dw[dw_ptr[..] ..].
 */
int64_t synth_count_rows(int64_t npairs, int32_t nper, const uint8_t *keep,
                         const int64_t *path_ptr, const int32_t *node_k, const int32_t *dnj,
                         int64_t *row_ptr, int32_t *row_pair, int32_t *row_period)
{
    int64_t r = 0, nnz = 0;
    if (row_ptr) row_ptr[0] = 0;
    for (int64_t p = 0; p < npairs; ++p)
        for (int32_t t = 0; t < nper; ++t) {
            const int64_t q = p * nper + t;
            if (!keep[q]) continue;
            for (int64_t a = path_ptr[q]; a < path_ptr[q + 1]; ++a)
                nnz += dnj[(int64_t)node_k[a] * nper + t];
            if (row_pair) row_pair[r] = (int32_t)p;
            if (row_period) row_period[r] = t;
            ++r;
            if (row_ptr) row_ptr[r] = nnz;
        }
    return r;
}

void synth_fill_rows(int64_t m, int32_t nz, int32_t nper, const int64_t *row_ptr,
                     const int32_t *row_pair, const int32_t *row_period,
                     const int64_t *path_ptr, const int32_t *node_k, const double *node_len,
                     const double *cvel, const int32_t *dj0, const int32_t *dnj,
                     const int64_t *dw_ptr, const double *dw,
                     const double *m_true, int32_t *col, double *val, double *gm)
{
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < m; ++r) {
        const int32_t t = row_period[r];
        const int64_t q = (int64_t)row_pair[r] * nper + t;
        int64_t e = row_ptr[r];
        double acc = 0.0;
        for (int64_t a = path_ptr[q]; a < path_ptr[q + 1]; ++a) {
            const int64_t kt = (int64_t)node_k[a] * nper + t;
            const double s = -node_len[a] / cvel[t];
            const double *w = dw + dw_ptr[kt];
            const int64_t base = (int64_t)node_k[a] * nz + dj0[kt];
            for (int32_t b = 0; b < dnj[kt]; ++b, ++e) {
                const double g = s * w[b];
                col[e] = (int32_t)(base + b);
                val[e] = g;
                if (m_true) acc += g * m_true[base + b];
            }
        }
        if (gm) gm[r] = acc;
    }
}
