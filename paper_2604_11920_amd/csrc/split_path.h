// Bilinear split of a ray polyline over the lateral grid (the interpolation
// coefficients of eq. (1)): for every lateral node a path touches, the path
// integral of that node's bilinear hat function, in km.  Shared by the
// device assembly (one workgroup per path) and a host check; plain IEEE
// double arithmetic with no contraction, so both give the same bits.
//
// A piece (two consecutive points, at most h/4 long) is cut where it
// crosses an x or a y grid line (at most one of each); every sub-piece of
// positive length lies in one cell, and the bilinear corner weights are
// quadratic along it, so Simpson's rule on the sub-piece is exact.  The
// contributions of a path to one node are summed in the order the
// sub-pieces occur along the path, as the first contribution plus the
// blocked sum of the rest (see sum_contributions).
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define LSQR_HD __host__ __device__
#else
#define LSQR_HD
#endif

namespace lsqr {

struct SplitGrid {
    double h;        // node spacing (degrees); node (ix, iy) sits at (ix h, iy h)
    double km;       // kilometres per degree
    int nx, ny;      // lateral nodes, k = iy nx + ix
};

// Fraction along a piece (one coordinate from a0 to a1 = a0 + da) where it
// crosses a grid line, NaN when both ends lie between the same two lines.
LSQR_HD inline double split_crossing(double a0, double a1, double da, double h)
{
#pragma clang fp contract(off)
    const double i0 = floor(a0 / h), i1 = floor(a1 / h);
    if (i0 == i1) return NAN;
    const double xc = (i0 > i1 ? i0 : i1) * h;
    return (xc - a0) / da;
}

// Lower and upper of two crossing fractions, a NaN operand ignored.
LSQR_HD inline double split_lo(double a, double b)
{
    return isnan(a) ? b : isnan(b) ? a : (b < a ? b : a);
}
LSQR_HD inline double split_hi(double a, double b)
{
    return isnan(a) ? b : isnan(b) ? a : (b > a ? b : a);
}

// Records of piece i -> i+1 (x0, y0 to x1, y1; length len in degrees, as the
// ray tracer measured it): up to three sub-pieces, four corner records each,
// written to node[] / val[] in order (sub-piece, then corners k, k+1,
// k+nx, k+nx+1).  Returns the number of records (0 .. 12).
LSQR_HD inline int split_piece(double x0, double y0, double x1, double y1, double len,
                               const SplitGrid &g, int64_t *node, double *val)
{
#pragma clang fp contract(off)
    const double dx = x1 - x0, dy = y1 - y0;
    double t1 = split_lo(split_crossing(x0, x1, dx, g.h), split_crossing(y0, y1, dy, g.h));
    double t2 = split_hi(split_crossing(x0, x1, dx, g.h), split_crossing(y0, y1, dy, g.h));
    if (isnan(t1)) t1 = 1.0;
    if (isnan(t2)) t2 = 1.0;
    const double ta[3] = {0.0, t1, t2}, tb[3] = {t1, t2, 1.0};
    int r = 0;
    for (int q = 0; q < 3; ++q) {
        const double seg = ((tb[q] - ta[q]) * len) * g.km;
        if (!(seg > 0.0)) continue;
        const double ax = x0 + ta[q] * dx, ay = y0 + ta[q] * dy;
        const double bx = x0 + tb[q] * dx, by = y0 + tb[q] * dy;
        const double mx = 0.5 * (ax + bx), my = 0.5 * (ay + by);
        int64_t ci = (int64_t)floor(mx / g.h), cj = (int64_t)floor(my / g.h);
        ci = ci < 0 ? 0 : ci > g.nx - 2 ? g.nx - 2 : ci;
        cj = cj < 0 ? 0 : cj > g.ny - 2 ? g.ny - 2 : cj;
        const double fci = (double)ci, fcj = (double)cj;
        double w[3][4];
        const double xs[3] = {ax, mx, bx}, ys[3] = {ay, my, by};
        for (int e = 0; e < 3; ++e) {
            const double fx = xs[e] / g.h - fci, fy = ys[e] / g.h - fcj;
            w[e][0] = (1.0 - fx) * (1.0 - fy);
            w[e][1] = fx * (1.0 - fy);
            w[e][2] = (1.0 - fx) * fy;
            w[e][3] = fx * fy;
        }
        const double s6 = seg / 6.0;
        const int64_t k = cj * g.nx + ci;
        const int64_t nodes[4] = {k, k + 1, k + g.nx, k + g.nx + 1};
        for (int c = 0; c < 4; ++c) {
            node[r] = nodes[c];
            val[r] = s6 * ((w[0][c] + 4.0 * w[1][c]) + w[2][c]);
            ++r;
        }
    }
    return r;
}

// The sum of one node's contributions c[0], c[1], ..., c[n-1] (in path order,
// read through at(j)): c[0] plus the blocked sum of the rest, which for
// fewer than 8 terms adds them one by one to zero and for 8 .. 128 terms
// keeps eight running sums over consecutive blocks of eight, combines them
// as ((s0+s1)+(s2+s3))+((s4+s5)+(s6+s7)) and adds the leftover terms one by
// one.  n - 1 > 128 is not supported (returns NaN).
template <class At>
LSQR_HD inline double sum_contributions(int n, At at)
{
#pragma clang fp contract(off)
    const int r = n - 1;
    double rest;
    if (r < 8) {
        rest = 0.0;
        for (int j = 1; j < n; ++j) rest = rest + at(j);
    } else if (r <= 128) {
        double s[8];
        for (int j = 0; j < 8; ++j) s[j] = at(1 + j);
        int i = 8;
        for (; i < r - (r % 8); i += 8)
            for (int j = 0; j < 8; ++j) s[j] = s[j] + at(1 + i + j);
        rest = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
        for (; i < r; ++i) rest = rest + at(1 + i);
    } else {
        return NAN;
    }
    return at(0) + rest;
}

}  // namespace lsqr
