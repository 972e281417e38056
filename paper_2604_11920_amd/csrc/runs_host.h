// Host-side builders of the index formats (plain C++, no HIP): row groups of
// the data rows (forward product), node runs of the data block and their
// padded layouts (transposed product).  All read only the CSR structure.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <thread>
#include <vector>

namespace lsqr {

// Node runs of the data block (the transposed product's storage): for every
// lateral node k (columns [k nz, (k+1) nz), eq. 7) the data rows reaching it in
// ascending order, each with its maximal stretch of consecutive depths.  Built
// from the CSR structure; `src` / `dst` give, per run, the CSR position of its
// first value and its node-major position (for the value gather on the device).
struct NodeRuns {
    std::vector<int64_t> nrp;       // [nnodes+1]
    std::vector<int64_t> nvq;       // [4 nnodes+1]
    std::vector<uint32_t> row, src, dst;
    std::vector<uint16_t> desc;
    std::vector<int32_t> order;
};

inline bool build_node_runs_host(int64_t m, int64_t n, int nz, const int64_t *rp, const int32_t *ci,
                          NodeRuns &R)
{
    const int64_t nnz = rp[m];
    if (nz < 1 || nz > 64 || n % nz != 0 || nnz >= ((int64_t)1 << 32) || m >= ((int64_t)1 << 32))
        return false;
    const int64_t nn = n / nz;
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (nnz < (1 << 20)) nt = 1;
    // run starts: first entry of a row, a gap in the columns, or a new node
    auto is_start = [&](int64_t i, int64_t p) {
        return p == rp[i] || ci[p] != ci[p - 1] + 1 || ci[p] % nz == 0;
    };
    std::vector<std::vector<int64_t>> cnt(nt, std::vector<int64_t>((size_t)nn, 0));
    {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t]() {
                auto &c = cnt[t];
                for (int64_t i = m * t / nt; i < m * (t + 1) / nt; ++i)
                    for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
                        if (is_start(i, p)) ++c[(size_t)(ci[p] / nz)];
            });
        for (auto &x : th) x.join();
    }
    // node-major positions: node k, then thread order (= ascending rows)
    R.nrp.assign((size_t)nn + 1, 0);
    for (int64_t k = 0; k < nn; ++k) {
        int64_t tot = 0;
        for (unsigned t = 0; t < nt; ++t) {
            const int64_t c = cnt[t][(size_t)k];
            cnt[t][(size_t)k] = R.nrp[(size_t)k] + tot;      // becomes the cursor
            tot += c;
        }
        R.nrp[(size_t)k + 1] = R.nrp[(size_t)k] + tot;
    }
    const int64_t nr = R.nrp[(size_t)nn];
    R.row.resize((size_t)nr);
    R.src.resize((size_t)nr);
    R.dst.resize((size_t)nr);
    R.desc.resize((size_t)nr);
    {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t]() {
                auto &cur = cnt[t];
                for (int64_t i = m * t / nt; i < m * (t + 1) / nt; ++i) {
                    int64_t r = -1;
                    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                        if (is_start(i, p)) {
                            r = cur[(size_t)(ci[p] / nz)]++;
                            R.row[(size_t)r] = (uint32_t)i;
                            R.src[(size_t)r] = (uint32_t)p;
                            R.desc[(size_t)r] = (uint16_t)((ci[p] % nz) << 8);
                        }
                        R.desc[(size_t)r] = (uint16_t)(R.desc[(size_t)r] + 1);
                    }
                }
            });
        for (auto &x : th) x.join();
    }
    // value positions (node-major, runs in order) and the quarter offsets
    R.nvq.assign((size_t)(4 * nn + 1), 0);
    int64_t off = 0;
    for (int64_t k = 0; k < nn; ++k) {
        const int64_t r0 = R.nrp[(size_t)k], r1 = R.nrp[(size_t)k + 1], c = r1 - r0;
        for (int64_t r = r0; r < r1; ++r) {
            R.dst[(size_t)r] = (uint32_t)off;
            off += R.desc[(size_t)r] & 255;
        }
        // quarter w of the node's runs starts at run r0 + c w / 4 (as in the kernel)
        for (int w = 0; w < 4; ++w) {
            const int64_t q = r0 + c * w / 4;
            R.nvq[(size_t)(4 * k + w)] = q < r1 ? (int64_t)R.dst[(size_t)q] : off;
        }
    }
    R.nvq[(size_t)(4 * nn)] = off;
    R.order.resize((size_t)nn);
    for (int64_t k = 0; k < nn; ++k) R.order[(size_t)k] = (int32_t)k;
    std::stable_sort(R.order.begin(), R.order.end(), [&](int32_t x, int32_t y) {
        return R.nrp[(size_t)x + 1] - R.nrp[(size_t)x] > R.nrp[(size_t)y + 1] - R.nrp[(size_t)y];
    });
    return off == nnz;
}

// Row order of the node runs: the runs of row i are rrid[rrp[i] .. rrp[i+1]),
// node-major run indices in ascending node (= column) order, so a row's
// per-run partial sums are added in the order of its stored entries.  A
// stable counting sort of the node-major runs by row.
inline void row_order_of_runs(const NodeRuns &R, int64_t m, std::vector<int64_t> &rrp,
                              std::vector<uint32_t> &rrid)
{
    const int64_t nr = (int64_t)R.row.size();
    rrp.assign((size_t)m + 1, 0);
    for (int64_t r = 0; r < nr; ++r) ++rrp[(size_t)R.row[(size_t)r] + 1];
    for (int64_t i = 0; i < m; ++i) rrp[(size_t)i + 1] += rrp[(size_t)i];
    std::vector<int64_t> fill(rrp.begin(), rrp.end() - 1);
    rrid.resize((size_t)nr);
    for (int64_t r = 0; r < nr; ++r) rrid[(size_t)fill[(size_t)R.row[(size_t)r]]++] = (uint32_t)r;
}

// Row groups with local columns (forward product): the data rows are cut, in
// order, into groups of consecutive rows whose columns together number at
// most cap (the rays of one path at all its periods cross the same lateral
// nodes, so their columns largely coincide).  Per group its sorted column
// list; per stored entry the position of its column in that list (u16), so a
// workgroup stages the group's part of D v in LDS once and its rows read it
// there.  gp[g] = first row of group g (gp[ng] = m); gcp[g] = offset of its
// list in gcol.  Every slot is below the size of its group's list, hence below
// cap.  Returns false when some row alone has more than cap distinct columns,
// cap is not in [1, 65536], or m >= 2^31.
struct RowGroups {
    std::vector<int32_t> gp;
    std::vector<int64_t> gcp;
    std::vector<int32_t> gcol;
    std::vector<uint16_t> slot;
};

inline bool build_row_groups_host(int64_t m, int64_t n, const int64_t *rp, const int32_t *ci,
                                  int cap, RowGroups &R)
{
    if (cap < 1 || cap > 65536 || m >= ((int64_t)1 << 31) || m < 0) return false;
    R.gp.clear(); R.gcp.clear(); R.gcol.clear();
    R.gp.push_back(0);
    // group boundaries: a row joins the open group while the union fits
    std::vector<int32_t> stamp((size_t)n, -1);
    int32_t g = 0;
    int64_t cnt = 0;
    for (int64_t i = 0; i < m; ++i) {
        int64_t fresh = 0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) fresh += stamp[(size_t)ci[p]] != g;
        if (cnt + fresh > cap && i > R.gp.back()) {    // close the group before row i
            R.gp.push_back((int32_t)i);
            ++g;
            cnt = 0;
            fresh = rp[i + 1] - rp[i];                  // columns of a row are distinct
        }
        if (fresh > cap) return false;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) stamp[(size_t)ci[p]] = g;
        cnt += fresh;
    }
    if (m > 0) R.gp.push_back((int32_t)m);
    const int64_t ng = (int64_t)R.gp.size() - 1;
    // column lists and slots, groups split over threads
    std::vector<std::vector<int32_t>> lists((size_t)ng);
    R.slot.assign((size_t)(m > 0 ? rp[m] : 0), 0);
    const int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            std::vector<int32_t> seen((size_t)n, -1), at((size_t)n, 0);
            for (int64_t k = t; k < ng; k += nt) {
                std::vector<int32_t> &L = lists[(size_t)k];
                const int64_t p0 = rp[R.gp[(size_t)k]], p1 = rp[R.gp[(size_t)k + 1]];
                for (int64_t p = p0; p < p1; ++p)
                    if (seen[(size_t)ci[p]] != (int32_t)k) { seen[(size_t)ci[p]] = (int32_t)k; L.push_back(ci[p]); }
                std::sort(L.begin(), L.end());
                for (size_t q = 0; q < L.size(); ++q) at[(size_t)L[q]] = (int32_t)q;
                for (int64_t p = p0; p < p1; ++p) R.slot[(size_t)p] = (uint16_t)at[(size_t)ci[p]];
            }
        });
    for (auto &x : th) x.join();
    R.gcp.assign((size_t)ng + 1, 0);
    for (int64_t k = 0; k < ng; ++k) R.gcp[(size_t)k + 1] = R.gcp[(size_t)k] + (int64_t)lists[(size_t)k].size();
    R.gcol.resize((size_t)R.gcp.back());
    for (int64_t k = 0; k < ng; ++k)
        std::copy(lists[(size_t)k].begin(), lists[(size_t)k].end(), R.gcol.begin() + R.gcp[(size_t)k]);
    return true;
}

// Depth-pair layout of the node-run values (W = 2; W = 4 and W = 8 group
// four and eight depths the same way): each run is stored from a position
// that is a multiple of W, preceded by iz0 mod W zeros and followed by zeros
// up to a multiple of W, so that depths Wk .. Wk+W-1 of a run share one
// aligned W-element word at run start + Wk - (iz0 - iz0 mod W).  dst[r] =
// position of run r's first value; nvq as in NodeRuns (the padded start of
// each quarter of a node's runs); total = the padded length (a multiple of
// W).  Returns false when it does not fit 32-bit positions or W is not 2, 4
// or 8.
inline bool pair_layout_host(const NodeRuns &R, int64_t nn, std::vector<uint32_t> &dst,
                             std::vector<int64_t> &nvq, int64_t &total, int W = 2)
{
    if (W != 2 && W != 4 && W != 8) return false;
    const int64_t nr = R.nrp[(size_t)nn];
    dst.resize((size_t)nr);
    nvq.assign((size_t)(4 * nn + 1), 0);
    int64_t off = 0;
    for (int64_t k = 0; k < nn; ++k) {
        const int64_t r0 = R.nrp[(size_t)k], r1 = R.nrp[(size_t)k + 1], c = r1 - r0;
        int w = 0;
        for (int64_t r = r0; r <= r1; ++r) {
            for (; w < 4 && r0 + c * w / 4 == r; ++w) nvq[(size_t)(4 * k + w)] = off;
            if (r == r1) break;
            const int iz0 = R.desc[(size_t)r] >> 8, len = R.desc[(size_t)r] & 255;
            const int pre = iz0 & (W - 1);
            dst[(size_t)r] = (uint32_t)(off + pre);
            off += (len + pre + W - 1) & ~(W - 1);
        }
    }
    nvq[(size_t)(4 * nn)] = off;
    total = off;
    return off + 2 < ((int64_t)1 << 32);
}

}  // namespace lsqr
