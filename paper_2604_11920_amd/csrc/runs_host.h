// Host-side builders of the compressed index formats (plain C++, no HIP):
// depth runs of the data rows and run masks (forward product), node runs and
// node masks of the data block (transposed product).  All read only the CSR
// structure; the masked formats index the existing CSR / CSC value arrays.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <thread>
#include <vector>

namespace lsqr {

// Depth runs of a CSR: maximal stretches of consecutive columns within a row
// (eq. 7 orders unknowns depth fastest, so each lateral node of a ray gives a
// run of depths), split at 255 entries.  run = (first column << 8) | length;
// roff = offset of the run's first value within its row.  Returns false when
// the format cannot hold the matrix (row longer than 65535 or n >= 2^24).
inline bool build_runs_host(int64_t m, int64_t n, const int64_t *rp, const int32_t *ci,
                     std::vector<int64_t> &run_ptr, std::vector<uint32_t> &runs,
                     std::vector<uint16_t> &roff)
{
    if (n >= (1 << 24)) return false;
    for (int64_t i = 0; i < m; ++i)
        if (rp[i + 1] - rp[i] > 65535) return false;
    run_ptr.assign((size_t)m + 1, 0);
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (rp[m] < (1 << 20)) nt = 1;
    auto is_start = [&](int64_t i, int64_t p, int64_t len) {
        return p == rp[i] || ci[p] != ci[p - 1] + 1 || len == 255;
    };
    {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t]() {
                for (int64_t i = m * t / nt; i < m * (t + 1) / nt; ++i) {
                    int64_t cnt = 0, len = 0;
                    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                        if (is_start(i, p, len)) { ++cnt; len = 0; }
                        ++len;
                    }
                    run_ptr[i + 1] = cnt;
                }
            });
        for (auto &x : th) x.join();
    }
    for (int64_t i = 0; i < m; ++i) run_ptr[i + 1] += run_ptr[i];
    runs.resize((size_t)run_ptr[m]);
    roff.resize((size_t)run_ptr[m]);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            for (int64_t i = m * t / nt; i < m * (t + 1) / nt; ++i) {
                int64_t r = run_ptr[i] - 1, len = 0;
                for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                    if (is_start(i, p, len)) {
                        if (r >= run_ptr[i]) runs[r] = ((uint32_t)ci[p - len] << 8) | (uint32_t)len;
                        ++r;
                        len = 0;
                        roff[r] = (uint16_t)(p - rp[i]);
                    }
                    ++len;
                }
                if (r >= run_ptr[i]) runs[r] = ((uint32_t)ci[rp[i + 1] - len] << 8) | (uint32_t)len;
            }
        });
    for (auto &x : th) x.join();
    return true;
}

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

// XCD bands of the lateral nodes for the transposed product: the node range
// [0, nn) is cut into nb contiguous bands of about equal cost (stored values
// plus 8 per run), each band's nodes sorted by decreasing run count (stable).
// Band x occupies order[seg[x] .. seg[x+1]).  The kernel gives band x to the
// workgroups that the dispatcher places on XCD x, so the t entries of the rays
// that cross a band are reused from that XCD's L2.
inline void xcd_band_order(const NodeRuns &R, int64_t nn, int nb, std::vector<int32_t> &order,
                           std::vector<int32_t> &seg)
{
    std::vector<int64_t> pre((size_t)nn + 1, 0);
    for (int64_t k = 0; k < nn; ++k)
        pre[(size_t)k + 1] = pre[(size_t)k] + (R.nvq[(size_t)(4 * k + 4)] - R.nvq[(size_t)(4 * k)]) +
                             8 * (R.nrp[(size_t)k + 1] - R.nrp[(size_t)k]);
    seg.assign((size_t)nb + 1, 0);
    for (int x = 1; x < nb; ++x) {
        const int64_t target = (int64_t)(((__int128)pre[(size_t)nn] * x) / nb);
        seg[(size_t)x] = (int32_t)(std::lower_bound(pre.begin(), pre.end(), target) - pre.begin());
        if (seg[(size_t)x] < seg[(size_t)x - 1]) seg[(size_t)x] = seg[(size_t)x - 1];
    }
    seg[(size_t)nb] = (int32_t)nn;
    order.resize((size_t)nn);
    for (int64_t k = 0; k < nn; ++k) order[(size_t)k] = (int32_t)k;
    for (int x = 0; x < nb; ++x)
        std::stable_sort(order.begin() + seg[(size_t)x], order.begin() + seg[(size_t)x + 1],
                         [&](int32_t a, int32_t b) {
                             return R.nrp[(size_t)a + 1] - R.nrp[(size_t)a] >
                                    R.nrp[(size_t)b + 1] - R.nrp[(size_t)b];
                         });
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

// Run masks of the data rows (forward product over the CSR values).  A run is
// a maximal stretch of consecutive columns inside a row.  Bit p of the global
// mask (word p / 64, bit p % 64) is set when stored entry p starts a run;
// base[w] = number of runs starting before word w; rcol[r] = first column of
// run r minus the offset of its first entry inside its row, so the column of
// entry p in row i, run r, is rcol[r] + (p - row_ptr[i]).  Needs nnz < 2^32.
struct RowMasks {
    std::vector<uint64_t> mask;     // [ceil(nnz / 64)]
    std::vector<uint32_t> base;     // [ceil(nnz / 64)]
    std::vector<int32_t> rcol;      // [runs]
};

inline bool build_row_masks_host(int64_t m, const int64_t *rp, const int32_t *ci, RowMasks &R)
{
    const int64_t nnz = rp[m];
    if (nnz >= ((int64_t)1 << 32)) return false;
    const int64_t nw = (nnz + 63) / 64;
    R.mask.assign((size_t)nw, 0ull);
    R.base.assign((size_t)nw, 0u);
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (nnz < (1 << 20)) nt = 1;
    auto start = [&](int64_t i, int64_t p) { return p == rp[i] || ci[p] != ci[p - 1] + 1; };
    // bits: threads own whole mask words (entry ranges split at multiples of 64)
    {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t]() {
                const int64_t w0 = nw * t / nt, w1 = nw * (t + 1) / nt;
                if (w0 >= w1) return;
                // first row holding entry 64 w0
                int64_t i = std::upper_bound(rp, rp + m + 1, 64 * w0) - rp - 1;
                for (int64_t p = 64 * w0; p < std::min(64 * w1, nnz); ++p) {
                    while (rp[i + 1] <= p) ++i;
                    if (start(i, p)) R.mask[(size_t)(p >> 6)] |= 1ull << (p & 63);
                }
            });
        for (auto &x : th) x.join();
    }
    uint64_t runs = 0;
    for (int64_t w = 0; w < nw; ++w) {
        R.base[(size_t)w] = (uint32_t)runs;
        runs += (uint64_t)__builtin_popcountll(R.mask[(size_t)w]);
    }
    if (runs >= ((uint64_t)1 << 32)) return false;
    R.rcol.resize((size_t)runs);
    {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t]() {
                for (int64_t i = m * t / nt; i < m * (t + 1) / nt; ++i)
                    for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
                        if (start(i, p)) {
                            const int64_t w = p >> 6;
                            const uint64_t below = R.mask[(size_t)w] & ((1ull << (p & 63)) - 1);
                            const int64_t r = (int64_t)R.base[(size_t)w] + __builtin_popcountll(below);
                            R.rcol[(size_t)r] = (int32_t)(ci[p] - (p - rp[i]));
                        }
            });
        for (auto &x : th) x.join();
    }
    return true;
}

// Node masks of the data block (transposed product over the CSC values).  For
// lateral node k (columns [k nz, (k+1) nz), eq. 7): rows[rp_k .. rp_{k+1}) =
// the data rows reaching the node, ascending, cut into chunks of 64; chunk c
// of all nodes (global chunk index) has nz mask words, bit l of word
// mask[c nz + iz] set when row 64 (c - chunk0_k) + l of node k has an entry in
// column k nz + iz.  The entries of a column sit in the CSC in ascending row
// order, so the set bits, in order, enumerate the column's values.  qoff
// [(k 4 + w) nz + iz] = CSC position of the first value of column k nz + iz
// in quarter w of the node's chunks (wave w of the workgroup takes chunks
// [chunk0 + c w / 4, chunk0 + c (w+1) / 4)).  order = nodes by decreasing
// chunk count (stable).
struct NodeMasks {
    std::vector<int64_t> rptr;      // [nnodes+1] into rows
    std::vector<uint32_t> rows;     // [node rows]
    std::vector<int64_t> cptr;      // [nnodes+1] first global chunk of a node
    std::vector<uint64_t> mask;     // [chunks * nz]
    std::vector<int64_t> qoff;      // [nnodes * 4 * nz]
    std::vector<int32_t> order;     // [nnodes]
};

inline bool build_node_masks_host(int64_t m, int64_t n, int nz, const int64_t *rp,
                                  const int32_t *ci, NodeMasks &R)
{
    const int64_t nnz = rp[m];
    if (nz < 1 || nz > 32 || n % nz != 0 || m >= ((int64_t)1 << 32)) return false;
    const int64_t nn = n / nz;
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (nnz < (1 << 20)) nt = 1;
    // (row, node) pairs: entries of one node are contiguous inside a row
    std::vector<std::vector<int64_t>> cnt(nt, std::vector<int64_t>((size_t)nn, 0));
    {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t]() {
                auto &c = cnt[t];
                for (int64_t i = m * t / nt; i < m * (t + 1) / nt; ++i)
                    for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
                        if (p == rp[i] || ci[p] / nz != ci[p - 1] / nz) ++c[(size_t)(ci[p] / nz)];
            });
        for (auto &x : th) x.join();
    }
    R.rptr.assign((size_t)nn + 1, 0);
    for (int64_t k = 0; k < nn; ++k) {
        int64_t tot = 0;
        for (unsigned t = 0; t < nt; ++t) {
            const int64_t c = cnt[t][(size_t)k];
            cnt[t][(size_t)k] = R.rptr[(size_t)k] + tot;      // becomes the cursor
            tot += c;
        }
        R.rptr[(size_t)k + 1] = R.rptr[(size_t)k] + tot;
    }
    R.cptr.assign((size_t)nn + 1, 0);
    for (int64_t k = 0; k < nn; ++k)
        R.cptr[(size_t)k + 1] = R.cptr[(size_t)k] + (R.rptr[(size_t)k + 1] - R.rptr[(size_t)k] + 63) / 64;
    R.rows.resize((size_t)R.rptr[(size_t)nn]);
    R.mask.assign((size_t)(R.cptr[(size_t)nn] * nz), 0ull);
    {
        // a thread's rows land in disjoint slots; the mask bits are set in a
        // second pass split by node, so every mask word has one writer
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t]() {
                auto &cur = cnt[t];
                for (int64_t i = m * t / nt; i < m * (t + 1) / nt; ++i)
                    for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
                        if (p == rp[i] || ci[p] / nz != ci[p - 1] / nz)
                            R.rows[(size_t)cur[(size_t)(ci[p] / nz)]++] = (uint32_t)i;
            });
        for (auto &x : th) x.join();
    }
    {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t]() {
                for (int64_t k = nn * t / nt; k < nn * (t + 1) / nt; ++k)
                    for (int64_t q = R.rptr[(size_t)k]; q < R.rptr[(size_t)k + 1]; ++q) {
                        const int64_t i = R.rows[(size_t)q], idx = q - R.rptr[(size_t)k];
                        const int64_t chunk = R.cptr[(size_t)k] + idx / 64;
                        // the row's entries in node k: binary search the row's columns
                        const int32_t *b = ci + rp[i], *e = ci + rp[i + 1];
                        for (const int32_t *c = std::lower_bound(b, e, (int32_t)(k * nz));
                             c < e && *c < (k + 1) * nz; ++c)
                            R.mask[(size_t)(chunk * nz + (*c - k * nz))] |= 1ull << (idx & 63);
                    }
            });
        for (auto &x : th) x.join();
    }
    // quarter offsets: column start (CSC) plus the set bits of earlier chunks
    std::vector<int64_t> colcnt((size_t)n + 1, 0);
    for (int64_t p = 0; p < nnz; ++p) ++colcnt[(size_t)ci[p] + 1];
    for (int64_t j = 0; j < n; ++j) colcnt[(size_t)j + 1] += colcnt[(size_t)j];
    R.qoff.assign((size_t)(nn * 4 * nz), 0);
    for (int64_t k = 0; k < nn; ++k) {
        const int64_t c0 = R.cptr[(size_t)k], nc = R.cptr[(size_t)k + 1] - c0;
        for (int iz = 0; iz < nz; ++iz) {
            int64_t pos = colcnt[(size_t)(k * nz + iz)];
            int64_t c = 0;
            for (int w = 0; w < 4; ++w) {
                const int64_t cw = nc * w / 4;
                for (; c < cw; ++c) pos += __builtin_popcountll(R.mask[(size_t)((c0 + c) * nz + iz)]);
                R.qoff[(size_t)((k * 4 + w) * nz + iz)] = pos;
            }
        }
    }
    R.order.resize((size_t)nn);
    for (int64_t k = 0; k < nn; ++k) R.order[(size_t)k] = (int32_t)k;
    std::stable_sort(R.order.begin(), R.order.end(), [&](int32_t x, int32_t y) {
        return R.cptr[(size_t)x + 1] - R.cptr[(size_t)x] > R.cptr[(size_t)y + 1] - R.cptr[(size_t)y];
    });
    return true;
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

// Run-slice layout of the node runs (k_adj_slices).  Per node, its runs are
// ordered by first depth, then by decreasing length, then by row (a stable
// order), and cut into slices of up to 64 runs that share a first depth.  A
// slice's padded length L is its longest run rounded up to a multiple of W;
// it occupies L * 64 values from off[s]: step k (depths kW .. kW+W-1 of every
// run) holds lane j's W values at off[s] + k 64 W + j W.  Lanes without a
// run (the last slice of a first depth) and depths past a run's end hold
// zeros; their row is 0.  dst[r] = off[s] + j W for run r in lane j of
// slice s, so value e of run r sits at dst[r] + (e / W) 64 W + e mod W.
// total = padded values.  Rows must fit 32 bits (node runs already do).
struct RunSlices {
    std::vector<int64_t> sptr;      // [nn+1]
    std::vector<int64_t> off;       // [nslices]
    std::vector<uint16_t> desc;     // [nslices] (iz0 << 8) | L
    std::vector<uint32_t> row;      // [64 nslices]
    std::vector<uint64_t> dst;      // [nruns]
    int64_t total = 0;
};

inline void slice_layout_host(const NodeRuns &R, int64_t nn, int W, RunSlices &S)
{
    const int64_t nr = R.nrp[(size_t)nn];
    // slice counts per node (threads over nodes), then offsets, then fill
    std::vector<int64_t> cnt((size_t)nn, 0), vals((size_t)nn, 0);
    std::vector<std::vector<uint32_t>> ord((size_t)nn);
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (nr < (1 << 20)) nt = 1;
    auto key_less = [&](uint32_t x, uint32_t y) {
        const int ix = R.desc[x] >> 8, iy = R.desc[y] >> 8;
        if (ix != iy) return ix < iy;
        const int lx = R.desc[x] & 255, ly = R.desc[y] & 255;
        if (lx != ly) return lx > ly;
        return x < y;
    };
    {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t]() {
                for (int64_t k = nn * t / nt; k < nn * (t + 1) / nt; ++k) {
                    const int64_t r0 = R.nrp[(size_t)k], r1 = R.nrp[(size_t)k + 1];
                    auto &o = ord[(size_t)k];
                    o.resize((size_t)(r1 - r0));
                    for (int64_t r = r0; r < r1; ++r) o[(size_t)(r - r0)] = (uint32_t)r;
                    std::sort(o.begin(), o.end(), key_less);
                    int64_t ns = 0, nv = 0;
                    for (size_t i = 0; i < o.size();) {
                        const int iz0 = R.desc[o[i]] >> 8;
                        const int L = (((R.desc[o[i]] & 255) + W - 1) / W) * W;   // longest first
                        size_t j = i;
                        while (j < o.size() && j - i < 64 && (R.desc[o[j]] >> 8) == iz0) ++j;
                        ++ns;
                        nv += (int64_t)L * 64;
                        i = j;
                    }
                    cnt[(size_t)k] = ns;
                    vals[(size_t)k] = nv;
                }
            });
        for (auto &x : th) x.join();
    }
    S.sptr.assign((size_t)nn + 1, 0);
    std::vector<int64_t> voff((size_t)nn + 1, 0);
    for (int64_t k = 0; k < nn; ++k) {
        S.sptr[(size_t)k + 1] = S.sptr[(size_t)k] + cnt[(size_t)k];
        voff[(size_t)k + 1] = voff[(size_t)k] + vals[(size_t)k];
    }
    const int64_t nsl = S.sptr[(size_t)nn];
    S.total = voff[(size_t)nn];
    S.off.resize((size_t)nsl);
    S.desc.resize((size_t)nsl);
    S.row.assign((size_t)nsl * 64, 0u);
    S.dst.resize((size_t)nr);
    {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t]() {
                for (int64_t k = nn * t / nt; k < nn * (t + 1) / nt; ++k) {
                    const auto &o = ord[(size_t)k];
                    int64_t sl = S.sptr[(size_t)k], off = voff[(size_t)k];
                    for (size_t i = 0; i < o.size();) {
                        const int iz0 = R.desc[o[i]] >> 8;
                        const int L = (((R.desc[o[i]] & 255) + W - 1) / W) * W;
                        S.off[(size_t)sl] = off;
                        S.desc[(size_t)sl] = (uint16_t)((iz0 << 8) | L);
                        size_t j = i;
                        for (; j < o.size() && j - i < 64 && (R.desc[o[j]] >> 8) == iz0; ++j) {
                            const int lane = (int)(j - i);
                            S.row[(size_t)(sl * 64 + lane)] = R.row[o[j]];
                            S.dst[o[j]] = (uint64_t)(off + (int64_t)lane * W);
                        }
                        off += (int64_t)L * 64;
                        ++sl;
                        i = j;
                    }
                }
            });
        for (auto &x : th) x.join();
    }
}

}  // namespace lsqr
