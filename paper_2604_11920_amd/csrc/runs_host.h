// Host-side builders of the run formats (plain C++, no HIP): depth runs of
// the data rows (forward product) and node runs of the data block
// (transposed product).  Both read only the CSR structure.
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

}  // namespace lsqr
