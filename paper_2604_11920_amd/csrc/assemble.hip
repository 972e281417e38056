// Device-side assembly of the data block G from the rays (per path: crossed
// lateral nodes and path lengths; per period: phase velocity and depth
// kernel).  The host derives the row structure (path-major rows, nnz per row
// = nodes x kernel depths) from the small ray arrays; one wave per row then
// writes the row's columns and values on the device.
#include <math.h>

#include <vector>

#include "ctx.h"
#include "split_path.h"

namespace {

// ------------------------------------------------------ bilinear split --
constexpr int kSplitCap = 4096;          // corner records of one path (LDS)
constexpr int kSplitMaxGroup = 129;      // contributions to one node

// Exclusive prefix sum of v over the 256 threads (ascending thread order);
// *tot receives the total.  Every thread must call it.
__device__ int block_excl_scan(int v, int *ws, int *tot)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) ws[wid] = x;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wid; ++w) before += ws[w];
    *tot = ws[0] + ws[1] + ws[2] + ws[3];
    __syncthreads();
    return before + x - v;
}

// One workgroup per path: the corner records of its pieces in path order
// into LDS (key = node << 12 | record position, so sorting the keys groups
// the records by node and keeps path order inside a node), a bitonic sort
// of the keys, then one thread per group start sums the group
// (sum_contributions) and the positive ones are numbered in node order.
// Count pass (node_k == nullptr): cnt[p] = nodes kept.  Fill pass: the
// nodes and lengths at node_ptr[p] ... *err |= 1 when a path has more than
// kSplitCap records, 2 when a node has more than kSplitMaxGroup.
__global__ __launch_bounds__(256) void k_split_paths(int64_t npaths, const int64_t *pt_ptr,
                                                     const double *px, const double *py,
                                                     const double *plen, lsqr::SplitGrid g,
                                                     int64_t *cnt, const int64_t *node_ptr,
                                                     int32_t *node_k, double *node_len, int *err)
{
    __shared__ uint64_t key[kSplitCap];
    __shared__ double val[kSplitCap];
    __shared__ int ws[4];
    const int tid = threadIdx.x;
    for (int64_t p = blockIdx.x; p < npaths; p += gridDim.x) {
        const int64_t p0 = pt_ptr[p], npc = pt_ptr[p + 1] - p0 - 1;
        int nrec = 0;
        bool over = false;
        for (int64_t c0 = 0; c0 < npc; c0 += 256) {
            const int64_t i = p0 + c0 + tid;
            int64_t nb[12];
            double vb[12];
            int r = 0;
            if (c0 + tid < npc) r = lsqr::split_piece(px[i], py[i], px[i + 1], py[i + 1], plen[i], g, nb, vb);
            int tot = 0;
            const int off = block_excl_scan(r, ws, &tot);
            if (nrec + tot > kSplitCap) { over = true; break; }       // uniform
            for (int j = 0; j < r; ++j) {
                const int pos = nrec + off + j;
                key[pos] = ((uint64_t)nb[j] << 12) | (uint64_t)pos;
                val[pos] = vb[j];
            }
            nrec += tot;
        }
        if (over) {
            if (tid == 0) { atomicOr(err, 1); if (!node_k) cnt[p] = 0; }
            __syncthreads();
            continue;
        }
        int n2 = 1;
        while (n2 < nrec) n2 <<= 1;
        for (int j = nrec + tid; j < n2; j += 256) key[j] = ~(uint64_t)0;
        __syncthreads();
        for (int k = 2; k <= n2; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = tid; i < n2; i += 256) {
                    const int q = i ^ j;
                    if (q > i) {
                        const uint64_t a = key[i], b = key[q];
                        const bool up = (i & k) == 0;
                        if ((a > b) == up) { key[i] = b; key[q] = a; }
                    }
                }
                __syncthreads();
            }
        int kept = 0;
        const int64_t out0 = node_k ? node_ptr[p] : 0;
        for (int c0 = 0; c0 < nrec; c0 += 256) {
            const int j = c0 + tid;
            int keep = 0;
            double sum = 0.0;
            uint64_t node = 0;
            if (j < nrec) {
                node = key[j] >> 12;
                if (j == 0 || (key[j - 1] >> 12) != node) {
                    int e = j + 1;
                    while (e < nrec && (key[e] >> 12) == node) ++e;
                    if (e - j > kSplitMaxGroup) {
                        atomicOr(err, 2);
                    } else {
                        sum = lsqr::sum_contributions(e - j, [&](int q) { return val[key[j + q] & 4095u]; });
                        keep = sum > 0.0;
                    }
                }
            }
            int tot = 0;
            const int off = block_excl_scan(keep, ws, &tot);
            if (keep && node_k) {
                node_k[out0 + kept + off] = (int32_t)node;
                node_len[out0 + kept + off] = sum;
            }
            kept += tot;
        }
        if (!node_k && tid == 0) cnt[p] = kept;
        __syncthreads();
    }
}

// Checks device-resident node arrays: bit 1 a negative node, bit 2 a
// non-finite length; kmax = the largest node.
__global__ void k_check_nodes(int64_t nn, const int32_t *node_k, const double *node_len,
                              int *flag, int *kmax)
{
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nn;
         a += (int64_t)gridDim.x * blockDim.x) {
        const int k = node_k[a];
        if (k < 0) atomicOr(flag, 1);
        if (!isfinite(node_len[a])) atomicOr(flag, 2);
        atomicMax(kmax, k);
    }
}

// Row r = (path rpair[r], period rper[r]); entry i of the row, i = a nj + b:
// node a of the path, depth j0 + b; value (-len_a / c_t) w_t[b], the same
// two FP64 operations in the same order as the generator.
__global__ __launch_bounds__(lsqr::kBlock) void k_assemble(
    int64_t m, int nz, const int64_t *rp, const int32_t *rpair, const int32_t *rper,
    const int64_t *node_ptr, const int32_t *node_k, const double *node_len, const double *cvel,
    const int32_t *j0, const int32_t *nj, const int64_t *w_ptr, const double *w, int32_t *col,
    double *val)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (lsqr::kBlock / 64);
    for (int64_t r = (int64_t)blockIdx.x * (lsqr::kBlock / 64) + (threadIdx.x >> 6); r < m;
         r += waves) {
        const int p = rpair[r], t = rper[r];
        const int64_t s0 = rp[r], e = rp[r + 1];
        const int q = nj[t];
        const int64_t a0 = node_ptr[p];
        const int base = j0[t];
        const double c = cvel[t];
        const double *wt = w + w_ptr[t];
        for (int64_t i = s0 + lane; i < e; i += 64) {
            const int64_t off = i - s0;
            const int64_t a = a0 + off / q;
            const int b = (int)(off % q);
            const double s = -node_len[a] / c;
            col[i] = node_k[a] * nz + base + b;
            val[i] = s * wt[b];
        }
    }
}

// Validates the rays and derives the row structure on the host.
lsqr_status ray_rows(const lsqr_rays *R, std::vector<int64_t> *rp, std::vector<int32_t> *rpair,
                     std::vector<int32_t> *rper, int64_t *m_out, int64_t *nnz_out)
{
    if (!R) return lsqr::fail(nullptr, LSQR_E_INVALID_ARG, "rays is NULL");
    if (R->npairs < 0 || R->nper < 1 || R->nz < 1)
        return lsqr::fail(nullptr, LSQR_E_INVALID_ARG, "npairs >= 0, nper >= 1 and nz >= 1 required");
    if (R->npairs >= ((int64_t)1 << 31))
        return lsqr::fail(nullptr, LSQR_E_UNSUPPORTED, "npairs must be below 2^31");
    if (!R->node_ptr || !R->cvel || !R->j0 || !R->nj || !R->w_ptr || (R->npairs > 0 && !R->keep))
        return lsqr::fail(nullptr, LSQR_E_INVALID_ARG, "ray arrays are NULL");
    const int64_t P = R->npairs, T = R->nper;
    if (R->node_ptr[0] != 0) return lsqr::fail(nullptr, LSQR_E_INVALID_ARG, "node_ptr[0] must be 0");
    for (int64_t p = 0; p < P; ++p)
        if (R->node_ptr[p + 1] < R->node_ptr[p])
            return lsqr::fail(nullptr, LSQR_E_INVALID_ARG, "node_ptr must be non-decreasing");
    const int64_t nn = R->node_ptr[P];
    if (nn > 0 && (!R->node_k || !R->node_len))
        return lsqr::fail(nullptr, LSQR_E_INVALID_ARG, "node arrays are NULL");
    if (R->node_mem != LSQR_MEM_HOST && R->node_mem != LSQR_MEM_DEVICE)
        return lsqr::fail(nullptr, LSQR_E_INVALID_ARG, "unknown memory kind of the node arrays");
    int64_t kmax = -1;
    if (R->node_mem == LSQR_MEM_HOST) {
        for (int64_t a = 0; a < nn; ++a) {
            if (R->node_k[a] < 0) return lsqr::fail(nullptr, LSQR_E_INVALID_ARG, "node_k must be >= 0");
            if (!isfinite(R->node_len[a])) return lsqr::fail(nullptr, LSQR_E_NONFINITE, "non-finite node_len");
            kmax = R->node_k[a] > kmax ? R->node_k[a] : kmax;
        }
    }                              // device arrays: checked by lsqr_assemble_rays
    if (R->w_ptr[0] != 0) return lsqr::fail(nullptr, LSQR_E_INVALID_ARG, "w_ptr[0] must be 0");
    for (int64_t t = 0; t < T; ++t) {
        if (R->j0[t] < 0 || R->nj[t] < 0 || (int64_t)R->j0[t] + R->nj[t] > R->nz)
            return lsqr::fail(nullptr, LSQR_E_INVALID_ARG, "depth kernel outside 0 .. nz-1");
        if (R->w_ptr[t + 1] - R->w_ptr[t] != R->nj[t])
            return lsqr::fail(nullptr, LSQR_E_INVALID_ARG, "w_ptr[t+1] - w_ptr[t] must equal nj[t]");
        if (!isfinite(R->cvel[t]) || R->cvel[t] == 0.0)
            return lsqr::fail(nullptr, LSQR_E_INVALID_ARG, "cvel must be finite and nonzero");
    }
    if (R->w_ptr[T] > 0 && !R->w) return lsqr::fail(nullptr, LSQR_E_INVALID_ARG, "w is NULL");
    for (int64_t i = 0; i < R->w_ptr[T]; ++i)
        if (!isfinite(R->w[i])) return lsqr::fail(nullptr, LSQR_E_NONFINITE, "non-finite depth weight");
    if ((kmax + 1) * (int64_t)R->nz >= ((int64_t)1 << 31))
        return lsqr::fail(nullptr, LSQR_E_UNSUPPORTED, "columns must be below 2^31");
    int64_t m = 0, nnz = 0;
    if (rp) rp->assign(1, 0);
    for (int64_t p = 0; p < P; ++p) {
        const int64_t nk = R->node_ptr[p + 1] - R->node_ptr[p];
        for (int64_t t = 0; t < T; ++t) {
            if (!R->keep[p * T + t]) continue;
            nnz += nk * R->nj[t];
            ++m;
            if (rp) {
                rp->push_back(nnz);
                rpair->push_back((int32_t)p);
                rper->push_back((int32_t)t);
            }
        }
    }
    if (m >= ((int64_t)1 << 31)) return lsqr::fail(nullptr, LSQR_E_UNSUPPORTED, "m must be below 2^31");
    *m_out = m;
    *nnz_out = nnz;
    return LSQR_OK;
}

// A temporary device copy of a host array, from the caller's allocator.
struct Staged {
    void *p = nullptr;
    size_t bytes = 0;
};

template <class T>
hipError_t upload(lsqr::Allocator &al, std::vector<Staged> &held, T **d, const T *h, int64_t count,
                  hipStream_t st)
{
    *d = nullptr;
    if (count <= 0) return hipSuccess;
    const size_t bytes = (size_t)count * sizeof(T);
    *d = (T *)al.get(bytes);
    if (!*d) return hipErrorOutOfMemory;
    held.push_back({(void *)*d, bytes});
    return hipMemcpyAsync(*d, h, bytes, hipMemcpyHostToDevice, st);
}

}  // namespace

extern "C" {

lsqr_status lsqr_rays_size(const lsqr_rays *rays, int64_t *m, int64_t *nnz)
{
    if (!m || !nnz) return lsqr::fail(nullptr, LSQR_E_INVALID_ARG, "m and nnz must not be NULL");
    return ray_rows(rays, nullptr, nullptr, nullptr, m, nnz);
}

lsqr_status lsqr_assemble_rays(const lsqr_rays *rays, void *stream, lsqr_alloc_fn alloc,
                               lsqr_free_fn dealloc, void *alloc_user, int64_t *row_ptr,
                               int32_t *col_idx, double *val)
{
    std::vector<int64_t> rp;
    std::vector<int32_t> rpair, rper;
    int64_t m = 0, nnz = 0;
    lsqr_status s = ray_rows(rays, &rp, &rpair, &rper, &m, &nnz);
    if (s != LSQR_OK) return s;
    if (!row_ptr || (nnz > 0 && (!col_idx || !val)))
        return lsqr::fail(nullptr, LSQR_E_INVALID_ARG, "output arrays are NULL");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(row_ptr, rp.data(), (m + 1) * sizeof(int64_t),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nnz > 0) {
        const lsqr_rays &R = *rays;
        int32_t *d_rpair = nullptr, *d_rper = nullptr, *d_k = nullptr, *d_j0 = nullptr, *d_nj = nullptr;
        int64_t *d_np = nullptr, *d_wp = nullptr;
        double *d_len = nullptr, *d_c = nullptr, *d_w = nullptr;
        const int64_t nn = R.node_ptr[R.npairs];
        lsqr::Allocator al;
        al.alloc = alloc;
        al.dealloc = dealloc;
        al.user = alloc_user;
        std::vector<Staged> held;
        hipError_t u = hipSuccess;
        if (u == hipSuccess) u = upload(al, held, &d_rpair, rpair.data(), m, st);
        if (u == hipSuccess) u = upload(al, held, &d_rper, rper.data(), m, st);
        if (u == hipSuccess) u = upload(al, held, &d_np, R.node_ptr, R.npairs + 1, st);
        if (R.node_mem == LSQR_MEM_DEVICE) {
            d_k = const_cast<int32_t *>(R.node_k);
            d_len = const_cast<double *>(R.node_len);
            // nodes >= 0, lengths finite, columns below 2^31: checked here
            int *d_flag = nullptr;
            int hf[2] = {0, -1};
            if (nn > 0) {
                u = upload(al, held, &d_flag, hf, 2, st);
                if (u == hipSuccess) {
                    hipLaunchKernelGGL(k_check_nodes, dim3((unsigned)std::min<int64_t>((nn + 255) / 256, 4096)),
                                       dim3(256), 0, st, nn, R.node_k, R.node_len, d_flag, d_flag + 1);
                    u = hipGetLastError();
                }
                if (u == hipSuccess) u = hipMemcpyAsync(hf, d_flag, sizeof(hf), hipMemcpyDeviceToHost, st);
                if (u == hipSuccess) u = hipStreamSynchronize(st);
                if (u == hipSuccess && (hf[0] || ((int64_t)hf[1] + 1) * R.nz >= ((int64_t)1 << 31))) {
                    for (const Staged &h : held) al.put(h.p, h.bytes);
                    return lsqr::fail(nullptr, (hf[0] & 2) ? LSQR_E_NONFINITE : (hf[0] & 1) ? LSQR_E_INVALID_ARG
                                                                                               : LSQR_E_UNSUPPORTED,
                                      (hf[0] & 2) ? "non-finite node_len" : (hf[0] & 1) ? "node_k must be >= 0"
                                                                                       : "columns must be below 2^31");
                }
            }
        } else {
            if (u == hipSuccess) u = upload(al, held, &d_k, R.node_k, nn, st);
            if (u == hipSuccess) u = upload(al, held, &d_len, R.node_len, nn, st);
        }
        if (u == hipSuccess) u = upload(al, held, &d_c, R.cvel, (int64_t)R.nper, st);
        if (u == hipSuccess) u = upload(al, held, &d_j0, R.j0, (int64_t)R.nper, st);
        if (u == hipSuccess) u = upload(al, held, &d_nj, R.nj, (int64_t)R.nper, st);
        if (u == hipSuccess) u = upload(al, held, &d_wp, R.w_ptr, (int64_t)R.nper + 1, st);
        if (u == hipSuccess) u = upload(al, held, &d_w, R.w, R.w_ptr[R.nper], st);
        if (u == hipSuccess) {
            const int64_t blocks = std::min<int64_t>((m + 3) / 4, 4096);
            hipLaunchKernelGGL(k_assemble, dim3((unsigned)std::max<int64_t>(blocks, 1)),
                               dim3(lsqr::kBlock), 0, st, m, (int)R.nz, row_ptr, d_rpair, d_rper,
                               d_np, d_k, d_len, d_c, d_j0, d_nj, d_wp, d_w, col_idx, val);
            u = hipGetLastError();
        }
        hipError_t w = hipStreamSynchronize(st);
        if (u == hipSuccess) u = w;
        for (const Staged &h : held) al.put(h.p, h.bytes);
        e = u;
    } else if (e == hipSuccess) {
        e = hipStreamSynchronize(st);
    }
    if (e != hipSuccess)
        return lsqr::fail(nullptr, e == hipErrorOutOfMemory ? LSQR_E_OOM : LSQR_E_DEVICE,
                          std::string("assembly: ") + hipGetErrorString(e));
    return LSQR_OK;
}

lsqr_status lsqr_split_polylines(const lsqr_polylines *P, void *stream, lsqr_alloc_fn alloc,
                                 lsqr_free_fn dealloc, void *alloc_user, int64_t *node_ptr,
                                 int32_t *node_k, double *node_len)
{
    using lsqr::fail;
    if (!P || !node_ptr) return fail(nullptr, LSQR_E_INVALID_ARG, "poly and node_ptr must not be NULL");
    if ((node_k == nullptr) != (node_len == nullptr))
        return fail(nullptr, LSQR_E_INVALID_ARG, "node_k and node_len: both or neither");
    const int64_t np = P->npaths;
    if (np < 0 || P->nx < 2 || P->ny < 2 || !(P->h > 0.0) || !isfinite(P->h) ||
        !(P->km_per_deg > 0.0) || !isfinite(P->km_per_deg))
        return fail(nullptr, LSQR_E_INVALID_ARG, "npaths >= 0, nx, ny >= 2, h > 0 and km_per_deg > 0 required");
    if ((int64_t)P->nx * P->ny >= ((int64_t)1 << 31))
        return fail(nullptr, LSQR_E_UNSUPPORTED, "nx ny must be below 2^31");
    if (!P->pt_ptr) return fail(nullptr, LSQR_E_INVALID_ARG, "pt_ptr is NULL");
    if (P->pt_ptr[0] != 0) return fail(nullptr, LSQR_E_INVALID_ARG, "pt_ptr[0] must be 0");
    for (int64_t p = 0; p < np; ++p)
        if (P->pt_ptr[p + 1] < P->pt_ptr[p])
            return fail(nullptr, LSQR_E_INVALID_ARG, "pt_ptr must be non-decreasing");
    const int64_t npt = P->pt_ptr[np];
    if (npt > 0 && (!P->px || !P->py || !P->plen))
        return fail(nullptr, LSQR_E_INVALID_ARG, "point arrays are NULL");
    for (int64_t i = 0; i < npt; ++i)
        if (!isfinite(P->px[i]) || !isfinite(P->py[i]))
            return fail(nullptr, LSQR_E_NONFINITE, "non-finite point");
    for (int64_t p = 0; p < np; ++p)
        for (int64_t i = P->pt_ptr[p]; i + 1 < P->pt_ptr[p + 1]; ++i) {
            if (!isfinite(P->plen[i]) || P->plen[i] < 0.0)
                return fail(nullptr, LSQR_E_NONFINITE, "piece lengths must be finite and >= 0");
            if (!(fabs(P->px[i + 1] - P->px[i]) < P->h) || !(fabs(P->py[i + 1] - P->py[i]) < P->h))
                return fail(nullptr, LSQR_E_INVALID_ARG, "a piece spans a whole cell (|dx| or |dy| >= h)");
        }
    hipStream_t st = (hipStream_t)stream;
    lsqr::Allocator al;
    al.alloc = alloc;
    al.dealloc = dealloc;
    al.user = alloc_user;
    std::vector<Staged> held;
    const int64_t *d_pt = nullptr;
    const double *d_x = nullptr, *d_y = nullptr, *d_l = nullptr;
    int64_t *d_cnt = nullptr, *d_np = nullptr;
    int *d_err = nullptr;
    hipError_t u = hipSuccess;
    u = upload(al, held, const_cast<int64_t **>(&d_pt), P->pt_ptr, np + 1, st);
    if (u == hipSuccess) u = upload(al, held, const_cast<double **>(&d_x), P->px, npt, st);
    if (u == hipSuccess) u = upload(al, held, const_cast<double **>(&d_y), P->py, npt, st);
    if (u == hipSuccess) u = upload(al, held, const_cast<double **>(&d_l), P->plen, npt, st);
    std::vector<int64_t> cnt((size_t)np + 1, 0);
    int herr = 0;
    if (u == hipSuccess) u = upload(al, held, &d_cnt, cnt.data(), np + 1, st);
    if (u == hipSuccess) u = upload(al, held, &d_err, &herr, 1, st);
    const lsqr::SplitGrid g{P->h, P->km_per_deg, P->nx, P->ny};
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(np, 8192));
    if (u == hipSuccess && np > 0) {
        hipLaunchKernelGGL(k_split_paths, dim3(grid), dim3(256), 0, st, np, d_pt, d_x, d_y, d_l, g,
                           d_cnt, (const int64_t *)nullptr, (int32_t *)nullptr, (double *)nullptr,
                           d_err);
        u = hipGetLastError();
    }
    if (u == hipSuccess) u = hipMemcpyAsync(cnt.data(), d_cnt, np * sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (u == hipSuccess) u = hipMemcpyAsync(&herr, d_err, sizeof(int), hipMemcpyDeviceToHost, st);
    if (u == hipSuccess) u = hipStreamSynchronize(st);
    lsqr_status s = LSQR_OK;
    if (u == hipSuccess && herr)
        s = fail(nullptr, LSQR_E_UNSUPPORTED, (herr & 1) ? "a path has more than 4096 corner records"
                                                         : "a node receives more than 129 contributions");
    if (u == hipSuccess && s == LSQR_OK) {
        node_ptr[0] = 0;
        for (int64_t p = 0; p < np; ++p) node_ptr[p + 1] = node_ptr[p] + cnt[(size_t)p];
        if (node_k && np > 0) {
            u = upload(al, held, &d_np, node_ptr, np + 1, st);
            if (u == hipSuccess) {
                hipLaunchKernelGGL(k_split_paths, dim3(grid), dim3(256), 0, st, np, d_pt, d_x, d_y,
                                   d_l, g, d_cnt, (const int64_t *)d_np, node_k, node_len, d_err);
                u = hipGetLastError();
            }
            if (u == hipSuccess) u = hipStreamSynchronize(st);
        }
    }
    (void)hipStreamSynchronize(st);
    for (const Staged &h : held) al.put(h.p, h.bytes);
    if (u != hipSuccess)
        return fail(nullptr, u == hipErrorOutOfMemory ? LSQR_E_OOM : LSQR_E_DEVICE,
                    std::string("polyline split: ") + hipGetErrorString(u));
    return s;
}

}  // extern "C"
