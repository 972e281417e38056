// Device-side assembly of the data block G from the rays (per path: crossed
// lateral nodes and path lengths; per period: phase velocity and depth
// kernel).  The host derives the row structure (path-major rows, nnz per row
// = nodes x kernel depths) from the small ray arrays; one wave per row then
// writes the row's columns and values on the device.
#include <math.h>

#include <vector>

#include "ctx.h"

namespace {

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
    int64_t kmax = -1;
    for (int64_t a = 0; a < nn; ++a) {
        if (R->node_k[a] < 0) return lsqr::fail(nullptr, LSQR_E_INVALID_ARG, "node_k must be >= 0");
        if (!isfinite(R->node_len[a])) return lsqr::fail(nullptr, LSQR_E_NONFINITE, "non-finite node_len");
        kmax = R->node_k[a] > kmax ? R->node_k[a] : kmax;
    }
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
        if (u == hipSuccess) u = upload(al, held, &d_k, R.node_k, nn, st);
        if (u == hipSuccess) u = upload(al, held, &d_len, R.node_len, nn, st);
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

}  // extern "C"
