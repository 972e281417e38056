// Device transpose CSR -> CSC.
//
// The transposed product of LSQR reads G^T from a stored copy instead of
// scattering with atomics.  The copy is built once per system: a stable LSD
// radix sort of (column, nnz position) pairs on the column bits keeps the
// row-major order inside every column, so rows are ascending within a column
// and the result is independent of scheduling (bitwise reproducible).
#include <rocprim/device/device_radix_sort.hpp>

#include "internal.h"

namespace lsqr {

void *Allocator::get(size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (alloc) return alloc(bytes, user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void Allocator::put(void *p, size_t bytes)
{
    if (!p) return;
    if (alloc) {
        if (dealloc) dealloc(p, bytes, user);
        return;
    }
    (void)hipFree(p);
}

__global__ void k_copy_keys(int64_t nnz, const int32_t *col, uint32_t *keys, uint32_t *pos)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        keys[e] = (uint32_t)col[e];
        pos[e] = (uint32_t)e;
    }
}

// row id of every stored entry (one wave per row)
__global__ void k_row_ids(int64_t m, const int64_t *rp, int32_t *rowid)
{
    const int lane = threadIdx.x & 63;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < m;
         i += ((int64_t)gridDim.x * blockDim.x) >> 6)
        for (int64_t e = rp[i] + lane; e < rp[i + 1]; e += 64) rowid[e] = (int32_t)i;
}

__global__ void k_gather_csc(int64_t nnz, const uint32_t *perm, const int32_t *rowid,
                             const double *val, int32_t *crow, double *cval)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t e = perm[p];
        crow[p] = rowid[e];
        cval[p] = val[e];
    }
}

// col_ptr[c] = first position whose key >= c
__global__ void k_col_ptr(int64_t nnz, int64_t n, const uint32_t *keys, int64_t *cp)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = keys[p];
        const int64_t prev = p == 0 ? -1 : (int64_t)keys[p - 1];
        for (int64_t c = prev + 1; c <= k; ++c) cp[c] = p;
    }
}

__global__ void k_col_ptr_tail(int64_t nnz, int64_t n, const uint32_t *keys, int64_t *cp)
{
    const int64_t last = nnz > 0 ? (int64_t)keys[nnz - 1] : -1;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= n;
         c += (int64_t)gridDim.x * blockDim.x)
        if (c > last) cp[c] = nnz;
}

static int grid_for(int64_t work)
{
    int64_t b = (work + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

hipError_t build_transpose(hipStream_t st, Allocator &al, int64_t m, int64_t n, int64_t nnz,
                           const int64_t *rp, const int32_t *ci, const double *val,
                           int64_t *col_ptr, int32_t *row_idx, double *cval, std::string &err)
{
    if (nnz >= ((int64_t)1 << 32)) {
        err = "transpose: nnz must be below 2^32";
        return hipErrorInvalidValue;
    }
    if (nnz == 0) {
        hipLaunchKernelGGL(k_col_ptr_tail, dim3(grid_for(n + 1)), dim3(256), 0, st, nnz, n,
                           (const uint32_t *)nullptr, col_ptr);
        return hipGetLastError();
    }
    const size_t kb = (size_t)nnz * sizeof(uint32_t);
    uint32_t *k0 = (uint32_t *)al.get(kb), *k1 = (uint32_t *)al.get(kb);
    uint32_t *p0 = (uint32_t *)al.get(kb), *p1 = (uint32_t *)al.get(kb);
    int32_t *rowid = (int32_t *)al.get((size_t)nnz * sizeof(int32_t));
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    hipError_t rc = hipSuccess;
    unsigned end_bit = 1;
    while (end_bit < 32 && ((int64_t)1 << end_bit) < n) ++end_bit;
    if (!k0 || !k1 || !p0 || !p1 || !rowid) {
        err = "transpose: allocation failed";
        rc = hipErrorOutOfMemory;
        goto out;
    }
    hipLaunchKernelGGL(k_copy_keys, dim3(grid_for(nnz)), dim3(256), 0, st, nnz, ci, k0, p0);
    hipLaunchKernelGGL(k_row_ids, dim3(grid_for(m * 64)), dim3(256), 0, st, m, rp, rowid);
    {
        rocprim::double_buffer<uint32_t> keys(k0, k1);
        rocprim::double_buffer<uint32_t> vals(p0, p1);
        rc = rocprim::radix_sort_pairs(nullptr, tmp_bytes, keys, vals, (size_t)nnz, 0, end_bit, st);
        if (rc != hipSuccess) { err = "transpose: radix sort sizing failed"; goto out; }
        tmp = al.get(tmp_bytes);
        if (!tmp) { err = "transpose: allocation failed"; rc = hipErrorOutOfMemory; goto out; }
        rc = rocprim::radix_sort_pairs(tmp, tmp_bytes, keys, vals, (size_t)nnz, 0, end_bit, st);
        if (rc != hipSuccess) { err = "transpose: radix sort failed"; goto out; }
        hipLaunchKernelGGL(k_gather_csc, dim3(grid_for(nnz)), dim3(256), 0, st, nnz,
                           vals.current(), rowid, val, row_idx, cval);
        hipLaunchKernelGGL(k_col_ptr, dim3(grid_for(nnz)), dim3(256), 0, st, nnz, n,
                           keys.current(), col_ptr);
        hipLaunchKernelGGL(k_col_ptr_tail, dim3(grid_for(n + 1)), dim3(256), 0, st, nnz, n,
                           keys.current(), col_ptr);
        rc = hipGetLastError();
        if (rc == hipSuccess) rc = hipStreamSynchronize(st);
        if (rc != hipSuccess) err = "transpose: kernel launch failed";
    }
out:
    if (rc != hipSuccess) (void)hipStreamSynchronize(st);
    al.put(tmp, tmp_bytes);
    al.put(k0, kb); al.put(k1, kb); al.put(p0, kb); al.put(p1, kb);
    al.put(rowid, (size_t)nnz * sizeof(int32_t));
    return rc;
}

}  // namespace lsqr
