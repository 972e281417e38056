// Learned column scaling: per-column features, the MLP 6 -> 64 -> 64 -> 1
// (GELU, softplus output) for inference in BF16 (weights and activations
// rounded to nearest-even, FP32 accumulation), and FP32 training kernels
// (forward/backward per sample, per-parameter gradient sums in a fixed order,
// Adam).  The multiplier softplus(z) scales the Jacobi column scale.
#include <math.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "ctx.h"
#include "lsqr_kernels.cuh"

using namespace lsqr;

namespace {

constexpr int H = 64;
constexpr int NF = 6;
// flat parameter layout: W1 [H][NF], b1 [H], W2 [H][H], b2 [H], W3 [H], b3 [1]
constexpr int OW1 = 0, OB1 = OW1 + H * NF, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H,
              OB3 = OW3 + H, NP = OB3 + 1;
static_assert(NP == LSQR_MLP_NPARAMS, "parameter count");

__device__ __forceinline__ float gelu(float x)
{
    return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad(float x)
{
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
           x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

__device__ __forceinline__ float softplus(float z)
{
    return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));
}

__device__ __forceinline__ float sigmoid(float z) { return 0.5f * (1.0f + tanhf(0.5f * z)); }

// FP32 -> BF16 -> FP32, round to nearest even (finite inputs)
__device__ __forceinline__ float bf16r(float x)
{
    uint32_t u = __float_as_uint(x);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return __uint_as_float(u & 0xFFFF0000u);
}

// ----------------------------------------------------------------- features --
__global__ void k_row_centroid(int64_t m, int nz, const int64_t *rp, const int32_t *ci,
                               const double *va, double *cen)
{
    const int lane = threadIdx.x & 63;
    const double zden = nz > 1 ? (double)(nz - 1) : 1.0;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < m;
         i += ((int64_t)gridDim.x * blockDim.x) >> 6) {
        double sa = 0.0, sz = 0.0;
        for (int64_t e = rp[i] + lane; e < rp[i + 1]; e += 64) {
            const double a = fabs(va[e]);
            sa += a;
            sz += a * (double)(ci[e] % nz);
        }
        sa = group_sum<64>(sa);
        sz = group_sum<64>(sz);
        if (lane == 0) cen[i] = sa > 0.0 ? sz / sa / zden : 0.0;
    }
}

__global__ void k_col_features(int n, int nx, int ny, int nz, double w, double damp,
                               const int64_t *cp, const int32_t *ri, const double *cv,
                               const double *cen, float *feat)
{
    const int lane = threadIdx.x & 63;
    const double zden = nz > 1 ? (double)(nz - 1) : 1.0;
    for (int j = (int)((((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6)); j < n;
         j += (int)(((int64_t)gridDim.x * blockDim.x) >> 6)) {
        double g2 = 0.0, ca = 0.0, c1 = 0.0, c2 = 0.0;
        for (int64_t p = cp[j] + lane; p < cp[j + 1]; p += 64) {
            const double g = cv[p], a = fabs(g), c = cen[ri[p]];
            g2 += g * g;
            ca += a;
            c1 += a * c;
            c2 += a * c * c;
        }
        g2 = group_sum<64>(g2);
        ca = group_sum<64>(ca);
        c1 = group_sum<64>(c1);
        c2 = group_sum<64>(c2);
        if (lane == 0) {
            const int iz = j % nz, ixy = j / nz, ix = ixy % nx, iy = ixy / nx;
            const int sxy = nx * nz;
            int deg = 0;
            double nb = 0.0;
            auto hit = [&](int q) { return (double)(cp[q + 1] - cp[q]); };
            if (ix > 0) { nb += hit(j - nz); ++deg; }
            if (ix < nx - 1) { nb += hit(j + nz); ++deg; }
            if (iy > 0) { nb += hit(j - sxy); ++deg; }
            if (iy < ny - 1) { nb += hit(j + sxy); ++deg; }
            if (iz > 0) { nb += hit(j - 1); ++deg; }
            if (iz < nz - 1) { nb += hit(j + 1); ++deg; }
            const double colnorm2 = g2 + w * w * (double)(deg * deg + deg) + damp * damp;
            const double mean = ca > 0.0 ? c1 / ca : 0.0;
            const double var = ca > 0.0 ? c2 / ca - mean * mean : 0.0;
            float *f = feat + (int64_t)j * NF;
            f[0] = (float)(0.5 * log10(colnorm2));
            f[1] = (float)log1p(hit(j));
            f[2] = (float)((double)iz / zden);
            f[3] = (float)mean;
            f[4] = (float)sqrt(var > 0.0 ? var : 0.0);
            f[5] = (float)log1p(deg > 0 ? nb / (double)deg : 0.0);
        }
    }
}

// ---------------------------------------------------------------- inference --
struct Norm {
    float mean[NF], inv_std[NF];
};

// Means over the system's columns of the features flagged in `mask` (FP64,
// one workgroup, fixed order: strided per-thread sums, then a fixed tree).
__global__ __launch_bounds__(256) void k_feature_means(int n, const float *feat, unsigned mask,
                                                       double *out)
{
    __shared__ double acc[NF][256];
    for (int f = 0; f < NF; ++f) {
        double sum = 0.0;
        if ((mask >> f) & 1u)
            for (int j = threadIdx.x; j < n; j += 256) sum += (double)feat[(int64_t)j * NF + f];
        acc[f][threadIdx.x] = sum;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int f = 0; f < NF; ++f) acc[f][threadIdx.x] += acc[f][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < NF) out[threadIdx.x] = n > 0 ? acc[threadIdx.x][0] / (double)n : 0.0;
}

// d_j = djac_j * softplus(z_j), BF16 weights and activations, FP32 sums.
// Features flagged in `mask` are centred on the system's own means (sysmean).
__global__ __launch_bounds__(256) void k_mlp_infer(int n, const float *params, Norm nrm,
                                                   unsigned mask, const double *sysmean,
                                                   const float *feat, const double *djac,
                                                   double *d)
{
    __shared__ float W[NP];
    __shared__ float mu[NF];
    for (int i = threadIdx.x; i < NP; i += blockDim.x) W[i] = bf16r(params[i]);
    if (threadIdx.x < NF)
        mu[threadIdx.x] = ((mask >> threadIdx.x) & 1u) ? (float)sysmean[threadIdx.x]
                                                         : nrm.mean[threadIdx.x];
    __syncthreads();
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        float x[NF];
        for (int f = 0; f < NF; ++f)
            x[f] = bf16r((feat[(int64_t)j * NF + f] - mu[f]) * nrm.inv_std[f]);
        float h1[H];
        for (int k = 0; k < H; ++k) {
            float a = W[OB1 + k];
            for (int f = 0; f < NF; ++f) a = fmaf(W[OW1 + k * NF + f], x[f], a);
            h1[k] = bf16r(gelu(a));
        }
        float z = W[OB3];
        for (int k = 0; k < H; ++k) {
            float a = W[OB2 + k];
            for (int l = 0; l < H; ++l) a = fmaf(W[OW2 + k * H + l], h1[l], a);
            z = fmaf(W[OW3 + k], bf16r(gelu(a)), z);
        }
        d[j] = djac[j] * (double)softplus(z);
    }
}

// ----------------------------------------------------------------- training --
// Per sample (FP32): forward, loss term and the deltas needed for the weight
// gradients.  Stored per sample: h1, h2, d1, d2 [H] and dz; per-workgroup
// partial sums of the squared residual.
__global__ __launch_bounds__(256) void k_mlp_fwd_bwd(int B, const float *params, const float *x,
                                                     const float *target, float *h1o, float *h2o,
                                                     float *d1o, float *d2o, float *dzo,
                                                     double *part)
{
    __shared__ float W[NP];
    __shared__ double lds[4];
    for (int i = threadIdx.x; i < NP; i += blockDim.x) W[i] = params[i];
    __syncthreads();
    double sq = 0.0;
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
        float xv[NF];
        for (int f = 0; f < NF; ++f) xv[f] = x[(int64_t)b * NF + f];
        float a1[H], h1[H];
        for (int k = 0; k < H; ++k) {
            float a = W[OB1 + k];
            for (int f = 0; f < NF; ++f) a = fmaf(W[OW1 + k * NF + f], xv[f], a);
            a1[k] = a;
            h1[k] = gelu(a);
            h1o[(int64_t)b * H + k] = h1[k];
        }
        float a2[H];
        float z = W[OB3];
        for (int k = 0; k < H; ++k) {
            float a = W[OB2 + k];
            for (int l = 0; l < H; ++l) a = fmaf(W[OW2 + k * H + l], h1[l], a);
            a2[k] = a;
            const float h2 = gelu(a);
            h2o[(int64_t)b * H + k] = h2;
            z = fmaf(W[OW3 + k], h2, z);
        }
        const float sp = softplus(z);
        const float r = logf(sp) - target[b];
        sq += (double)r * (double)r;
        const float dz = 2.0f * r / (float)B * sigmoid(z) / sp;
        dzo[b] = dz;
        for (int k = 0; k < H; ++k) {
            a2[k] = dz * W[OW3 + k] * gelu_grad(a2[k]);      // d2
            d2o[(int64_t)b * H + k] = a2[k];
        }
        for (int l = 0; l < H; ++l) {
            float s = 0.0f;
            for (int k = 0; k < H; ++k) s = fmaf(W[OW2 + k * H + l], a2[k], s);
            d1o[(int64_t)b * H + l] = s * gelu_grad(a1[l]);
        }
    }
    const double tot = block_sum(sq, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// One thread per parameter: its gradient as a sum over the batch in sample
// order (FP64 accumulation).
__global__ void k_mlp_wgrad(int B, const float *x, const float *h1, const float *h2,
                            const float *d1, const float *d2, const float *dz, float *grad)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NP) return;
    double s = 0.0;
    if (p < OB1) {
        const int k = p / NF, f = p % NF;
        for (int b = 0; b < B; ++b) s += (double)d1[(int64_t)b * H + k] * (double)x[(int64_t)b * NF + f];
    } else if (p < OW2) {
        const int k = p - OB1;
        for (int b = 0; b < B; ++b) s += (double)d1[(int64_t)b * H + k];
    } else if (p < OB2) {
        const int k = (p - OW2) / H, l = (p - OW2) % H;
        for (int b = 0; b < B; ++b) s += (double)d2[(int64_t)b * H + k] * (double)h1[(int64_t)b * H + l];
    } else if (p < OW3) {
        const int k = p - OB2;
        for (int b = 0; b < B; ++b) s += (double)d2[(int64_t)b * H + k];
    } else if (p < OB3) {
        const int k = p - OW3;
        for (int b = 0; b < B; ++b) s += (double)dz[b] * (double)h2[(int64_t)b * H + k];
    } else {
        for (int b = 0; b < B; ++b) s += (double)dz[b];
    }
    grad[p] = (float)s;
}

__global__ void k_adam(float *params, float *m, float *v, const float *g, float lr, float b1c,
                       float b2c)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NP) return;
    const float gi = g[p];
    const float mi = 0.9f * m[p] + 0.1f * gi;
    const float vi = 0.999f * v[p] + 0.001f * gi * gi;
    m[p] = mi;
    v[p] = vi;
    params[p] -= lr * (mi / b1c) / (sqrtf(vi / b2c) + 1e-8f);
}

}  // namespace

struct lsqr_trainer {
    hipStream_t st = nullptr;
    lsqr::Allocator al;
    int max_batch = 0;
    int t = 0;
    float *params = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    float *h1 = nullptr, *h2 = nullptr, *d1 = nullptr, *d2 = nullptr, *dz = nullptr;
    double *part = nullptr, *sum = nullptr;
    double *hsum = nullptr;
    int grid = 1;
    std::string err;
};

// Device buffers of a trainer and their sizes (bytes), in one place so that
// creation and release agree.
static void trainer_buffers(lsqr_trainer *t, void **(&ptrs)[11], size_t (&bytes)[11])
{
    const size_t B = (size_t)t->max_batch;
    void **p[11] = {(void **)&t->params, (void **)&t->m, (void **)&t->v, (void **)&t->grad,
                    (void **)&t->h1, (void **)&t->h2, (void **)&t->d1, (void **)&t->d2,
                    (void **)&t->dz, (void **)&t->part, (void **)&t->sum};
    const size_t b[11] = {NP * 4, NP * 4, NP * 4, NP * 4, B * H * 4, B * H * 4, B * H * 4,
                          B * H * 4, B * 4, 1024 * 8, 8};
    for (int i = 0; i < 11; ++i) { ptrs[i] = p[i]; bytes[i] = b[i]; }
}

static void trainer_free(lsqr_trainer *t)
{
    void **ptrs[11];
    size_t bytes[11];
    trainer_buffers(t, ptrs, bytes);
    for (int i = 0; i < 11; ++i)
        if (*ptrs[i]) t->al.put(*ptrs[i], bytes[i]);
    if (t->hsum) (void)hipHostFree(t->hsum);
    delete t;
}

// Scratch of lsqr_mlp_scale_noalloc: the Jacobi scale of up to
// LSQR_NOALLOC_MAX_COLS columns followed by the NF feature means.  Host code
// never passes this name to a kernel or a copy: it reads the array's device
// address once per device (hipGetSymbolAddress) and uses that address.
static __device__ __align__(256) double scratch[LSQR_NOALLOC_MAX_COLS + NF];

static std::mutex g_scratch_mu;
static std::vector<double *> g_scratch_ptr;      // per device; null until looked up

static lsqr_status scratch_address(lsqr_ctx *c, double **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    const int dev = c->device;
    if (dev < 0) return fail(c, LSQR_E_DEVICE, "invalid device of the context");
    if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        double *p = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(c, LSQR_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                              hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LSQR_OK;
}

extern "C" {

lsqr_status lsqr_column_features(lsqr_ctx *c, float *feat)
{
    if (!c || !feat) return fail(c, LSQR_E_INVALID_ARG, "ctx and feat must not be NULL");
    DeviceGuard dg(c->device);
    const Problem &P = c->P;
    double *cen = ctx_alloc<double>(c, std::max<int64_t>(P.m, 1));
    if (!cen) return fail(c, LSQR_E_OOM, "device allocation failed");
    const int gr = (int)std::min<int64_t>(std::max<int64_t>((P.m * 64 + 255) / 256, 1), 65536);
    hipLaunchKernelGGL(k_row_centroid, dim3(gr), dim3(256), 0, c->st, P.m, P.nz, c->rp, c->ci,
                       c->va, cen);
    const int gc = (int)std::min<int64_t>(std::max<int64_t>((P.n * 64 + 255) / 256, 1), 65536);
    hipLaunchKernelGGL(k_col_features, dim3(gc), dim3(256), 0, c->st, (int)P.n, P.nx, P.ny, P.nz,
                       P.w, P.damp, c->cp, c->ri, c->cv, cen, feat);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->st));
    ctx_release(c, cen);
    return LSQR_OK;
}

// Inference with the Jacobi scale and the feature means in djac [n + NF].
static lsqr_status mlp_scale_into(lsqr_ctx *c, const float *params, const Norm &nrm,
                                  unsigned centre, const float *feat, double *d, double *djac)
{
    const Problem &P = c->P;
    double *sysmean = djac + P.n;
    launch_jacobi(c->st, P, c->C64, djac);
    hipLaunchKernelGGL(k_feature_means, dim3(1), dim3(256), 0, c->st, (int)P.n, feat, centre,
                       sysmean);
    const int g = (int)std::min<int64_t>((P.n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_mlp_infer, dim3(std::max(g, 1)), dim3(256), 0, c->st, (int)P.n, params,
                       nrm, centre, (const double *)sysmean, feat, (const double *)djac, d);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return LSQR_OK;
}

static lsqr_status mlp_scale_args(lsqr_ctx *c, const float *params, const float *mean,
                                  const float *std, unsigned centre, const float *feat, double *d,
                                  Norm &nrm)
{
    if (!c || !params || !mean || !std || !feat || !d)
        return fail(c, LSQR_E_INVALID_ARG, "arguments must not be NULL");
    if (centre >> NF) return fail(c, LSQR_E_INVALID_ARG, "centre flags only features 0..5");
    for (int f = 0; f < NF; ++f) {
        if (!(std[f] > 0.0f) || !isfinite(std[f]) || !isfinite(mean[f]))
            return fail(c, LSQR_E_INVALID_ARG, "standardisation must be finite with std > 0");
        nrm.mean[f] = mean[f];
        nrm.inv_std[f] = 1.0f / std[f];
    }
    return LSQR_OK;
}

lsqr_status lsqr_mlp_scale(lsqr_ctx *c, const float *params, const float *mean, const float *std,
                           unsigned centre, const float *feat, double *d)
{
    Norm nrm;
    lsqr_status s = mlp_scale_args(c, params, mean, std, centre, feat, d, nrm);
    if (s != LSQR_OK) return s;
    DeviceGuard dg(c->device);
    double *djac = ctx_alloc<double>(c, c->P.n + NF);
    if (!djac) return fail(c, LSQR_E_OOM, "device allocation failed");
    s = mlp_scale_into(c, params, nrm, centre, feat, d, djac);
    ctx_release(c, djac);
    return s;
}

lsqr_status lsqr_mlp_scale_noalloc(lsqr_ctx *c, const float *params, const float *mean,
                                   const float *std, unsigned centre, const float *feat, double *d)
{
    Norm nrm;
    lsqr_status s = mlp_scale_args(c, params, mean, std, centre, feat, d, nrm);
    if (s != LSQR_OK) return s;
    if (c->P.n > LSQR_NOALLOC_MAX_COLS)
        return fail(c, LSQR_E_INVALID_ARG,
                    "lsqr_mlp_scale_noalloc: n = " + std::to_string(c->P.n) +
                        " columns exceeds the static scratch of " +
                        std::to_string((long long)LSQR_NOALLOC_MAX_COLS) +
                        " (use lsqr_mlp_scale)");
    DeviceGuard dg(c->device);
    double *djac = nullptr;
    s = scratch_address(c, &djac);
    if (s != LSQR_OK) return s;
    // every element the kernels read is written first in the same call (the
    // Jacobi scale of all n columns, then the NF means): nothing to clear
    return mlp_scale_into(c, params, nrm, centre, feat, d, djac);
}

static thread_local std::string t_err;

lsqr_status lsqr_trainer_create(int max_batch, const float *params, void *stream,
                                lsqr_alloc_fn alloc, lsqr_free_fn dealloc, void *alloc_user,
                                lsqr_trainer **out)
{
    if (!out || !params || max_batch < 1) {
        t_err = "invalid arguments";
        return LSQR_E_INVALID_ARG;
    }
    *out = nullptr;
    lsqr_trainer *t = new lsqr_trainer();
    t->st = (hipStream_t)stream;
    t->al.alloc = alloc;
    t->al.dealloc = dealloc;
    t->al.user = alloc_user;
    t->max_batch = max_batch;
    t->grid = std::min(1024, (max_batch + 255) / 256);
    void **ptrs[11];
    size_t bytes[11];
    trainer_buffers(t, ptrs, bytes);
    bool ok = true;
    for (int i = 0; i < 11 && ok; ++i) ok = (*ptrs[i] = t->al.get(bytes[i])) != nullptr;
    ok = ok && hipHostMalloc((void **)&t->hsum, 8, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        trainer_free(t);
        t_err = "device allocation failed";
        return LSQR_E_OOM;
    }
    if (hipMemcpy(t->params, params, NP * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(t->m, 0, NP * 4) != hipSuccess || hipMemset(t->v, 0, NP * 4) != hipSuccess) {
        trainer_free(t);
        t_err = "device copy failed";
        return LSQR_E_DEVICE;
    }
    *out = t;
    return LSQR_OK;
}

static lsqr_status trainer_grad(lsqr_trainer *t, int batch, const float *x, const float *target,
                                double *loss)
{
    hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3(t->grid), dim3(256), 0, t->st, batch, t->params, x,
                       target, t->h1, t->h2, t->d1, t->d2, t->dz, t->part);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((NP + 255) / 256), dim3(256), 0, t->st, batch, x, t->h1,
                       t->h2, t->d1, t->d2, t->dz, t->grad);
    if (loss) {
        launch_sum_partials(t->st, t->part, t->grid, t->sum);
        if (hipMemcpyAsync(t->hsum, t->sum, 8, hipMemcpyDeviceToHost, t->st) != hipSuccess ||
            hipStreamSynchronize(t->st) != hipSuccess) {
            t->err = "device copy failed";
            return LSQR_E_DEVICE;
        }
        *loss = t->hsum[0] / (double)batch;
    }
    if (hipGetLastError() != hipSuccess) {
        t->err = "kernel launch failed";
        return LSQR_E_DEVICE;
    }
    return LSQR_OK;
}

lsqr_status lsqr_trainer_grad(lsqr_trainer *t, int batch, const float *x, const float *target,
                              float *grad, double *loss)
{
    if (!t || !x || !target || batch < 1 || batch > t->max_batch) return LSQR_E_INVALID_ARG;
    lsqr_status s = trainer_grad(t, batch, x, target, loss);
    if (s != LSQR_OK) return s;
    if (grad && hipMemcpyAsync(grad, t->grad, NP * 4, hipMemcpyDeviceToDevice, t->st) != hipSuccess)
        return LSQR_E_DEVICE;
    return hipStreamSynchronize(t->st) == hipSuccess ? LSQR_OK : LSQR_E_DEVICE;
}

lsqr_status lsqr_trainer_step(lsqr_trainer *t, int batch, const float *x, const float *target,
                              float lr, double *loss)
{
    if (!t || !x || !target || batch < 1 || batch > t->max_batch || !(lr > 0.0f)) return LSQR_E_INVALID_ARG;
    lsqr_status s = trainer_grad(t, batch, x, target, loss);
    if (s != LSQR_OK) return s;
    t->t += 1;
    const float b1c = 1.0f - powf(0.9f, (float)t->t), b2c = 1.0f - powf(0.999f, (float)t->t);
    hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, t->st, t->params, t->m, t->v,
                       t->grad, lr, b1c, b2c);
    return hipGetLastError() == hipSuccess ? LSQR_OK : LSQR_E_DEVICE;
}

lsqr_status lsqr_trainer_params(const lsqr_trainer *t, float *params, float *params_device)
{
    if (!t || (!params && !params_device)) return LSQR_E_INVALID_ARG;
    if (params && hipMemcpyAsync(params, t->params, NP * 4, hipMemcpyDeviceToHost, t->st) != hipSuccess)
        return LSQR_E_DEVICE;
    if (params_device &&
        hipMemcpyAsync(params_device, t->params, NP * 4, hipMemcpyDeviceToDevice, t->st) != hipSuccess)
        return LSQR_E_DEVICE;
    return hipStreamSynchronize(t->st) == hipSuccess ? LSQR_OK : LSQR_E_DEVICE;
}

void lsqr_trainer_destroy(lsqr_trainer *t)
{
    if (!t) return;
    if (t->st) (void)hipStreamSynchronize(t->st);
    trainer_free(t);
}

}  // extern "C"
