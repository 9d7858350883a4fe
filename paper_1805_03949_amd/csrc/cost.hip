// Learned cost model of a work item: a 12 -> 64 -> 64 -> 1 ReLU perceptron in
// FP32 with hand-written forward, backward and Adam kernels.
//
// The paper observes that the computational weight of an element cannot be
// estimated a priori and that the number of Gauss points, used as the METIS
// weight, balances poorly (abstract; Section 4.1, Figures lb_resp/lb_iter).
// The batched assembly records the cycles every work item takes; this model
// learns log(cycles) from item features and orders the work queue.
//
// Layouts: parameters W1[64][12], b1[64], W2[64][64], b2[64], W3[64], b3;
// features row-major [n][12]; activations row-major [n][64].
// Gradients are reduced in a fixed order (per chunk of 64 samples in
// ascending order, then chunks in ascending order), so training is
// deterministic.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "fea_internal.h"

namespace fea {

constexpr int NI = 12, NH = 64;
constexpr int OW1 = 0, OB1 = OW1 + NH * NI, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH, NPAR = OB3 + 1;
static_assert(NPAR == FEA_COST_PARAMS, "parameter count");
constexpr int CHUNK = 64;

// Forward pass, one thread per sample; parameters staged in LDS. When
// h1/h2/z are given the activations are stored for the backward pass.
__global__ void __launch_bounds__(256) k_mlp_forward(const float *P, const float *mean, const float *scale,
                                                     const float *X, int64_t n, float *y, float *z_out,
                                                     float *h1_out, float *h2_out)
{
    __shared__ float sP[NPAR];
    __shared__ float sM[NI], sS[NI];
    for (int i = threadIdx.x; i < NPAR; i += 256) sP[i] = P[i];
    if (threadIdx.x < NI) {
        sM[threadIdx.x] = mean[threadIdx.x];
        sS[threadIdx.x] = scale[threadIdx.x];
    }
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    float z[NI], h1[NH];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        z[k] = (X[s * NI + k] - sM[k]) / sS[k];
        if (z_out) z_out[s * NI + k] = z[k];
    }
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        float a = sP[OB1 + j];
#pragma unroll
        for (int k = 0; k < NI; ++k) a += sP[OW1 + j * NI + k] * z[k];
        h1[j] = a > 0.f ? a : 0.f;
        if (h1_out) h1_out[s * NH + j] = h1[j];
    }
    float out = sP[OB3];
    for (int i = 0; i < NH; ++i) {
        float a = sP[OB2 + i];
#pragma unroll
        for (int j = 0; j < NH; ++j) a += sP[OW2 + i * NH + j] * h1[j];
        const float h = a > 0.f ? a : 0.f;
        if (h2_out) h2_out[s * NH + i] = h;
        out += sP[OW3 + i] * h;
    }
    y[s] = out;
}

// Backward pass per sample: dy = 2 (y - t) / n, da2 = dy W3 (.) [h2 > 0],
// da1 = (W2^T da2) (.) [h1 > 0]. Also the squared residual for the loss.
__global__ void __launch_bounds__(256) k_mlp_backward(const float *P, const float *y, const float *t,
                                                      int64_t n, const float *h1, const float *h2,
                                                      float *dy_out, float *da1_out, float *da2_out,
                                                      float *r2_out)
{
    __shared__ float sW2[NH * NH];
    __shared__ float sW3[NH];
    for (int i = threadIdx.x; i < NH * NH; i += 256) sW2[i] = P[OW2 + i];
    if (threadIdx.x < NH) sW3[threadIdx.x] = P[OW3 + threadIdx.x];
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const float r = y[s] - t[s];
    const float dy = 2.f * r / (float)n;
    dy_out[s] = dy;
    r2_out[s] = r * r;
    float da2[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        da2[i] = h2[s * NH + i] > 0.f ? dy * sW3[i] : 0.f;
        da2_out[s * NH + i] = da2[i];
    }
    for (int j = 0; j < NH; ++j) {
        float a = 0.f;
#pragma unroll
        for (int i = 0; i < NH; ++i) a += sW2[i * NH + j] * da2[i];
        da1_out[s * NH + j] = h1[s * NH + j] > 0.f ? a : 0.f;
    }
}

// Partial gradients of one chunk of CHUNK samples, summed in sample order.
// part[c][p] for every parameter p; part[c][NPAR] = sum of squared residuals.
__global__ void __launch_bounds__(256) k_mlp_grad_chunk(const float *z, const float *h1, const float *h2,
                                                        const float *dy, const float *da1,
                                                        const float *da2, const float *r2, int64_t n,
                                                        float *part)
{
    __shared__ float sz[CHUNK][NI], sh1[CHUNK][NH], sh2[CHUNK][NH], sd1[CHUNK][NH], sd2[CHUNK][NH];
    __shared__ float sdy[CHUNK], sr2[CHUNK];
    const int64_t s0 = (int64_t)blockIdx.x * CHUNK;
    const int cn = (int)std::min<int64_t>(CHUNK, n - s0);
    for (int i = threadIdx.x; i < cn * NH; i += 256) {
        const int s = i / NH, j = i % NH;
        sh1[s][j] = h1[(s0 + s) * NH + j];
        sh2[s][j] = h2[(s0 + s) * NH + j];
        sd1[s][j] = da1[(s0 + s) * NH + j];
        sd2[s][j] = da2[(s0 + s) * NH + j];
    }
    for (int i = threadIdx.x; i < cn * NI; i += 256) sz[i / NI][i % NI] = z[(s0 + i / NI) * NI + i % NI];
    for (int i = threadIdx.x; i < cn; i += 256) {
        sdy[i] = dy[s0 + i];
        sr2[i] = r2[s0 + i];
    }
    __syncthreads();
    float *out = part + (int64_t)blockIdx.x * (NPAR + 1);
    for (int p = threadIdx.x; p <= NPAR; p += 256) {
        float acc = 0.f;
        if (p < OB1) {
            const int j = (p - OW1) / NI, k = (p - OW1) % NI;
            for (int s = 0; s < cn; ++s) acc += sd1[s][j] * sz[s][k];
        } else if (p < OW2) {
            const int j = p - OB1;
            for (int s = 0; s < cn; ++s) acc += sd1[s][j];
        } else if (p < OB2) {
            const int i = (p - OW2) / NH, j = (p - OW2) % NH;
            for (int s = 0; s < cn; ++s) acc += sd2[s][i] * sh1[s][j];
        } else if (p < OW3) {
            const int i = p - OB2;
            for (int s = 0; s < cn; ++s) acc += sd2[s][i];
        } else if (p < OB3) {
            const int i = p - OW3;
            for (int s = 0; s < cn; ++s) acc += sdy[s] * sh2[s][i];
        } else if (p == OB3) {
            for (int s = 0; s < cn; ++s) acc += sdy[s];
        } else {
            for (int s = 0; s < cn; ++s) acc += sr2[s];
        }
        out[p] = acc;
    }
}

// Sum of the chunk partials in chunk order; loss = sum r^2 / n.
__global__ void k_mlp_grad_final(const float *part, int64_t nchunks, int64_t n, float *grad, float *loss)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p > NPAR) return;
    float acc = 0.f;
    for (int64_t c = 0; c < nchunks; ++c) acc += part[c * (NPAR + 1) + p];
    if (p < NPAR) {
        if (grad) grad[p] = acc;
    } else if (loss) {
        *loss = acc / (float)n;
    }
}

__global__ void k_adam(float *P, float *m, float *v, const float *g, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= NPAR) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.f - b1) * gp;
    const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    P[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

// Per-feature mean and population standard deviation, one workgroup per
// feature, fixed reduction order.
__global__ void __launch_bounds__(256) k_norm(const float *X, int64_t n, float *mean, float *scale)
{
    __shared__ double s1[256], s2[256];
    const int k = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t s = threadIdx.x; s < n; s += 256) {
        const double x = X[s * NI + k];
        a += x;
        b += x * x;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s1[threadIdx.x] += s1[threadIdx.x + off];
            s2[threadIdx.x] += s2[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mu = s1[0] / (double)n;
        const double var = std::max(0.0, s2[0] / (double)n - mu * mu);
        const double sd = sqrt(var);
        mean[k] = (float)mu;
        scale[k] = sd > 1e-12 ? (float)sd : 1.f;
    }
}

__global__ void k_log_cycles(const uint64_t *c, int64_t n, float *t)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) t[i] = logf((float)(c[i] > 0 ? c[i] : 1));
}

}  // namespace fea

using namespace fea;

struct fea_cost {
    int device = 0;
    float *P = nullptr, *m = nullptr, *v = nullptr, *g = nullptr, *mean = nullptr, *scale = nullptr;
    float *loss = nullptr;
    int64_t step = 0;
    // activations workspace
    float *ws = nullptr;
    int64_t ws_n = 0;
};

namespace {

uint64_t splitmix(uint64_t &x)
{
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// standard normal by Box-Muller from a SplitMix64 stream
double normal(uint64_t &x)
{
    const double u1 = ((splitmix(x) >> 11) + 1.0) * 0x1.0p-53;
    const double u2 = (splitmix(x) >> 11) * 0x1.0p-53;
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

void destroy_cost(fea_cost *c)
{
    if (!c) return;
    void *bufs[] = {c->P, c->m, c->v, c->g, c->mean, c->scale, c->loss, c->ws};
    for (void *p : bufs) dfree(p);
    delete c;
}

// workspace: z[n][12], h1, h2, da1, da2 [n][64], y, dy, r2 [n], partials
int ensure_ws(fea_cost *c, int64_t n)
{
    if (c->ws && c->ws_n >= n) return FEA_OK;
    dfree(c->ws);
    c->ws = nullptr;
    c->ws_n = 0;
    const int64_t nch = (n + CHUNK - 1) / CHUNK;
    const size_t floats = (size_t)n * (NI + 4 * NH + 3) + (size_t)nch * (NPAR + 1);
    int rc = dalloc((void **)&c->ws, sizeof(float) * std::max<size_t>(floats, 1));
    if (rc) return rc;
    c->ws_n = n;
    return FEA_OK;
}

struct Ws {
    float *z, *h1, *h2, *da1, *da2, *y, *dy, *r2, *part;
};

Ws carve(const fea_cost *c, int64_t n)
{
    Ws w;
    float *p = c->ws;
    w.z = p; p += n * NI;
    w.h1 = p; p += n * NH;
    w.h2 = p; p += n * NH;
    w.da1 = p; p += n * NH;
    w.da2 = p; p += n * NH;
    w.y = p; p += n;
    w.dy = p; p += n;
    w.r2 = p; p += n;
    w.part = p;
    return w;
}

int grad_impl(const fea_cost *c, const float *X, const float *t, int64_t n, float *grad, float *loss,
              hipStream_t s)
{
    Ws w = carve(c, n);
    const unsigned nb = grid_for(n, 256);
    k_mlp_forward<<<nb, 256, 0, s>>>(c->P, c->mean, c->scale, X, n, w.y, w.z, w.h1, w.h2);
    k_mlp_backward<<<nb, 256, 0, s>>>(c->P, w.y, t, n, w.h1, w.h2, w.dy, w.da1, w.da2, w.r2);
    const int64_t nch = (n + CHUNK - 1) / CHUNK;
    k_mlp_grad_chunk<<<(unsigned)nch, 256, 0, s>>>(w.z, w.h1, w.h2, w.dy, w.da1, w.da2, w.r2, n, w.part);
    k_mlp_grad_final<<<grid_for(NPAR + 1, 256), 256, 0, s>>>(w.part, nch, n, grad, loss);
    FEA_HIP(hipGetLastError());
    return FEA_OK;
}

int check(const fea_cost *c)
{
    if (!c) return set_error(FEA_EINVAL, "cost model is NULL");
    int dev = 0;
    FEA_HIP(hipGetDevice(&dev));
    if (dev != c->device) return set_error(FEA_EINVAL, "cost model lives on device %d", c->device);
    return FEA_OK;
}

const char kMagic[8] = {'F', 'E', 'A', 'C', 'O', 'S', 'T', '1'};
const char kArch[8] = {'g', 'f', 'x', '9', '5', '0', 0, 0};
const uint32_t kVersion = 1;

}  // namespace

extern "C" int fea_cost_create(uint64_t seed, fea_cost **out)
{
    clear_error();
    if (!out) return set_error(FEA_EINVAL, "out is NULL");
    *out = nullptr;
    fea_cost *c = new (std::nothrow) fea_cost();
    if (!c) return set_error(FEA_ENOMEM, "host allocation failed");
    int rc = 0;
    (void)hipGetDevice(&c->device);
    float **bufs[] = {&c->P, &c->m, &c->v, &c->g};
    for (float **b : bufs)
        if (!rc) rc = dalloc((void **)b, sizeof(float) * NPAR);
    if (!rc) rc = dalloc((void **)&c->mean, sizeof(float) * NI);
    if (!rc) rc = dalloc((void **)&c->scale, sizeof(float) * NI);
    if (!rc) rc = dalloc((void **)&c->loss, sizeof(float));
    if (rc) {
        destroy_cost(c);
        return rc;
    }
    std::vector<float> P(NPAR, 0.f), zero(NPAR, 0.f), mean(NI, 0.f), scale(NI, 1.f);
    uint64_t st = seed;
    for (int i = 0; i < NH * NI; ++i) P[OW1 + i] = (float)(normal(st) * sqrt(2.0 / NI));
    for (int i = 0; i < NH * NH; ++i) P[OW2 + i] = (float)(normal(st) * sqrt(2.0 / NH));
    for (int i = 0; i < NH; ++i) P[OW3 + i] = (float)(normal(st) * sqrt(2.0 / NH));
    hipError_t e = hipMemcpy(c->P, P.data(), sizeof(float) * NPAR, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->m, zero.data(), sizeof(float) * NPAR, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->v, zero.data(), sizeof(float) * NPAR, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->mean, mean.data(), sizeof(float) * NI, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->scale, scale.data(), sizeof(float) * NI, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        destroy_cost(c);
        return set_error(FEA_EHIP, "upload failed: %s", hipGetErrorString(e));
    }
    *out = c;
    return FEA_OK;
}

extern "C" void fea_cost_destroy(fea_cost *c) { destroy_cost(c); }

extern "C" int fea_cost_get_params(const fea_cost *c, float *params)
{
    clear_error();
    if (!c || !params) return set_error(FEA_EINVAL, "cost model and params are required");
    FEA_HIP(hipMemcpy(params, c->P, sizeof(float) * NPAR, hipMemcpyDeviceToHost));
    return FEA_OK;
}

extern "C" int fea_cost_set_params(fea_cost *c, const float *params)
{
    clear_error();
    if (!c || !params) return set_error(FEA_EINVAL, "cost model and params are required");
    FEA_HIP(hipMemcpy(c->P, params, sizeof(float) * NPAR, hipMemcpyHostToDevice));
    return FEA_OK;
}

extern "C" int fea_cost_set_norm(fea_cost *c, const float *mean, const float *scale)
{
    clear_error();
    if (!c || !mean || !scale) return set_error(FEA_EINVAL, "cost model, mean and scale are required");
    for (int k = 0; k < NI; ++k)
        if (!(scale[k] > 0.f)) return set_error(FEA_EINVAL, "scale[%d] must be positive", k);
    FEA_HIP(hipMemcpy(c->mean, mean, sizeof(float) * NI, hipMemcpyHostToDevice));
    FEA_HIP(hipMemcpy(c->scale, scale, sizeof(float) * NI, hipMemcpyHostToDevice));
    return FEA_OK;
}

extern "C" int fea_cost_fit_norm(fea_cost *c, const float *feats, int64_t n, hipStream_t s)
{
    clear_error();
    int rc = check(c);
    if (rc) return rc;
    if (n <= 0 || !feats) return set_error(FEA_EINVAL, "need features");
    k_norm<<<NI, 256, 0, s>>>(feats, n, c->mean, c->scale);
    FEA_HIP(hipGetLastError());
    return FEA_OK;
}

extern "C" int fea_cost_predict(const fea_cost *c, const float *feats, int64_t n, float *pred, hipStream_t s)
{
    clear_error();
    int rc = check(c);
    if (rc) return rc;
    if (n < 0 || (n > 0 && (!feats || !pred))) return set_error(FEA_EINVAL, "bad arguments");
    if (n) k_mlp_forward<<<grid_for(n, 256), 256, 0, s>>>(c->P, c->mean, c->scale, feats, n, pred, nullptr, nullptr, nullptr);
    FEA_HIP(hipGetLastError());
    return FEA_OK;
}

extern "C" int fea_cost_grad(const fea_cost *c, const float *feats, const float *target, int64_t n,
                             float *grad, float *loss, hipStream_t s)
{
    clear_error();
    int rc = check(c);
    if (rc) return rc;
    if (n <= 0 || !feats || !target) return set_error(FEA_EINVAL, "bad arguments");
    if ((rc = ensure_ws(const_cast<fea_cost *>(c), n))) return rc;
    return grad_impl(c, feats, target, n, grad, loss, s);
}

extern "C" int fea_cost_train(fea_cost *c, const float *feats, const float *target, int64_t n, int steps,
                              float lr, float *loss_hist, hipStream_t s)
{
    clear_error();
    int rc = check(c);
    if (rc) return rc;
    if (n <= 0 || steps < 0 || !feats || !target || !(lr > 0.f)) return set_error(FEA_EINVAL, "bad arguments");
    if ((rc = ensure_ws(c, n))) return rc;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int k = 0; k < steps; ++k) {
        if ((rc = grad_impl(c, feats, target, n, c->g, loss_hist ? loss_hist + k : c->loss, s))) return rc;
        c->step += 1;
        const float c1 = 1.f - powf(b1, (float)c->step), c2 = 1.f - powf(b2, (float)c->step);
        k_adam<<<grid_for(NPAR, 256), 256, 0, s>>>(c->P, c->m, c->v, c->g, lr, b1, b2, eps, c1, c2);
    }
    FEA_HIP(hipGetLastError());
    return FEA_OK;
}

extern "C" int fea_cost_log_cycles(const uint64_t *cycles, int64_t n, float *target, hipStream_t s)
{
    clear_error();
    if (n < 0 || (n > 0 && (!cycles || !target))) return set_error(FEA_EINVAL, "bad arguments");
    if (n) k_log_cycles<<<grid_for(n, 256), 256, 0, s>>>(cycles, n, target);
    FEA_HIP(hipGetLastError());
    return FEA_OK;
}

extern "C" int fea_cost_save(const fea_cost *c, const char *path)
{
    clear_error();
    if (!c || !path) return set_error(FEA_EINVAL, "cost model and path are required");
    std::vector<float> P(NPAR), m(NPAR), v(NPAR), mean(NI), scale(NI);
    FEA_HIP(hipDeviceSynchronize());
    FEA_HIP(hipMemcpy(P.data(), c->P, sizeof(float) * NPAR, hipMemcpyDeviceToHost));
    FEA_HIP(hipMemcpy(m.data(), c->m, sizeof(float) * NPAR, hipMemcpyDeviceToHost));
    FEA_HIP(hipMemcpy(v.data(), c->v, sizeof(float) * NPAR, hipMemcpyDeviceToHost));
    FEA_HIP(hipMemcpy(mean.data(), c->mean, sizeof(float) * NI, hipMemcpyDeviceToHost));
    FEA_HIP(hipMemcpy(scale.data(), c->scale, sizeof(float) * NI, hipMemcpyDeviceToHost));
    FILE *f = fopen(path, "wb");
    if (!f) return set_error(FEA_EINVAL, "cannot write %s", path);
    bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(&kVersion, 4, 1, f) == 1 && fwrite(kArch, 1, 8, f) == 8 &&
              fwrite(mean.data(), 4, NI, f) == NI && fwrite(scale.data(), 4, NI, f) == NI &&
              fwrite(P.data(), 4, NPAR, f) == NPAR && fwrite(m.data(), 4, NPAR, f) == NPAR &&
              fwrite(v.data(), 4, NPAR, f) == NPAR && fwrite(&c->step, 8, 1, f) == 1;
    fclose(f);
    if (!ok) return set_error(FEA_EINVAL, "short write to %s", path);
    return FEA_OK;
}

extern "C" int fea_cost_load(fea_cost *c, const char *path)
{
    clear_error();
    if (!c || !path) return set_error(FEA_EINVAL, "cost model and path are required");
    FILE *f = fopen(path, "rb");
    if (!f) return set_error(FEA_EINVAL, "cannot read %s", path);
    char magic[8], arch[8];
    uint32_t ver = 0;
    std::vector<float> P(NPAR), m(NPAR), v(NPAR), mean(NI), scale(NI);
    int64_t step = 0;
    bool ok = fread(magic, 1, 8, f) == 8 && fread(&ver, 4, 1, f) == 1 && fread(arch, 1, 8, f) == 8 &&
              fread(mean.data(), 4, NI, f) == NI && fread(scale.data(), 4, NI, f) == NI &&
              fread(P.data(), 4, NPAR, f) == NPAR && fread(m.data(), 4, NPAR, f) == NPAR &&
              fread(v.data(), 4, NPAR, f) == NPAR && fread(&step, 8, 1, f) == 1;
    fclose(f);
    if (!ok || memcmp(magic, kMagic, 8) != 0 || ver != kVersion || memcmp(arch, kArch, 8) != 0)
        return set_error(FEA_EINVAL, "%s is not a cost-model checkpoint of this version", path);
    FEA_HIP(hipMemcpy(c->P, P.data(), sizeof(float) * NPAR, hipMemcpyHostToDevice));
    FEA_HIP(hipMemcpy(c->m, m.data(), sizeof(float) * NPAR, hipMemcpyHostToDevice));
    FEA_HIP(hipMemcpy(c->v, v.data(), sizeof(float) * NPAR, hipMemcpyHostToDevice));
    FEA_HIP(hipMemcpy(c->mean, mean.data(), sizeof(float) * NI, hipMemcpyHostToDevice));
    FEA_HIP(hipMemcpy(c->scale, scale.data(), sizeof(float) * NI, hipMemcpyHostToDevice));
    c->step = step;
    return FEA_OK;
}
