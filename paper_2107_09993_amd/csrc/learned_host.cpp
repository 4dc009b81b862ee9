// C ABI of the learned pivot proposer: network handles, training, scoring,
// top-k pivot selection and the pivoted skyline calls.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/skycell.h"
#include "common.h"
#include "host_internal.h"
#include "mlp.h"

#define fail skycell::set_error
#define ok skycell::clear_error

struct skycell_mlp {
    int device = -1;
    int d = 0;
    int g = 0;
    uint32_t count = 0;
    int step = 0;
    float grad_scale = 0.0f;
    void *mem = nullptr;      // one allocation: master, m1, m2, grad, loss, bfloat16 copy
    float *master = nullptr, *m1 = nullptr, *m2 = nullptr, *grad = nullptr, *loss = nullptr;
    skycell::MlpDevice net{};
};

namespace skycell {

static size_t aligned(size_t v) { return (v + 255) & ~(size_t)255; }

static int mlp_alloc(int d, int g, skycell_mlp **out)
{
    skycell_mlp *m = new skycell_mlp;
    m->d = d;
    m->g = g;
    m->count = mlp_num_params(d);
    const size_t vec = aligned((size_t)m->count * 4);
    const size_t bytes = 4 * vec + 256 + kMlpDeviceBytes;
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        return fail(SKYCELL_E_NODEV, "no current HIP device");
    }
    if (hipMalloc(&m->mem, bytes) != hipSuccess) {
        delete m;
        return fail(SKYCELL_E_NOMEM, "hipMalloc of %zu bytes for the network failed", bytes);
    }
    char *p = (char *)m->mem;
    m->master = (float *)p;
    m->m1 = (float *)(p + vec);
    m->m2 = (float *)(p + 2 * vec);
    m->grad = (float *)(p + 3 * vec);
    m->loss = (float *)(p + 4 * vec);
    m->net = mlp_device_view(p + 4 * vec + 256);
    if (hipMemset(m->mem, 0, bytes) != hipSuccess) {
        (void)hipFree(m->mem);
        delete m;
        return fail(SKYCELL_E_HIP, "hipMemset of the network failed");
    }
    *out = m;
    return SKYCELL_OK;
}

static int check_handle(const skycell_mlp *m)
{
    if (m == nullptr) return fail(SKYCELL_E_INVAL, "network handle is NULL");
    int dev = -1;
    SKYCELL_HIP_CHECK(hipGetDevice(&dev));
    if (dev != m->device)
        return fail(SKYCELL_E_INVAL, "the network lives on device %d, device %d is current", m->device, dev);
    return SKYCELL_OK;
}

static int check_points(const float *points, int64_t ld, int64_t n)
{
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(SKYCELL_E_INVAL, "n = %lld out of range", (long long)n);
    if (ld < n) return fail(SKYCELL_E_INVAL, "ld = %lld is below n = %lld", (long long)ld, (long long)n);
    if (n > 0 && points == nullptr) return fail(SKYCELL_E_INVAL, "points is NULL");
    return SKYCELL_OK;
}

// SplitMix64 (Steele, Lea and Flood, 2014) of seed + i, as a uniform in [0, 1).
static double splitmix_uniform(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static std::vector<float> glorot_init(int d, uint64_t seed)
{
    std::vector<float> p(mlp_num_params(d), 0.0f);
    const int F = 2 * d;
    auto fill = [&](uint32_t off, uint32_t count, int fan_in, int fan_out) {
        const double a = std::sqrt(6.0 / (double)(fan_in + fan_out));
        for (uint32_t i = 0; i < count; ++i) p[off + i] = (float)((2.0 * splitmix_uniform(seed, off + i) - 1.0) * a);
    };
    fill(mlp_off_w1(), kMlpHidden * F, F, kMlpHidden);
    fill(mlp_off_w2(d), kMlpHidden * kMlpHidden, kMlpHidden, kMlpHidden);
    fill(mlp_off_w3(d), kMlpHidden, kMlpHidden, 1);
    return p;
}

static int upload_params(skycell_mlp *m, const float *host)
{
    SKYCELL_HIP_CHECK(hipMemcpy(m->master, host, (size_t)m->count * 4, hipMemcpyHostToDevice));
    SKYCELL_HIP_CHECK(hipMemset(m->m1, 0, (size_t)m->count * 4));
    SKYCELL_HIP_CHECK(hipMemset(m->m2, 0, (size_t)m->count * 4));
    m->step = 0;
    SKYCELL_HIP_CHECK(launch_mlp_pack(m->master, m->count, m->d, m->net, nullptr));
    SKYCELL_HIP_CHECK(hipDeviceSynchronize());
    return SKYCELL_OK;
}

static int backward(skycell_mlp *m, const float *points, int64_t ld, const uint8_t *labels, int64_t n,
                    float *loss_out, hipStream_t st)
{
    SKYCELL_HIP_CHECK(launch_mlp_backward(points, ld, (uint32_t)n, m->d, m->g, m->net, labels, m->grad, m->loss,
                                          m->count, device_cus(m->device), st));
    m->grad_scale = n > 0 ? (float)(1.0 / (double)n) : 0.0f;
    if (loss_out != nullptr) SKYCELL_HIP_CHECK(launch_mlp_mean_loss(m->loss, m->grad_scale, loss_out, st));
    return SKYCELL_OK;
}

static int adam(skycell_mlp *m, float lr, hipStream_t st)
{
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return fail(SKYCELL_E_INVAL, "learning rate %g is not a finite value >= 0", lr);
    m->step += 1;
    AdamArgs a;
    a.lr = lr;
    a.beta1 = 0.9f;
    a.beta2 = 0.999f;
    a.eps = 1e-8f;
    a.corr1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)m->step)));
    a.corr2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)m->step)));
    a.grad_scale = m->grad_scale;
    SKYCELL_HIP_CHECK(launch_mlp_adam(m->master, m->m1, m->m2, m->grad, m->count, m->d, m->net, a, st));
    return SKYCELL_OK;
}

// Pivot scratch (and, for the scored path, a logits buffer of n floats) from
// the library's per-(device, stream) cache.
static int pivot_scratch(int dev, hipStream_t st, int64_t n_logits, PivotScratch *ps, float **logits)
{
    const size_t base = pivot_scratch_layout(nullptr, nullptr);
    void *ptr = nullptr;
    int rc = cached_buffer(kCachePivots, dev, st, base + aligned((size_t)n_logits * 4 + 4), &ptr);
    if (rc != SKYCELL_OK) return rc;
    pivot_scratch_layout(ps, (char *)ptr);
    if (logits) *logits = (float *)((char *)ptr + base);
    return SKYCELL_OK;
}

// skycell_compute with pivots: `scored` picks them with the network first.
static int compute_with(const float *points, int64_t n, int32_t d, int32_t grid_res, const int32_t *pivot_idx,
                        int32_t k, skycell_mlp *mlp, int32_t *out_idx, int32_t *out_count, uint64_t *stats,
                        hipStream_t st)
{
    int rc = validate(points, SKYCELL_DTYPE_F32, n, d, grid_res, 16, out_idx, out_count);
    if (rc != SKYCELL_OK) return rc;
    if (k < 0 || k > kMaxPivots) return fail(SKYCELL_E_INVAL, "k = %d is outside [0, %d]", k, kMaxPivots);
    if (mlp == nullptr && k > 0 && pivot_idx == nullptr) return fail(SKYCELL_E_INVAL, "pivot_idx is NULL");
    if (mlp != nullptr) {
        if ((rc = check_handle(mlp)) != SKYCELL_OK) return rc;
        if (mlp->d != d) return fail(SKYCELL_E_INVAL, "the network takes d = %d, the points have d = %d", mlp->d, d);
    }
    int g = 0;
    if ((rc = resolve_grid(n, d, SKYCELL_DTYPE_F32, grid_res, &g)) != SKYCELL_OK) return rc;
    if (n == 0) {
        SKYCELL_HIP_CHECK(launch_write_zero_count(out_count, st));
        return ok();
    }
    int dev = 0;
    SKYCELL_HIP_CHECK(hipGetDevice(&dev));
    const uint32_t kk = (uint32_t)(k < n ? k : n);
    PivotArgs piv;
    piv.k = kk;
    float *logits = nullptr;
    if ((rc = pivot_scratch(dev, st, mlp ? n : 0, &piv.ps, &logits)) != SKYCELL_OK) return rc;
    if (mlp != nullptr && kk > 0) {
        SKYCELL_HIP_CHECK(launch_mlp_forward(points, n, (uint32_t)n, d, mlp->g, mlp->net, logits, device_cus(dev), st));
        SKYCELL_HIP_CHECK(launch_topk(logits, (uint32_t)n, kk, piv.ps.idx, piv.ps, st));
        piv.idx = piv.ps.idx;
    } else {
        piv.idx = pivot_idx;
    }
    const size_t need = workspace_layout(n, d, grid_desc(d, g).cells, nullptr, nullptr);
    void *ws = nullptr;
    if ((rc = cached_buffer(kCacheWorkspace, dev, st, need, &ws)) != SKYCELL_OK) return rc;
    return run_pipeline(points, SKYCELL_DTYPE_F32, n, d, g, 16, out_idx, out_count, ws, stats, st, &piv);
}

}  // namespace skycell

using namespace skycell;

extern "C" {

int skycell_mlp_num_params(int32_t d, int64_t *count)
{
    if (count == nullptr) return fail(SKYCELL_E_INVAL, "count is NULL");
    if (d < 1 || d > SKYCELL_MAX_D) return fail(SKYCELL_E_INVAL, "d = %d is outside [1, %d]", d, SKYCELL_MAX_D);
    *count = (int64_t)mlp_num_params(d);
    return ok();
}

int skycell_mlp_create(int32_t d, int32_t grid_res, uint64_t seed, skycell_mlp_t *mlp)
{
    if (mlp == nullptr) return fail(SKYCELL_E_INVAL, "mlp is NULL");
    *mlp = nullptr;
    if (d < 1 || d > SKYCELL_MAX_D) return fail(SKYCELL_E_INVAL, "d = %d is outside [1, %d]", d, SKYCELL_MAX_D);
    if (grid_res < 1) return fail(SKYCELL_E_INVAL, "grid_res = %d is not >= 1", grid_res);
    skycell_mlp *m = nullptr;
    int rc = mlp_alloc(d, grid_res, &m);
    if (rc != SKYCELL_OK) return rc;
    const std::vector<float> init = glorot_init(d, seed);
    if ((rc = upload_params(m, init.data())) != SKYCELL_OK) {
        (void)hipFree(m->mem);
        delete m;
        return rc;
    }
    *mlp = m;
    return ok();
}

int skycell_mlp_destroy(skycell_mlp_t mlp)
{
    if (mlp == nullptr) return ok();
    (void)hipDeviceSynchronize();
    (void)hipFree(mlp->mem);
    delete mlp;
    return ok();
}

int skycell_mlp_set_params(skycell_mlp_t mlp, const float *params, int64_t count)
{
    int rc = check_handle(mlp);
    if (rc != SKYCELL_OK) return rc;
    if (params == nullptr) return fail(SKYCELL_E_INVAL, "params is NULL");
    if (count != (int64_t)mlp->count) return fail(SKYCELL_E_INVAL, "count = %lld, the network has %u parameters", (long long)count, mlp->count);
    if ((rc = upload_params(mlp, params)) != SKYCELL_OK) return rc;
    return ok();
}

int skycell_mlp_get_params(skycell_mlp_t mlp, float *params, int64_t count)
{
    int rc = check_handle(mlp);
    if (rc != SKYCELL_OK) return rc;
    if (params == nullptr) return fail(SKYCELL_E_INVAL, "params is NULL");
    if (count != (int64_t)mlp->count) return fail(SKYCELL_E_INVAL, "count = %lld, the network has %u parameters", (long long)count, mlp->count);
    SKYCELL_HIP_CHECK(hipDeviceSynchronize());
    SKYCELL_HIP_CHECK(hipMemcpy(params, mlp->master, (size_t)count * 4, hipMemcpyDeviceToHost));
    return ok();
}

int skycell_mlp_get_grads(skycell_mlp_t mlp, float *grads, int64_t count)
{
    int rc = check_handle(mlp);
    if (rc != SKYCELL_OK) return rc;
    if (grads == nullptr) return fail(SKYCELL_E_INVAL, "grads is NULL");
    if (count != (int64_t)mlp->count) return fail(SKYCELL_E_INVAL, "count = %lld, the network has %u parameters", (long long)count, mlp->count);
    SKYCELL_HIP_CHECK(hipDeviceSynchronize());
    SKYCELL_HIP_CHECK(hipMemcpy(grads, mlp->grad, (size_t)count * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < count; ++i) grads[i] *= mlp->grad_scale;
    return ok();
}

int skycell_mlp_set_grads(skycell_mlp_t mlp, const float *grads, int64_t count)
{
    int rc = check_handle(mlp);
    if (rc != SKYCELL_OK) return rc;
    if (grads == nullptr) return fail(SKYCELL_E_INVAL, "grads is NULL");
    if (count != (int64_t)mlp->count) return fail(SKYCELL_E_INVAL, "count = %lld, the network has %u parameters", (long long)count, mlp->count);
    SKYCELL_HIP_CHECK(hipDeviceSynchronize());
    SKYCELL_HIP_CHECK(hipMemcpy(mlp->grad, grads, (size_t)count * 4, hipMemcpyHostToDevice));
    mlp->grad_scale = 1.0f;
    return ok();
}

int skycell_mlp_score(skycell_mlp_t mlp, const float *points, int64_t ld, int64_t n, float *logits, void *stream)
{
    int rc = check_handle(mlp);
    if (rc != SKYCELL_OK) return rc;
    if ((rc = check_points(points, ld, n)) != SKYCELL_OK) return rc;
    if (n > 0 && logits == nullptr) return fail(SKYCELL_E_INVAL, "logits is NULL");
    if (n == 0) return ok();
    SKYCELL_HIP_CHECK(launch_mlp_forward(points, ld, (uint32_t)n, mlp->d, mlp->g, mlp->net, logits,
                                         device_cus(mlp->device), (hipStream_t)stream));
    return ok();
}

int skycell_mlp_backward(skycell_mlp_t mlp, const float *points, int64_t ld, const uint8_t *labels, int64_t n,
                         float *loss_out, void *stream)
{
    int rc = check_handle(mlp);
    if (rc != SKYCELL_OK) return rc;
    if ((rc = check_points(points, ld, n)) != SKYCELL_OK) return rc;
    if (n > 0 && labels == nullptr) return fail(SKYCELL_E_INVAL, "labels is NULL");
    if ((rc = backward(mlp, points, ld, labels, n, loss_out, (hipStream_t)stream)) != SKYCELL_OK) return rc;
    return ok();
}

int skycell_mlp_adam_step(skycell_mlp_t mlp, float lr, void *stream)
{
    int rc = check_handle(mlp);
    if (rc != SKYCELL_OK) return rc;
    if ((rc = adam(mlp, lr, (hipStream_t)stream)) != SKYCELL_OK) return rc;
    return ok();
}

int skycell_mlp_train_step(skycell_mlp_t mlp, const float *points, int64_t ld, const uint8_t *labels, int64_t n,
                           float lr, float *loss_out, void *stream)
{
    int rc = check_handle(mlp);
    if (rc != SKYCELL_OK) return rc;
    if ((rc = check_points(points, ld, n)) != SKYCELL_OK) return rc;
    if (n > 0 && labels == nullptr) return fail(SKYCELL_E_INVAL, "labels is NULL");
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return fail(SKYCELL_E_INVAL, "learning rate %g is not a finite value >= 0", lr);
    if ((rc = backward(mlp, points, ld, labels, n, loss_out, (hipStream_t)stream)) != SKYCELL_OK) return rc;
    if ((rc = adam(mlp, lr, (hipStream_t)stream)) != SKYCELL_OK) return rc;
    return ok();
}

static const char kMlpMagic[8] = {'S', 'K', 'Y', 'M', 'L', 'P', '0', '1'};

int skycell_mlp_save(skycell_mlp_t mlp, const char *path)
{
    int rc = check_handle(mlp);
    if (rc != SKYCELL_OK) return rc;
    if (path == nullptr) return fail(SKYCELL_E_INVAL, "path is NULL");
    std::vector<float> buf((size_t)mlp->count * 3);
    SKYCELL_HIP_CHECK(hipDeviceSynchronize());
    SKYCELL_HIP_CHECK(hipMemcpy(buf.data(), mlp->master, (size_t)mlp->count * 4, hipMemcpyDeviceToHost));
    SKYCELL_HIP_CHECK(hipMemcpy(buf.data() + mlp->count, mlp->m1, (size_t)mlp->count * 4, hipMemcpyDeviceToHost));
    SKYCELL_HIP_CHECK(hipMemcpy(buf.data() + 2 * (size_t)mlp->count, mlp->m2, (size_t)mlp->count * 4, hipMemcpyDeviceToHost));
    FILE *f = fopen(path, "wb");
    if (f == nullptr) return fail(SKYCELL_E_INVAL, "cannot open %s for writing", path);
    const int32_t hdr[4] = {mlp->d, mlp->g, mlp->step, (int32_t)mlp->count};
    bool good = fwrite(kMlpMagic, 1, 8, f) == 8 && fwrite(hdr, 4, 4, f) == 4 &&
                fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    good = (fclose(f) == 0) && good;
    if (!good) return fail(SKYCELL_E_INVAL, "writing %s failed", path);
    return ok();
}

int skycell_mlp_load(const char *path, skycell_mlp_t *mlp)
{
    if (mlp == nullptr) return fail(SKYCELL_E_INVAL, "mlp is NULL");
    *mlp = nullptr;
    if (path == nullptr) return fail(SKYCELL_E_INVAL, "path is NULL");
    FILE *f = fopen(path, "rb");
    if (f == nullptr) return fail(SKYCELL_E_INVAL, "cannot open %s", path);
    char magic[8];
    int32_t hdr[4];
    if (fread(magic, 1, 8, f) != 8 || memcmp(magic, kMlpMagic, 8) != 0 || fread(hdr, 4, 4, f) != 4) {
        fclose(f);
        return fail(SKYCELL_E_INVAL, "%s is not a network file", path);
    }
    const int d = hdr[0], g = hdr[1], step = hdr[2];
    if (d < 1 || d > SKYCELL_MAX_D || g < 1 || step < 0 || hdr[3] != (int32_t)mlp_num_params(d)) {
        fclose(f);
        return fail(SKYCELL_E_INVAL, "%s has an invalid header", path);
    }
    std::vector<float> buf((size_t)hdr[3] * 3);
    const bool good = fread(buf.data(), 4, buf.size(), f) == buf.size();
    fclose(f);
    if (!good) return fail(SKYCELL_E_INVAL, "%s is truncated", path);
    skycell_mlp *m = nullptr;
    int rc = mlp_alloc(d, g, &m);
    if (rc != SKYCELL_OK) return rc;
    if ((rc = upload_params(m, buf.data())) != SKYCELL_OK ||
        hipMemcpy(m->m1, buf.data() + m->count, (size_t)m->count * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->m2, buf.data() + 2 * (size_t)m->count, (size_t)m->count * 4, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(m->mem);
        delete m;
        return rc != SKYCELL_OK ? rc : fail(SKYCELL_E_HIP, "uploading %s failed", path);
    }
    m->step = step;
    *mlp = m;
    return ok();
}

int skycell_skyline_labels(const int32_t *idx, const int32_t *count, int64_t n, uint8_t *labels, void *stream)
{
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(SKYCELL_E_INVAL, "n = %lld out of range", (long long)n);
    if (n == 0) return ok();
    if (idx == nullptr || count == nullptr || labels == nullptr) return fail(SKYCELL_E_INVAL, "a pointer is NULL");
    SKYCELL_HIP_CHECK(launch_labels(idx, count, (uint32_t)n, labels, (hipStream_t)stream));
    return ok();
}

int skycell_topk(const float *scores, int64_t n, int32_t k, int32_t *out_idx, void *stream)
{
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(SKYCELL_E_INVAL, "n = %lld out of range", (long long)n);
    if (k < 1 || k > kMaxPivots) return fail(SKYCELL_E_INVAL, "k = %d is outside [1, %d]", k, kMaxPivots);
    if (n == 0) return ok();
    if (scores == nullptr || out_idx == nullptr) return fail(SKYCELL_E_INVAL, "a pointer is NULL");
    int dev = 0;
    SKYCELL_HIP_CHECK(hipGetDevice(&dev));
    PivotScratch ps;
    hipStream_t st = (hipStream_t)stream;
    int rc = pivot_scratch(dev, st, 0, &ps, nullptr);
    if (rc != SKYCELL_OK) return rc;
    const uint32_t kk = (uint32_t)(k < n ? k : n);
    SKYCELL_HIP_CHECK(launch_topk(scores, (uint32_t)n, kk, out_idx, ps, st));
    return ok();
}

int skycell_compute_with_pivots(const float *points, int64_t n, int32_t d, int32_t grid_res,
                                const int32_t *pivot_idx, int32_t k, int32_t *out_idx, int32_t *out_count,
                                uint64_t *stats, void *stream)
{
    int rc = compute_with(points, n, d, grid_res, pivot_idx, k, nullptr, out_idx, out_count, stats,
                          (hipStream_t)stream);
    return rc != SKYCELL_OK ? rc : ok();
}

int skycell_compute_pivoted(const float *points, int64_t n, int32_t d, int32_t grid_res, skycell_mlp_t mlp,
                            int32_t k, int32_t *out_idx, int32_t *out_count, uint64_t *stats, void *stream)
{
    if (mlp == nullptr) return fail(SKYCELL_E_INVAL, "network handle is NULL");
    int rc = compute_with(points, n, d, grid_res, nullptr, k, mlp, out_idx, out_count, stats, (hipStream_t)stream);
    return rc != SKYCELL_OK ? rc : ok();
}

}  // extern "C"
