// Learned pivot proposer: a 2d -> 64 -> 64 -> 1 perceptron (ReLU, logistic
// output) that scores points by how likely they are to be skyline points.  It
// only chooses pivots for the exact pre-filter; every output of the skyline
// path is still decided by exact dominance tests.
//
// All matrix products run on the gfx950 matrix cores as
// v_mfma_f32_16x16x16_bf16 with float32 accumulation.  The products are taken
// transposed, H^T = W * X^T, so that the 16 columns of a tile are 16 points
// and the rows are hidden units: the accumulator layout of one layer (lane l
// holds point l%16, units 4*(l/16)..+3 of each 16-unit block) is then exactly
// the B-operand layout the next layer needs, and activations never leave the
// registers in the forward pass.  The weight-gradient products contract over
// points instead; their operands are transposed through LDS.
//
// Features of a point x for g columns per dimension: x[k] and the fractional
// position t - floor(t), t = x[k] * g (binary32), of x inside its column of
// Equation 1 (k < d).  Features, weights and hidden activations are rounded to
// bfloat16 (to nearest, ties to even) before every product.
#include "common.h"
#include "mlp.h"
#include "../../include/skycell.h"

namespace skycell {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMlpThreads = 256;
constexpr int kMlpWaves = kMlpThreads / kWave;

__device__ __forceinline__ uint16_t bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x4 load_frag(const uint16_t *p)
{
    const uint2 v = *(const uint2 *)p;
    bf16x4 r;
    r[0] = (short)(v.x & 0xFFFFu);
    r[1] = (short)(v.x >> 16);
    r[2] = (short)(v.y & 0xFFFFu);
    r[3] = (short)(v.y >> 16);
    return r;
}

// Feature k of point p (k < 2d), binary32.
__device__ __forceinline__ float feature(const float *__restrict__ pts, int64_t ld, uint32_t p, int d,
                                         float gf, int k)
{
    const int kk = k < d ? k : k - d;
    const float x = pts[(size_t)kk * ld + p];
    if (k < d) return x;
    const float t = __fmul_rn(x, gf);
    return __fsub_rn(t, floorf(t));
}

// B operand of the first layer for the wave's 16-point tile: lane l holds
// features 16s + 4*(l/16) + e of point l%16.
template <int KS>
__device__ __forceinline__ void load_features(const float *__restrict__ pts, int64_t ld, uint32_t p,
                                              bool valid, int d, float gf, int grp, bf16x4 (&X)[KS])
{
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 16 * s + 4 * grp + e;
            const float f = (valid && k < 2 * d) ? feature(pts, ld, p, d, gf, k) : 0.0f;
            X[s][e] = (short)bf16_rne(f);
        }
}

// ------------------------------------------------------------------ forward
template <int KS>
__global__ __launch_bounds__(kMlpThreads) void k_mlp_forward(const float *__restrict__ pts, int64_t ld,
                                                             uint32_t n, int d, float gf,
                                                             MlpDevice net, float *__restrict__ logits)
{
    const int l = __lane_id(), col = l & 15, grp = l >> 4;
    bf16x4 A1[4][KS], A2[4][4];
    f32x4 B1[4], B2[4], W3[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int s = 0; s < KS; ++s) A1[m][s] = load_frag(net.w1 + (16 * m + col) * kMlpFeatPad + 16 * s + 4 * grp);
#pragma unroll
        for (int s = 0; s < 4; ++s) A2[m][s] = load_frag(net.w2 + (16 * m + col) * kMlpHidden + 16 * s + 4 * grp);
        B1[m] = *(const f32x4 *)(net.b1 + 16 * m + 4 * grp);
        B2[m] = *(const f32x4 *)(net.b2 + 16 * m + 4 * grp);
        W3[m] = *(const f32x4 *)(net.w3 + 16 * m + 4 * grp);
    }
    const float b3 = net.b3[0];

    const uint32_t tiles = (n + 15u) / 16u;
    const uint32_t nwaves = gridDim.x * kMlpWaves;
    for (uint32_t t = blockIdx.x * kMlpWaves + threadIdx.x / kWave; t < tiles; t += nwaves) {
        const uint32_t p = t * 16u + (uint32_t)col;
        const bool valid = p < n;
        bf16x4 X[KS];
        load_features<KS>(pts, ld, p, valid, d, gf, grp, X);

        bf16x4 H1[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < KS; ++s) acc = mfma16(A1[m][s], X[s], acc);
#pragma unroll
            for (int e = 0; e < 4; ++e) H1[m][e] = (short)bf16_rne(fmaxf(acc[e] + B1[m][e], 0.0f));
        }
        float z = 0.0f;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 4; ++s) acc = mfma16(A2[m][s], H1[s], acc);
#pragma unroll
            for (int e = 0; e < 4; ++e) z += bf16_val(bf16_rne(fmaxf(acc[e] + B2[m][e], 0.0f))) * W3[m][e];
        }
        z += __shfl_xor(z, 16);
        z += __shfl_xor(z, 32);
        if (grp == 0 && valid) logits[p] = z + b3;
    }
}

// ------------------------------------------------------------------ backward
// Per 16-point tile of every wave: the forward pass again, the logistic loss,
// the gradient back through both layers, and the weight-gradient products
// (contracting over the tile's points) accumulated in registers.  The tile loop
// is uniform over the workgroup so that workgroup barriers can separate the
// LDS writes of the transposes from their reads.
template <int KS>
__global__ __launch_bounds__(kMlpThreads) void k_mlp_backward(const float *__restrict__ pts, int64_t ld,
                                                              uint32_t n, int d, float gf, MlpDevice net,
                                                              const uint8_t *__restrict__ labels,
                                                              float *__restrict__ grad,
                                                              float *__restrict__ loss_sum)
{
    __shared__ __align__(16) uint16_t s_w1[kMlpHidden * kMlpFeatPad];
    __shared__ __align__(16) uint16_t s_w2[kMlpHidden * kMlpHidden];
    __shared__ __align__(16) uint16_t s_w2t[kMlpHidden * kMlpHidden];
    // per wave: [unit][point] tiles of dpre2, h1, dpre1 (64 x 16) and of the features (KF x 16)
    __shared__ __align__(16) uint16_t s_t[kMlpWaves][3 * kMlpHidden * 16 + kMlpFeatPad * 16];

    for (int i = threadIdx.x; i < kMlpHidden * kMlpFeatPad; i += kMlpThreads) s_w1[i] = net.w1[i];
    for (int i = threadIdx.x; i < kMlpHidden * kMlpHidden; i += kMlpThreads) {
        s_w2[i] = net.w2[i];
        s_w2t[i] = net.w2t[i];
    }

    const int l = __lane_id(), col = l & 15, grp = l >> 4;
    const int wave = threadIdx.x / kWave;
    uint16_t *t_d2 = s_t[wave];
    uint16_t *t_h1 = t_d2 + kMlpHidden * 16;
    uint16_t *t_d1 = t_h1 + kMlpHidden * 16;
    uint16_t *t_x = t_d1 + kMlpHidden * 16;

    f32x4 B1[4], B2[4], W3[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        B1[m] = *(const f32x4 *)(net.b1 + 16 * m + 4 * grp);
        B2[m] = *(const f32x4 *)(net.b2 + 16 * m + 4 * grp);
        W3[m] = *(const f32x4 *)(net.w3 + 16 * m + 4 * grp);
    }
    const float b3 = net.b3[0];

    f32x4 gW2[4][4], gW1[4][KS];
    float gw3[4][4], gb2[4][4], gb1[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            gW2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
            gw3[a][b] = gb2[a][b] = gb1[a][b] = 0.0f;
        }
#pragma unroll
        for (int s = 0; s < KS; ++s) gW1[a][s] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    float lsum = 0.0f, gb3 = 0.0f;
    __syncthreads();

    const uint32_t tiles = (n + 15u) / 16u;
    const uint32_t block_tiles = (tiles + kMlpWaves - 1) / kMlpWaves;
    for (uint32_t bt = blockIdx.x; bt < block_tiles; bt += gridDim.x) {
        const uint32_t t = bt * kMlpWaves + (uint32_t)wave;
        const uint32_t p = t * 16u + (uint32_t)col;
        const bool valid = t < tiles && p < n;
        bf16x4 X[KS];
        load_features<KS>(pts, ld, p, valid, d, gf, grp, X);

        // forward
        bf16x4 H1[4];
        bool mask1[4][4], mask2[4][4];
        float h2[4][4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < KS; ++s)
                acc = mfma16(load_frag(s_w1 + (16 * m + col) * kMlpFeatPad + 16 * s + 4 * grp), X[s], acc);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float v = acc[e] + B1[m][e];
                mask1[m][e] = v > 0.0f;
                H1[m][e] = (short)bf16_rne(fmaxf(v, 0.0f));
            }
        }
        float z = 0.0f;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc = mfma16(load_frag(s_w2 + (16 * m + col) * kMlpHidden + 16 * s + 4 * grp), H1[s], acc);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float v = acc[e] + B2[m][e];
                mask2[m][e] = v > 0.0f;
                h2[m][e] = bf16_val(bf16_rne(fmaxf(v, 0.0f)));
                z += h2[m][e] * W3[m][e];
            }
        }
        z += __shfl_xor(z, 16);
        z += __shfl_xor(z, 32);
        z += b3;

        // loss and output gradient (unscaled: the mean is taken at the update)
        const float y = valid ? (float)labels[p] : 0.0f;
        const float sig = 1.0f / (1.0f + __expf(-z));
        const float dz = valid ? sig - y : 0.0f;
        if (grp == 0 && valid) {
            lsum += fmaxf(z, 0.0f) - y * z + log1pf(__expf(-fabsf(z)));
            gb3 += dz;
        }

        // second layer
        bf16x4 D2[4];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                gw3[m][e] += dz * h2[m][e];
                const float g = mask2[m][e] ? dz * W3[m][e] : 0.0f;
                gb2[m][e] += g;
                D2[m][e] = (short)bf16_rne(g);
                const int unit = 16 * m + 4 * grp + e;
                t_d2[unit * 16 + col] = (uint16_t)D2[m][e];
                t_h1[unit * 16 + col] = (uint16_t)H1[m][e];
            }
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int e = 0; e < 4; ++e) t_x[(16 * s + 4 * grp + e) * 16 + col] = (uint16_t)X[s][e];

        // first layer: dh1 = W2^T dpre2
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc = mfma16(load_frag(s_w2t + (16 * m + col) * kMlpHidden + 16 * s + 4 * grp), D2[s], acc);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float g = mask1[m][e] ? acc[e] : 0.0f;
                gb1[m][e] += g;
                t_d1[(16 * m + 4 * grp + e) * 16 + col] = bf16_rne(g);
            }
        }
        __syncthreads();

        // weight gradients, contracting over the tile's 16 points
        bf16x4 TH1[4], TX[KS];
#pragma unroll
        for (int m = 0; m < 4; ++m) TH1[m] = load_frag(t_h1 + (16 * m + col) * 16 + 4 * grp);
#pragma unroll
        for (int s = 0; s < KS; ++s) TX[s] = load_frag(t_x + (16 * s + col) * 16 + 4 * grp);
#pragma unroll
        for (int mj = 0; mj < 4; ++mj) {
            const bf16x4 TD2 = load_frag(t_d2 + (16 * mj + col) * 16 + 4 * grp);
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) gW2[mj][mi] = mfma16(TD2, TH1[mi], gW2[mj][mi]);
        }
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) {
            const bf16x4 TD1 = load_frag(t_d1 + (16 * mi + col) * 16 + 4 * grp);
#pragma unroll
            for (int s = 0; s < KS; ++s) gW1[mi][s] = mfma16(TD1, TX[s], gW1[mi][s]);
        }
        __syncthreads();
    }

    // flush: matrix gradients straight from the accumulator layout
    const int F = 2 * d;
    float *gw1 = grad + mlp_off_w1();
    float *gw2 = grad + mlp_off_w2(d);
#pragma unroll
    for (int mj = 0; mj < 4; ++mj)
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                atomicAdd(&gw2[(16 * mj + 4 * grp + e) * kMlpHidden + 16 * mi + col], gW2[mj][mi][e]);
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int f = 16 * s + col;
            if (f < F)
#pragma unroll
                for (int e = 0; e < 4; ++e) atomicAdd(&gw1[(16 * mi + 4 * grp + e) * F + f], gW1[mi][s][e]);
        }
    // per-unit vectors: sum over the 16 lanes that hold the same units
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float a = gw3[m][e], b = gb2[m][e], c = gb1[m][e];
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                a += __shfl_xor(a, off);
                b += __shfl_xor(b, off);
                c += __shfl_xor(c, off);
            }
            if (col == 0) {
                const int unit = 16 * m + 4 * grp + e;
                atomicAdd(&grad[mlp_off_w3(d) + unit], a);
                atomicAdd(&grad[mlp_off_b2(d) + unit], b);
                atomicAdd(&grad[mlp_off_b1(d) + unit], c);
            }
        }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lsum += __shfl_xor(lsum, off);
        gb3 += __shfl_xor(gb3, off);
    }
    if (l == 0) {
        atomicAdd(&grad[mlp_off_b3(d)], gb3);
        atomicAdd(loss_sum, lsum);
    }
}

// ------------------------------------------------------------------ update
// Writes parameter i (flat layout) into the bfloat16 copy the kernels read.
__device__ __forceinline__ void pack_param(const MlpDevice &net, int d, uint32_t i, float v)
{
    const uint32_t F = 2u * (uint32_t)d;
    const uint16_t h = bf16_rne(v);
    if (i < mlp_off_b1(d)) {
        net.w1[(i / F) * kMlpFeatPad + i % F] = h;
    } else if (i < mlp_off_w2(d)) {
        net.b1[i - mlp_off_b1(d)] = bf16_val(h);
    } else if (i < mlp_off_b2(d)) {
        const uint32_t j = i - mlp_off_w2(d);
        net.w2[j] = h;
        net.w2t[(j % kMlpHidden) * kMlpHidden + j / kMlpHidden] = h;
    } else if (i < mlp_off_w3(d)) {
        net.b2[i - mlp_off_b2(d)] = bf16_val(h);
    } else if (i < mlp_off_b3(d)) {
        net.w3[i - mlp_off_w3(d)] = bf16_val(h);
    } else {
        net.b3[0] = bf16_val(h);
    }
}

__global__ void k_mlp_pack(const float *__restrict__ master, uint32_t count, int d, MlpDevice net)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) pack_param(net, d, i, master[i]);
}

__global__ void k_mlp_adam(float *__restrict__ master, float *__restrict__ m1, float *__restrict__ m2,
                           const float *__restrict__ grad, uint32_t count, int d, MlpDevice net,
                           AdamArgs a)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float g = grad[i] * a.grad_scale;
    const float m = a.beta1 * m1[i] + (1.0f - a.beta1) * g;
    const float v = a.beta2 * m2[i] + (1.0f - a.beta2) * g * g;
    m1[i] = m;
    m2[i] = v;
    const float p = master[i] - a.lr * (m * a.corr1) / (sqrtf(v * a.corr2) + a.eps);
    master[i] = p;
    pack_param(net, d, i, p);
}

__global__ void k_fill_f32(float *__restrict__ p, uint32_t count, float v)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

__global__ void k_mean_loss(const float *__restrict__ loss_sum, float inv_n, float *__restrict__ out)
{
    out[0] = loss_sum[0] * inv_n;
}

// ------------------------------------------------------------------ labels
__global__ void k_fill_u8(uint8_t *__restrict__ p, uint32_t count, uint8_t v)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

__global__ void k_labels_scatter(const int32_t *__restrict__ idx, const int32_t *__restrict__ count,
                                 uint32_t n, uint8_t *__restrict__ labels)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t c = count[0];
    if (c <= 0 || j >= (uint32_t)c || j >= n) return;
    const int32_t i = idx[j];
    if (i >= 0 && (uint32_t)i < n) labels[i] = 1;
}

// ------------------------------------------------------------------ launchers
static inline dim3 blocks_for(uint64_t count, int per = 256)
{
    uint64_t b = (count + per - 1) / per;
    return dim3((unsigned)(b ? b : 1));
}

// Workgroups of the forward and backward grid-stride loops: enough to fill the
// GPU several times over, fewer for small inputs.
static inline unsigned mlp_blocks(uint32_t n, int num_cus, int per_cu)
{
    const uint64_t tiles = (n + 15u) / 16u;
    uint64_t b = (tiles + kMlpWaves - 1) / kMlpWaves;
    const uint64_t cap = (uint64_t)num_cus * per_cu;
    if (b > cap) b = cap;
    return (unsigned)(b ? b : 1);
}

hipError_t launch_mlp_forward(const float *pts, int64_t ld, uint32_t n, int d, int g, const MlpDevice &net,
                              float *logits, int num_cus, hipStream_t st)
{
    const dim3 grid(mlp_blocks(n, num_cus, 8));
    if (2 * d <= 16)
        hipLaunchKernelGGL(k_mlp_forward<1>, grid, dim3(kMlpThreads), 0, st, pts, ld, n, d, (float)g, net, logits);
    else
        hipLaunchKernelGGL(k_mlp_forward<2>, grid, dim3(kMlpThreads), 0, st, pts, ld, n, d, (float)g, net, logits);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const float *pts, int64_t ld, uint32_t n, int d, int g, const MlpDevice &net,
                               const uint8_t *labels, float *grad, float *loss_sum, uint32_t count,
                               int num_cus, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_f32, blocks_for(count), dim3(256), 0, st, grad, count, 0.0f);
    hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(64), 0, st, loss_sum, 1u, 0.0f);
    if (n == 0) return hipGetLastError();
    const dim3 grid(mlp_blocks(n, num_cus, 2));
    if (2 * d <= 16)
        hipLaunchKernelGGL(k_mlp_backward<1>, grid, dim3(kMlpThreads), 0, st, pts, ld, n, d, (float)g, net,
                           labels, grad, loss_sum);
    else
        hipLaunchKernelGGL(k_mlp_backward<2>, grid, dim3(kMlpThreads), 0, st, pts, ld, n, d, (float)g, net,
                           labels, grad, loss_sum);
    return hipGetLastError();
}

hipError_t launch_mlp_mean_loss(const float *loss_sum, float inv_n, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_mean_loss, dim3(1), dim3(1), 0, st, loss_sum, inv_n, out);
    return hipGetLastError();
}

hipError_t launch_mlp_pack(const float *master, uint32_t count, int d, const MlpDevice &net, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_pack, blocks_for(count), dim3(256), 0, st, master, count, d, net);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *master, float *m1, float *m2, const float *grad, uint32_t count, int d,
                           const MlpDevice &net, const AdamArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_adam, blocks_for(count), dim3(256), 0, st, master, m1, m2, grad, count, d, net, a);
    return hipGetLastError();
}

hipError_t launch_labels(const int32_t *idx, const int32_t *count, uint32_t n, uint8_t *labels, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u8, blocks_for(n), dim3(256), 0, st, labels, n, (uint8_t)0);
    hipLaunchKernelGGL(k_labels_scatter, blocks_for(n), dim3(256), 0, st, idx, count, n, labels);
    return hipGetLastError();
}

}  // namespace skycell
