// Learned pivot proposer: parameter layout and launchers (kernels in mlp.hip,
// pivot selection and pre-filter in pivot.hip).
#pragma once

#include "common.h"

namespace skycell {

constexpr int kMlpHidden = 64;
constexpr int kMlpFeatPad = 32;   // feature rows of the first weight matrix, zero padded (2d <= 32)

// Flat float32 parameter vector: W1 [64][2d], b1 [64], W2 [64][64], b2 [64],
// w3 [64], b3 [1]; matrices are output-unit major.
__host__ __device__ constexpr uint32_t mlp_off_w1() { return 0u; }
__host__ __device__ constexpr uint32_t mlp_off_b1(int d) { return (uint32_t)(kMlpHidden * 2 * d); }
__host__ __device__ constexpr uint32_t mlp_off_w2(int d) { return mlp_off_b1(d) + kMlpHidden; }
__host__ __device__ constexpr uint32_t mlp_off_b2(int d) { return mlp_off_w2(d) + kMlpHidden * kMlpHidden; }
__host__ __device__ constexpr uint32_t mlp_off_w3(int d) { return mlp_off_b2(d) + kMlpHidden; }
__host__ __device__ constexpr uint32_t mlp_off_b3(int d) { return mlp_off_w3(d) + kMlpHidden; }
__host__ __device__ constexpr uint32_t mlp_num_params(int d) { return mlp_off_b3(d) + 1u; }

// The bfloat16 copy of the weights the kernels read (biases and the output
// vector as float32 holding bfloat16 values), carved from one allocation.
struct MlpDevice {
    uint16_t *w1;    // [64][kMlpFeatPad], columns >= 2d stay zero
    uint16_t *w2;    // [64][64]
    uint16_t *w2t;   // [64][64], transpose of w2 (for the backward pass)
    float *b1, *b2, *w3, *b3;
};

constexpr size_t kMlpDeviceBytes = 21504;

inline MlpDevice mlp_device_view(void *base)
{
    char *p = (char *)base;
    MlpDevice v;
    v.w1 = (uint16_t *)(p + 0);
    v.w2 = (uint16_t *)(p + 4096);
    v.w2t = (uint16_t *)(p + 12288);
    v.b1 = (float *)(p + 20480);
    v.b2 = (float *)(p + 20736);
    v.w3 = (float *)(p + 20992);
    v.b3 = (float *)(p + 21248);
    return v;
}

struct AdamArgs {
    float lr, beta1, beta2, eps;
    float corr1, corr2;   // 1 / (1 - beta^t)
    float grad_scale;     // 1 / points of the last backward pass
};

hipError_t launch_mlp_forward(const float *pts, int64_t ld, uint32_t n, int d, int g, const MlpDevice &net,
                              float *logits, int num_cus, hipStream_t st);
hipError_t launch_mlp_backward(const float *pts, int64_t ld, uint32_t n, int d, int g, const MlpDevice &net,
                               const uint8_t *labels, float *grad, float *loss_sum, uint32_t count,
                               int num_cus, hipStream_t st);
hipError_t launch_mlp_mean_loss(const float *loss_sum, float inv_n, float *out, hipStream_t st);
hipError_t launch_mlp_pack(const float *master, uint32_t count, int d, const MlpDevice &net, hipStream_t st);
hipError_t launch_mlp_adam(float *master, float *m1, float *m2, const float *grad, uint32_t count, int d,
                           const MlpDevice &net, const AdamArgs &a, hipStream_t st);
hipError_t launch_labels(const int32_t *idx, const int32_t *count, uint32_t n, uint8_t *labels, hipStream_t st);

// ---- pivots (pivot.hip) ----
constexpr int kMaxPivots = 4096;

// Scratch of the top-k selection and the pivot table, carved from one allocation.
struct PivotScratch {
    uint32_t *hist;     // [2048] digit histogram
    uint32_t *state;    // [16] selection state
    uint64_t *sel;      // [kMaxPivots] selected (inverted key, index) pairs
    int32_t *idx;       // [kMaxPivots] pivot indices, best first
    uint32_t *pkeys;    // [kMaxPivots * kMaxD] order-preserving keys of the pivots
    uint64_t *pfine;    // [kMaxPivots * 2] packed screening columns of the pivots
};
size_t pivot_scratch_layout(PivotScratch *ps, char *base);

hipError_t launch_topk(const float *scores, uint32_t n, uint32_t k, int32_t *out_idx, const PivotScratch &ps,
                       hipStream_t st);
hipError_t launch_pivot_gather(const float *pts, uint32_t n, int d, const int32_t *idx, uint32_t k,
                               const PivotScratch &ps, uint32_t *ctr, hipStream_t st);
// gated: screen a sample first and run the full pass only when the pivots
// remove at least 1 in 100 of its points of surviving cells
hipError_t launch_pivot_prune(const float *pts, uint32_t n, const GridDesc &gd, const Workspace &ws,
                              const PivotScratch &ps, uint32_t k, uint64_t *stats, bool gated, hipStream_t st);

}  // namespace skycell
