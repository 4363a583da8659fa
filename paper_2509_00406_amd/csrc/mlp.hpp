// The learned per-triangle density psi(z): a 6 -> 64 -> 64 -> 1 softplus network
// (project-defined; the paper has no learned component). Trainable parameters
// are packed as W1 (64 x 6), b1 (64), W2 (64 x 64), b2 (64), w3 (64), b3 (1),
// row-major; the input scale s_in (6) and output scale s_out are fixed:
//   psi(z) = s_out (w3 . sp(W2 sp(W1 (s_in * z) + b1) + b2) + b3),  sp = softplus.
// FP32 master copy and Adam moments for training; a BF16 copy for evaluation.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mad.h"

namespace mad {

constexpr int kHid = 64;
constexpr int kMlpParams = kHid * 6 + kHid + kHid * kHid + kHid + kHid + 1;  // 4673
constexpr int kOffW1 = 0, kOffB1 = kHid * 6, kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid,
              kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid;
constexpr int kPsi = 28;  // network outputs per element: value, dpsi/dz (6), packed d2psi/dz2 (21)

// one network evaluation pass over a term's triangles (patch order)
struct MlpHeadLaunch {
    const double* x;          // [nv][3]
    const double* normals;    // [nv][3]
    const int32_t* stencil;   // [n][3] global vertices
    const double* rest;       // SoA [8][n]
    int64_t n;
    const uint16_t* wbf;      // BF16 parameters, packed order
    float s_in[6];
    float s_out;
    float* xh;                // SoA [6][n] scaled features s_in * z (written by the feature pass)
    float* psi;               // SoA [28][n]
    int32_t n_cu;             // compute units: the network pass runs at most one workgroup per CU (its registers
                              // allow one wave per SIMD; its LDS operand tables are built once per workgroup)
};
// feature pass (one lane per triangle, FP64 features rounded to FP32 and scaled), then the
// network pass reading them
hipError_t launch_mlp_head(const MlpHeadLaunch& L, hipStream_t s);

// area-weighted unit vertex normals by a fixed-order gather over each vertex's triangles
hipError_t launch_vertex_normals(const double* x, int64_t nv, const int32_t* vf_ptr, const int32_t* vf,
                                 const int32_t* tris, double* normals, hipStream_t s);

// training: loss and gradient over samples idx[base, base + count) (idx may be NULL: identity)
struct MlpTrainLaunch {
    const float* z;           // [N][6]
    const float* W;           // [N]
    const float* dW;          // [N][6]
    const int32_t* idx;
    int64_t base, count;
    const float* params;      // FP32 master [kMlpParams]
    float s_in[6];
    float s_out;
    float c_e, c_g[6], lam_g;
    float* partial;           // [n_waves][kMlpParams + 1]
    int n_waves;
};
hipError_t launch_mlp_train(const MlpTrainLaunch& L, hipStream_t s);
// sum the per-wave partials in a fixed order: grad [kMlpParams], loss [1]
hipError_t launch_mlp_reduce(const float* partial, int n_waves, float* grad, float* loss, hipStream_t s);
// Adam on the master copy (step t >= 1, read on the device), then refresh the BF16 copy
hipError_t launch_mlp_adam(float* params, float* m, float* v, const float* grad, const int64_t* step, float lr,
                           float beta1, float beta2, float eps, uint16_t* wbf, hipStream_t s);
hipError_t launch_mlp_to_bf16(const float* params, uint16_t* wbf, hipStream_t s);
hipError_t launch_mlp_step_incr(int64_t* step, hipStream_t s);

}  // namespace mad

struct mad_mlp {
    int device = 0;
    float s_in[6] = {1, 1, 1, 1, 1, 1};
    float s_out = 1.0f;
    float* d_params = nullptr;     // FP32 master
    float* d_m = nullptr;          // Adam first moment
    float* d_v = nullptr;          // Adam second moment
    uint16_t* d_wbf = nullptr;     // BF16 evaluation copy
    float* d_grad = nullptr;
    float* d_loss = nullptr;
    int64_t* d_step = nullptr;     // Adam step counter (device, so a training loop needs no host sync)
    float* d_partial = nullptr;
    int partial_waves = 0;
};
