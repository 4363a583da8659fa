// Kernels of the learned per-triangle density (project-defined; no paper
// counterpart): passive vertex normals, the network pass that produces psi and
// its first and second derivatives with respect to the six features for every
// triangle, and the training pass (loss, gradient, Adam).
//
// Network pass. Forward mode is seeded on the six (scaled) features: layer 1's
// unit k carries, in closed form, sp(a1) and its first derivatives
// sigma(a1) W1[k,i] (second derivatives sigma'(a1) W1[k,i] W1[k,j]). Layer 2's
// value and first-order channels, the transposed contraction u = W2^T v that
// folds layer 2's second-order channels into one, and the layer-1 part of the
// second derivatives are contractions over the 64 units and run on the matrix
// cores (v_mfma_f32_16x16x32_bf16; see k_mlp_head). Weights and products of
// two weights are exact in one or two BF16 terms; every activation is split
// into three BF16 terms (hi + mid + lo carries all 24 bits of an FP32
// significand), so the MFMAs reproduce FP32 products with FP32 accumulation.
#include <hip/hip_runtime.h>

#include <cmath>

#include "mlp.hpp"
#include "terms.hpp"

namespace mad {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short short8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float softplusf(float a) { return fmaxf(a, 0.0f) + log1pf(expf(-fabsf(a))); }
__device__ __forceinline__ float logisticf(float a) {
    const float e = expf(-fabsf(a));
    const float r = 1.0f / (1.0f + e);
    return a >= 0.0f ? r : e * r;
}

// softplus and logistic of a from one exponential, with the hardware exp2, log2 and reciprocal
// (about one ulp each; used by the network pass): e = exp(-|a|), with the product -|a| log2(e) carried
// to twice FP32 precision so that e keeps its relative accuracy for large |a|; sigma = 1/(1+e)
// (a >= 0) or e/(1+e); softplus = max(a, 0) + log1p(e), with log1p(e) = log(u) e / (u - 1),
// u = 1 + e rounded, and e itself where u rounds to 1: the method of D. Goldberg, "What every computer
// scientist should know about floating-point arithmetic" (ACM Computing Surveys, 1991), Theorem 4.
// Relative error within five FP32 ulps of FP64 log1p / exp over |a| <= 80 in an FP32 emulation with every
// hardware result rounded to nearest or one ulp off either way.
__device__ __forceinline__ void softplus_logistic(float a, float& sp, float& sg) {
    constexpr float kL2E = 1.44269502162933349609375f;          // log2(e) rounded to FP32
    constexpr float kL2ELo = 1.925963033500011079e-8f;          // log2(e) - kL2E
    constexpr float kLn2 = 0.693147180559945309f;
    const float x = -fabsf(a);
    const float t = x * kL2E;
    const float tl = fmaf(x, kL2E, -t) + x * kL2ELo;
    float e = __builtin_amdgcn_exp2f(t);
    e = fmaf(e, tl * kLn2, e);
    const float u = 1.0f + e;
    const float r = __builtin_amdgcn_rcpf(u);
    sg = a >= 0.0f ? r : e * r;
    const float um1 = u - 1.0f;
    const float l1p = um1 == 0.0f ? e : (__builtin_amdgcn_logf(u) * kLn2) * (e * __builtin_amdgcn_rcpf(um1));
    sp = fmaxf(a, 0.0f) + l1p;
}

// ---- vertex normals ------------------------------------------------------------------------------
__global__ void k_vertex_normals(const double* x, int64_t nv, const int32_t* vf_ptr, const int32_t* vf,
                                 const int32_t* tris, double* normals) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        double n0 = 0.0, n1 = 0.0, n2 = 0.0;
        for (int32_t q = vf_ptr[v]; q < vf_ptr[v + 1]; ++q) {
            const int32_t* t = tris + 3 * (int64_t)vf[q];
            const double* a = x + 3 * (int64_t)t[0];
            const double* b = x + 3 * (int64_t)t[1];
            const double* c = x + 3 * (int64_t)t[2];
            const double e1x = b[0] - a[0], e1y = b[1] - a[1], e1z = b[2] - a[2];
            const double e2x = c[0] - a[0], e2y = c[1] - a[1], e2z = c[2] - a[2];
            n0 += e1y * e2z - e1z * e2y;
            n1 += e1z * e2x - e1x * e2z;
            n2 += e1x * e2y - e1y * e2x;
        }
        const double l = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
        const double il = l > 0.0 ? 1.0 / l : 0.0;
        normals[3 * v] = n0 * il;
        normals[3 * v + 1] = n1 * il;
        normals[3 * v + 2] = n2 * il;
    }
}

hipError_t launch_vertex_normals(const double* x, int64_t nv, const int32_t* vf_ptr, const int32_t* vf,
                                 const int32_t* tris, double* normals, hipStream_t s) {
    if (nv <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((nv + 255) / 256, 16384);
    hipLaunchKernelGGL(k_vertex_normals, dim3((unsigned)blocks), dim3(256), 0, s, x, nv, vf_ptr, vf, tris, normals);
    return hipGetLastError();
}

// ---- network pass --------------------------------------------------------------------------------
// feature channel c >= 7: the packed upper pair (i, j) of Packed<6>
__host__ __device__ constexpr int pair_i(int q) { return q < 6 ? 0 : q < 11 ? 1 : q < 15 ? 2 : q < 18 ? 3 : q < 20 ? 4 : 5; }
__host__ __device__ constexpr int pair_j(int q) {
    return q < 6 ? q : q < 11 ? q - 5 : q < 15 ? q - 9 : q < 18 ? q - 12 : q < 20 ? q - 14 : 5;
}
static_assert(Packed<6>::at(pair_i(13), pair_j(13)) == 13 && Packed<6>::at(pair_i(20), pair_j(20)) == 20,
              "pair tables follow Packed<6>");

// features z of triangle e (FP64): same formulas as the element term's shell_features
__device__ __forceinline__ void features_at(const MlpHeadLaunch& L, int64_t e, double (&z)[6]) {
    const int32_t* st = L.stencil + 3 * e;
    double xs[9], in[17];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xs[3 * s + c] = L.x[3 * (int64_t)st[s] + c];
            in[8 + 3 * s + c] = L.normals[3 * (int64_t)st[s] + c];
        }
#pragma unroll
    for (int k = 0; k < 8; ++k) in[k] = L.rest[(int64_t)k * L.n + e];
    double r[6];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        r[i] = xs[3 + i] - xs[i];
        r[3 + i] = xs[6 + i] - xs[i];
    }
    shell_features<double>(r, in, z);
}

// wave-scope ordering of LDS accesses between the lanes of one wave
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// three BF16 terms of an FP32 value (hi + mid + lo reproduces its 24 significand bits), stored
// into element j of three operand vectors
__device__ __forceinline__ void split3(float v, bf16x8& h, bf16x8& m, bf16x8& l, int j) {
    const __bf16 a = (__bf16)v;
    const float r = v - (float)a;
    const __bf16 b = (__bf16)r;
    h[j] = a;
    m[j] = b;
    l[j] = (__bf16)(r - (float)b);
}

// One wave evaluates 16 triangles at a time (one per MFMA column). With v = w3 * sigma(a2) and
// u = W2^T v, the network's derivatives with respect to the scaled features xh are
//   dpsi/dxh_i        = sum_k u_k sigma(a1_k) W1[k,i]
//   d2psi/dxh_i dxh_j = sum_k u_k sigma'(a1_k) W1[k,i] W1[k,j] + sum_m w3_m sigma'(a2_m) g_mi g_mj,
// g_mi = sum_k W2[m,k] sigma(a1_k) W1[k,i] (layer 2's first-order channels). Three groups of contractions run
// on the matrix cores (v_mfma_f32_16x16x32_bf16):
//   a2 - b2 = W2 sp(a1), g_i = W2 (sigma(a1) W1[:,i])   W2 exact in BF16 (held in registers as the A operand),
//                                                      the seven activation channels in three BF16 terms;
//   u = W2^T v                                         v in three BF16 terms, W2^T read from LDS;
//   S1[t,q] = sum_k (u sigma') C[k,q]                  C[k,q] = W1[k,i_q] W1[k,j_q] over the 21 packed pairs, a
//                                                      product of two BF16 values (16 significant bits: exactly
//                                                      two BF16 terms), built once per workgroup in LDS; u sigma'
//                                                      in three terms: the layer-1 part of the second derivatives.
// A product of three-term by two-term operands drops only the lo x lo part (2^-24 relative), so every
// contraction reproduces FP32 products with FP32 accumulation. The layer-2 part of the second derivatives (a
// rank-6 sum per triangle) and the first derivatives are per-triangle VALU work. (Moving the six first-order
// channels to constant operands G_i = W2 diag(W1[:,i]) in LDS, split once, cut the VALU instructions by a
// quarter but ran slower: at one wave per SIMD the extra MFMA chains and LDS reads were not hidden.)
// Layouts (16x16x32 MFMA): B operand lane l holds column l % 16 and k = 32 ks + 8 (l / 16) + j; A operand lane
// l holds row l % 16 and the same k; accumulators hold rows 4 (l / 16) + jj of column l % 16.
constexpr int kHeadWaves = 4;
constexpr int kLdsRow = kHid + 8;   // BF16 row stride of the LDS operand tables (144 B: 16-byte reads spread over banks)

struct HeadSmem {   // byte offsets into the network pass's dynamic LDS
    static constexpr int w1 = 0;                                   // float [64][6]
    static constexpr int b1 = w1 + kHid * 6 * 4;                   // float [64]
    static constexpr int b2 = b1 + kHid * 4;
    static constexpr int w3 = b2 + kHid * 4;
    static constexpr int w2t = w3 + kHid * 4;                      // bf16 [k][kLdsRow]: W2 transposed
    static constexpr int c = w2t + kHid * kLdsRow * 2;             // bf16 [2][32][kLdsRow]: C hi, lo (q >= 21: 0)
    static constexpr int t = c + 2 * 32 * kLdsRow * 2;             // float [waves][16][kHid + 1]
    static constexpr int bytes = t + kHeadWaves * 16 * (kHid + 1) * 4;
};
static_assert(HeadSmem::w2t % 16 == 0 && HeadSmem::c % 16 == 0 && HeadSmem::t % 16 == 0,
              "16-byte LDS operand reads");
static_assert(HeadSmem::bytes <= 160 * 1024, "network pass LDS fits a CU");
static_assert(kOffW2 % 8 == 0 && kHid % 8 == 0, "16-byte reads of W2 rows from the BF16 parameters");

// a product of two BF16 values (exact in FP32) as hi + lo BF16 terms, both exact
__device__ __forceinline__ void split2_exact(float p, uint16_t& hi, uint16_t& lo) {
    hi = f2bf(p);
    lo = f2bf(p - bf2f(hi));
}

__device__ __forceinline__ bf16x8 lds_bf16x8(const uint16_t* p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const short8*>(p));
}

__global__ __launch_bounds__(kHeadWaves * 64) void k_mlp_head(MlpHeadLaunch L) {
    extern __shared__ __align__(16) unsigned char head_smem[];
    float* sW1 = reinterpret_cast<float*>(head_smem + HeadSmem::w1);
    float* sB1 = reinterpret_cast<float*>(head_smem + HeadSmem::b1);
    float* sB2 = reinterpret_cast<float*>(head_smem + HeadSmem::b2);
    float* sW3 = reinterpret_cast<float*>(head_smem + HeadSmem::w3);
    uint16_t* sW2T = reinterpret_cast<uint16_t*>(head_smem + HeadSmem::w2t);
    uint16_t* sC = reinterpret_cast<uint16_t*>(head_smem + HeadSmem::c);
    for (int i = threadIdx.x; i < kHid * 6; i += blockDim.x) sW1[i] = bf2f(L.wbf[kOffW1 + i]);
    for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
        sB1[i] = bf2f(L.wbf[kOffB1 + i]);
        sB2[i] = bf2f(L.wbf[kOffB2 + i]);
        sW3[i] = bf2f(L.wbf[kOffW3 + i]);
    }
    for (int idx = threadIdx.x; idx < kHid * kHid; idx += blockDim.x)
        sW2T[(idx % kHid) * kLdsRow + idx / kHid] = L.wbf[kOffW2 + idx];
    for (int idx = threadIdx.x; idx < 32 * kHid; idx += blockDim.x) {
        const int q = idx / kHid, k = idx % kHid;
        const float p = q < 21 ? bf2f(L.wbf[kOffW1 + k * 6 + pair_i(q)]) * bf2f(L.wbf[kOffW1 + k * 6 + pair_j(q)]) : 0.0f;
        uint16_t hi, lo;
        split2_exact(p, hi, lo);
        sC[(0 * 32 + q) * kLdsRow + k] = hi;
        sC[(1 * 32 + q) * kLdsRow + k] = lo;
    }
    __syncthreads();
    const float b3 = bf2f(L.wbf[kOffB3]);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, col = lane & 15;
    float (*T)[kHid + 1] = reinterpret_cast<float (*)[kHid + 1]>(head_smem + HeadSmem::t) + wave * 16;
    // A operand (all seven forward channels): W2 rows m = 16 mt + col, k = 32 ks + 8 g + j, as 16-byte global
    // reads (the BF16 parameters are their own allocation, and kOffW2 and every row start are multiples of 8)
    short8 A[4][2];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
            A[mt][ks] = *reinterpret_cast<const short8*>(L.wbf + kOffW2 + (16 * mt + col) * kHid + 32 * ks + 8 * g);
    const int64_t tiles = (L.n + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * kHeadWaves + wave; tile < tiles;
         tile += (int64_t)gridDim.x * kHeadWaves) {
        const int64_t e = tile * 16 + col;
        const bool valid = e < L.n;
        float xh[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) xh[i] = valid ? L.xh[(int64_t)i * L.n + e] : 0.0f;
        // layer 1 at this lane's 16 units (B layout): sp(a1) and sigma(a1), each split into three BF16 terms
        float s1[2][8];
        bf16x8 b0h[2], b0m[2], b0l[2];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = 32 * ks + 8 * g + j;
                float a = sB1[k];
#pragma unroll
                for (int i = 0; i < 6; ++i) a = fmaf(sW1[k * 6 + i], xh[i], a);
                float sp, sg;
                softplus_logistic(a, sp, sg);
                s1[ks][j] = sg;
                split3(sp, b0h[ks], b0m[ks], b0l[ks], j);
            }
        // channel 0: the value through layer 2
        float P0 = 0.0f, PH[21];
#pragma unroll
        for (int q = 0; q < 21; ++q) PH[q] = 0.0f;
        float v[4][4], ws2p[4][4], a2g[6][4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const bf16x8 a = __builtin_bit_cast(bf16x8, A[mt][ks]);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0h[ks], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0m[ks], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0l[ks], acc, 0, 0, 0);
            }
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int m = 16 * mt + 4 * g + jj;
                const float a2 = acc[jj] + sB2[m];
                float sp, sg;
                softplus_logistic(a2, sp, sg);
                v[mt][jj] = sW3[m] * sg;
                ws2p[mt][jj] = sW3[m] * sg * (1.0f - sg);
                P0 = fmaf(sW3[m], sp, P0);
            }
        }
        // channels 1..6: g_i = W2 (sigma(a1) W1[:,i]), the B operand split per channel
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            bf16x8 bh[2], bm[2], bl[2];
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
#pragma unroll
                for (int j = 0; j < 8; ++j) split3(s1[ks][j] * sW1[(32 * ks + 8 * g + j) * 6 + i], bh[ks], bm[ks], bl[ks], j);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const bf16x8 a = __builtin_bit_cast(bf16x8, A[mt][ks]);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh[ks], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bm[ks], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl[ks], acc, 0, 0, 0);
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) a2g[i][mt][jj] = acc[jj];
            }
        }
        // second-order part through layer 2's nonlinearity: sum_m w3 sigma'(a2) g_mi g_mj
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    const float t = ws2p[mt][jj] * a2g[i][mt][jj];
#pragma unroll
                    for (int j2 = i; j2 < 6; ++j2) PH[Packed<6>::at(i, j2)] = fmaf(t, a2g[j2][mt][jj], PH[Packed<6>::at(i, j2)]);
                }
            }
        // u = W2^T v: v to LDS as [triangle][unit], read back as the A operand (rows = triangles)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) T[col][16 * mt + 4 * g + jj] = v[mt][jj];
        wave_sync();
        bf16x8 vh[2], vm[2], vl[2];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int j = 0; j < 8; ++j) split3(T[col][32 * ks + 8 * g + j], vh[ks], vm[ks], vl[ks], j);
        f32x4 U[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            U[nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                // B operand: W2[m][k], m = 32 ks + 8 g + j, k = 16 nt + col (a row of W2^T)
                const bf16x8 b = lds_bf16x8(sW2T + (16 * nt + col) * kLdsRow + 32 * ks + 8 * g);
                U[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vh[ks], b, U[nt], 0, 0, 0);
                U[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vm[ks], b, U[nt], 0, 0, 0);
                U[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vl[ks], b, U[nt], 0, 0, 0);
            }
        }
        wave_sync();   // every lane has read v before u overwrites it
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) T[4 * g + jj][16 * nt + col] = U[nt][jj];
        wave_sync();
        // first derivatives over this lane's 16 units; u sigma' split as the A operand of the layer-1
        // second-order contraction (rows = triangles, the same lane distribution as the B layout)
        float Pg[6] = {0, 0, 0, 0, 0, 0};
        bf16x8 uh[2], um[2], ul[2];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = 32 * ks + 8 * g + j;
                const float u = T[col][k];
                const float us = u * s1[ks][j];
#pragma unroll
                for (int i = 0; i < 6; ++i) Pg[i] = fmaf(us, sW1[k * 6 + i], Pg[i]);
                split3(us * (1.0f - s1[ks][j]), uh[ks], um[ks], ul[ks], j);
            }
        f32x4 S1[2];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            S1[nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const uint16_t* crow = sC + (16 * nt + col) * kLdsRow + 32 * ks + 8 * g;
                const bf16x8 ch = lds_bf16x8(crow), cl = lds_bf16x8(crow + 32 * kLdsRow);
                S1[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(uh[ks], ch, S1[nt], 0, 0, 0);
                S1[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(um[ks], ch, S1[nt], 0, 0, 0);
                S1[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ul[ks], ch, S1[nt], 0, 0, 0);
                S1[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(uh[ks], cl, S1[nt], 0, 0, 0);
                S1[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(um[ks], cl, S1[nt], 0, 0, 0);
            }
        }
        wave_sync();   // u is read before the layer-2 second derivatives overwrite it
        // sum over the four lanes holding the same triangle
        P0 += __shfl_xor(P0, 16);
        P0 += __shfl_xor(P0, 32);
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            Pg[i] += __shfl_xor(Pg[i], 16);
            Pg[i] += __shfl_xor(Pg[i], 32);
        }
#pragma unroll
        for (int q = 0; q < 21; ++q) {
            PH[q] += __shfl_xor(PH[q], 16);
            PH[q] += __shfl_xor(PH[q], 32);
        }
        if (g == 0) {
#pragma unroll
            for (int q = 0; q < 21; ++q) T[col][q] = PH[q];
        }
        if (valid && g == 0) {
            // back to z: dpsi/dz_i = s_out s_in[i] dpsi/dxh_i, likewise for the second derivatives
            L.psi[e] = L.s_out * (P0 + b3);
#pragma unroll
            for (int i = 0; i < 6; ++i) L.psi[(int64_t)(1 + i) * L.n + e] = L.s_out * L.s_in[i] * Pg[i];
        }
        wave_sync();
        // second derivatives: the layer-1 part (S1 rows = triangles 4 g + jj, column q = 16 nt + col) plus
        // the layer-2 part from LDS
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int q = 16 * nt + col;
            if (q < 21) {
                const float sc = L.s_out * L.s_in[pair_i(q)] * L.s_in[pair_j(q)];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int t = 4 * g + jj;
                    const int64_t et = tile * 16 + t;
                    if (et < L.n) L.psi[(int64_t)(7 + q) * L.n + et] = sc * (S1[nt][jj] + T[t][q]);
                }
            }
        }
        wave_sync();   // the layer-2 part is read before the next tile writes v
    }
}

__global__ __launch_bounds__(256) void k_mlp_features(MlpHeadLaunch L) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < L.n; e += (int64_t)gridDim.x * blockDim.x) {
        double z[6];
        features_at(L, e, z);
#pragma unroll
        for (int i = 0; i < 6; ++i) L.xh[(int64_t)i * L.n + e] = float(z[i]) * L.s_in[i];
    }
}

hipError_t launch_mlp_head(const MlpHeadLaunch& L, hipStream_t s) {
    if (L.n <= 0) return hipSuccess;
    {
        const int64_t blocks = std::min<int64_t>((L.n + 255) / 256, 16384);
        hipLaunchKernelGGL(k_mlp_features, dim3((unsigned)blocks), dim3(256), 0, s, L);
    }
    const int64_t tiles = (L.n + 15) / 16;
    const int64_t blocks = std::min<int64_t>((tiles + kHeadWaves - 1) / kHeadWaves, std::max(L.n_cu, 1));
    hipLaunchKernelGGL(k_mlp_head, dim3((unsigned)blocks), dim3(kHeadWaves * 64), HeadSmem::bytes, s, L);
    return hipGetLastError();
}

// ---- training ------------------------------------------------------------------------------------
// One wave per sample at a time, lane m = hidden unit m. Forward mode carries the six tangents
// d/dxh (xh = s_in * z) through both layers; reverse mode then differentiates
//   loss = (psi - W)^2 / (c_e B) + lam_g sum_i (dpsi/dz_i - dW_i)^2 / (c_g[i] B)   (B = batch size)
// with respect to every parameter. Each wave accumulates its samples' gradients in registers and
// writes one partial row; the rows are summed in a fixed order afterwards.
constexpr int kTrainBlock = 256;
constexpr int kW2Pad = kHid + 1;   // padded LDS rows: lane m reading row m is bank-conflict free

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ __launch_bounds__(kTrainBlock) void k_mlp_train(MlpTrainLaunch L) {
    __shared__ float sW2[kHid * kW2Pad];
    __shared__ float sX[kTrainBlock / 64][kHid][8];    // per wave: h1, T1 (6), pad
    __shared__ float sD[kTrainBlock / 64][kHid][8];    // per wave: delta2, G2a (6), pad
    for (int i = threadIdx.x; i < kHid * kHid; i += blockDim.x)
        sW2[(i / kHid) * kW2Pad + i % kHid] = L.params[kOffW2 + i];
    __syncthreads();
    const int m = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int gw = blockIdx.x * (blockDim.x >> 6) + wv;   // global wave
    float w1[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) w1[i] = L.params[kOffW1 + m * 6 + i];
    const float b1 = L.params[kOffB1 + m], b2 = L.params[kOffB2 + m], w3 = L.params[kOffW3 + m];
    const float b3 = L.params[kOffB3];
    float gW2[kHid];
#pragma unroll
    for (int k = 0; k < kHid; ++k) gW2[k] = 0.0f;
    float gW1[6] = {0, 0, 0, 0, 0, 0};
    float gb1 = 0.0f, gb2 = 0.0f, gw3 = 0.0f, gb3 = 0.0f, loss = 0.0f;
    const float inv_b = 1.0f / float(L.count);
    // every wave runs the same number of rounds (the block barriers below need it); a wave past the
    // end of the batch evaluates sample 0 of the batch with zero weight
    const int64_t rounds = (L.count + L.n_waves - 1) / L.n_waves;
    for (int64_t it = 0; it < rounds; ++it) {
        const int64_t q = gw + it * L.n_waves;
        const bool active = q < L.count;
        const int64_t qi = active ? q : 0;
        const int64_t smp = L.idx ? (int64_t)L.idx[L.base + qi] : L.base + qi;
        const float wgt = active ? inv_b : 0.0f;
        float xh[6], dWt[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            xh[i] = L.z[smp * 6 + i] * L.s_in[i];
            dWt[i] = L.dW[smp * 6 + i];
        }
        const float Wt = L.W[smp];
        // layer 1 (unit m)
        float a1 = b1;
#pragma unroll
        for (int i = 0; i < 6; ++i) a1 = fmaf(w1[i], xh[i], a1);
        const float h1 = softplusf(a1), d1 = logisticf(a1), d1p = d1 * (1.0f - d1);
        sX[wv][m][0] = h1;
#pragma unroll
        for (int i = 0; i < 6; ++i) sX[wv][m][1 + i] = d1 * w1[i];
        __syncthreads();
        // layer 2 (unit m): a2 = W2[m, :] h1 + b2, T2a[m, i] = W2[m, :] T1[:, i]
        float a2 = b2, t2a[6] = {0, 0, 0, 0, 0, 0};
        for (int k = 0; k < kHid; ++k) {
            const float w = sW2[m * kW2Pad + k];
            a2 = fmaf(w, sX[wv][k][0], a2);
#pragma unroll
            for (int i = 0; i < 6; ++i) t2a[i] = fmaf(w, sX[wv][k][1 + i], t2a[i]);
        }
        const float h2 = softplusf(a2), d2 = logisticf(a2), d2p = d2 * (1.0f - d2);
        // output: psi^ = w3 . h2 + b3, g^_i = w3 . (d2 T2a[:, i])
        const float ps = wave_sum(w3 * h2) + b3;
        float gh[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) gh[i] = wave_sum(w3 * d2 * t2a[i]);
        const float psi = L.s_out * ps;
        const float rr = 2.0f * (psi - Wt) * wgt / L.c_e * L.s_out;            // dloss / dpsi^
        float qq[6];
        float lg = 0.0f;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const float dz = L.s_out * L.s_in[i] * gh[i] - dWt[i];
            lg += dz * dz / L.c_g[i];
            qq[i] = 2.0f * L.lam_g * dz * wgt / L.c_g[i] * L.s_out * L.s_in[i];  // dloss / dg^_i
        }
        loss += ((psi - Wt) * (psi - Wt) / L.c_e + L.lam_g * lg) * wgt;
        // reverse through the output layer and layer 2's nonlinearity
        float qt = 0.0f, g2a[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            qt = fmaf(qq[i], t2a[i], qt);
            g2a[i] = d2 * w3 * qq[i];                 // dloss / dT2a[m, i]
        }
        gw3 += rr * h2 + d2 * qt;
        gb3 += rr;
        const float delta2 = d2p * w3 * qt + d2 * rr * w3;   // dloss / da2[m]
        gb2 += delta2;
        sD[wv][m][0] = delta2;
#pragma unroll
        for (int i = 0; i < 6; ++i) sD[wv][m][1 + i] = g2a[i];
        __syncthreads();
        // dW2[m, k] += delta2[m] h1[k] + sum_i G2a[m, i] T1[k, i]
#pragma unroll
        for (int k = 0; k < kHid; ++k) {
            float acc = delta2 * sX[wv][k][0];
#pragma unroll
            for (int i = 0; i < 6; ++i) acc = fmaf(g2a[i], sX[wv][k][1 + i], acc);
            gW2[k] += acc;
        }
        // unit k = m of layer 1: dh1[k] = sum_m W2[m, k] delta2[m], dT1[k, i] = sum_m W2[m, k] G2a[m, i]
        float dh1 = 0.0f, dT1[6] = {0, 0, 0, 0, 0, 0};
        for (int mm = 0; mm < kHid; ++mm) {
            const float w = sW2[mm * kW2Pad + m];
            dh1 = fmaf(w, sD[wv][mm][0], dh1);
#pragma unroll
            for (int i = 0; i < 6; ++i) dT1[i] = fmaf(w, sD[wv][mm][1 + i], dT1[i]);
        }
        float dd1 = 0.0f;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            dd1 = fmaf(w1[i], dT1[i], dd1);
            gW1[i] += d1 * dT1[i];                      // through T1 = d1 W1
        }
        const float delta1 = d1p * dd1 + d1 * dh1;     // dloss / da1[m]
        gb1 += delta1;
#pragma unroll
        for (int i = 0; i < 6; ++i) gW1[i] += delta1 * xh[i];
        __syncthreads();   // sX / sD are rewritten by the next sample
    }
    float* out = L.partial + (int64_t)gw * (kMlpParams + 1);
    if (gw < L.n_waves) {
#pragma unroll
        for (int i = 0; i < 6; ++i) out[kOffW1 + m * 6 + i] = gW1[i];
        out[kOffB1 + m] = gb1;
#pragma unroll
        for (int k = 0; k < kHid; ++k) out[kOffW2 + m * kHid + k] = gW2[k];
        out[kOffB2 + m] = gb2;
        out[kOffW3 + m] = gw3;
        if (m == 0) {
            out[kOffB3] = gb3;
            out[kMlpParams] = loss;
        }
    }
}

hipError_t launch_mlp_train(const MlpTrainLaunch& L, hipStream_t s) {
    const int per_block = kTrainBlock / 64;
    if (L.n_waves % per_block != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_train, dim3(L.n_waves / per_block), dim3(kTrainBlock), 0, s, L);
    return hipGetLastError();
}

__global__ void k_mlp_reduce(const float* partial, int n_waves, float* grad, float* loss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > kMlpParams) return;
    float acc = 0.0f;
    for (int w = 0; w < n_waves; ++w) acc += partial[(int64_t)w * (kMlpParams + 1) + i];
    if (i < kMlpParams) grad[i] = acc;
    else *loss = acc;
}

hipError_t launch_mlp_reduce(const float* partial, int n_waves, float* grad, float* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, s, partial, n_waves, grad,
                       loss);
    return hipGetLastError();
}

__global__ void k_mlp_adam(float* params, float* m, float* v, const float* grad, const int64_t* step, float lr,
                           float beta1, float beta2, float eps, uint16_t* wbf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kMlpParams) return;
    const float t = float(*step);
    const float g = grad[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * g;
    const float vi = beta2 * v[i] + (1.0f - beta2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - powf(beta1, t));
    const float vh = vi / (1.0f - powf(beta2, t));
    const float p = params[i] - lr * mh / (sqrtf(vh) + eps);
    params[i] = p;
    wbf[i] = f2bf(p);
}

hipError_t launch_mlp_adam(float* params, float* m, float* v, const float* grad, const int64_t* step, float lr,
                           float beta1, float beta2, float eps, uint16_t* wbf, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, params, m, v, grad, step, lr,
                       beta1, beta2, eps, wbf);
    return hipGetLastError();
}

__global__ void k_mlp_to_bf16(const float* params, uint16_t* wbf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kMlpParams) wbf[i] = f2bf(params[i]);
}

hipError_t launch_mlp_to_bf16(const float* params, uint16_t* wbf, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_to_bf16, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, params, wbf);
    return hipGetLastError();
}

__global__ void k_step_incr(int64_t* step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *step += 1;
}

hipError_t launch_mlp_step_incr(int64_t* step, hipStream_t s) {
    hipLaunchKernelGGL(k_step_incr, dim3(1), dim3(64), 0, s, step);
    return hipGetLastError();
}

}  // namespace mad
