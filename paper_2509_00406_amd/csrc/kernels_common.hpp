// Helpers shared by the assembly kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "element.hpp"
#include "mad_internal.hpp"
#include "terms.hpp"

namespace mad {

constexpr int kBlock = 256;

__device__ __forceinline__ void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }

// Finiteness by an integer test of the exponent bits, after an empty asm has hidden the value's
// origin: the element kernels are compiled with -ffinite-math-only (so that arithmetic on the
// structurally zero channels of the duals folds away), under which a floating-point test could be
// folded to "finite". The hardware still computes IEEE results; this reads them.
__device__ __forceinline__ bool finite(float v) {
    uint32_t u = __float_as_uint(v);
    asm volatile("" : "+v"(u));
    return (u & 0x7f800000u) != 0x7f800000u;
}
__device__ __forceinline__ bool finite(double v) {
    uint64_t u = (uint64_t)__double_as_longlong(v);
    asm volatile("" : "+v"(u));
    return (u & 0x7ff0000000000000ull) != 0x7ff0000000000000ull;
}

// triangle quality 4 sqrt(3) A / (l0^2 + l1^2 + l2^2): 1 for equilateral, 0 for degenerate
__device__ __forceinline__ double tri_quality3(const double* a, const double* b, const double* c) {
    const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    const double e3[3] = {c[0] - b[0], c[1] - b[1], c[2] - b[2]};
    const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double l2 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2] + e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2] +
                      e3[0] * e3[0] + e3[1] * e3[1] + e3[2] * e3[2];
    const double area2 = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    return l2 > 0.0 ? 2.0 * 1.7320508075688772 * area2 / l2 : 0.0;
}
__device__ __forceinline__ double tri_quality2(const double* a, const double* b, const double* c) {
    const double e1[2] = {b[0] - a[0], b[1] - a[1]}, e2[2] = {c[0] - a[0], c[1] - a[1]};
    const double e3[2] = {c[0] - b[0], c[1] - b[1]};
    const double l2 = e1[0] * e1[0] + e1[1] * e1[1] + e2[0] * e2[0] + e2[1] * e2[1] + e3[0] * e3[0] + e3[1] * e3[1];
    const double area2 = fabs(e1[0] * e2[1] - e1[1] * e2[0]);
    return l2 > 0.0 ? 2.0 * 1.7320508075688772 * area2 / l2 : 0.0;
}

// worst current-triangle quality of an element (diamonds: the worse of its two faces)
template <class Term> __device__ __forceinline__ double quality(const double* xs) {
    if constexpr (Term::NS == 3 && Term::D == 3) {
        return tri_quality3(xs, xs + 3, xs + 6);
    } else if constexpr (Term::NS == 3 && Term::D == 2) {
        return tri_quality2(xs, xs + 2, xs + 4);
    } else if constexpr (Term::NS == 4) {
        const double q1 = tri_quality3(xs, xs + 3, xs + 6);   // (x0, x1, x2)
        const double q2 = tri_quality3(xs, xs + 9, xs + 3);   // (x0, x3, x1)
        return q1 < q2 ? q1 : q2;
    } else {
        return 1.0;
    }
}

// Number of per-element inputs a term's energy reads: rest data, then (shell-feature terms) the
// three unit vertex normals, then (learned density) the 28 network outputs.
template <class Term> constexpr int n_inputs() {
    return (Term::NREST + Term::NAUX + Term::NPSI + Term::NVD) > 0 ? Term::NREST + Term::NAUX + Term::NPSI + Term::NVD
                                                                    : 1;
}

// Gather one element's inputs: rest SoA [NREST][n], normals [nv][3] at the element's global
// vertices gv[], network outputs SoA [28][n] (FP32), the caller's per-vertex data [nv][NVD] at gv[].
template <class Term>
__device__ __forceinline__ void gather_inputs(double (&in)[n_inputs<Term>()], const double* rest, int64_t n, int64_t e,
                                              const double* normals, const int* gv, const float* psi,
                                              const double* vdata) {
#pragma unroll
    for (int k = 0; k < Term::NREST; ++k) in[k] = rest[(int64_t)k * n + e];
    if constexpr (Term::NAUX > 0) {
#pragma unroll
        for (int s = 0; s < 3; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) in[Term::NREST + 3 * s + c] = normals[(int64_t)gv[s] * 3 + c];
    }
    if constexpr (Term::NPSI > 0) {
#pragma unroll
        for (int k = 0; k < Term::NPSI; ++k) in[Term::NREST + Term::NAUX + k] = double(psi[(int64_t)k * n + e]);
    }
    if constexpr (Term::NVD > 0) {
        constexpr int B = Term::NREST + Term::NAUX + Term::NPSI;
#pragma unroll
        for (int s = 0; s < Term::NS; ++s)
#pragma unroll
            for (int k = 0; k < Term::NVD; ++k) in[B + s * Term::NVD + k] = vdata[(int64_t)gv[s] * Term::NVD + k];
    }
}

// An element's outputs are all finite iff the sum of their magnitudes is (a NaN or an infinity
// anywhere reaches the sum; finite outputs cannot overflow it at the magnitudes that occur here).
template <class Term, typename T>
__device__ __forceinline__ bool out_finite(const ElemOut<Term, T>& o, int mode) {
    constexpr int NF = Term::NS * Term::D;
    T acc = T(0);
    if (mode >= 1) {
#pragma unroll
        for (int i = 0; i < NF; ++i) acc += fabs(o.g[i]);
    }
    if (mode >= 2) {
#pragma unroll
        for (int i = 0; i < Packed<Term::KR>::N; ++i) acc += fabs(o.hr[i]);
    }
    return finite(o.f) && finite(acc);
}

template <class Term, typename T, typename U>
__device__ __forceinline__ void convert_out(const ElemOut<Term, U>& in, ElemOut<Term, T>& out) {
    constexpr int NF = Term::NS * Term::D;
    out.f = in.f;
#pragma unroll
    for (int i = 0; i < NF; ++i) out.g[i] = T(in.g[i]);
#pragma unroll
    for (int i = 0; i < Packed<Term::KR>::N; ++i) out.hr[i] = T(in.hr[i]);
}

__device__ __forceinline__ void block_reduce_store(double v, double* red, double* out) {
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// sum of red[0, kBlock) in a fixed tree order, whatever the workgroup size (at least kBlock threads, all of
// them calling); red is already filled and visible to every lane
__device__ __forceinline__ void block_sum_store(double* red, double* out) {
#pragma unroll
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

}  // namespace mad
