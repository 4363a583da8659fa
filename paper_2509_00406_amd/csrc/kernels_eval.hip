// Element evaluation and atomic assembly kernels (Sec. 5.5, Sec. 6.2), the
// deterministic FP64 energy reduction, and a fill kernel for zeroing outputs.
//
// One workgroup per patch: the patch's elements of one term are contiguous in
// the device arrays, so a workgroup touches a compact set of vertices and its
// scattered updates stay in the local L2 slice. Each lane evaluates whole
// elements; the local gradient and Hessian live in registers; global updates
// are hardware floating-point atomic adds (global_atomic_add_f32/_f64).
#include <hip/hip_runtime.h>

#include "element.hpp"
#include "mad_internal.hpp"
#include "terms.hpp"

namespace mad {

constexpr int kBlock = 256;

__device__ __forceinline__ void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }

__device__ __forceinline__ bool finite(double v) { return isfinite(v); }

// triangle quality 4 sqrt(3) A / (l0^2 + l1^2 + l2^2), 1 for equilateral, 0 for degenerate
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

template <class Term, typename T>
__device__ __forceinline__ void scatter(const ElemOut<Term, T>& o, const int* vs, int e, const EvalLaunch& L,
                                        bool want_grad, bool want_hess) {
    constexpr int NS = Term::NS, D = Term::D, NF = NS * D;
    if (want_grad) {
        T* g = static_cast<T*>(L.grad);
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < D; ++c) atomic_add(g + (int64_t)vs[s] * D + c, o.g[s * D + c]);
    }
    if (want_hess) {
        T* h = static_cast<T*>(L.hess);
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                const int32_t slot = L.slots[(int64_t)(s * NS + t) * L.n + e];
                T* blk = h + (int64_t)slot * (D * D);
#pragma unroll
                for (int c = 0; c < D; ++c)
#pragma unroll
                    for (int c2 = 0; c2 < D; ++c2)
                        atomic_add(blk + c * D + c2, o.h[Packed<NF>::at(s * D + c, t * D + c2)]);
            }
    }
}

template <class Term, typename T>
__device__ __forceinline__ bool out_finite(const ElemOut<Term, T>& o, int mode) {
    constexpr int NF = Term::NS * Term::D;
    bool ok = finite(o.f);
    if (mode >= 1) {
#pragma unroll
        for (int i = 0; i < NF; ++i) ok = ok && finite(double(o.g[i]));
    }
    if (mode >= 2) {
#pragma unroll
        for (int i = 0; i < Packed<NF>::N; ++i) ok = ok && finite(double(o.h[i]));
    }
    return ok;
}

template <class Term, typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_eval(EvalLaunch L) {
    constexpr int NS = Term::NS, D = Term::D, NF = NS * D, NR = Term::NREST;
    __shared__ double red[kBlock];
    const int p = blockIdx.x;
    const int beg = L.elem_ptr[p], end = L.elem_ptr[p + 1];
    double esum = 0.0;
    bool bad = false;
    for (int e = beg + (int)threadIdx.x; e < end; e += kBlock) {
        int vs[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) vs[s] = L.stencil[(int64_t)e * NS + s];
        double xs[NF];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < D; ++c) xs[s * D + c] = L.x[(int64_t)vs[s] * D + c];
        double rest[NR > 0 ? NR : 1];
#pragma unroll
        for (int k = 0; k < NR; ++k) rest[k] = L.rest[(int64_t)k * L.n + e];

        ElemOut<Term, T> o;
        if constexpr (MODE == 3 && sizeof(T) == 4) {
            // FP32 path; near-degenerate elements (or a non-converged projection) redo in FP64
            bool fb = quality<Term>(xs) < L.qmin;
            if (!fb) fb = !element_eval<Term, T, MODE>(xs, rest, L.prm, L.eps, o);
            if (fb) {
                ElemOut<Term, double> o64;
                element_eval<Term, double, MODE>(xs, rest, L.prm, L.eps, o64);
                o.f = o64.f;
#pragma unroll
                for (int i = 0; i < NF; ++i) o.g[i] = T(o64.g[i]);
#pragma unroll
                for (int i = 0; i < Packed<NF>::N; ++i) o.h[i] = T(o64.h[i]);
                atomicAdd(L.fallbacks, 1ull);
            }
        } else {
            element_eval<Term, T, MODE>(xs, rest, L.prm, L.eps, o);
        }
        esum += o.f;
        bad = bad || !out_finite<Term, T>(o, MODE);
        if constexpr (MODE >= 1) scatter<Term, T>(o, vs, e, L, L.want_grad != 0, MODE >= 2);
    }
    if (bad) atomicOr(L.flags, 1);
    red[threadIdx.x] = esum;
    __syncthreads();
#pragma unroll
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) L.partial[p] = red[0];
}

template <class Term, typename T>
static hipError_t launch_mode(const EvalLaunch& L, hipStream_t s) {
    dim3 grid(L.n_patch), block(kBlock);
    switch (L.mode) {
    case 0: hipLaunchKernelGGL((k_eval<Term, T, 0>), grid, block, 0, s, L); break;
    case 1: hipLaunchKernelGGL((k_eval<Term, T, 1>), grid, block, 0, s, L); break;
    case 2: hipLaunchKernelGGL((k_eval<Term, T, 2>), grid, block, 0, s, L); break;
    case 3: hipLaunchKernelGGL((k_eval<Term, T, 3>), grid, block, 0, s, L); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class Term>
static hipError_t launch_prec(const EvalLaunch& L, hipStream_t s) {
    return L.prec == MAD_F32 ? launch_mode<Term, float>(L, s) : launch_mode<Term, double>(L, s);
}

hipError_t launch_eval(const EvalLaunch& L, hipStream_t s) {
    if (L.n_patch <= 0) return hipSuccess;
    switch (L.kind) {
    case K_EDGE_SQLEN: return launch_prec<TermEdgeSqlen>(L, s);
    case K_TRI_AREA: return launch_prec<TermTriArea>(L, s);
    case K_DIRICHLET: return launch_prec<TermDirichlet>(L, s);
    case K_STVK: return launch_prec<TermStVK>(L, s);
    case K_BENDING: return launch_prec<TermBending>(L, s);
    case K_SYMDIR: return launch_prec<TermSymDir>(L, s);
    default: return hipErrorInvalidValue;
    }
}

// ---- fused patch kernel: LDS staging and accumulation --------------------------------------------
// One workgroup per patch runs every term's elements of that patch. x of the patch's vertices is
// staged in LDS; element gradients and Hessian blocks are summed into LDS with LDS atomics
// (only upper blocks r <= c are kept; the lower block is the transpose); then each touched entry
// is written to HBM once: a plain store if no other patch touches it, else one atomic add.

__host__ __device__ constexpr size_t align16(size_t b) { return (b + 15) & ~size_t(15); }

template <typename T>
__device__ __forceinline__ void lds_add(T* p, T v) { atomicAdd(p, v); }

template <typename T>
__device__ __forceinline__ void flush_store(T* p, T v, bool excl) {
    if (excl) *p = v;
    else atomic_add(p, v);
}

template <class Term, typename T, int MODE>
__device__ __forceinline__ void patch_term(const PatchLaunch& L, const PatchTermArgs& A, int p, const double* sx,
                                           T* sg, T* sh, double& esum, bool& bad) {
    constexpr int NS = Term::NS, D = Term::D, NF = NS * D, NR = Term::NREST, DD = D * D;
    const int beg = A.elem_ptr[p], end = A.elem_ptr[p + 1];
    for (int e = beg + (int)threadIdx.x; e < end; e += kBlock) {
        int lv[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) lv[s] = A.lvert[(int64_t)s * A.n + e];
        double xs[NF];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < D; ++c) xs[s * D + c] = sx[lv[s] * D + c];
        double rest[NR > 0 ? NR : 1];
#pragma unroll
        for (int k = 0; k < NR; ++k) rest[k] = A.rest[(int64_t)k * A.n + e];
        ElemOut<Term, T> o;
        if constexpr (MODE == 3 && sizeof(T) == 4) {
            bool fb = quality<Term>(xs) < L.qmin;
            if (!fb) fb = !element_eval<Term, T, MODE>(xs, rest, A.prm, L.eps, o);
            if (fb) {
                ElemOut<Term, double> o64;
                element_eval<Term, double, MODE>(xs, rest, A.prm, L.eps, o64);
                o.f = o64.f;
#pragma unroll
                for (int i = 0; i < NF; ++i) o.g[i] = T(o64.g[i]);
#pragma unroll
                for (int i = 0; i < Packed<NF>::N; ++i) o.h[i] = T(o64.h[i]);
                atomicAdd(L.fallbacks, 1ull);
            }
        } else {
            element_eval<Term, T, MODE>(xs, rest, A.prm, L.eps, o);
        }
        esum += o.f;
        bad = bad || !out_finite<Term, T>(o, MODE);
        if constexpr (MODE >= 1) {
            if (L.want_grad) {
#pragma unroll
                for (int s = 0; s < NS; ++s)
#pragma unroll
                    for (int c = 0; c < D; ++c) lds_add(sg + lv[s] * D + c, o.g[s * D + c]);
            }
        }
        if constexpr (MODE >= 2) {
            int k = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int t = s; t < NS; ++t, ++k) {
                    const uint32_t w = A.lslot[(int64_t)k * A.n + e];
                    T* blk = sh + (int)(w & 0x3fffu) * DD;
                    const uint32_t flag = w >> 14;
#pragma unroll
                    for (int c = 0; c < D; ++c)
#pragma unroll
                        for (int c2 = 0; c2 < D; ++c2) {
                            const T v = o.h[Packed<NF>::at(s * D + c, t * D + c2)];
                            if (s == t) {
                                lds_add(blk + c * D + c2, v);
                            } else if (flag == 0u) {
                                lds_add(blk + c * D + c2, v);
                            } else if (flag == 1u) {
                                lds_add(blk + c2 * D + c, v);
                            } else {
                                lds_add(blk + c * D + c2, v);
                                lds_add(blk + c2 * D + c, v);
                            }
                        }
                }
        }
    }
}

template <typename T, int MODE, int D>
__global__ __launch_bounds__(kBlock) void k_eval_patch(PatchLaunch L) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kBlock];
    constexpr int DD = D * D;
    const int p = blockIdx.x;
    const int lv0 = L.lv_ptr[p], nlv = L.lv_ptr[p + 1] - lv0;
    const int lb0 = L.lb_ptr[p], nlb = L.lb_ptr[p + 1] - lb0;
    double* sx = reinterpret_cast<double*>(smem);
    T* sg = reinterpret_cast<T*>(smem + align16((size_t)nlv * D * sizeof(double)));
    T* sh = reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(sg) +
                                 (MODE >= 1 ? align16((size_t)nlv * D * sizeof(T)) : 0));
    for (int i = threadIdx.x; i < nlv * D; i += kBlock) {
        const int v = L.lv_global[lv0 + i / D];
        sx[i] = L.x[(int64_t)v * D + (i % D)];
        if constexpr (MODE >= 1) sg[i] = T(0);
    }
    if constexpr (MODE >= 2)
        for (int i = threadIdx.x; i < nlb * DD; i += kBlock) sh[i] = T(0);
    __syncthreads();

    double esum = 0.0;
    bool bad = false;
    for (int t = 0; t < L.n_terms; ++t) {
        const PatchTermArgs& A = L.terms[t];
        if constexpr (D == 3) {
            switch (A.kind) {
            case K_STVK: patch_term<TermStVK, T, MODE>(L, A, p, sx, sg, sh, esum, bad); break;
            case K_BENDING: patch_term<TermBending, T, MODE>(L, A, p, sx, sg, sh, esum, bad); break;
            case K_TRI_AREA: patch_term<TermTriArea, T, MODE>(L, A, p, sx, sg, sh, esum, bad); break;
            case K_EDGE_SQLEN: patch_term<TermEdgeSqlen, T, MODE>(L, A, p, sx, sg, sh, esum, bad); break;
            default: break;
            }
        } else if constexpr (D == 2) {
            if (A.kind == K_SYMDIR) patch_term<TermSymDir, T, MODE>(L, A, p, sx, sg, sh, esum, bad);
        } else {
            if (A.kind == K_DIRICHLET) patch_term<TermDirichlet, T, MODE>(L, A, p, sx, sg, sh, esum, bad);
        }
    }
    if (bad) atomicOr(L.flags, 1);
    __syncthreads();

    if constexpr (MODE >= 1) {
        if (L.want_grad) {
            T* G = static_cast<T*>(L.grad);
            for (int i = threadIdx.x; i < nlv * D; i += kBlock) {
                const int k = lv0 + i / D;
                flush_store(G + (int64_t)L.lv_global[k] * D + (i % D), sg[i], L.lv_excl[k] != 0);
            }
        }
    }
    if constexpr (MODE >= 2) {
        T* H = static_cast<T*>(L.hess);
        for (int i = threadIdx.x; i < nlb * DD; i += kBlock) {
            const int b = lb0 + i / DD, k = i % DD;
            const int32_t g = L.lb_gidx[b], gt = L.lb_gidxT[b];
            const bool ex = L.lb_excl[b] != 0;
            const T v = sh[i];
            flush_store(H + (int64_t)g * DD + k, v, ex);
            if (gt != g) flush_store(H + (int64_t)gt * DD + (k % D) * D + k / D, v, ex);
        }
    }
    red[threadIdx.x] = esum;
    __syncthreads();
#pragma unroll
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) L.partial[p] = red[0];
}

template <typename T, int D>
static size_t lds_for(int mode, int32_t max_lv, int32_t max_lb) {
    size_t b = align16((size_t)max_lv * D * sizeof(double));
    if (mode >= 1) b += align16((size_t)max_lv * D * sizeof(T));
    if (mode >= 2) b += (size_t)max_lb * D * D * sizeof(T);
    return b;
}

size_t patch_lds_bytes(int var_dim, int prec, int mode, int32_t max_lv, int32_t max_lb) {
    const bool f32 = prec == MAD_F32;
    switch (var_dim) {
    case 1: return f32 ? lds_for<float, 1>(mode, max_lv, max_lb) : lds_for<double, 1>(mode, max_lv, max_lb);
    case 2: return f32 ? lds_for<float, 2>(mode, max_lv, max_lb) : lds_for<double, 2>(mode, max_lv, max_lb);
    default: return f32 ? lds_for<float, 3>(mode, max_lv, max_lb) : lds_for<double, 3>(mode, max_lv, max_lb);
    }
}

template <typename T, int D>
static hipError_t launch_patch_mode(const PatchLaunch& L, hipStream_t s) {
    dim3 grid(L.n_patch), block(kBlock);
    const size_t sh = L.lds_bytes;
    switch (L.mode) {
    case 0: hipLaunchKernelGGL((k_eval_patch<T, 0, D>), grid, block, sh, s, L); break;
    case 1: hipLaunchKernelGGL((k_eval_patch<T, 1, D>), grid, block, sh, s, L); break;
    case 2: hipLaunchKernelGGL((k_eval_patch<T, 2, D>), grid, block, sh, s, L); break;
    case 3: hipLaunchKernelGGL((k_eval_patch<T, 3, D>), grid, block, sh, s, L); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_eval_patch(const PatchLaunch& L, hipStream_t s) {
    if (L.n_patch <= 0) return hipSuccess;
    const bool f32 = L.prec == MAD_F32;
    switch (L.var_dim) {
    case 1: return f32 ? launch_patch_mode<float, 1>(L, s) : launch_patch_mode<double, 1>(L, s);
    case 2: return f32 ? launch_patch_mode<float, 2>(L, s) : launch_patch_mode<double, 2>(L, s);
    case 3: return f32 ? launch_patch_mode<float, 3>(L, s) : launch_patch_mode<double, 3>(L, s);
    default: return hipErrorInvalidValue;
    }
}

// ---- fill ----------------------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}
__global__ void k_fill_u128(uint4* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

hipError_t launch_fill(void* ptr, int64_t n_elems, int elem_bytes, hipStream_t s) {
    const int64_t bytes = n_elems * elem_bytes;
    if (bytes <= 0) return hipSuccess;
    const int64_t n16 = ((uintptr_t)ptr % 16 == 0) ? bytes / 16 : 0;
    if (n16 > 0) {
        const int64_t blocks = std::min<int64_t>((n16 + 255) / 256, 8192);
        hipLaunchKernelGGL(k_fill_u128, dim3((unsigned)blocks), dim3(256), 0, s, (uint4*)ptr, n16);
    }
    const int64_t rem = (bytes - n16 * 16) / 4;
    if (rem > 0) {
        const int64_t blocks = std::min<int64_t>((rem + 255) / 256, 8192);
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)((char*)ptr + n16 * 16), rem);
    }
    return hipGetLastError();
}

// ---- deterministic FP64 energy reduction (Sec. 5.5 global reduction) ----------------------------
// partial[t * n_patch + p]; patches of component c are [comp_patch_ptr[c], comp_patch_ptr[c+1]).
// One workgroup; each lane sums a fixed strided subset in a fixed order, then a fixed tree.
__global__ __launch_bounds__(kBlock) void k_energy_reduce(const double* partial, int n_terms, int n_patch,
                                                          const int32_t* comp_patch_ptr, int n_comp, int batched,
                                                          double* energy) {
    __shared__ double red[kBlock];
    double total = 0.0;
    for (int c = 0; c < n_comp; ++c) {
        const int pb = comp_patch_ptr[c], pe = comp_patch_ptr[c + 1];
        const int np = pe - pb;
        double acc = 0.0;
        for (int t = 0; t < n_terms; ++t)
            for (int i = (int)threadIdx.x; i < np; i += kBlock) acc += partial[(int64_t)t * n_patch + pb + i];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            total += red[0];
            if (batched) energy[1 + c] = red[0];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) energy[0] = total;
}

hipError_t launch_energy_reduce(const double* partial, int n_terms, int n_patch, const int32_t* comp_patch_ptr,
                                int n_comp, bool batched, double* energy, hipStream_t s) {
    hipLaunchKernelGGL(k_energy_reduce, dim3(1), dim3(kBlock), 0, s, partial, n_terms, n_patch, comp_patch_ptr,
                       n_comp, batched ? 1 : 0, energy);
    return hipGetLastError();
}

}  // namespace mad
