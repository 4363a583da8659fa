// Device-wide atomic and colored assembly (Sec. 5.5, Sec. 6.2), the
// deterministic FP64 energy reduction, and a fill kernel for zeroing outputs.
//
// One kernel per term and one workgroup per patch: the patch's elements of
// that term are contiguous in the device arrays. Each lane evaluates whole
// elements with the local gradient and Hessian in registers, then adds every
// stencil entry to the global gradient / block-CSR values with hardware
// floating-point atomics (global_atomic_add_f32/_f64), as the paper does.
// The colored variant (PLAIN) runs one launch per color over chunks of
// elements of that color, which share no vertex, and adds with plain
// read-add-writes.
#include "kernels_common.hpp"

namespace mad {

// add into a global entry: a hardware atomic, or (colored scatter, PLAIN) a plain read-add-write
template <bool PLAIN, typename T>
__device__ __forceinline__ void global_add(T* p, T v) {
    if constexpr (PLAIN) *p += v;
    else atomic_add(p, v);
}

template <class Term, typename T, int MODE, bool PLAIN>
__device__ __forceinline__ void scatter_global(const ElemOut<Term, T>& o, const int* vs, int e, const EvalLaunch& L,
                                               bool want_grad) {
    constexpr int NS = Term::NS, D = Term::D;
    if (want_grad) {
        T* g = static_cast<T*>(L.grad);
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < D; ++c) global_add<PLAIN>(g + (int64_t)vs[s] * D + c, o.g[s * D + c]);
    }
    if constexpr (MODE >= 2) {
        const T te = T(L.eps > 0.0 ? L.eps : 0.0);
        if (L.hvp) {
            // matrix-free: y += H_j v_j
            T vl[NS * D], yl[NS * D];
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int c = 0; c < D; ++c) vl[s * D + c] = T(L.v[(int64_t)vs[s] * D + c]);
            hvp_apply<Term, MODE, T>(o, te, vl, yl);
            T* y = static_cast<T*>(L.y);
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int c = 0; c < D; ++c) global_add<PLAIN>(y + (int64_t)vs[s] * D + c, yl[s * D + c]);
            return;
        }
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
                        global_add<PLAIN>(blk + c * D + c2, hfull<Term, MODE>(o, s * D + c, t * D + c2, te));
            }
    }
}

template <class Term, typename T, int MODE, bool PLAIN>
__global__ __launch_bounds__(kBlock) void k_eval(EvalLaunch L) {
    constexpr int NS = Term::NS, D = Term::D, NF = NS * D;
    __shared__ double red[kBlock];
    const int p = (int)blockIdx.x + L.chunk0;
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
            for (int c = 0; c < D; ++c) {
                xs[s * D + c] = L.x[(int64_t)vs[s] * D + c];
                bad = bad || !finite(xs[s * D + c]);
            }
        double rest[n_inputs<Term>()];
        gather_inputs<Term>(rest, L.rest, L.n, e, L.normals, vs, L.psi, L.vdata);

        ElemOut<Term, T> o;
        if constexpr (MODE == 3 && sizeof(T) == 4) {
            // near-degenerate elements, or a projection that did not converge, redo in FP64
            bool fb = quality<Term>(xs) < L.qmin;
            if (!fb) fb = !element_eval<Term, T, MODE>(xs, rest, L.prm, L.eps, o);
            if (fb) {
                ElemOut<Term, double> o64;
                element_eval<Term, double, MODE>(xs, rest, L.prm, L.eps, o64);
                convert_out(o64, o);
                atomicAdd(L.fallbacks, 1ull);
            }
        } else {
            element_eval<Term, T, MODE>(xs, rest, L.prm, L.eps, o);
        }
        esum += o.f;
        bad = bad || !out_finite<Term, T>(o, MODE);
        if constexpr (MODE >= 1) scatter_global<Term, T, MODE, PLAIN>(o, vs, e, L, L.want_grad != 0);
    }
    if (bad) atomicOr(L.flags, 1);
    block_reduce_store(esum, red, L.partial + (L.slot_map ? L.slot_map[p] : p));
}

template <class Term, typename T, bool PLAIN>
static hipError_t launch_mode_t(const EvalLaunch& L, hipStream_t s) {
    dim3 grid(L.n_patch), block(kBlock);
    switch (L.mode) {
    case 0: hipLaunchKernelGGL((k_eval<Term, T, 0, PLAIN>), grid, block, 0, s, L); break;
    case 1: hipLaunchKernelGGL((k_eval<Term, T, 1, PLAIN>), grid, block, 0, s, L); break;
    case 2: hipLaunchKernelGGL((k_eval<Term, T, 2, PLAIN>), grid, block, 0, s, L); break;
    case 3: hipLaunchKernelGGL((k_eval<Term, T, 3, PLAIN>), grid, block, 0, s, L); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class Term, typename T>
static hipError_t launch_mode(const EvalLaunch& L, hipStream_t s) {
    return L.plain ? launch_mode_t<Term, T, true>(L, s) : launch_mode_t<Term, T, false>(L, s);
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
    case K_SHELL_TRI: return launch_prec<TermShellTri>(L, s);
    case K_MLP: return launch_prec<TermMLP>(L, s);
    case K_SPRING: return launch_prec<TermSpring>(L, s);
    case K_INERTIA: return launch_prec<TermInertia>(L, s);
    case K_RES_EDGE: return launch_prec<TermResEdge>(L, s);
    case K_RES_POSITION: return launch_prec<TermResPosition>(L, s);
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

// zero block list[i] (words 32-bit words each) of hess
__global__ void k_zero_blocks(uint32_t* hess, const int32_t* list, int64_t n, int words) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * words) return;
    const int64_t b = i / words;
    hess[(int64_t)list[b] * words + (i - b * words)] = 0u;
}

hipError_t launch_zero_blocks(void* hess, const int32_t* list, int64_t n, int dd, int elem_bytes, hipStream_t s) {
    const int words = dd * elem_bytes / 4;
    const int64_t total = n * words;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_blocks, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (uint32_t*)hess, list, n,
                       words);
    return hipGetLastError();
}

__global__ void k_zero_counters(int32_t* a, int32_t* b) {
    if (threadIdx.x == 0 && a) *a = 0;
    if (threadIdx.x == 1 && b) *b = 0;
}

hipError_t launch_zero_counters(int32_t* a, int32_t* b, hipStream_t s) {
    if (!a && !b) return hipSuccess;
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, a, b);
    return hipGetLastError();
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
// One workgroup per component: each lane sums a fixed strided subset in a fixed order, then a fixed
// tree. With several components a second one-workgroup pass sums the component energies the same way.
__global__ __launch_bounds__(kBlock) void k_energy_comp(const double* partial, int n_terms, int n_patch,
                                                        const int32_t* comp_patch_ptr, int batched, double* energy,
                                                        double* comp_out) {
    __shared__ double red[kBlock];
    const int c = blockIdx.x;
    const int pb = comp_patch_ptr[c], pe = comp_patch_ptr[c + 1];
    double acc = 0.0;
    for (int t = 0; t < n_terms; ++t) {
        const double* pt = partial + (int64_t)t * n_patch;
        int i = pb + (int)threadIdx.x;
        // eight loads in flight, then the additions in the same order as one at a time
        for (; i + 7 * kBlock < pe; i += 8 * kBlock) {
            double v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = pt[i + k * kBlock];
#pragma unroll
            for (int k = 0; k < 8; ++k) acc += v[k];
        }
        for (; i < pe; i += kBlock) acc += pt[i];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (batched) energy[1 + c] = red[0];
        if (gridDim.x == 1) energy[0] = red[0];
        else comp_out[c] = red[0];
    }
}

__global__ __launch_bounds__(kBlock) void k_energy_total(const double* comp, int n_comp, double* energy) {
    __shared__ double red[kBlock];
    double acc = 0.0;
    for (int i = (int)threadIdx.x; i < n_comp; i += kBlock) acc += comp[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) energy[0] = red[0];
}

hipError_t launch_energy_reduce(const double* partial, int n_terms, int n_patch, const int32_t* comp_patch_ptr,
                                int n_comp, bool batched, double* energy, double* comp_scratch, hipStream_t s) {
    hipLaunchKernelGGL(k_energy_comp, dim3(n_comp), dim3(kBlock), 0, s, partial, n_terms, n_patch, comp_patch_ptr,
                       batched ? 1 : 0, energy, comp_scratch);
    if (n_comp > 1) hipLaunchKernelGGL(k_energy_total, dim3(1), dim3(kBlock), 0, s, comp_scratch, n_comp, energy);
    return hipGetLastError();
}

}  // namespace mad
