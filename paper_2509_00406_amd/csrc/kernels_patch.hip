// Fused patch assembly: one workgroup per patch evaluates every term's
// elements of that patch (the term fusion the paper names as future work,
// Sec. 6 and Sec. 8), with the patch's vertex positions staged in LDS and the
// element gradients / Hessian blocks summed in LDS (only upper blocks r <= c
// are kept; the lower block is the transpose). Each entry only this patch
// touches is then written to HBM once with a plain store; an entry several
// patches touch is written to a halo slot per patch, and a gather kernel sums
// those slots in a fixed order and writes the entry once. No global atomics.
//
// FP32 elements that are near-degenerate (triangle quality below a threshold)
// or whose eigen-decomposition did not converge keep their FP64 energy here
// and are queued; a second, small kernel redoes their derivatives and clamp
// in FP64 and adds them with atomics.
#include "kernels_common.hpp"

namespace mad {

__host__ __device__ constexpr size_t align16(size_t b) { return (b + 15) & ~size_t(15); }

template <typename T>
__device__ __forceinline__ void lds_add(T* p, T v) { atomicAdd(p, v); }


// queued FP32 element: term << 29 | gradient-already-assembled << 28 | element
constexpr uint32_t kFbTermShift = 29;
constexpr uint32_t kFbGradDone = 1u << 28;
constexpr uint32_t kFbElemMask = kFbGradDone - 1u;

// One lock per workgroup over the patch's Hessian blocks in LDS: one wave at a time adds its unit's
// blocks. Lane 0 takes it for the whole wave (all lanes converged); it is released once the wave's
// LDS writes have completed. The spin is bounded (`spins` attempts, a launch parameter): past the bound
// the internal-error flag is raised and the wave adds nothing, so every wave ends and no block is ever
// added without the lock.
__device__ __forceinline__ bool wave_lock(int* lock, int32_t* flags, int spins) {
    for (int spin = 0; spin < spins; ++spin) {
        int got = 0;
        if ((threadIdx.x & 63) == 0) {
            int expected = 0;
            got = __hip_atomic_compare_exchange_strong(lock, &expected, 1, __ATOMIC_ACQUIRE, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP)
                      ? 1
                      : 0;
        }
        got = __shfl(got, 0);
        if (got) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            return true;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    if ((threadIdx.x & 63) == 0) atomicOr(flags + 1, kFlagLockTimeout);
    return false;
}

__device__ __forceinline__ void wave_unlock(int* lock, bool held) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (held && (threadIdx.x & 63) == 0) __hip_atomic_store(lock, 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// Add the Hessian blocks of the wave's elements (one per lane, `have` lanes only) into the patch's
// blocks in LDS with plain read-add-writes: the lanes of one segment touch disjoint blocks, the
// segments go one after another, and the lock keeps the other waves of the workgroup out. The block
// values are computed before the lock is taken; under it, a segment reads all its entries, then
// writes them back summed (one LDS round trip per segment). An element whose stencil names one
// vertex twice (two pairs landing in one block) makes the wave add pair by pair instead.
// Called by all 64 lanes of the wave together.
template <class Term, typename T, int MODE>
__device__ __forceinline__ void add_blocks(const PatchLaunch& L, const PatchTermArgs& A, int e, bool have,
                                           const ElemOut<Term, T>& o, T te, T* sh, int* lock) {
    constexpr int NS = Term::NS, D = Term::D, DD = D * D, NP = NS * (NS + 1) / 2;
    uint32_t wv[NP];
    int seg = -1;
    bool degen = false;
    if (have) {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            wv[k] = A.lslot[(int64_t)k * A.n + e];
            degen = degen || (wv[k] >> 14) == 2u;
        }
        seg = A.lseg[e];
    } else {
#pragma unroll
        for (int k = 0; k < NP; ++k) wv[k] = 0u;
    }
    const int nseg = wave_max(seg) + 1;
    if (nseg == 0) return;
    // entry (k, c, c2) of pair k: the diagonal pairs keep their upper half (c2 >= c)
    T hv[NP][DD];
    {
        int k = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int t = s; t < NS; ++t, ++k)
#pragma unroll
                for (int c = 0; c < D; ++c)
#pragma unroll
                    for (int c2 = 0; c2 < D; ++c2) {
                        if (s == t && c2 < c) continue;
                        hv[k][c * D + c2] = hfull<Term, MODE>(o, s * D + c, t * D + c2, te);
                    }
    }
    const bool held = wave_lock(lock, L.flags, L.lock_spins);
    if (!held) return;   // flagged: the evaluation's Hessian is reported invalid
    if (__ballot(degen) != 0ull) {
        // rare: some pair lands in a diagonal block without s == t; add pair by pair
        int k = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int t = s; t < NS; ++t, ++k) {
                T* blk = sh + (int)(wv[k] & 0x3fffu) * DD;
                const uint32_t flag = wv[k] >> 14;
                for (int g = 0; g < nseg; ++g) {
                    if (seg != g) continue;
                    if (s == t) {
#pragma unroll
                        for (int c = 0; c < D; ++c)
#pragma unroll
                            for (int c2 = c; c2 < D; ++c2) blk[c * D + c2] += hv[k][c * D + c2];
                    } else if (flag == 2u) {
#pragma unroll
                        for (int c = 0; c < D; ++c)
#pragma unroll
                            for (int c2 = c; c2 < D; ++c2) blk[c * D + c2] += hv[k][c * D + c2] + hv[k][c2 * D + c];
                    } else {
#pragma unroll
                        for (int c = 0; c < D; ++c)
#pragma unroll
                            for (int c2 = 0; c2 < D; ++c2)
                                blk[(flag == 1u) ? (c2 * D + c) : (c * D + c2)] += hv[k][c * D + c2];
                    }
                }
            }
    } else {
        for (int g = 0; g < nseg; ++g) {
            if (seg != g) continue;
            // row by row of the stencil's pairs (s, t >= s): read the row's blocks, then write them back
            // summed. Each block is read and written at fixed offsets from its base, so the compiler pairs
            // entries into two-address LDS instructions; a block stored as (c, r) (the transpose of the
            // element's (s, t) block) receives the transpose of the element's values instead.
            int k0 = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                T cur[NS][DD];
#pragma unroll
                for (int t = s; t < NS; ++t) {
                    const T* blk = sh + (int)(wv[k0 + (t - s)] & 0x3fffu) * DD;
#pragma unroll
                    for (int c = 0; c < D; ++c)
#pragma unroll
                        for (int c2 = 0; c2 < D; ++c2) {
                            if (s == t && c2 < c) continue;
                            cur[t][c * D + c2] = blk[c * D + c2];
                        }
                }
#pragma unroll
                for (int t = s; t < NS; ++t) {
                    const int k = k0 + (t - s);
                    T* blk = sh + (int)(wv[k] & 0x3fffu) * DD;
                    const bool tr = s != t && (wv[k] >> 14) == 1u;
#pragma unroll
                    for (int c = 0; c < D; ++c)
#pragma unroll
                        for (int c2 = 0; c2 < D; ++c2) {
                            if (s == t && c2 < c) continue;
                            blk[c * D + c2] = cur[t][c * D + c2] + (tr ? hv[k][c2 * D + c] : hv[k][c * D + c2]);
                        }
                }
                k0 += NS - s;
            }
        }
    }
    wave_unlock(lock, held);
}

// Element e (one per lane; lanes with e >= e_end have none) of one term of patch p. Called by all
// 64 lanes of a wave together (the Hessian blocks are added wave by wave, see add_blocks).
template <class Term, typename T, int MODE>
__device__ __forceinline__ void patch_term(const PatchLaunch& L, const PatchTermArgs& A, int term, int p, int e,
                                           int e_end, const double* sx, T* sg, T* sh, T* sy, int* lock, double& esum,
                                           bool& bad) {
    constexpr int NS = Term::NS, D = Term::D, NF = NS * D;
    const int lv0 = L.lv_ptr[p];
    const T te = T(L.eps > 0.0 ? L.eps : 0.0);
    ElemOut<Term, T> o{};
    bool blocks = false;   // this lane adds a Hessian into the patch's blocks
    if (e < e_end) {
        int lv[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) lv[s] = A.lvert[(int64_t)s * A.n + e];
        double xs[NF];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < D; ++c) xs[s * D + c] = sx[lv[s] * D + c];
        double rest[n_inputs<Term>()];
        if constexpr (Term::NAUX > 0 || Term::NVD > 0) {
            int gv[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) gv[s] = L.lv_global[lv0 + lv[s]];
            gather_inputs<Term>(rest, A.rest, A.n, e, L.normals, gv, A.psi, A.vdata);
        } else {
            gather_inputs<Term>(rest, A.rest, A.n, e, nullptr, nullptr, nullptr, nullptr);
        }
        if constexpr (MODE == 3) {
            // FP32: near-degenerate elements (quality below qmin) are queued whole for the FP64 redo.
            // Every other element assembles its gradient before the eigen-decomposition (so neither
            // it nor the inputs stay live across the Jacobi loop); an FP32 element whose
            // decomposition does not converge is queued for its Hessian only. The primal value (the
            // energy) is FP64 on every path, so the energy stays here and the reduction stays
            // deterministic.
            bool queued = false;
            if constexpr (sizeof(T) == 4) {
                if (quality<Term>(xs) < L.qmin) {
                    ElemOut<Term, double> op;
                    element_eval<Term, double, 0>(xs, rest, A.prm, L.eps, op);
                    esum += op.f;
                    bad = bad || !finite(op.f);
                    const int k = atomicAdd(L.fb_count, 1);
                    if (k < L.fb_cap) L.fb_list[k] = ((uint32_t)term << kFbTermShift) | (uint32_t)e;
                    atomicAdd(L.fallbacks, 1ull);
                    queued = true;
                }
            }
            if (!queued) {
                T Aq[Packed<Term::KR>::N];
                element_derivs<Term, T, 3>(xs, rest, A.prm, o, Aq);
                esum += o.f;
                {
                    T ga = T(0);
#pragma unroll
                    for (int i = 0; i < NF; ++i) ga += fabs(o.g[i]);
                    bad = bad || !finite(o.f) || !finite(ga);
                }
                if (L.want_grad) {
#pragma unroll
                    for (int s = 0; s < NS; ++s)
#pragma unroll
                        for (int c = 0; c < D; ++c) lds_add(sg + lv[s] * D + c, o.g[s * D + c]);
                }
                const bool conv = element_clamp<Term, T>(Aq, L.eps, o);
                if (sizeof(T) == 4 && !conv) {
                    const int k = atomicAdd(L.fb_count, 1);
                    if (k < L.fb_cap) L.fb_list[k] = ((uint32_t)term << kFbTermShift) | kFbGradDone | (uint32_t)e;
                    atomicAdd(L.fallbacks, 1ull);
                } else {
                    T ha = T(0);
#pragma unroll
                    for (int i = 0; i < Packed<Term::KR>::N; ++i) ha += fabs(o.hr[i]);
                    bad = bad || !finite(ha);
                    blocks = true;
                }
            }
        } else {
            element_eval<Term, T, MODE>(xs, rest, A.prm, L.eps, o);
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
            blocks = MODE >= 2;
        }
        if constexpr (MODE >= 2) {
            if (L.hvp && blocks) {
                // matrix-free: y += H_j v_j (sh holds the patch's v, sy its product)
                T vl[NF], yl[NF];
#pragma unroll
                for (int s = 0; s < NS; ++s)
#pragma unroll
                    for (int c = 0; c < D; ++c) vl[s * D + c] = sh[lv[s] * D + c];
                hvp_apply<Term, MODE, T>(o, te, vl, yl);
#pragma unroll
                for (int s = 0; s < NS; ++s)
#pragma unroll
                    for (int c = 0; c < D; ++c) lds_add(sy + lv[s] * D + c, yl[s * D + c]);
            }
        }
    }
    if constexpr (MODE >= 2) {
        if (!L.hvp) add_blocks<Term, T, MODE>(L, A, e, blocks, o, te, sh, lock);
    }
}

template <typename T, int MODE, int D, int FAM, int BLK>
__device__ __forceinline__ void eval_patch_one(const PatchLaunch& L, int p, unsigned char* smem, double* red,
                                               int* s_next, int* lock, int* s_terms) {
    constexpr int DD = D * D;
    const int lv0 = L.lv_ptr[p], nlv = L.lv_ptr[p + 1] - lv0;
    const int lb0 = L.lb_ptr[p], nlb = L.lb_ptr[p + 1] - lb0;
    double* sx = reinterpret_cast<double*>(smem);
    T* sg = reinterpret_cast<T*>(smem + align16((size_t)nlv * D * sizeof(double)));
    T* sh = reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(sg) +
                                 (MODE >= 1 ? align16((size_t)nlv * D * sizeof(T)) : 0));
    // matrix-free mode: the block area holds the patch's v, then its product y
    T* sy = (MODE >= 2 && L.hvp) ? sh + align16((size_t)nlv * D * sizeof(T)) / sizeof(T) : nullptr;
    if (threadIdx.x == 0) {
        *s_next = 0;
        *lock = 0;
    }
    // the patch's element range of each term, in unit order (read by every unit below)
    if (threadIdx.x < L.n_terms) {
        const int tt = L.term_order[threadIdx.x];
        const int b = L.terms[tt].elem_ptr[p];
        s_terms[2 * threadIdx.x] = b;
        s_terms[2 * threadIdx.x + 1] = L.terms[tt].elem_ptr[p + 1] - b;
    }
    if (threadIdx.x < kMaxPatchUnits) red[threadIdx.x] = 0.0;   // per-unit energies
    bool bad_x = false;
    // one vertex per thread: its index read once, its D coordinates loaded together
    for (int i = threadIdx.x; i < nlv; i += BLK) {
        const int64_t v = L.lv_global[lv0 + i];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const double xv = L.x[v * D + c];
            sx[i * D + c] = xv;
            bad_x = bad_x || !finite(xv);
            if constexpr (MODE >= 1) sg[i * D + c] = T(0);
            if constexpr (MODE >= 2) {
                if (L.hvp) {
                    sh[i * D + c] = T(L.v[v * D + c]);
                    sy[i * D + c] = T(0);
                }
            }
        }
    }
    if (bad_x) atomicOr(L.flags, 1);
    if constexpr (MODE >= 2) {
        if (!L.hvp) {
            // 16-byte LDS writes (the block area starts 16-byte aligned), then the tail
            const int nw = nlb * DD;
            float4* sh4 = reinterpret_cast<float4*>(sh);
            const int n4 = (nw * (int)sizeof(T)) / 16;
            for (int i = threadIdx.x; i < n4; i += BLK) sh4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            for (int i = n4 * (16 / (int)sizeof(T)) + threadIdx.x; i < nw; i += BLK) sh[i] = T(0);
        }
    }
    __syncthreads();

    bool bad = false;
    // Work units are chunks of 64 consecutive elements of one term; each wave takes the next unit from
    // an LDS counter, the costliest terms' units first (greedy list scheduling: a wave that finishes
    // early takes more units, so the four waves of the patch end close together). Which wave runs a
    // unit varies from run to run, so each unit's energy is summed over its lanes in a fixed order
    // into a slot of its own, and the slots are summed in a fixed order at the end.
    static_assert(kMaxPatchUnits <= BLK, "one energy slot per unit");
    const int lane = threadIdx.x & 63;
    for (;;) {
        int u = 0;
        if (lane == 0) u = atomicAdd(s_next, 1);
        u = __builtin_amdgcn_readfirstlane(__shfl(u, 0));
        const int unit = u;
        double esum = 0.0;
        int t = -1, first = 0, last = 0;
        for (int k = 0; k < L.n_terms; ++k) {
            const int b = s_terms[2 * k], n = s_terms[2 * k + 1];
            const int nc = (n + 63) >> 6;
            if (u < nc) {
                t = L.term_order[k];
                first = b + (u << 6);
                last = min(b + n, first + 64);
                break;
            }
            u -= nc;
        }
        // the same for every lane of the wave: kept in scalar registers, so the term's arguments are
        // scalar loads and the dispatch below a scalar branch
        t = __builtin_amdgcn_readfirstlane(t);
        first = __builtin_amdgcn_readfirstlane(first);
        last = __builtin_amdgcn_readfirstlane(last);
        if (t < 0) break;
        const PatchTermArgs& A = L.terms[t];
        const int e0 = first + lane;
        if constexpr (D == 3) {
            switch (A.kind) {
            case K_EDGE_SQLEN:
                patch_term<TermEdgeSqlen, T, MODE>(L, A, t, p, e0, last, sx, sg, sh, sy, lock, esum, bad);
                break;
            case K_SPRING: patch_term<TermSpring, T, MODE>(L, A, t, p, e0, last, sx, sg, sh, sy, lock, esum, bad); break;
            case K_RES_EDGE:
                patch_term<TermResEdge, T, MODE>(L, A, t, p, e0, last, sx, sg, sh, sy, lock, esum, bad);
                break;
            case K_RES_POSITION:
                patch_term<TermResPosition, T, MODE>(L, A, t, p, e0, last, sx, sg, sh, sy, lock, esum, bad);
                break;
            case K_INERTIA:
                patch_term<TermInertia, T, MODE>(L, A, t, p, e0, last, sx, sg, sh, sy, lock, esum, bad);
                break;
            case K_STVK:
                if constexpr (FAM != 2) patch_term<TermStVK, T, MODE>(L, A, t, p, e0, last, sx, sg, sh, sy, lock, esum, bad);
                break;
            case K_BENDING:
                if constexpr (FAM != 2) patch_term<TermBending, T, MODE>(L, A, t, p, e0, last, sx, sg, sh, sy, lock, esum, bad);
                break;
            case K_TRI_AREA:
                if constexpr (FAM != 2) patch_term<TermTriArea, T, MODE>(L, A, t, p, e0, last, sx, sg, sh, sy, lock, esum, bad);
                break;
            case K_SHELL_TRI:
                if constexpr (FAM == 1) patch_term<TermShellTri, T, MODE>(L, A, t, p, e0, last, sx, sg, sh, sy, lock, esum, bad);
                break;
            case K_MLP:
                if constexpr (FAM == 1) patch_term<TermMLP, T, MODE>(L, A, t, p, e0, last, sx, sg, sh, sy, lock, esum, bad);
                break;
            default: break;
            }
        } else if constexpr (D == 2) {
            if (A.kind == K_SYMDIR)
                patch_term<TermSymDir, T, MODE>(L, A, t, p, e0, last, sx, sg, sh, sy, lock, esum, bad);
        } else {
            if (A.kind == K_DIRICHLET)
                patch_term<TermDirichlet, T, MODE>(L, A, t, p, e0, last, sx, sg, sh, sy, lock, esum, bad);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) esum += __shfl_down(esum, o);
        if (lane == 0 && unit < kMaxPatchUnits) red[unit] = esum;
    }
    if (bad) atomicOr(L.flags, 1);
    __syncthreads();

    // flush: entries only this patch touches go straight to the output; shared entries go to their
    // halo slot and are summed by the gather kernel
    // one vertex's D gradient entries, or one row of a D x D block, per thread: the patch's index lists
    // are read once per vertex / block row, and each thread writes D consecutive values
    if constexpr (MODE >= 1) {
        if (L.want_grad) {
            T* G = static_cast<T*>(L.grad);
            T* HG = static_cast<T*>(L.halo_g);
            for (int i = threadIdx.x; i < nlv; i += BLK) {
                const int32_t h = L.lv_halo[lv0 + i];
                T* dst = h < 0 ? G + (int64_t)L.lv_global[lv0 + i] * D : HG + (int64_t)h * D;
#pragma unroll
                for (int c = 0; c < D; ++c) dst[c] = sg[i * D + c];
            }
        }
    }
    if constexpr (MODE >= 2) {
        if (L.hvp) {
            T* Y = static_cast<T*>(L.y);
            T* HY = static_cast<T*>(L.halo_y);
            for (int i = threadIdx.x; i < nlv * D; i += BLK) {
                const int k = lv0 + i / D, c = i % D;
                const int32_t h = L.lv_halo[k];
                if (h < 0) Y[(int64_t)L.lv_global[k] * D + c] = sy[i];
                else HY[(int64_t)h * D + c] = sy[i];
            }
        }
    }
    if constexpr (MODE >= 2) {
        if (L.hvp) {
            block_sum_store(red, L.partial + p);
            return;
        }
        T* H = static_cast<T*>(L.hess);
        T* HH = static_cast<T*>(L.halo_h);
        for (int i = threadIdx.x; i < nlb * D; i += BLK) {
            const int bl = i / D, r = i % D;
            const int32_t h = L.lb_halo[lb0 + bl];
            const int32_t g = L.lb_gidx[lb0 + bl], gt = L.lb_gidxT[lb0 + bl];
            const T* blk = sh + bl * DD;
            // row r of the block; a diagonal block keeps only its upper half in LDS
            T row[D];
#pragma unroll
            for (int c = 0; c < D; ++c) row[c] = (g == gt && c < r) ? blk[c * D + r] : blk[r * D + c];
            T* dst = h >= 0 ? HH + (int64_t)h * DD + r * D : H + (int64_t)g * DD + r * D;
#pragma unroll
            for (int c = 0; c < D; ++c) dst[c] = row[c];
            if (h < 0 && gt != g) {
                // row r of the transposed block (c, r) is column r of this one
                T* dt = H + (int64_t)gt * DD + r * D;
#pragma unroll
                for (int c = 0; c < D; ++c) dt[c] = blk[c * D + r];
            }
        }
    }
    block_sum_store(red, L.partial + p);
}

// One patch per workgroup, or (persistent) a grid sized to the device whose workgroups take
// patches from a counter in the given order (largest first) until every patch is taken.
template <typename T, int MODE, int D, int FAM, int BLK>
__device__ __forceinline__ void eval_patch_body(const PatchLaunch& L) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kMaxPatchUnits];
    __shared__ int next, unit_next, block_lock;
    __shared__ int term_range[2 * sizeof(PatchLaunch::term_order) / sizeof(int)];   // (first, count) per term
    if (!L.persistent) {
        eval_patch_one<T, MODE, D, FAM, BLK>(L, blockIdx.x, smem, red, &unit_next, &block_lock, term_range);
        return;
    }
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(L.work_counter, 1);
        __syncthreads();
        const int k = next;
        __syncthreads();   // every lane has read `next` before it is overwritten
        if (k >= L.n_patch) break;
        eval_patch_one<T, MODE, D, FAM, BLK>(L, L.work_order[k], smem, red, &unit_next, &block_lock, term_range);
        __syncthreads();   // the flush has read LDS before the next patch clears it
    }
}

// FAM: the term family compiled into an instantiation. 0: the catalogue; 1: the catalogue and the
// shell-feature terms (analytic and learned per-triangle densities), whose register needs would
// otherwise burden the catalogue's kernel; 2: light terms only (edge, spring, vertex and residual
// terms: 3 x 3 reduced Hessians), held to fewer registers for more waves per SIMD, since such
// elements wait on memory more than they compute.
// FP32 families 0 and 1: the compiler is held to 256 registers so two waves share each SIMD (the
// second wave hides the latency of the long dependent rotation chains).
// BLK: threads per workgroup (the tile): 256 (four waves; two workgroups share a CU) or, for FP32, 512
// (eight waves; one workgroup holds the CU's LDS for larger patches, or two light workgroups share it).
template <int MODE, int D, int FAM, int BLK>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(2))) void k_eval_patch_f32(PatchLaunch L) {
    eval_patch_body<float, MODE, D, FAM, BLK>(L);
}
template <int MODE, int D, int BLK>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(4))) void k_eval_patch_light_f32(PatchLaunch L) {
    eval_patch_body<float, MODE, D, 2, BLK>(L);
}
template <int MODE, int D, int FAM>
__global__ __launch_bounds__(kBlock) void k_eval_patch_f64(PatchLaunch L) {
    eval_patch_body<double, MODE, D, FAM, kBlock>(L);
}

// ---- gather of shared entries --------------------------------------------------------------------
template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_gather(GatherLaunch G) {
    constexpr int DD = D * D;
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x, stride = (int64_t)gridDim.x * kBlock;
    if (G.want_hess) {
        // one shared block per lane: its index lists read once, each halo partial read whole, the sum and its
        // transpose written row by row (the partials are summed in slot order, as for every entry before)
        T* H = static_cast<T*>(G.hess);
        const T* HH = static_cast<const T*>(G.halo_h);
        for (int64_t b = tid; b < (int64_t)G.n_gb; b += stride) {
            T v[DD];
#pragma unroll
            for (int k = 0; k < DD; ++k) v[k] = T(0);
            for (int j = G.gb_ptr[b]; j < G.gb_ptr[b + 1]; ++j) {
                const T* src = HH + (int64_t)G.gb_src[j] * DD;
#pragma unroll
                for (int k = 0; k < DD; ++k) v[k] += src[k];
            }
            const int32_t g = G.gb_gidx[b], gt = G.gb_gidxT[b];
            T* dst = H + (int64_t)g * DD;
#pragma unroll
            for (int k = 0; k < DD; ++k) dst[k] = v[k];
            if (gt != g) {
                T* dt = H + (int64_t)gt * DD;
#pragma unroll
                for (int r = 0; r < D; ++r)
#pragma unroll
                    for (int c = 0; c < D; ++c) dt[r * D + c] = v[c * D + r];
            }
        }
        for (int64_t i = tid; i < (int64_t)G.n_orphan_block * DD; i += stride)
            H[(int64_t)G.orphan_block[i / DD] * DD + i % DD] = T(0);
    }
    if (G.want_grad) {
        T* GR = static_cast<T*>(G.grad);
        const T* HG = static_cast<const T*>(G.halo_g);
        for (int64_t b = tid; b < (int64_t)G.n_gv; b += stride) {
            T v[D];
#pragma unroll
            for (int c = 0; c < D; ++c) v[c] = T(0);
            for (int j = G.gv_ptr[b]; j < G.gv_ptr[b + 1]; ++j) {
                const T* src = HG + (int64_t)G.gv_src[j] * D;
#pragma unroll
                for (int c = 0; c < D; ++c) v[c] += src[c];
            }
            T* dst = GR + (int64_t)G.gv_vert[b] * D;
#pragma unroll
            for (int c = 0; c < D; ++c) dst[c] = v[c];
        }
        for (int64_t i = tid; i < (int64_t)G.n_orphan_vert * D; i += stride)
            GR[(int64_t)G.orphan_vert[i / D] * D + i % D] = T(0);
    }
}

template <typename T>
static hipError_t launch_gather_t(const GatherLaunch& G, hipStream_t s) {
    const int64_t work = std::max<int64_t>({(int64_t)G.n_gb, (int64_t)G.n_gv, (int64_t)G.n_orphan_block * G.var_dim *
                                                                              G.var_dim});
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + kBlock - 1) / kBlock, 8192));
    switch (G.var_dim) {
    case 1: hipLaunchKernelGGL((k_gather<T, 1>), dim3(blocks), dim3(kBlock), 0, s, G); break;
    case 2: hipLaunchKernelGGL((k_gather<T, 2>), dim3(blocks), dim3(kBlock), 0, s, G); break;
    case 3: hipLaunchKernelGGL((k_gather<T, 3>), dim3(blocks), dim3(kBlock), 0, s, G); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gather(const GatherLaunch& G, hipStream_t s) {
    if (!G.want_grad && !G.want_hess) return hipSuccess;
    return G.prec == MAD_F32 ? launch_gather_t<float>(G, s) : launch_gather_t<double>(G, s);
}

// ---- FP64 redo of queued FP32 elements -----------------------------------------------------------
__device__ __forceinline__ int32_t find_block(const int32_t* rowptr, const int32_t* colidx, int32_t r, int32_t c) {
    int32_t lo = rowptr[r], hi = rowptr[r + 1] - 1;
    while (lo <= hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        const int32_t m = colidx[mid];
        if (m == c) return mid;
        if (m < c) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

template <class Term>
__device__ __forceinline__ void fallback_elem(const FallbackLaunch& F, const FallbackTerm& A, int e, bool grad_done) {
    constexpr int NS = Term::NS, D = Term::D, NF = NS * D, DD = D * D;
    int vs[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) vs[s] = A.stencil[(int64_t)e * NS + s];
    double xs[NF];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int c = 0; c < D; ++c) xs[s * D + c] = F.x[(int64_t)vs[s] * D + c];
    double rest[n_inputs<Term>()];
    gather_inputs<Term>(rest, A.rest, A.n, e, F.normals, vs, A.psi, A.vdata);
    ElemOut<Term, double> o;
    element_eval<Term, double, 3>(xs, rest, A.prm, F.eps, o);
    if (!out_finite<Term, double>(o, 3)) atomicOr(F.flags, 1);
    if (F.want_grad && !grad_done) {
        float* G = static_cast<float*>(F.grad);
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < D; ++c) atomic_add(G + (int64_t)vs[s] * D + c, float(o.g[s * D + c]));
    }
    const double te = F.eps > 0.0 ? F.eps : 0.0;
    if (F.hvp) {
        // matrix-free: add H_j v_j to y
        double vl[NF], yl[NF];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < D; ++c) vl[s * D + c] = F.v[(int64_t)vs[s] * D + c];
        hvp_apply<Term, 3, double>(o, te, vl, yl);
        float* Y = static_cast<float*>(F.y);
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < D; ++c) atomic_add(Y + (int64_t)vs[s] * D + c, float(yl[s * D + c]));
        return;
    }
    float* H = static_cast<float*>(F.hess);
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            const int32_t b = find_block(F.rowptr, F.colidx, vs[s], vs[t]);
            if (b < 0) {
                atomicOr(F.flags + 1, kFlagRedoBlockMissing);
                continue;
            }
#pragma unroll
            for (int c = 0; c < D; ++c)
#pragma unroll
                for (int c2 = 0; c2 < D; ++c2)
                    atomic_add(H + (int64_t)b * DD + c * D + c2, float(hfull<Term, 3>(o, s * D + c, t * D + c2, te)));
        }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_fallback(FallbackLaunch F) {
    const int queued = *F.fb_count;
    const int cnt = min(queued, F.fb_cap);
    // a queue smaller than the number of queued elements dropped some: the evaluation is not valid
    if (queued > F.fb_cap && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(F.flags + 1, kFlagQueueOverflow);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < cnt; i += gridDim.x * kBlock) {
        const uint32_t w = F.fb_list[i];
        const int t = (int)(w >> kFbTermShift), e = (int)(w & kFbElemMask);
        const bool grad_done = (w & kFbGradDone) != 0;
        const FallbackTerm& A = F.terms[t];
        if constexpr (D == 3) {
            switch (A.kind) {
            case K_STVK: fallback_elem<TermStVK>(F, A, e, grad_done); break;
            case K_BENDING: fallback_elem<TermBending>(F, A, e, grad_done); break;
            case K_TRI_AREA: fallback_elem<TermTriArea>(F, A, e, grad_done); break;
            case K_EDGE_SQLEN: fallback_elem<TermEdgeSqlen>(F, A, e, grad_done); break;
            case K_SPRING: fallback_elem<TermSpring>(F, A, e, grad_done); break;
            case K_INERTIA: fallback_elem<TermInertia>(F, A, e, grad_done); break;
            case K_RES_EDGE: fallback_elem<TermResEdge>(F, A, e, grad_done); break;
            case K_RES_POSITION: fallback_elem<TermResPosition>(F, A, e, grad_done); break;
            case K_SHELL_TRI: fallback_elem<TermShellTri>(F, A, e, grad_done); break;
            case K_MLP: fallback_elem<TermMLP>(F, A, e, grad_done); break;
            default: break;
            }
        } else if constexpr (D == 2) {
            if (A.kind == K_SYMDIR) fallback_elem<TermSymDir>(F, A, e, grad_done);
        } else {
            if (A.kind == K_DIRICHLET) fallback_elem<TermDirichlet>(F, A, e, grad_done);
        }
    }
}

// ---- launchers ----------------------------------------------------------------------------------
template <typename T, int D>
static size_t lds_for(int mode, int32_t max_lv, int32_t max_lb, bool hvp) {
    size_t b = align16((size_t)max_lv * D * sizeof(double));
    if (mode >= 1) b += align16((size_t)max_lv * D * sizeof(T));
    if (mode >= 2) b += hvp ? 2 * align16((size_t)max_lv * D * sizeof(T)) : (size_t)max_lb * D * D * sizeof(T);
    return b;
}

size_t patch_lds_bytes(int var_dim, int prec, int mode, int32_t max_lv, int32_t max_lb, bool hvp) {
    const bool f32 = prec == MAD_F32;
    switch (var_dim) {
    case 1: return f32 ? lds_for<float, 1>(mode, max_lv, max_lb, hvp) : lds_for<double, 1>(mode, max_lv, max_lb, hvp);
    case 2: return f32 ? lds_for<float, 2>(mode, max_lv, max_lb, hvp) : lds_for<double, 2>(mode, max_lv, max_lb, hvp);
    default: return f32 ? lds_for<float, 3>(mode, max_lv, max_lb, hvp) : lds_for<double, 3>(mode, max_lv, max_lb, hvp);
    }
}

// workgroups of a persistent launch: as many as are resident on the device at once
template <typename K>
static int persistent_grid(K kernel, const PatchLaunch& L, int blk) {
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, blk, L.lds_bytes) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return std::max(1, std::min(L.n_patch, std::max(L.n_cu, 1) * per_cu));
}

template <int MODE, int D, int FAM, int BLK>
static void launch_patch_f32(const PatchLaunch& L, hipStream_t s) {
    const dim3 block(BLK);
    if constexpr (FAM == 2) {
        const dim3 grid(L.persistent ? persistent_grid(k_eval_patch_light_f32<MODE, D, BLK>, L, BLK) : L.n_patch);
        hipLaunchKernelGGL((k_eval_patch_light_f32<MODE, D, BLK>), grid, block, L.lds_bytes, s, L);
    } else {
        const dim3 grid(L.persistent ? persistent_grid(k_eval_patch_f32<MODE, D, FAM, BLK>, L, BLK) : L.n_patch);
        hipLaunchKernelGGL((k_eval_patch_f32<MODE, D, FAM, BLK>), grid, block, L.lds_bytes, s, L);
    }
}

template <int MODE, int D, int FAM>
static void launch_patch_variant(bool f32, const PatchLaunch& L, hipStream_t s) {
    if (f32) {
        if (L.block == 512) launch_patch_f32<MODE, D, FAM, 512>(L, s);
        else launch_patch_f32<MODE, D, FAM, kBlock>(L, s);
    } else {
        const dim3 grid(L.persistent ? persistent_grid(k_eval_patch_f64<MODE, D, FAM>, L, kBlock) : L.n_patch);
        hipLaunchKernelGGL((k_eval_patch_f64<MODE, D, FAM>), grid, dim3(kBlock), L.lds_bytes, s, L);
    }
}

template <int MODE, int D>
static void launch_patch_kernel(bool f32, const PatchLaunch& L, hipStream_t s) {
    if constexpr (D == 3) {
        if (L.shell) {
            launch_patch_variant<MODE, D, 1>(f32, L, s);
            return;
        }
        if (L.light) {
            launch_patch_variant<MODE, D, 2>(f32, L, s);
            return;
        }
    }
    launch_patch_variant<MODE, D, 0>(f32, L, s);
}

template <typename T, int D>
static hipError_t launch_patch_mode(const PatchLaunch& L, hipStream_t s) {
    const bool f32 = sizeof(T) == 4;
    switch (L.mode) {
    case 0: launch_patch_kernel<0, D>(f32, L, s); break;
    case 1: launch_patch_kernel<1, D>(f32, L, s); break;
    case 2: launch_patch_kernel<2, D>(f32, L, s); break;
    case 3: launch_patch_kernel<3, D>(f32, L, s); break;
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

hipError_t launch_fallback(const FallbackLaunch& F, hipStream_t s) {
    const dim3 grid(256), block(kBlock);
    switch (F.var_dim) {
    case 1: hipLaunchKernelGGL(k_fallback<1>, grid, block, 0, s, F); break;
    case 2: hipLaunchKernelGGL(k_fallback<2>, grid, block, 0, s, F); break;
    case 3: hipLaunchKernelGGL(k_fallback<3>, grid, block, 0, s, F); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mad
