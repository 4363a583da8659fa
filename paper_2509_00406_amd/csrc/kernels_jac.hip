// Residual terms: the global residual vector and the sparse Jacobian (Sec. 4.1 Eq. 3, Sec. 6.1).
// Each element owns NRES consecutive rows of J (element e of a term: rows row_off + e NRES ...), and
// each row holds the element's stencil DOFs v * D + c in ascending order, so the pattern is fixed by
// the stencils and every value is written once by its owner: no atomics, no assembly pass. The local
// Jacobian comes from first-order duals over the element's (translation-reduced) coordinates, mapped
// back to the stencil DOFs exactly as the gradient is.
#include "kernels_common.hpp"

namespace mad {

template <class Term, typename T>
__global__ __launch_bounds__(256) void k_jacobian(JacLaunch L, int t) {
    constexpr int NS = Term::NS, D = Term::D, KR = Term::KR, NF = NS * D, M = Term::NRES;
    const JacTerm& A = L.terms[t];
    // one element per lane, in element order: consecutive lanes write consecutive rows
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= A.n) return;
    int vs[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) vs[s] = A.stencil[e * NS + s];
    // stencil vertices in ascending order: the row's column order
    int ord[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) ord[s] = s;
#pragma unroll
    for (int a = 1; a < NS; ++a)
#pragma unroll
        for (int b = a; b > 0; --b)
            if (vs[ord[b - 1]] > vs[ord[b]]) {
                const int tmp = ord[b];
                ord[b] = ord[b - 1];
                ord[b - 1] = tmp;
            }
    const int64_t row0 = A.row_off + e * M;
    const int64_t nz0 = A.nz_off + e * M * NF;
    if (L.pattern) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            L.rowptr[row0 + m] = (int32_t)(nz0 + (int64_t)m * NF);
#pragma unroll
            for (int j = 0; j < NF; ++j) L.colidx[nz0 + (int64_t)m * NF + j] = vs[ord[j / D]] * D + j % D;
        }
        return;
    }
    double xs[NF];
    bool bad = false;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int c = 0; c < D; ++c) {
            xs[s * D + c] = L.x[(int64_t)vs[s] * D + c];
            bad = bad || !finite(xs[s * D + c]);
        }
    double rest[n_inputs<Term>()];
    gather_inputs<Term>(rest, A.rest, A.n, e, nullptr, vs, nullptr, A.vdata);
    double r[KR];
    if constexpr (Term::TI) {
#pragma unroll
        for (int s = 1; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < D; ++c) r[(s - 1) * D + c] = xs[s * D + c] - xs[c];
    } else {
#pragma unroll
        for (int k = 0; k < KR; ++k) r[k] = xs[k];
    }
    using S1 = D1<KR, T>;
    S1 q[KR], res[M];
#pragma unroll
    for (int k = 0; k < KR; ++k) q[k] = var<S1>(k, r[k]);
    Term::template residual<S1>(q, rest, A.prm, res);
    T* vals = static_cast<T*>(L.vals);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        // the row over the stencil DOFs: (D_NS (x) I)^T applied to the reduced row
        T jx[NF];
        if constexpr (Term::TI) {
#pragma unroll
            for (int c = 0; c < D; ++c) {
                T j0 = T(0);
#pragma unroll
                for (int s = 1; s < NS; ++s) {
                    jx[s * D + c] = res[m].g[(s - 1) * D + c];
                    j0 -= res[m].g[(s - 1) * D + c];
                }
                jx[c] = j0;
            }
        } else {
#pragma unroll
            for (int k = 0; k < NF; ++k) jx[k] = res[m].g[k];
        }
        L.r[row0 + m] = res[m].v;
        bad = bad || !finite(res[m].v);
#pragma unroll
        for (int j = 0; j < NF; ++j) {
            const T v = jx[ord[j / D] * D + j % D];
            vals[nz0 + (int64_t)m * NF + j] = v;
            bad = bad || !finite(v);
        }
    }
    if (bad) atomicOr(L.flags, 1);
}

template <class Term>
static hipError_t launch_jac_term(const JacLaunch& L, int t, hipStream_t s) {
    const int64_t n = L.terms[t].n;
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (L.prec == MAD_F32) hipLaunchKernelGGL((k_jacobian<Term, float>), grid, block, 0, s, L, t);
    else hipLaunchKernelGGL((k_jacobian<Term, double>), grid, block, 0, s, L, t);
    return hipGetLastError();
}

hipError_t launch_jacobian(const JacLaunch& L, hipStream_t s) {
    for (int t = 0; t < L.n_terms; ++t) {
        hipError_t e = hipSuccess;
        switch (L.terms[t].kind) {
        case K_RES_POSITION: e = launch_jac_term<TermResPosition>(L, t, s); break;
        case K_RES_EDGE: e = launch_jac_term<TermResEdge>(L, t, s); break;
        default: e = hipErrorInvalidValue; break;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace mad
