// One element: forward-mode derivatives over the stencil (Sec. 6.2), the
// optional eigenvalue clamp of the local Hessian (Sec. 7.1 Hessian
// filtering), and the map back to the stencil DOFs.
//
// Active variables are the KR = (NS-1)*D relative coordinates
// r = (D_NS (x) I_D) x with D_NS = [-1 | I] (see terms.hpp). Then
//   g_x = (D_NS (x) I)^T g_r,   H_x = (D_NS (x) I)^T H_r (D_NS (x) I),
// and H_x annihilates the D translation directions exactly.
//
// Clamp in the reduced space: let Q (NS x NS-1) be the orthonormal Helmert
// basis of the complement of the constant vector. Because H_x maps
// translations to zero, H_x = (Q (x) I) Hq (Q (x) I)^T with
// Hq = (W (x) I)^T H_r (W (x) I), W = D_NS Q, and the eigenpairs of H_x are
// those of Hq lifted by (Q (x) I) plus the D translations with eigenvalue 0.
// So clamp(H_x) = (Q (x) I) clamp(Hq) (Q (x) I)^T + max(0, eps) T, with T
// the translation projector. The eigen-decomposition runs on a KR x KR matrix
// instead of an NS*D x NS*D one (6 instead of 9 for a triangle in 3D, 9
// instead of 12 for a diamond).
#pragma once
#include <type_traits>

#include "dual.hpp"

namespace mad {

// Helmert basis: column i (0..NS-2) is (-1, ..., -1, i+1, 0, ...) / sqrt((i+1)(i+2)).
__device__ __forceinline__ constexpr double helmert(int s, int i) {
    return s <= i ? -1.0 / (i == 0 ? 1.4142135623730951 : (i == 1 ? 2.449489742783178 : 3.4641016151377544))
                  : (s == i + 1 ? double(i + 1) / (i == 0 ? 1.4142135623730951
                                                          : (i == 1 ? 2.449489742783178 : 3.4641016151377544))
                                : 0.0);
}
// W = D_NS Q: W[s][i] = Q[s+1][i] - Q[0][i]
__device__ __forceinline__ constexpr double wmat(int s, int i) { return helmert(s + 1, i) - helmert(0, i); }

// Result of one element: energy, the stencil gradient, and the Hessian kept in reduced form
// (KR x KR packed): for MODE 2 the raw Hessian in relative coordinates, for MODE 3 the clamped
// Hessian in Helmert coordinates. hfull() expands any stencil entry on demand.
template <class Term, typename T>
struct ElemOut {
    static constexpr int NF = Term::NS * Term::D;
    double f;
    T g[NF];
    T hr[Packed<Term::KR>::N];
};

// entry (i, j) of the stencil Hessian (i, j in 0..NS*D-1) from the reduced form; te = clamp floor
template <class Term, int MODE, typename T>
__device__ __forceinline__ T hfull(const ElemOut<Term, T>& o, int i, int j, T te) {
    constexpr int NS = Term::NS, D = Term::D, KR = Term::KR;
    if constexpr (!Term::TI) return o.hr[Packed<KR>::at(i, j)];   // seeded on the stencil DOFs
    const int si = i / D, ci = i % D, sj = j / D, cj = j % D;
    T acc = T(0);
    if constexpr (MODE == 2) {
        // H_x = (D_NS (x) I)^T H_r (D_NS (x) I)
#pragma unroll
        for (int a = 1; a < NS; ++a) {
            if (si != 0 && a != si) continue;
#pragma unroll
            for (int b = 1; b < NS; ++b) {
                if (sj != 0 && b != sj) continue;
                const T hv = o.hr[Packed<KR>::at((a - 1) * D + ci, (b - 1) * D + cj)];
                acc += ((si == 0) != (sj == 0)) ? -hv : hv;
            }
        }
    } else {
        // clamp(H_x) = (Q (x) I) clamp(Hq) (Q (x) I)^T + max(0, eps) T
#pragma unroll
        for (int a = 0; a < NS - 1; ++a) {
            const double qa = helmert(si, a);
            if (qa == 0.0) continue;
#pragma unroll
            for (int b = 0; b < NS - 1; ++b) {
                const double qb = helmert(sj, b);
                if (qb == 0.0) continue;
                acc += T(qa * qb) * o.hr[Packed<KR>::at(a * D + ci, b * D + cj)];
            }
        }
        if (ci == cj) acc += te * T(1.0 / NS);
    }
    return acc;
}

// Matrix-free product of one element's Hessian with the stencil vector v (Sec. 6.2, matrix-free
// mode): y = H_x v from the reduced form, without expanding H_x. MODE 2: H_x = (D (x) I)^T H_r (D (x) I),
// so u = (D (x) I) v (relative coordinates), w = H_r u, y = (D (x) I)^T w. MODE 3: H_x = (Q (x) I) Hc
// (Q (x) I)^T + te T, so u = (Q (x) I)^T v, w = Hc u, y = (Q (x) I) w + te T v (T the translation projector).
template <class Term, int MODE, typename T>
__device__ __forceinline__ void hvp_apply(const ElemOut<Term, T>& o, T te, const T (&v)[Term::NS * Term::D],
                                          T (&y)[Term::NS * Term::D]) {
    constexpr int NS = Term::NS, D = Term::D, KR = Term::KR;
    if constexpr (!Term::TI) {
        // seeded on the stencil DOFs: y = H v (the clamp, if any, is already in hr)
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            T acc = T(0);
#pragma unroll
            for (int j = 0; j < KR; ++j) acc += o.hr[Packed<KR>::at(i, j)] * v[j];
            y[i] = acc;
        }
        return;
    }
    T u[KR], w[KR];
    if constexpr (MODE == 2) {
#pragma unroll
        for (int s = 1; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < D; ++c) u[(s - 1) * D + c] = v[s * D + c] - v[c];
    } else {
#pragma unroll
        for (int a = 0; a < NS - 1; ++a)
#pragma unroll
            for (int c = 0; c < D; ++c) {
                T acc = T(0);
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const double q = helmert(s, a);
                    if (q != 0.0) acc += T(q) * v[s * D + c];
                }
                u[a * D + c] = acc;
            }
    }
#pragma unroll
    for (int i = 0; i < KR; ++i) {
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < KR; ++j) acc += o.hr[Packed<KR>::at(i, j)] * u[j];
        w[i] = acc;
    }
    if constexpr (MODE == 2) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
            T y0 = T(0);
#pragma unroll
            for (int s = 1; s < NS; ++s) {
                y[s * D + c] = w[(s - 1) * D + c];
                y0 -= w[(s - 1) * D + c];
            }
            y[c] = y0;
        }
    } else {
#pragma unroll
        for (int c = 0; c < D; ++c) {
            T vs = T(0);
#pragma unroll
            for (int s = 0; s < NS; ++s) vs += v[s * D + c];
            const T tv = te * vs * T(1.0 / NS);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                T acc = tv;
#pragma unroll
                for (int a = 0; a < NS - 1; ++a) {
                    const double q = helmert(s, a);
                    if (q != 0.0) acc += T(q) * w[a * D + c];
                }
                y[s * D + c] = acc;
            }
        }
    }
}

// hardware reciprocal / square root / reciprocal square root: approximate (about 1 ulp) in FP32,
// IEEE in FP64
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double frsq(double x) { return 1.0 / sqrt(x); }

// ---- symmetric eigen-decomposition: Jacobi rotations in round-robin order --------------------
// A sweep visits every pair (p, q) once, grouped into rounds of disjoint pairs (circle method
// over M = N rounded up to even players; pairs with the padding player are skipped): the parallel
// ordering of R. P. Brent and F. T. Luk, "The solution of singular-value and symmetric eigenvalue
// problems on multiprocessor arrays" (SIAM J. Sci. Stat. Comput., 1985). Rotations
// in one round touch disjoint (p, q) planes, so their parameters depend only on entries no other
// rotation of the round changes: they are computed together, giving independent instruction
// streams. The rotation zeroing a_pq uses t = tan(phi) = sgn(d) 2 a_pq / (|d| + sqrt(d^2 + 4 a_pq^2)),
// d = a_qq - a_pp (the smaller root of t^2 + 2 t d / (2 a_pq) - 1 = 0), c = 1/sqrt(1 + t^2),
// s = t c, and A <- J^T A J, V <- V J with J_pp = J_qq = c, J_pq = s, J_qp = -s.
//
// Scaled rotations (the idea of the fast Givens transformation of W. M. Gentleman, 1973, and
// S. Hammarling, 1974, applied to Jacobi rotations): the off-diagonal entries and the eigenvector
// columns are kept with a diagonal scale, a_ij = d_i d_j b_ij (i != j) and V = W diag(d), while the diagonal of A is kept as is. A
// rotation in the (p, q) plane multiplies d_p and d_q by c; the stored entries then change by one
// fused multiply-add each, b_ip -= t (d_q / d_p) b_iq and b_iq += t (d_p / d_q) b_ip (the same for
// W's columns), where the plain rotation needs two products and a multiply-add. The reciprocals
// e = 1/d are carried along (e <- e sqrt(1 + t^2)), so no division is needed. c >= 1/sqrt(2), so
// after s sweeps d >= 2^(-s (N - 1) / 2): no underflow in FP32 within the sweep limit, and the
// stored entries grow by at most the inverse.
// On return A's diagonal holds the eigenvalues and W diag(d) the eigenvectors. The matrix is
// scaled to max |a_ij| = 1 first (and the eigenvalues scaled back) so squares cannot overflow.
// Returns whether the off-diagonal mass fell below tol of the Frobenius norm within max_sweeps.
__host__ __device__ constexpr int rr_players(int n) { return n + (n & 1); }
// pair k of round r of the circle method over M players: one of the two members
__host__ __device__ constexpr int rr_a(int M, int r, int k) { return k == 0 ? M - 1 : (r + k) % (M - 1); }
__host__ __device__ constexpr int rr_b(int M, int r, int k) { return k == 0 ? r : (r - k + (M - 1)) % (M - 1); }

// off-diagonal mass (of the unscaled entries) below tol of the Frobenius norm
template <int N, typename T>
__device__ __forceinline__ bool jacobi_converged(const T (&A)[Packed<N>::N], const T (&dsc)[N], T tol) {
    T off = T(0), dg = T(0);
#pragma unroll
    for (int p = 0; p < N; ++p) {
        dg += A[Packed<N>::at(p, p)] * A[Packed<N>::at(p, p)];
#pragma unroll
        for (int q = p + 1; q < N; ++q) {
            const T a = dsc[p] * dsc[q] * A[Packed<N>::at(p, q)];
            off += a * a;
        }
    }
    return off <= tol * tol * (dg + T(2) * off);
}

// one sweep: every pair once, round by round
template <int N, typename T>
__device__ __forceinline__ void jacobi_sweep(T (&A)[Packed<N>::N], T (&W)[N][N], T (&dsc)[N], T (&inv)[N]) {
    constexpr int M = rr_players(N), H = M / 2;
#pragma unroll
    for (int r = 0; r < M - 1; ++r) {
        T tn[H], ta[H];
        // parameters of the round's rotations (independent of each other)
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const int a = rr_a(M, r, k), b = rr_b(M, r, k);
            if (a >= N || b >= N) continue;
            const int p = a < b ? a : b, q = a < b ? b : a;
            const T apq = dsc[p] * dsc[q] * A[Packed<N>::at(p, q)];
            const T d = A[Packed<N>::at(q, q)] - A[Packed<N>::at(p, p)];
            const T den = fabs(d) + fsqrt(d * d + T(4) * apq * apq);
            T t = (T(2) * apq) * frcp(den);
            t = d < T(0) ? -t : t;
            t = (apq == T(0)) ? T(0) : t;
            tn[k] = t;
            ta[k] = t * apq;
        }
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const int a = rr_a(M, r, k), b = rr_b(M, r, k);
            if (a >= N || b >= N) continue;
            const int p = a < b ? a : b, q = a < b ? b : a;
            const T t = tn[k];
            const T w = t * t + T(1);
            const T c = frsq(w);
            const T u = t * dsc[q] * inv[p], v = t * dsc[p] * inv[q];
            A[Packed<N>::at(p, p)] -= ta[k];
            A[Packed<N>::at(q, q)] += ta[k];
            A[Packed<N>::at(p, q)] = T(0);
#pragma unroll
            for (int i = 0; i < N; ++i) {
                if (i == p || i == q) continue;
                const T g = A[Packed<N>::at(i, p)], h = A[Packed<N>::at(i, q)];
                A[Packed<N>::at(i, p)] = g - u * h;
                A[Packed<N>::at(i, q)] = h + v * g;
            }
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const T g = W[i][p], h = W[i][q];
                W[i][p] = g - u * h;
                W[i][q] = h + v * g;
            }
            const T ic = w * c;
            dsc[p] *= c;
            dsc[q] *= c;
            inv[p] *= ic;
            inv[q] *= ic;
        }
    }
}

template <int N, typename T>
__device__ __forceinline__ bool jacobi_eig(T (&A)[Packed<N>::N], T (&W)[N][N], T (&dsc)[N], int max_sweeps, T tol) {
    T inv[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        dsc[i] = T(1);
        inv[i] = T(1);
#pragma unroll
        for (int j = 0; j < N; ++j) W[i][j] = (i == j) ? T(1) : T(0);
    }
    T amax = T(0);
#pragma unroll
    for (int i = 0; i < Packed<N>::N; ++i) amax = fmax(amax, fabs(A[i]));
    const T scale = amax > T(0) ? frcp(amax) : T(1);
#pragma unroll
    for (int i = 0; i < Packed<N>::N; ++i) A[i] *= scale;
    bool conv = jacobi_converged<N, T>(A, dsc, tol);
    if (!conv && max_sweeps > 0) {
        // the first sweep on its own: W is still the identity and the scales one there, so the
        // products with their structural zeros and ones fold away at compile time (the element
        // kernels are built without signed zeros and non-finite values)
        jacobi_sweep<N, T>(A, W, dsc, inv);
        // The test costs about a twentieth of a sweep. A dense 6x6 or 9x9 element Hessian rarely meets
        // the tolerance within two sweeps (in an FP32 emulation over the benchmark shell: no element
        // after one, 0.7% of the diamonds after two, never all 64 lanes of a wave), so for those sizes
        // the test starts after the third; a matrix that would have stopped sooner gets one or two
        // more sweeps, which only reduce its off-diagonal mass further. Small matrices are tested
        // after every sweep.
        constexpr int min_sweeps = N >= 6 ? 3 : 1;
        for (int sweep = 1;; ++sweep) {
            if (sweep >= min_sweeps && jacobi_converged<N, T>(A, dsc, tol)) {
                conv = true;
                break;
            }
            if (sweep == max_sweeps) break;
            jacobi_sweep<N, T>(A, W, dsc, inv);
        }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) A[Packed<N>::at(i, i)] *= amax > T(0) ? amax : T(1);
    return conv;
}

template <typename T> struct JacobiTol;
template <> struct JacobiTol<float> {
    static constexpr float tol = 1.0e-6f;
    static constexpr int sweeps = 15;
};
template <> struct JacobiTol<double> {
    static constexpr double tol = 1.0e-14;
    static constexpr int sweeps = 25;
};

// Derivatives of one element (modes 1-3): energy, stencil gradient, and the reduced Hessian --
// for MODE 2 the raw Hessian in relative coordinates (into out.hr), for MODE 3 the Hessian in
// Helmert coordinates Hq = (W (x) I)^T H_r (W (x) I) (into Aq, to be clamped by element_clamp).
template <class Term, typename T, int MODE>
__device__ __forceinline__ void element_derivs(const double* xs, const double* rest, const double* prm,
                                               ElemOut<Term, T>& out, T (&Aq)[Packed<Term::KR>::N]) {
    constexpr int NS = Term::NS, D = Term::D, KR = Term::KR;
    double r[KR];
    if constexpr (Term::TI) {
#pragma unroll
        for (int s = 1; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < D; ++c) r[(s - 1) * D + c] = xs[s * D + c] - xs[c];
    } else {
#pragma unroll
        for (int i = 0; i < KR; ++i) r[i] = xs[i];
    }
    using S = typename std::conditional<MODE == 1, D1<KR, T>, HD<KR, T>>::type;
    S f;
    if constexpr (Term::NRES > 0) {
        // residual term (Eq. 3): first-order duals give r and J; the scalar form is 1/2 |r|^2 with
        // gradient J^T r and the Gauss-Newton matrix J^T J in place of the Hessian
        using S1 = D1<KR, T>;
        S1 q[KR], res[Term::NRES];
#pragma unroll
        for (int i = 0; i < KR; ++i) q[i] = var<S1>(i, r[i]);
        Term::template residual<S1>(q, rest, prm, res);
        f = cst<S>(0.0);
#pragma unroll
        for (int m = 0; m < Term::NRES; ++m) {
            f.v += 0.5 * res[m].v * res[m].v;
            const T rv = T(res[m].v);
#pragma unroll
            for (int i = 0; i < KR; ++i) f.g[i] += rv * res[m].g[i];
            if constexpr (MODE >= 2) {
#pragma unroll
                for (int i = 0; i < KR; ++i)
#pragma unroll
                    for (int j = i; j < KR; ++j) f.h[Packed<KR>::at(i, j)] += res[m].g[i] * res[m].g[j];
            }
        }
    } else {
        S rs[KR];
#pragma unroll
        for (int i = 0; i < KR; ++i) rs[i] = var<S>(i, r[i]);
        f = Term::template energy<S>(rs, rest, prm);
    }
    out.f = f.v;
    if constexpr (!Term::TI) {
        // active variables are the stencil DOFs: no map back, no Helmert reduction
#pragma unroll
        for (int i = 0; i < KR; ++i) out.g[i] = f.g[i];
        if constexpr (MODE == 2) {
#pragma unroll
            for (int i = 0; i < Packed<KR>::N; ++i) out.hr[i] = f.h[i];
        } else if constexpr (MODE == 3) {
#pragma unroll
            for (int i = 0; i < Packed<KR>::N; ++i) Aq[i] = f.h[i];
        }
        return;
    }
#pragma unroll
    for (int c = 0; c < D; ++c) {
        T g0 = T(0);
#pragma unroll
        for (int s = 1; s < NS; ++s) {
            out.g[s * D + c] = f.g[(s - 1) * D + c];
            g0 -= f.g[(s - 1) * D + c];
        }
        out.g[c] = g0;
    }
    if constexpr (MODE == 2) {
#pragma unroll
        for (int i = 0; i < Packed<KR>::N; ++i) out.hr[i] = f.h[i];
    } else if constexpr (MODE == 3) {
#pragma unroll
        for (int i = 0; i < KR; ++i)
#pragma unroll
            for (int j = i; j < KR; ++j) {
                const int bi = i / D, ci = i % D, bj = j / D, cj = j % D;
                T acc = T(0);
#pragma unroll
                for (int a = 0; a < NS - 1; ++a) {
                    const double wa = wmat(a, bi);
                    if (wa == 0.0) continue;
#pragma unroll
                    for (int b = 0; b < NS - 1; ++b) {
                        const double wb = wmat(b, bj);
                        if (wb == 0.0) continue;
                        acc += T(wa * wb) * f.h[Packed<KR>::at(a * D + ci, b * D + cj)];
                    }
                }
                Aq[Packed<KR>::at(i, j)] = acc;
            }
    }
}

// clamp(Hq) = U diag(max(lambda, eps)) U^T into out.hr (U = V diag(dsc)); returns whether the eigen-decomposition
// converged
template <class Term, typename T>
__device__ __forceinline__ bool element_clamp(T (&A)[Packed<Term::KR>::N], double eps, ElemOut<Term, T>& out) {
    constexpr int KR = Term::KR;
    T V[KR][KR], dsc[KR];
    const bool conv = jacobi_eig<KR, T>(A, V, dsc, JacobiTol<T>::sweeps, JacobiTol<T>::tol);
    const T te = T(eps > 0.0 ? eps : 0.0);
#pragma unroll
    for (int i = 0; i < Packed<KR>::N; ++i) out.hr[i] = T(0);
#pragma unroll
    for (int m = 0; m < KR; ++m) {
        // eigenvector m is column m of V times dsc[m]: its scale squared goes with the eigenvalue
        const T lam = A[Packed<KR>::at(m, m)];
        const T lp = (lam > te ? lam : te) * (dsc[m] * dsc[m]);
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            const T li = lp * V[i][m];
#pragma unroll
            for (int j = i; j < KR; ++j) out.hr[Packed<KR>::at(i, j)] += li * V[j][m];
        }
    }
    return conv;
}

// Evaluate one element. MODE: 0 passive, 1 gradient, 2 Hessian, 3 clamped Hessian.
// xs: stencil DOFs (NS*D, FP64). Returns false if the eigen-decomposition did not converge.
template <class Term, typename T, int MODE>
__device__ __forceinline__ bool element_eval(const double* xs, const double* rest, const double* prm, double eps,
                                             ElemOut<Term, T>& out) {
    constexpr int NS = Term::NS, D = Term::D, KR = Term::KR;
    if constexpr (MODE == 0) {
        double r[KR];
        if constexpr (Term::TI) {
#pragma unroll
            for (int s = 1; s < NS; ++s)
#pragma unroll
                for (int c = 0; c < D; ++c) r[(s - 1) * D + c] = xs[s * D + c] - xs[c];
        } else {
#pragma unroll
            for (int i = 0; i < KR; ++i) r[i] = xs[i];
        }
        out.f = Term::template energy<double>(r, rest, prm);
        return true;
    } else {
        T A[Packed<KR>::N];
        element_derivs<Term, T, MODE>(xs, rest, prm, out, A);
        if constexpr (MODE == 3) return element_clamp<Term, T>(A, eps, out);
        return true;
    }
}

}  // namespace mad
