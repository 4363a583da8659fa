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

template <class Term, typename T>
struct ElemOut {
    static constexpr int NF = Term::NS * Term::D;
    double f;
    T g[NF];
    T h[Packed<NF>::N];
};

// ---- symmetric eigen-decomposition: cyclic Jacobi on a packed upper triangle ------------------
// On return A's diagonal holds the eigenvalues and V's columns the eigenvectors. Returns whether
// the off-diagonal mass fell below tol relative to the Frobenius norm within max_sweeps.
template <int N, typename T>
__device__ __forceinline__ bool jacobi_eig(T (&A)[Packed<N>::N], T (&V)[N][N], int max_sweeps, T tol) {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) V[i][j] = (i == j) ? T(1) : T(0);
    bool conv = false;
    for (int sweep = 0; sweep <= max_sweeps; ++sweep) {
        T off = T(0), dg = T(0);
#pragma unroll
        for (int p = 0; p < N; ++p) {
            dg += A[Packed<N>::at(p, p)] * A[Packed<N>::at(p, p)];
#pragma unroll
            for (int q = p + 1; q < N; ++q) off += A[Packed<N>::at(p, q)] * A[Packed<N>::at(p, q)];
        }
        if (off <= tol * tol * (dg + T(2) * off)) {
            conv = true;
            break;
        }
        if (sweep == max_sweeps) break;
#pragma unroll
        for (int p = 0; p < N - 1; ++p)
#pragma unroll
            for (int q = p + 1; q < N; ++q) {
                const T apq = A[Packed<N>::at(p, q)];
                const T app = A[Packed<N>::at(p, p)];
                const T aqq = A[Packed<N>::at(q, q)];
                const T theta = (aqq - app) / (T(2) * apq);
                T t = T(1) / (fabs(theta) + sqrt(theta * theta + T(1)));
                t = theta < T(0) ? -t : t;
                t = (apq == T(0)) ? T(0) : t;
                const T c = T(1) / sqrt(t * t + T(1));
                const T s = t * c;
                const T tau = s / (T(1) + c);
                A[Packed<N>::at(p, p)] = app - t * apq;
                A[Packed<N>::at(q, q)] = aqq + t * apq;
                A[Packed<N>::at(p, q)] = T(0);
#pragma unroll
                for (int r = 0; r < N; ++r) {
                    if (r == p || r == q) continue;
                    const T g = A[Packed<N>::at(r, p)], h = A[Packed<N>::at(r, q)];
                    A[Packed<N>::at(r, p)] = g - s * (h + g * tau);
                    A[Packed<N>::at(r, q)] = h + s * (g - h * tau);
                }
#pragma unroll
                for (int r = 0; r < N; ++r) {
                    const T g = V[r][p], h = V[r][q];
                    V[r][p] = g - s * (h + g * tau);
                    V[r][q] = h + s * (g - h * tau);
                }
            }
    }
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

// Evaluate one element. MODE: 0 passive, 1 gradient, 2 Hessian, 3 clamped Hessian.
// xs: stencil DOFs (NS*D, FP64). Returns false if the eigen-decomposition did not converge.
template <class Term, typename T, int MODE>
__device__ __forceinline__ bool element_eval(const double* xs, const double* rest, const double* prm, double eps,
                                             ElemOut<Term, T>& out) {
    constexpr int NS = Term::NS, D = Term::D, KR = Term::KR, NF = NS * D;
    double r[KR];
#pragma unroll
    for (int s = 1; s < NS; ++s)
#pragma unroll
        for (int c = 0; c < D; ++c) r[(s - 1) * D + c] = xs[s * D + c] - xs[c];

    if constexpr (MODE == 0) {
        out.f = Term::template energy<double>(r, rest, prm);
        return true;
    } else if constexpr (MODE == 1) {
        using S = D1<KR, T>;
        S rs[KR];
#pragma unroll
        for (int i = 0; i < KR; ++i) rs[i] = var<S>(i, r[i]);
        const S f = Term::template energy<S>(rs, rest, prm);
        out.f = f.v;
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
        return true;
    } else {
        using S = HD<KR, T>;
        S rs[KR];
#pragma unroll
        for (int i = 0; i < KR; ++i) rs[i] = var<S>(i, r[i]);
        const S f = Term::template energy<S>(rs, rest, prm);
        out.f = f.v;
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
            // H_x = (D_NS (x) I)^T H_r (D_NS (x) I), entry by entry
#pragma unroll
            for (int i = 0; i < NF; ++i)
#pragma unroll
                for (int j = i; j < NF; ++j) {
                    const int si = i / D, ci = i % D, sj = j / D, cj = j % D;
                    T acc = T(0);
#pragma unroll
                    for (int a = 1; a < NS; ++a) {
                        if (si != 0 && a != si) continue;
#pragma unroll
                        for (int b = 1; b < NS; ++b) {
                            if (sj != 0 && b != sj) continue;
                            const T hv = f.h[Packed<KR>::at((a - 1) * D + ci, (b - 1) * D + cj)];
                            const bool neg = (si == 0) != (sj == 0);
                            acc += neg ? -hv : hv;
                        }
                    }
                    out.h[Packed<NF>::at(i, j)] = acc;
                }
            return true;
        } else {
            // Hq = (W (x) I)^T H_r (W (x) I)
            T A[Packed<KR>::N];
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
                    A[Packed<KR>::at(i, j)] = acc;
                }
            T V[KR][KR];
            const bool conv = jacobi_eig<KR, T>(A, V, JacobiTol<T>::sweeps, JacobiTol<T>::tol);
            const T te = T(eps > 0.0 ? eps : 0.0);
#pragma unroll
            for (int i = 0; i < NF; ++i)
#pragma unroll
                for (int j = i; j < NF; ++j) out.h[Packed<NF>::at(i, j)] = ((i % D) == (j % D)) ? te / T(NS) : T(0);
#pragma unroll
            for (int m = 0; m < KR; ++m) {
                const T lam = A[Packed<KR>::at(m, m)];
                const T lp = lam > te ? lam : te;
                T u[NF];
#pragma unroll
                for (int s = 0; s < NS; ++s)
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        T acc = T(0);
#pragma unroll
                        for (int i = 0; i < NS - 1; ++i) {
                            const double q = helmert(s, i);
                            if (q == 0.0) continue;
                            acc += T(q) * V[i * D + c][m];
                        }
                        u[s * D + c] = acc;
                    }
#pragma unroll
                for (int i = 0; i < NF; ++i) {
                    const T li = lp * u[i];
#pragma unroll
                    for (int j = i; j < NF; ++j) out.h[Packed<NF>::at(i, j)] += li * u[j];
                }
            }
            return conv;
        }
    }
}

}  // namespace mad
