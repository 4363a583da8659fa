// Element energies of the term catalogue, written once over a generic active
// scalar S (double / D1 / HD, see dual.hpp).
//
// Every catalogued energy is invariant under translating all stencil DOFs
// together, so each term is a function of the NS-1 relative coordinates
// r_s = x_s - x_0 (s = 1..NS-1). Forward mode seeds those KR = (NS-1)*D
// relative coordinates as the active variables; the derivatives with respect
// to the stencil DOFs follow exactly through the fixed linear map
// x -> r (see element.hpp). This is the chain rule through a constant linear
// map, not an approximation.
#pragma once
#include "dual.hpp"

namespace mad {

enum TermKind { K_EDGE_SQLEN = 1, K_TRI_AREA = 2, K_DIRICHLET = 3, K_STVK = 4, K_BENDING = 5, K_SYMDIR = 6 };

template <typename S>
struct V3 {
    S x, y, z;
};

template <typename S> __device__ __forceinline__ V3<S> cross(const V3<S>& a, const V3<S>& b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename S> __device__ __forceinline__ S dot(const V3<S>& a, const V3<S>& b) {
    return a.x * b.x + a.y * b.y + a.z * b.z;
}

// Listing 1: squared edge length. r = x1 - x0.
struct TermEdgeSqlen {
    static constexpr int NS = 2, D = 3, KR = 3, NREST = 0;
    template <typename S> __device__ static S energy(const S* r, const double*, const double*) {
        return r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    }
};

// Sec. 7.6: triangle area 0.5 |(x1 - x0) x (x2 - x0)|.
struct TermTriArea {
    static constexpr int NS = 3, D = 3, KR = 6, NREST = 0;
    template <typename S> __device__ static S energy(const S* r, const double*, const double*) {
        const V3<S> a{r[0], r[1], r[2]}, b{r[3], r[4], r[5]};
        const V3<S> n = cross(a, b);
        return dsqrt(dot(n, n)) * 0.5;
    }
};

// Scalar Dirichlet energy 0.5 A |grad u|^2 with grad u = Dm^{-T} (u1 - u0, u2 - u0).
// rest = {Dm^{-1} row-major (4), rest area}.
struct TermDirichlet {
    static constexpr int NS = 3, D = 1, KR = 2, NREST = 5;
    template <typename S> __device__ static S energy(const S* r, const double* rest, const double*) {
        const S g0 = r[0] * rest[0] + r[1] * rest[2];
        const S g1 = r[0] * rest[1] + r[1] * rest[3];
        return (g0 * g0 + g1 * g1) * (0.5 * rest[4]);
    }
};

// StVK membrane: F = Ds Dm^{-1} (3x2), E = (F^T F - I)/2, A (mu tr(E^2) + lambda/2 tr(E)^2).
// r = (x_b - x_a, x_c - x_a); rest = {Dm^{-1} (4), rest area}; prm = {mu, lambda}.
struct TermStVK {
    static constexpr int NS = 3, D = 3, KR = 6, NREST = 5;
    template <typename S> __device__ static S energy(const S* r, const double* rest, const double* prm) {
        const double m00 = rest[0], m01 = rest[1], m10 = rest[2], m11 = rest[3];
        S f0[3], f1[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            f0[i] = r[i] * m00 + r[3 + i] * m10;
            f1[i] = r[i] * m01 + r[3 + i] * m11;
        }
        const S c00 = f0[0] * f0[0] + f0[1] * f0[1] + f0[2] * f0[2];
        const S c11 = f1[0] * f1[0] + f1[1] * f1[1] + f1[2] * f1[2];
        const S c01 = f0[0] * f1[0] + f0[1] * f1[1] + f0[2] * f1[2];
        const S e00 = (c00 + (-1.0)) * 0.5;
        const S e11 = (c11 + (-1.0)) * 0.5;
        const S e01 = c01 * 0.5;
        const S tr = e00 + e11;
        const S tr2 = e00 * e00 + e11 * e11 + (e01 * e01) * 2.0;
        return (tr2 * prm[0] + (tr * tr) * (0.5 * prm[1])) * rest[4];
    }
};

// Sec. 7.7 bending: k_b (A/3) (theta - theta_rest)^2 h^2 over the diamond (x0, x1, x2, x3),
// theta the signed dihedral angle about e = x1 - x0 between n1 = e x (x2 - x0) and
// n2 = (x3 - x0) x e. With a = x2 - x0, b = x3 - x0 the identity
// (n1 x n2) . e / |e| = -|e| (n1 . b) gives theta = atan2(-|e| (n1 . b), n1 . n2), which
// avoids the quartic cross product n1 x n2.
// r = (e, a, b); rest = {mean rest area, rest dihedral}; prm = {k_b, h}.
struct TermBending {
    static constexpr int NS = 4, D = 3, KR = 9, NREST = 2;
    template <typename S> __device__ static S energy(const S* r, const double* rest, const double* prm) {
        const V3<S> e{r[0], r[1], r[2]}, a{r[3], r[4], r[5]}, b{r[6], r[7], r[8]};
        const V3<S> n1 = cross(e, a);
        const V3<S> n2 = cross(b, e);
        const S c = dot(n1, n2);
        const S s = (dsqrt(dot(e, e)) * dot(n1, b)) * (-1.0);
        const S d = datan2(s, c) + (-rest[1]);
        return (d * d) * (prm[0] * rest[0] / 3.0 * prm[1] * prm[1]);
    }
};

// Sec. 7.2 symmetric Dirichlet: A (|J|_F^2 + |J^{-1}|_F^2), J = Ds Dm^{-1} (2x2);
// for 2x2 matrices |J^{-1}|_F^2 = |J|_F^2 / det(J)^2.
// r = (b - a, c - a) in UV; rest = {Dm^{-1} (4), rest area}.
struct TermSymDir {
    static constexpr int NS = 3, D = 2, KR = 4, NREST = 5;
    template <typename S> __device__ static S energy(const S* r, const double* rest, const double*) {
        const double m00 = rest[0], m01 = rest[1], m10 = rest[2], m11 = rest[3];
        const S j00 = r[0] * m00 + r[2] * m10, j01 = r[0] * m01 + r[2] * m11;
        const S j10 = r[1] * m00 + r[3] * m10, j11 = r[1] * m01 + r[3] * m11;
        const S det = j00 * j11 - j01 * j10;
        const S n = j00 * j00 + j01 * j01 + j10 * j10 + j11 * j11;
        return (n + n * drecip(det * det)) * rest[4];
    }
};

}  // namespace mad
