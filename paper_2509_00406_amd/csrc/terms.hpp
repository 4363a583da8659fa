// Element energies of the term catalogue, written once over a generic active
// scalar S (double / D1 / HD, see dual.hpp).
//
// Every catalogued energy is invariant under translating all stencil DOFs
// together, so each term is a function of the NS-1 relative coordinates
// r_s = x_s - x_0 (s = 1..NS-1). Forward mode seeds those KR = (NS-1)*D
// relative coordinates as the active variables; the derivatives with respect
// to the stencil DOFs follow exactly through the fixed linear map
// x -> r (see element.hpp). This is the chain rule through a constant linear
// map, not an approximation. A term that is not translation invariant (TI =
// false: the per-vertex inertia) seeds its stencil DOFs themselves, KR = NS*D.
// NVD: values the term reads per stencil vertex from a caller-owned vertex array.
#pragma once
#include "dual.hpp"

namespace mad {

enum TermKind {
    K_EDGE_SQLEN = 1, K_TRI_AREA = 2, K_DIRICHLET = 3, K_STVK = 4, K_BENDING = 5, K_SYMDIR = 6, K_MLP = 7, K_SHELL_TRI = 8,
    K_SPRING = 9, K_INERTIA = 10, K_RES_POSITION = 11, K_RES_EDGE = 12
};

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
    static constexpr int NS = 2, D = 3, KR = 3, NREST = 0, NAUX = 0, NPSI = 0, NVD = 0, NRES = 0;
    static constexpr bool TI = true;
    template <typename S> __device__ static S energy(const S* r, const double*, const double*) {
        return r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    }
};

// Sec. 7.1 mass-spring cloth, the spring of one edge: w (k/2) l^2 (|r|^2 / l^2 - 1)^2 with r = x1 - x0,
// l the rest length. rest = {l^2, 1 / l^2}, params = {k, w}.
struct TermSpring {
    static constexpr int NS = 2, D = 3, KR = 3, NREST = 2, NAUX = 0, NPSI = 0, NVD = 0, NRES = 0;
    static constexpr bool TI = true;
    template <typename S> __device__ static S energy(const S* r, const double* rest, const double* prm) {
        const S q = (r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) * rest[1] + (-1.0);
        return q * q * (0.5 * prm[0] * prm[1] * rest[0]);
    }
};

// Sec. 7.1 implicit-Euler inertia plus gravity at one vertex: (m/2) |x - xhat|^2 - w m g.x. Not
// translation invariant (TI = false): the active variables are the vertex's own coordinates x.
// Per-vertex inputs {m, xhat (3)} come from the caller's vertex array; params = {w, g (3)}.
struct TermInertia {
    static constexpr int NS = 1, D = 3, KR = 3, NREST = 0, NAUX = 0, NPSI = 0, NVD = 4, NRES = 0;
    static constexpr bool TI = false;
    template <typename S> __device__ static S energy(const S* x, const double* in, const double* prm) {
        const double m = in[0], wm = prm[0] * in[0];
        const S d0 = x[0] + (-in[1]), d1 = x[1] + (-in[2]), d2 = x[2] + (-in[3]);
        const S kin = (d0 * d0 + d1 * d1 + d2 * d2) * (0.5 * m);
        const S pot = x[0] * (-wm * prm[1]) + x[1] * (-wm * prm[2]) + x[2] * (-wm * prm[3]);
        return kin + pot;
    }
};

// Residual terms (Sec. 4.1, Eq. 3): NRES residuals per element. As scalar terms they contribute
// 1/2 |r|^2, and the element kernels assemble the Gauss-Newton matrix J^T J in place of the Hessian.
//
// Positional residual of one vertex (the paper's ActiveT<3> example): r = sqrt(w) (x - x_t), with
// {w, x_t} from the caller's per-vertex array. Not translation invariant.
struct TermResPosition {
    static constexpr int NS = 1, D = 3, KR = 3, NREST = 0, NAUX = 0, NPSI = 0, NVD = 4, NRES = 3;
    static constexpr bool TI = false;
    template <typename S> __device__ static void residual(const S* x, const double* in, const double*, S* out) {
        const double sw = sqrt(in[0]);
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c] = (x[c] + (-in[1 + c])) * sw;
    }
    template <typename S> __device__ static S energy(const S* x, const double* in, const double* prm) {
        S r[3];
        residual<S>(x, in, prm, r);
        return (r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) * 0.5;
    }
};

// Edge-length residual (a least-squares spring): r = sqrt(k) (|x1 - x0| - l), rest = {l}, params = {k}.
struct TermResEdge {
    static constexpr int NS = 2, D = 3, KR = 3, NREST = 1, NAUX = 0, NPSI = 0, NVD = 0, NRES = 1;
    static constexpr bool TI = true;
    template <typename S> __device__ static void residual(const S* r, const double* rest, const double* prm, S* out) {
        out[0] = (dsqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) + (-rest[0])) * sqrt(prm[0]);
    }
    template <typename S> __device__ static S energy(const S* r, const double* rest, const double* prm) {
        S q[1];
        residual<S>(r, rest, prm, q);
        return q[0] * q[0] * 0.5;
    }
};

// Sec. 7.6: triangle area 0.5 |(x1 - x0) x (x2 - x0)|.
struct TermTriArea {
    static constexpr int NS = 3, D = 3, KR = 6, NREST = 0, NAUX = 0, NPSI = 0, NVD = 0, NRES = 0;
    static constexpr bool TI = true;
    template <typename S> __device__ static S energy(const S* r, const double*, const double*) {
        const V3<S> a{r[0], r[1], r[2]}, b{r[3], r[4], r[5]};
        const V3<S> n = cross(a, b);
        return dsqrt(dot(n, n)) * 0.5;
    }
};

// Scalar Dirichlet energy 0.5 A |grad u|^2 with grad u = Dm^{-T} (u1 - u0, u2 - u0).
// rest = {Dm^{-1} row-major (4), rest area}.
struct TermDirichlet {
    static constexpr int NS = 3, D = 1, KR = 2, NREST = 5, NAUX = 0, NPSI = 0, NVD = 0, NRES = 0;
    static constexpr bool TI = true;
    template <typename S> __device__ static S energy(const S* r, const double* rest, const double*) {
        const S g0 = r[0] * rest[0] + r[1] * rest[2];
        const S g1 = r[0] * rest[1] + r[1] * rest[3];
        return (g0 * g0 + g1 * g1) * (0.5 * rest[4]);
    }
};

// StVK membrane: F = Ds Dm^{-1} (3x2), E = (F^T F - I)/2, A (mu tr(E^2) + lambda/2 tr(E)^2).
// r = (x_b - x_a, x_c - x_a); rest = {Dm^{-1} (4), rest area}; prm = {mu, lambda}.
struct TermStVK {
    static constexpr int NS = 3, D = 3, KR = 6, NREST = 5, NAUX = 0, NPSI = 0, NVD = 0, NRES = 0;
    static constexpr bool TI = true;
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
    static constexpr int NS = 4, D = 3, KR = 9, NREST = 2, NAUX = 0, NPSI = 0, NVD = 0, NRES = 0;
    static constexpr bool TI = true;
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
    static constexpr int NS = 3, D = 2, KR = 4, NREST = 5, NAUX = 0, NPSI = 0, NVD = 0, NRES = 0;
    static constexpr bool TI = true;
    template <typename S> __device__ static S energy(const S* r, const double* rest, const double*) {
        const double m00 = rest[0], m01 = rest[1], m10 = rest[2], m11 = rest[3];
        const S j00 = r[0] * m00 + r[2] * m10, j01 = r[0] * m01 + r[2] * m11;
        const S j10 = r[1] * m00 + r[3] * m10, j11 = r[1] * m01 + r[3] * m11;
        const S det = j00 * j11 - j01 * j10;
        const S n = j00 * j00 + j01 * j01 + j10 * j10 + j11 * j11;
        return (n + n * drecip(det * det)) * rest[4];
    }
};


// ---- per-triangle shell features (project-defined; the learned density's input) -----------------
// z = (E00, E11, E01, II00 - rII00, II11 - rII11, II01 - rII01): F = Ds Dm^{-1} (3x2),
// E = (F^T F - I)/2, N = [n_b - n_a, n_c - n_a] Dm^{-1} from the passive unit vertex normals,
// II = -(N^T F + F^T N)/2. rest = {Dm^{-1} (4), rest area, rest II (3), normals n_a, n_b, n_c (9)}.
// z is quadratic (E) and linear (II) in r.
template <typename S>
__device__ __forceinline__ void shell_features(const S* r, const double* rest, S (&z)[6]) {
    const double m00 = rest[0], m01 = rest[1], m10 = rest[2], m11 = rest[3];
    const double* na = rest + 8;
    S f0[3], f1[3];
    double n0[3], n1[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        f0[i] = r[i] * m00 + r[3 + i] * m10;
        f1[i] = r[i] * m01 + r[3 + i] * m11;
        const double d1 = na[3 + i] - na[i], d2 = na[6 + i] - na[i];
        n0[i] = d1 * m00 + d2 * m10;
        n1[i] = d1 * m01 + d2 * m11;
    }
    z[0] = (f0[0] * f0[0] + f0[1] * f0[1] + f0[2] * f0[2] + (-1.0)) * 0.5;
    z[1] = (f1[0] * f1[0] + f1[1] * f1[1] + f1[2] * f1[2] + (-1.0)) * 0.5;
    z[2] = (f0[0] * f1[0] + f0[1] * f1[1] + f0[2] * f1[2]) * 0.5;
    z[3] = (f0[0] * n0[0] + f0[1] * n0[1] + f0[2] * n0[2]) * (-1.0) + (-rest[5]);
    z[4] = (f1[0] * n1[0] + f1[1] * n1[1] + f1[2] * n1[2]) * (-1.0) + (-rest[6]);
    z[5] = (f1[0] * n0[0] + f1[1] * n0[1] + f1[2] * n0[2] + f0[0] * n1[0] + f0[1] * n1[1] + f0[2] * n1[2]) *
               (-0.5) + (-rest[7]);
}

// Analytic per-triangle shell density A W(z), W = mu (E00^2 + E11^2 + 2 E01^2)
// + lambda/2 (E00 + E11)^2 + k_b/2 (dII00^2 + dII11^2 + 2 dII01^2); prm = {mu, lambda, k_b}.
struct TermShellTri {
    static constexpr int NS = 3, D = 3, KR = 6, NREST = 8, NAUX = 9, NPSI = 0, NVD = 0, NRES = 0;
    static constexpr bool TI = true;
    template <typename S> __device__ static S energy(const S* r, const double* rest, const double* prm) {
        S z[6];
        shell_features(r, rest, z);
        const S tr = z[0] + z[1];
        const S m = z[0] * z[0] + z[1] * z[1] + (z[2] * z[2]) * 2.0;
        const S b = z[3] * z[3] + z[4] * z[4] + (z[5] * z[5]) * 2.0;
        return (m * prm[0] + (tr * tr) * (0.5 * prm[1]) + b * (0.5 * prm[2])) * rest[4];
    }
};

// Learned density A psi(z). The network's value, gradient and packed Hessian with respect to z
// at this element's features (28 numbers, computed by the network kernel) arrive after the
// normals: rest[17] = psi, rest[18 + i] = dpsi/dz_i, rest[24 + Packed<6>::at(i, j)] = d2psi/dz_i dz_j.
// With dz = z - val(z) (no value, exact first and second derivatives), the second-order Taylor
// form psi + sum_i psi_i dz_i + 1/2 sum_ij psi_ij dz_i dz_j carries exactly the value, gradient
// and Hessian of psi(z(r)) in hyper-dual arithmetic.
struct TermMLP {
    static constexpr int NS = 3, D = 3, KR = 6, NREST = 8, NAUX = 9, NPSI = 28, NVD = 0, NRES = 0;
    static constexpr bool TI = true;
    template <typename S> __device__ static S energy(const S* r, const double* rest, const double*) {
        S z[6];
        shell_features(r, rest, z);
        const double* ps = rest + 17;
        S acc = cst<S>(ps[0]);
        S dz[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            dz[i] = z[i] + (-val(z[i]));
            acc = acc + dz[i] * ps[1 + i];
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            acc = acc + (dz[i] * dz[i]) * (0.5 * ps[7 + Packed<6>::at(i, i)]);
#pragma unroll
            for (int j = i + 1; j < 6; ++j) acc = acc + (dz[i] * dz[j]) * ps[7 + Packed<6>::at(i, j)];
        }
        return acc * rest[4];
    }
};

}  // namespace mad
