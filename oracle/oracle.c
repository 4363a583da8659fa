/*
 * Plain FP64 CPU oracle (test infrastructure only; see oracle.h).
 *
 * Everything here is written for a reader checking it against the paper by
 * eye: dense hyper-dual numbers carry (value, gradient, full Hessian) over
 * the element's stencil DOFs (Sec. 5.1, Sec. 6.2), every energy is the
 * formula as stated, assembly is the serial sum of Eq. 2, and the Hessian
 * filter is a textbook cyclic Jacobi eigen-decomposition followed by the
 * eigenvalue clamp of Sec. 7.1. No blocking, no fusion, no reordering.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define KMAX 12

/* ------------------------------------------------------------------------- */
/* Hyper-dual scalar over k local variables (Sec. 5.1 "ActiveT", Sec. 6.2). */
/* ------------------------------------------------------------------------- */
typedef struct {
    int k;
    double v;
    double g[KMAX];
    double h[KMAX][KMAX];
} hd;

static hd hd_const(int k, double c) {
    hd r;
    memset(&r, 0, sizeof r);
    r.k = k;
    r.v = c;
    return r;
}

/* the i-th active variable with value v (seed: gradient e_i, zero Hessian) */
static hd hd_var(int k, int i, double v) {
    hd r = hd_const(k, v);
    if (i < k) r.g[i] = 1.0;
    return r;
}

static hd hd_add(hd a, hd b) {
    hd r = hd_const(a.k, a.v + b.v);
    for (int i = 0; i < a.k; ++i) {
        r.g[i] = a.g[i] + b.g[i];
        for (int j = 0; j < a.k; ++j) r.h[i][j] = a.h[i][j] + b.h[i][j];
    }
    return r;
}

static hd hd_sub(hd a, hd b) {
    hd r = hd_const(a.k, a.v - b.v);
    for (int i = 0; i < a.k; ++i) {
        r.g[i] = a.g[i] - b.g[i];
        for (int j = 0; j < a.k; ++j) r.h[i][j] = a.h[i][j] - b.h[i][j];
    }
    return r;
}

static hd hd_scale(hd a, double c) {
    hd r = hd_const(a.k, c * a.v);
    for (int i = 0; i < a.k; ++i) {
        r.g[i] = c * a.g[i];
        for (int j = 0; j < a.k; ++j) r.h[i][j] = c * a.h[i][j];
    }
    return r;
}

static hd hd_addc(hd a, double c) {
    a.v += c;
    return a;
}

/* product rule: (ab)'' = a b'' + b a'' + a' b'^T + b' a'^T */
static hd hd_mul(hd a, hd b) {
    hd r = hd_const(a.k, a.v * b.v);
    for (int i = 0; i < a.k; ++i) {
        r.g[i] = a.v * b.g[i] + b.v * a.g[i];
        for (int j = 0; j < a.k; ++j)
            r.h[i][j] = a.v * b.h[i][j] + b.v * a.h[i][j] + a.g[i] * b.g[j] + b.g[i] * a.g[j];
    }
    return r;
}

/* scalar chain rule for a unary f with f(a), f'(a), f''(a) */
static hd hd_unary(hd a, double f0, double f1, double f2) {
    hd r = hd_const(a.k, f0);
    for (int i = 0; i < a.k; ++i) {
        r.g[i] = f1 * a.g[i];
        for (int j = 0; j < a.k; ++j) r.h[i][j] = f1 * a.h[i][j] + f2 * a.g[i] * a.g[j];
    }
    return r;
}

/* chain rule for a binary f(a, b) with its first and second partials */
static hd hd_binary(hd a, hd b, double f0, double fa, double fb, double faa, double fbb, double fab) {
    hd r = hd_const(a.k, f0);
    for (int i = 0; i < a.k; ++i) {
        r.g[i] = fa * a.g[i] + fb * b.g[i];
        for (int j = 0; j < a.k; ++j)
            r.h[i][j] = fa * a.h[i][j] + fb * b.h[i][j] + faa * a.g[i] * a.g[j] + fbb * b.g[i] * b.g[j]
                        + fab * (a.g[i] * b.g[j] + b.g[i] * a.g[j]);
    }
    return r;
}

static hd hd_sq(hd a) { return hd_mul(a, a); }

static hd hd_recip(hd a) {
    double v = a.v;
    return hd_unary(a, 1.0 / v, -1.0 / (v * v), 2.0 / (v * v * v));
}

static hd hd_div(hd a, hd b) { return hd_mul(a, hd_recip(b)); }

static hd hd_sqrt(hd a) {
    double s = sqrt(a.v);
    return hd_unary(a, s, 0.5 / s, -0.25 / (s * a.v));
}

/* atan2(y, x): d/dy = x/r2, d/dx = -y/r2, d2/dy2 = -2xy/r4, d2/dx2 = 2xy/r4,
 * d2/dxdy = (y^2 - x^2)/r4 */
static hd hd_atan2(hd y, hd x) {
    double r2 = x.v * x.v + y.v * y.v;
    double r4 = r2 * r2;
    return hd_binary(y, x, atan2(y.v, x.v), x.v / r2, -y.v / r2, -2.0 * x.v * y.v / r4,
                     2.0 * x.v * y.v / r4, (y.v * y.v - x.v * x.v) / r4);
}

/* 3-vectors of hyper-duals */
typedef struct { hd c[3]; } hd3;

static hd3 hd3_sub(hd3 a, hd3 b) {
    hd3 r;
    for (int i = 0; i < 3; ++i) r.c[i] = hd_sub(a.c[i], b.c[i]);
    return r;
}

static hd hd3_dot(hd3 a, hd3 b) {
    hd r = hd_mul(a.c[0], b.c[0]);
    r = hd_add(r, hd_mul(a.c[1], b.c[1]));
    return hd_add(r, hd_mul(a.c[2], b.c[2]));
}

static hd3 hd3_cross(hd3 a, hd3 b) {
    hd3 r;
    r.c[0] = hd_sub(hd_mul(a.c[1], b.c[2]), hd_mul(a.c[2], b.c[1]));
    r.c[1] = hd_sub(hd_mul(a.c[2], b.c[0]), hd_mul(a.c[0], b.c[2]));
    r.c[2] = hd_sub(hd_mul(a.c[0], b.c[1]), hd_mul(a.c[1], b.c[0]));
    return r;
}

/* lift vertex s of the stencil (VarDim 3) as active variables 3s..3s+2 */
static hd3 lift3(int k, const double *xloc, int s) {
    hd3 r;
    for (int d = 0; d < 3; ++d) r.c[d] = hd_var(k, 3 * s + d, xloc[3 * s + d]);
    return r;
}

/* ------------------------------------------------------------------------- */
/* Element energies.                                                          */
/* ------------------------------------------------------------------------- */

/* Listing 1: squared edge length |x0 - x1|^2 (Op::EV, k = 6) */
static hd e_edge_sqlen(int k, const double *xloc) {
    hd3 d = hd3_sub(lift3(k, xloc, 0), lift3(k, xloc, 1));
    return hd3_dot(d, d);
}

/* Sec. 7.1 mass-spring cloth, spring of edge (x0, x1) with rest length l = rest[0]:
 * w * (k/2) l^2 (|x0 - x1|^2 / l^2 - 1)^2, params {k, w} (w: the potential's weight h^2). */
static hd e_spring(int k, const double *xloc, const double *rest, const double *prm) {
    double l2 = rest[0] * rest[0];
    hd3 d = hd3_sub(lift3(k, xloc, 0), lift3(k, xloc, 1));
    hd q = hd_addc(hd_scale(hd3_dot(d, d), 1.0 / l2), -1.0);
    return hd_scale(hd_sq(q), prm[1] * 0.5 * prm[0] * l2);
}

/* Sec. 7.1 implicit-Euler inertia plus gravity at one vertex: (m/2) |x - xhat|^2 - w m g.x,
 * rest = {m, xhat (3)} (xhat = x^n + h v^n), params {w, g (3)}. Not translation invariant. */
static hd e_inertia(int k, const double *xloc, const double *rest, const double *prm) {
    double m = rest[0];
    hd3 x = lift3(k, xloc, 0);
    hd acc = hd_const(k, 0.0);
    for (int c = 0; c < 3; ++c) {
        hd dc = hd_addc(x.c[c], -rest[1 + c]);
        acc = hd_add(acc, hd_scale(hd_sq(dc), 0.5 * m));
        acc = hd_add(acc, hd_scale(x.c[c], -prm[0] * m * prm[1 + c]));
    }
    return acc;
}

/* Residual terms (Sec. 4.1, Eq. 3). Positional residual of one vertex, the paper's ActiveT<3> example:
 * r = sqrt(w) (x - x_t), rest = {w, x_t (3)}. */
static int res_position(int k, const double *xloc, const double *rest, hd *out) {
    hd3 x = lift3(k, xloc, 0);
    double sw = sqrt(rest[0]);
    for (int c = 0; c < 3; ++c) out[c] = hd_scale(hd_addc(x.c[c], -rest[1 + c]), sw);
    return 3;
}

/* Edge-length residual (least-squares spring): r = sqrt(k_s) (|x0 - x1| - l), rest = {l}, params {k_s} */
static int res_edge(int k, const double *xloc, const double *rest, const double *prm, hd *out) {
    hd3 d = hd3_sub(lift3(k, xloc, 0), lift3(k, xloc, 1));
    out[0] = hd_scale(hd_addc(hd_sqrt(hd3_dot(d, d)), -rest[0]), sqrt(prm[0]));
    return 1;
}

/* residuals of one element with k active variables; returns m (0: not a residual kind) */
static int res_elem(int kind, int k, const double *prm, const double *rest, const double *xloc, hd *out) {
    switch (kind) {
    case OR_RES_POSITION: return res_position(k, xloc, rest, out);
    case OR_RES_EDGE: return res_edge(k, xloc, rest, prm, out);
    default: return 0;
    }
}

/* a residual term as a scalar term: f = 1/2 sum r_i^2, g = sum r_i grad r_i, and the Gauss-Newton
 * matrix sum grad r_i grad r_i^T in place of the Hessian */
static hd gauss_newton(int k, const hd *res, int m) {
    hd out = hd_const(k, 0.0);
    for (int i = 0; i < m; ++i) {
        out.v += 0.5 * res[i].v * res[i].v;
        for (int a = 0; a < k; ++a) {
            out.g[a] += res[i].v * res[i].g[a];
            for (int b = 0; b < k; ++b) out.h[a][b] += res[i].g[a] * res[i].g[b];
        }
    }
    return out;
}

/* Sec. 7.6: area 0.5 |(x1 - x0) x (x2 - x0)| (Op::FV, k = 9) */
static hd e_tri_area(int k, const double *xloc) {
    hd3 x0 = lift3(k, xloc, 0), x1 = lift3(k, xloc, 1), x2 = lift3(k, xloc, 2);
    hd3 n = hd3_cross(hd3_sub(x1, x0), hd3_sub(x2, x0));
    return hd_scale(hd_sqrt(hd3_dot(n, n)), 0.5);
}

/* Scalar Dirichlet energy 0.5 A |grad u|^2 of the piecewise-linear field u on a
 * triangle whose (passive) rest positions give Dm; grad u = Dm^{-T} (u1-u0, u2-u0). */
static hd e_dirichlet(int k, const double *xloc, const double *rest) {
    const double *mi = rest; /* Dm^{-1} row-major */
    double area = rest[4];
    hd u0 = hd_var(k, 0, xloc[0]), u1 = hd_var(k, 1, xloc[1]), u2 = hd_var(k, 2, xloc[2]);
    hd d1 = hd_sub(u1, u0), d2 = hd_sub(u2, u0);
    hd g0 = hd_add(hd_scale(d1, mi[0]), hd_scale(d2, mi[2]));
    hd g1 = hd_add(hd_scale(d1, mi[1]), hd_scale(d2, mi[3]));
    return hd_scale(hd_add(hd_sq(g0), hd_sq(g1)), 0.5 * area);
}

/* StVK membrane: F = Ds Dm^{-1} (3x2), E = (F^T F - I)/2,
 * f = A (mu tr(E^2) + lambda/2 tr(E)^2). */
static hd e_stvk(int k, const double *xloc, const double *rest, const double *prm) {
    const double *mi = rest;
    double area = rest[4], mu = prm[0], lam = prm[1];
    hd3 xa = lift3(k, xloc, 0), xb = lift3(k, xloc, 1), xc = lift3(k, xloc, 2);
    hd3 d1 = hd3_sub(xb, xa), d2 = hd3_sub(xc, xa);
    hd F[3][2];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 2; ++j)
            F[i][j] = hd_add(hd_scale(d1.c[i], mi[0 * 2 + j]), hd_scale(d2.c[i], mi[1 * 2 + j]));
    hd E[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            hd c = hd_mul(F[0][a], F[0][b]);
            c = hd_add(c, hd_mul(F[1][a], F[1][b]));
            c = hd_add(c, hd_mul(F[2][a], F[2][b]));
            E[a][b] = hd_scale(hd_addc(c, a == b ? -1.0 : 0.0), 0.5);
        }
    hd trE = hd_add(E[0][0], E[1][1]);
    hd trE2 = hd_add(hd_add(hd_sq(E[0][0]), hd_sq(E[1][1])), hd_add(hd_mul(E[0][1], E[1][0]), hd_mul(E[1][0], E[0][1])));
    hd psi = hd_add(hd_scale(trE2, mu), hd_scale(hd_sq(trE), 0.5 * lam));
    return hd_scale(psi, area);
}

/* dihedral angle of the diamond (x0, x1, x2, x3) about the edge e = x1 - x0:
 * n1 = e x (x2 - x0), n2 = (x3 - x0) x e, theta = atan2(((n1 x n2).e)/|e|, n1.n2) */
static hd dihedral(hd3 x0, hd3 x1, hd3 x2, hd3 x3) {
    hd3 e = hd3_sub(x1, x0);
    hd3 n1 = hd3_cross(e, hd3_sub(x2, x0));
    hd3 n2 = hd3_cross(hd3_sub(x3, x0), e);
    hd y = hd_div(hd3_dot(hd3_cross(n1, n2), e), hd_sqrt(hd3_dot(e, e)));
    hd xx = hd3_dot(n1, n2);
    return hd_atan2(y, xx);
}

/* Sec. 7.7: E_bend = k_b (A/3) (theta - theta')^2 h^2 */
static hd e_bending(int k, const double *xloc, const double *rest, const double *prm) {
    double abar = rest[0], theta0 = rest[1], kb = prm[0], ht = prm[1];
    hd th = dihedral(lift3(k, xloc, 0), lift3(k, xloc, 1), lift3(k, xloc, 2), lift3(k, xloc, 3));
    hd d = hd_addc(th, -theta0);
    return hd_scale(hd_sq(d), kb * abar / 3.0 * ht * ht);
}

/* Sec. 7.2: f = area (|J|_F^2 + |J^{-1}|_F^2), J = [b-a, c-a] [b_r-a_r, c_r-a_r]^{-1} */
static hd e_symdir(int k, const double *xloc, const double *rest) {
    const double *mi = rest;
    double area = rest[4];
    hd a[2], b[2], c[2];
    for (int d = 0; d < 2; ++d) {
        a[d] = hd_var(k, 0 + d, xloc[0 + d]);
        b[d] = hd_var(k, 2 + d, xloc[2 + d]);
        c[d] = hd_var(k, 4 + d, xloc[4 + d]);
    }
    hd J[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            J[i][j] = hd_add(hd_scale(hd_sub(b[i], a[i]), mi[0 * 2 + j]), hd_scale(hd_sub(c[i], a[i]), mi[1 * 2 + j]));
    hd det = hd_sub(hd_mul(J[0][0], J[1][1]), hd_mul(J[0][1], J[1][0]));
    hd idet = hd_recip(det);
    hd Ji[2][2];
    Ji[0][0] = hd_mul(J[1][1], idet);
    Ji[0][1] = hd_scale(hd_mul(J[0][1], idet), -1.0);
    Ji[1][0] = hd_scale(hd_mul(J[1][0], idet), -1.0);
    Ji[1][1] = hd_mul(J[0][0], idet);
    hd nJ = hd_const(k, 0.0), nJi = hd_const(k, 0.0);
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            nJ = hd_add(nJ, hd_sq(J[i][j]));
            nJi = hd_add(nJi, hd_sq(Ji[i][j]));
        }
    return hd_scale(hd_add(nJ, nJi), area);
}

/* ------------------------------------------------------------------------- */
/* Per-triangle shell features and densities (project-defined: the paper has  */
/* no learned component). z = (E00, E11, E01, dII00, dII11, dII01):           */
/*   F = Ds Dm^{-1} (3x2), E = (F^T F - I) / 2 (Green strain, rest frame);     */
/*   N = Dn Dm^{-1} with Dn = [n_b - n_a, n_c - n_a] from passive unit vertex  */
/*   normals; II = -(N^T F + F^T N) / 2; dII = II - rest II.                   */
/* rest data (8): Dm^{-1} (4, row-major), rest area, rest II (00, 11, 01).     */
/* aux (9): the current unit normals of the three vertices (not active).       */
/* ------------------------------------------------------------------------- */
static void shell_features(int k, const double *xloc, const double *rest, const double *nrm, hd z[6]) {
    const double *mi = rest;
    hd3 xa = lift3(k, xloc, 0), xb = lift3(k, xloc, 1), xc = lift3(k, xloc, 2);
    hd3 d1 = hd3_sub(xb, xa), d2 = hd3_sub(xc, xa);
    hd F[3][2];
    double N[3][2];
    for (int i = 0; i < 3; ++i) {
        double dn1 = nrm[3 + i] - nrm[i], dn2 = nrm[6 + i] - nrm[i];
        for (int j = 0; j < 2; ++j) {
            F[i][j] = hd_add(hd_scale(d1.c[i], mi[0 * 2 + j]), hd_scale(d2.c[i], mi[1 * 2 + j]));
            N[i][j] = dn1 * mi[0 * 2 + j] + dn2 * mi[1 * 2 + j];
        }
    }
    /* E[a][b] = (sum_i F[i][a] F[i][b] - delta_ab) / 2; II[a][b] = -(sum_i N[i][a] F[i][b] + F[i][a] N[i][b]) / 2 */
    static const int A[3] = {0, 1, 0}, B[3] = {0, 1, 1};
    for (int q = 0; q < 3; ++q) {
        int a = A[q], b = B[q];
        hd e = hd_const(k, 0.0), ii = hd_const(k, 0.0);
        for (int i = 0; i < 3; ++i) {
            e = hd_add(e, hd_mul(F[i][a], F[i][b]));
            ii = hd_add(ii, hd_add(hd_scale(F[i][b], N[i][a]), hd_scale(F[i][a], N[i][b])));
        }
        z[q] = hd_scale(hd_addc(e, a == b ? -1.0 : 0.0), 0.5);
        z[3 + q] = hd_addc(hd_scale(ii, -0.5), -rest[5 + q]);
    }
}

/* analytic density: W(z) = mu (E00^2 + E11^2 + 2 E01^2) + lambda/2 (E00 + E11)^2
 *                        + k_b/2 (dII00^2 + dII11^2 + 2 dII01^2); f = rest area * W */
static hd shell_density(const hd z[6], const double *prm) {
    double mu = prm[0], lam = prm[1], kb = prm[2];
    hd trE2 = hd_add(hd_add(hd_sq(z[0]), hd_sq(z[1])), hd_scale(hd_sq(z[2]), 2.0));
    hd trE = hd_add(z[0], z[1]);
    hd b2 = hd_add(hd_add(hd_sq(z[3]), hd_sq(z[4])), hd_scale(hd_sq(z[5]), 2.0));
    return hd_add(hd_add(hd_scale(trE2, mu), hd_scale(hd_sq(trE), 0.5 * lam)), hd_scale(b2, 0.5 * kb));
}

static hd e_shell_tri(int k, const double *xloc, const double *rest, const double *aux, const double *prm) {
    hd z[6];
    shell_features(k, xloc, rest, aux, z);
    return hd_scale(shell_density(z, prm), rest[4]);
}

/* softplus(a) = log(1 + e^a), evaluated without overflow; its derivatives are the
 * logistic sigma(a) and sigma(a) (1 - sigma(a)) */
static double softplus(double a) { return a > 0.0 ? a + log1p(exp(-a)) : log1p(exp(a)); }
static double logistic(double a) { return a >= 0.0 ? 1.0 / (1.0 + exp(-a)) : exp(a) / (1.0 + exp(a)); }
static hd hd_softplus(hd a) {
    double s = logistic(a.v);
    return hd_unary(a, softplus(a.v), s, s * (1.0 - s));
}

/* MLP parameter block: [H, s_out, s_in(6), W1(H x 6), b1(H), W2(H x H), b2(H), w3(H), b3],
 * psi(z) = s_out (w3 . sp(W2 sp(W1 (s_in * z) + b1) + b2) + b3), sp = softplus */
#define MLP_HMAX 64
static int mlp_layout(const double *prm, int *H, const double **sin_, const double **W1, const double **b1,
                      const double **W2, const double **b2, const double **w3, double *b3) {
    int h = (int)prm[0];
    if (h < 1 || h > MLP_HMAX || (double)h != prm[0]) return -1;
    *H = h;
    *sin_ = prm + 2;
    *W1 = prm + 8;
    *b1 = *W1 + 6 * h;
    *W2 = *b1 + h;
    *b2 = *W2 + h * h;
    *w3 = *b2 + h;
    *b3 = (*w3)[h];
    return 0;
}

static int mlp_psi(const double *prm, const hd z[6], hd *psi) {
    int H;
    const double *sin_, *W1, *b1, *W2, *b2, *w3;
    double b3;
    if (mlp_layout(prm, &H, &sin_, &W1, &b1, &W2, &b2, &w3, &b3) != 0) return -1;
    int k = z[0].k;
    hd xin[6];
    for (int i = 0; i < 6; ++i) xin[i] = hd_scale(z[i], sin_[i]);
    hd h1[MLP_HMAX], h2[MLP_HMAX];
    for (int n = 0; n < H; ++n) {
        hd a = hd_const(k, b1[n]);
        for (int i = 0; i < 6; ++i) a = hd_add(a, hd_scale(xin[i], W1[n * 6 + i]));
        h1[n] = hd_softplus(a);
    }
    for (int m = 0; m < H; ++m) {
        hd a = hd_const(k, b2[m]);
        for (int n = 0; n < H; ++n) a = hd_add(a, hd_scale(h1[n], W2[m * H + n]));
        h2[m] = hd_softplus(a);
    }
    hd out = hd_const(k, b3);
    for (int m = 0; m < H; ++m) out = hd_add(out, hd_scale(h2[m], w3[m]));
    *psi = hd_scale(out, prm[1]);
    return 0;
}

/* learned density: f = rest area * psi(z(x)) */
static int e_mlp(int k, const double *xloc, const double *rest, const double *aux, const double *prm, hd *out) {
    hd z[6], psi;
    shell_features(k, xloc, rest, aux, z);
    if (mlp_psi(prm, z, &psi) != 0) return -1;
    *out = hd_scale(psi, rest[4]);
    return 0;
}

static int kind_stencil(int kind) {
    switch (kind) {
    case OR_INERTIA: case OR_RES_POSITION: return 1;
    case OR_EDGE_SQLEN: case OR_SPRING: case OR_RES_EDGE: return 2;
    case OR_TRI_AREA: case OR_DIRICHLET: case OR_STVK: case OR_SYMDIR: case OR_MLP: case OR_SHELL_TRI: return 3;
    case OR_BENDING: return 4;
    default: return -1;
    }
}

static int kind_vardim(int kind) {
    switch (kind) {
    case OR_DIRICHLET: return 1;
    case OR_SYMDIR: return 2;
    case OR_EDGE_SQLEN: case OR_TRI_AREA: case OR_STVK: case OR_BENDING: case OR_MLP: case OR_SHELL_TRI:
    case OR_SPRING: case OR_INERTIA: case OR_RES_POSITION: case OR_RES_EDGE: return 3;
    default: return -1;
    }
}

/* evaluate one element with k active variables (k = 0: passive, value only) */
static int eval_elem(int kind, int k, const double *prm, const double *rest, const double *aux, const double *xloc,
                     hd *out) {
    switch (kind) {
    case OR_SHELL_TRI: *out = e_shell_tri(k, xloc, rest, aux, prm); return 0;
    case OR_MLP: return e_mlp(k, xloc, rest, aux, prm, out);
    case OR_EDGE_SQLEN: *out = e_edge_sqlen(k, xloc); return 0;
    case OR_TRI_AREA: *out = e_tri_area(k, xloc); return 0;
    case OR_DIRICHLET: *out = e_dirichlet(k, xloc, rest); return 0;
    case OR_STVK: *out = e_stvk(k, xloc, rest, prm); return 0;
    case OR_BENDING: *out = e_bending(k, xloc, rest, prm); return 0;
    case OR_SYMDIR: *out = e_symdir(k, xloc, rest); return 0;
    case OR_SPRING: *out = e_spring(k, xloc, rest, prm); return 0;
    case OR_INERTIA: *out = e_inertia(k, xloc, rest, prm); return 0;
    case OR_RES_POSITION: case OR_RES_EDGE: {
        hd res[3];
        int m = res_elem(kind, k, prm, rest, xloc, res);
        *out = gauss_newton(k, res, m);
        return 0;
    }
    default: return -1;
    }
}

/* ------------------------------------------------------------------------- */
/* Hessian filtering (Sec. 7.1): clamp eigenvalues of each term's local       */
/* Hessian from below. Cyclic Jacobi rotations (textbook symmetric Schur       */
/* decomposition), then out = Q diag(max(lambda, eps)) Q^T.                    */
/* ------------------------------------------------------------------------- */
int oracle_spd_project(int n, const double *Ain, double eps, double *out) {
    if (n <= 0 || n > KMAX) return -1;
    double A[KMAX][KMAX], Q[KMAX][KMAX];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            A[i][j] = 0.5 * (Ain[i * n + j] + Ain[j * n + i]);
            Q[i][j] = (i == j) ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0, fro = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                fro += A[i][j] * A[i][j];
                if (i != j) off += A[i][j] * A[i][j];
            }
        if (off <= 1e-30 * fro || fro == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                if (A[p][q] == 0.0) continue;
                double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                /* A <- A J (columns p, q), then A <- J^T A (rows p, q), Q <- Q J */
                for (int r = 0; r < n; ++r) {
                    double ap = A[r][p], aq = A[r][q];
                    A[r][p] = c * ap - s * aq;
                    A[r][q] = s * ap + c * aq;
                }
                for (int r = 0; r < n; ++r) {
                    double ap = A[p][r], aq = A[q][r];
                    A[p][r] = c * ap - s * aq;
                    A[q][r] = s * ap + c * aq;
                }
                for (int r = 0; r < n; ++r) {
                    double qp = Q[r][p], qq = Q[r][q];
                    Q[r][p] = c * qp - s * qq;
                    Q[r][q] = s * qp + c * qq;
                }
            }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int m = 0; m < n; ++m) {
                double lam = A[m][m] > eps ? A[m][m] : eps;
                acc += Q[i][m] * lam * Q[j][m];
            }
            out[i * n + j] = acc;
        }
    return 0;
}

int oracle_element(int kind, const double *params, const double *rest, const double *aux, const double *xloc,
                   int mode, double spd_eps, double *f, double *g, double *H) {
    int ss = kind_stencil(kind), vd = kind_vardim(kind);
    if (ss < 0 || vd < 0) return -1;
    int k = ss * vd;
    int kk = (mode & (OR_GRAD | OR_HESS)) ? k : 0;
    hd r;
    if (eval_elem(kind, kk, params, rest, aux, xloc, &r) != 0) return -1;
    if (f) *f = r.v;
    if (g && (mode & OR_GRAD))
        for (int i = 0; i < k; ++i) g[i] = r.g[i];
    if (H && (mode & OR_HESS)) {
        double tmp[KMAX * KMAX];
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) tmp[i * k + j] = r.h[i][j];
        if (mode & OR_SPD) return oracle_spd_project(k, tmp, spd_eps, H);
        memcpy(H, tmp, sizeof(double) * k * k);
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Topology: edges and edge diamonds (Sec. 6 pipeline input).                 */
/* ------------------------------------------------------------------------- */
typedef struct { int32_t lo, hi, face, from, to, opp; } erec;

static int erec_cmp(const void *pa, const void *pb) {
    const erec *a = pa, *b = pb;
    if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
    if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;
    if (a->face != b->face) return a->face < b->face ? -1 : 1;
    return 0;
}

int oracle_topology(int64_t nv, int64_t nt, const int32_t *tris, int64_t *n_edges, int32_t *edges,
                    int32_t *edge_nf, int64_t *n_diamonds, int32_t *diamonds, int32_t *diamond_faces) {
    erec *rec = malloc(sizeof(erec) * (size_t)(3 * nt + 1));
    if (!rec) return -4;
    for (int64_t f = 0; f < nt; ++f) {
        const int32_t *t = tris + 3 * f;
        for (int c = 0; c < 3; ++c) {
            if (t[c] < 0 || t[c] >= nv) { free(rec); return -1; }
        }
        if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2]) { free(rec); return -1; }
        for (int c = 0; c < 3; ++c) {
            erec *r = &rec[3 * f + c];
            r->from = t[c];
            r->to = t[(c + 1) % 3];
            r->opp = t[(c + 2) % 3];
            r->lo = r->from < r->to ? r->from : r->to;
            r->hi = r->from < r->to ? r->to : r->from;
            r->face = (int32_t)f;
        }
    }
    qsort(rec, (size_t)(3 * nt), sizeof(erec), erec_cmp);
    int64_t ne = 0, nd = 0;
    for (int64_t i = 0; i < 3 * nt;) {
        int64_t j = i;
        while (j < 3 * nt && rec[j].lo == rec[i].lo && rec[j].hi == rec[i].hi) ++j;
        edges[2 * ne] = rec[i].lo;
        edges[2 * ne + 1] = rec[i].hi;
        edge_nf[ne] = (int32_t)(j - i);
        if (j - i == 2) {
            /* f1 = rec[i] (lower face index after sorting), f2 = rec[i+1] */
            int32_t *d = diamonds + 4 * nd;
            d[0] = rec[i].from;
            d[1] = rec[i].to;
            d[2] = rec[i].opp;
            d[3] = rec[i + 1].opp;
            diamond_faces[2 * nd] = rec[i].face;
            diamond_faces[2 * nd + 1] = rec[i + 1].face;
            ++nd;
        }
        ++ne;
        i = j;
    }
    *n_edges = ne;
    *n_diamonds = nd;
    free(rec);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Rest data.                                                                 */
/* ------------------------------------------------------------------------- */
/* rest triangle in its own 2D frame: Dm = [[|e1|, e1.e2/|e1|], [0, |e1 x e2|/|e1|]] */
static int rest_frame(const double *X0, const double *X1, const double *X2, double *mi, double *area) {
    double e1[3], e2[3], c[3];
    for (int d = 0; d < 3; ++d) {
        e1[d] = X1[d] - X0[d];
        e2[d] = X2[d] - X0[d];
    }
    c[0] = e1[1] * e2[2] - e1[2] * e2[1];
    c[1] = e1[2] * e2[0] - e1[0] * e2[2];
    c[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    double cn = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    if (!(l1 > 0.0) || !(cn > 0.0)) return -2;
    double dm00 = l1, dm01 = (e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2]) / l1;
    double dm10 = 0.0, dm11 = cn / l1;
    double det = dm00 * dm11 - dm01 * dm10;
    mi[0] = dm11 / det;
    mi[1] = -dm01 / det;
    mi[2] = -dm10 / det;
    mi[3] = dm00 / det;
    *area = 0.5 * cn;
    return 0;
}

int oracle_rest_tri(int64_t nt, const int32_t *tris, const double *rest, double *dminv, double *area) {
    for (int64_t f = 0; f < nt; ++f) {
        const int32_t *t = tris + 3 * f;
        if (rest_frame(rest + 3 * t[0], rest + 3 * t[1], rest + 3 * t[2], dminv + 4 * f, area + f) != 0) return -2;
    }
    return 0;
}

int oracle_rest_diamond(int64_t nd, const int32_t *diamonds, const int32_t *diamond_faces,
                        const int32_t *tris, const double *rest, double *abar, double *theta0) {
    for (int64_t e = 0; e < nd; ++e) {
        double mi[4], a1, a2;
        const int32_t *t1 = tris + 3 * diamond_faces[2 * e], *t2 = tris + 3 * diamond_faces[2 * e + 1];
        if (rest_frame(rest + 3 * t1[0], rest + 3 * t1[1], rest + 3 * t1[2], mi, &a1) != 0) return -2;
        if (rest_frame(rest + 3 * t2[0], rest + 3 * t2[1], rest + 3 * t2[2], mi, &a2) != 0) return -2;
        abar[e] = 0.5 * (a1 + a2);
        double xl[12];
        for (int s = 0; s < 4; ++s)
            for (int d = 0; d < 3; ++d) xl[3 * s + d] = rest[3 * diamonds[4 * e + s] + d];
        hd th = dihedral(lift3(0, xl, 0), lift3(0, xl, 1), lift3(0, xl, 2), lift3(0, xl, 3));
        theta0[e] = th.v;
    }
    return 0;
}

/* area-weighted unit vertex normals: normalize(sum over incident triangles of
 * (x_b - x_a) x (x_c - x_a)); a vertex with no triangle (or a zero sum) gets 0 */
int oracle_vertex_normals(int64_t nv, int64_t nt, const int32_t *tris, const double *x, double *out) {
    memset(out, 0, sizeof(double) * (size_t)(3 * nv));
    for (int64_t f = 0; f < nt; ++f) {
        const int32_t *t = tris + 3 * f;
        const double *a = x + 3 * (int64_t)t[0], *b = x + 3 * (int64_t)t[1], *c = x + 3 * (int64_t)t[2];
        double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        for (int v = 0; v < 3; ++v)
            for (int d = 0; d < 3; ++d) out[3 * (int64_t)t[v] + d] += n[d];
    }
    for (int64_t v = 0; v < nv; ++v) {
        double *n = out + 3 * v;
        double l = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (l > 0.0)
            for (int d = 0; d < 3; ++d) n[d] /= l;
    }
    return 0;
}

/* per triangle [Dm^{-1} (4), rest area, rest II (3)]: the features' II evaluated on the rest
 * mesh with its own vertex normals */
int oracle_rest_shell(int64_t nv, int64_t nt, const int32_t *tris, const double *rest, double *out) {
    double *nrm = malloc(sizeof(double) * (size_t)(3 * (nv > 0 ? nv : 1)));
    if (!nrm) return -4;
    oracle_vertex_normals(nv, nt, tris, rest, nrm);
    for (int64_t f = 0; f < nt; ++f) {
        const int32_t *t = tris + 3 * f;
        double *o = out + 8 * f;
        if (rest_frame(rest + 3 * t[0], rest + 3 * t[1], rest + 3 * t[2], o, o + 4) != 0) { free(nrm); return -2; }
        o[5] = o[6] = o[7] = 0.0;
        double xl[9], aux[9];
        for (int a = 0; a < 3; ++a)
            for (int d = 0; d < 3; ++d) {
                xl[3 * a + d] = rest[3 * (int64_t)t[a] + d];
                aux[3 * a + d] = nrm[3 * (int64_t)t[a] + d];
            }
        hd z[6];
        shell_features(0, xl, o, aux, z);
        for (int q = 0; q < 3; ++q) o[5 + q] = z[3 + q].v;
    }
    free(nrm);
    return 0;
}

/* feature values z [nt][6] at positions x (normals from x over these triangles): the same
 * formulas as shell_features, in plain doubles (fast enough for millions of samples) */
int oracle_shell_features(int64_t nv, int64_t nt, const int32_t *tris, const double *rest8, const double *x,
                          double *z) {
    double *nrm = malloc(sizeof(double) * (size_t)(3 * (nv > 0 ? nv : 1)));
    if (!nrm) return -4;
    oracle_vertex_normals(nv, nt, tris, x, nrm);
    for (int64_t f = 0; f < nt; ++f) {
        const int32_t *t = tris + 3 * f;
        const double *mi = rest8 + 8 * f;
        const double *xa = x + 3 * (int64_t)t[0], *xb = x + 3 * (int64_t)t[1], *xc = x + 3 * (int64_t)t[2];
        const double *na = nrm + 3 * (int64_t)t[0], *nb = nrm + 3 * (int64_t)t[1], *nc = nrm + 3 * (int64_t)t[2];
        double F[3][2], N[3][2];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 2; ++j) {
                F[i][j] = (xb[i] - xa[i]) * mi[0 * 2 + j] + (xc[i] - xa[i]) * mi[1 * 2 + j];
                N[i][j] = (nb[i] - na[i]) * mi[0 * 2 + j] + (nc[i] - na[i]) * mi[1 * 2 + j];
            }
        static const int A[3] = {0, 1, 0}, B[3] = {0, 1, 1};
        for (int q = 0; q < 3; ++q) {
            int a = A[q], b = B[q];
            double e = 0.0, ii = 0.0;
            for (int i = 0; i < 3; ++i) {
                e += F[i][a] * F[i][b];
                ii += F[i][b] * N[i][a] + F[i][a] * N[i][b];
            }
            z[6 * f + q] = 0.5 * (e - (a == b ? 1.0 : 0.0));
            z[6 * f + 3 + q] = -0.5 * ii - mi[5 + q];
        }
    }
    free(nrm);
    return 0;
}

/* the analytic density W and dW/dz at n feature vectors (z seeded as 6 hyper-dual variables) */
int oracle_shell_density(int64_t n, const double *z, const double *params, double *W, double *dW) {
    for (int64_t i = 0; i < n; ++i) {
        hd zz[6];
        for (int q = 0; q < 6; ++q) zz[q] = hd_var(6, q, z[6 * i + q]);
        hd w = shell_density(zz, params);
        W[i] = w.v;
        if (dW)
            for (int q = 0; q < 6; ++q) dW[6 * i + q] = w.g[q];
    }
    return 0;
}

/* the network psi(z), and optionally dpsi/dz [n][6] and d2psi/dz2 [n][36] */
int oracle_mlp_eval(int64_t n, const double *z, const double *params, double *psi, double *dpsi, double *d2psi) {
    for (int64_t i = 0; i < n; ++i) {
        hd zz[6], p;
        for (int q = 0; q < 6; ++q) zz[q] = hd_var(6, q, z[6 * i + q]);
        if (mlp_psi(params, zz, &p) != 0) return -1;
        psi[i] = p.v;
        if (dpsi)
            for (int q = 0; q < 6; ++q) dpsi[6 * i + q] = p.g[q];
        if (d2psi)
            for (int q = 0; q < 6; ++q)
                for (int r = 0; r < 6; ++r) d2psi[36 * i + 6 * q + r] = p.h[q][r];
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Pattern (Sec. 6.1): sorted unique block pairs, prefix sum to row pointers. */
/* ------------------------------------------------------------------------- */
static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

int oracle_pattern(int64_t nv, int n_terms, const int64_t *n_elem, const int *stencil_size,
                   const int32_t *const *stencils, int32_t *rowptr, int32_t *colidx, int64_t *nnzb) {
    int64_t total = nv;
    for (int t = 0; t < n_terms; ++t) total += n_elem[t] * stencil_size[t] * stencil_size[t];
    int64_t *keys = malloc(sizeof(int64_t) * (size_t)(total > 0 ? total : 1));
    if (!keys) return -4;
    int64_t m = 0;
    for (int64_t i = 0; i < nv; ++i) keys[m++] = i * nv + i;
    for (int t = 0; t < n_terms; ++t) {
        int ss = stencil_size[t];
        for (int64_t e = 0; e < n_elem[t]; ++e) {
            const int32_t *s = stencils[t] + ss * e;
            for (int a = 0; a < ss; ++a) {
                if (s[a] < 0 || s[a] >= nv) { free(keys); return -1; }
                for (int b = 0; b < ss; ++b) keys[m++] = (int64_t)s[a] * nv + s[b];
            }
        }
    }
    qsort(keys, (size_t)m, sizeof(int64_t), cmp_i64);
    int64_t u = 0;
    for (int64_t i = 0; i < m; ++i)
        if (i == 0 || keys[i] != keys[i - 1]) keys[u++] = keys[i];
    *nnzb = u;
    if (u > 2147483647LL) { free(keys); return -3; }
    if (colidx) {
        for (int64_t i = 0; i <= nv; ++i) rowptr[i] = 0;
        for (int64_t i = 0; i < u; ++i) rowptr[keys[i] / nv + 1] += 1;
        for (int64_t i = 0; i < nv; ++i) rowptr[i + 1] += rowptr[i];
        for (int64_t i = 0; i < u; ++i) colidx[i] = (int32_t)(keys[i] % nv);
    }
    free(keys);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Energy reduction (Sec. 5.5): Neumaier compensated summation.                */
/* ------------------------------------------------------------------------- */
double oracle_neumaier_sum(int64_t n, const double *v) {
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double t = s + v[i];
        if (fabs(s) >= fabs(v[i])) c += (s - t) + v[i];
        else c += (v[i] - t) + s;
        s = t;
    }
    return s + c;
}

/* ------------------------------------------------------------------------- */
/* Evaluation and assembly (Eq. 1-2).                                         */
/* ------------------------------------------------------------------------- */
static int64_t find_block(const int32_t *rowptr, const int32_t *colidx, int32_t r, int32_t c) {
    int32_t lo = rowptr[r], hi = rowptr[r + 1] - 1;
    while (lo <= hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (colidx[mid] == c) return mid;
        if (colidx[mid] < c) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

/* doubles of per-element rest data of a kind */
static int rest_stride_of(int kind) {
    switch (kind) {
    case OR_BENDING: return 2;
    case OR_DIRICHLET: case OR_STVK: case OR_SYMDIR: return 5;
    case OR_SHELL_TRI: case OR_MLP: return 8;
    case OR_SPRING: case OR_RES_EDGE: return 1;
    case OR_INERTIA: case OR_RES_POSITION: return 4;
    default: return 0;
    }
}

int oracle_eval(int64_t nv, int var_dim, int n_terms, const int *kind, const int64_t *n_elem,
                const int32_t *const *stencil, const double *const *rest, const double *const *params,
                const double *x, int mode, double spd_eps, const char *row_mask, const int32_t *rowptr,
                const int32_t *colidx, double *energy, double *esum_abs, double *grad, double *gscale,
                double *hess, double *hscale) {
    const int d = var_dim;
    int64_t nnzb = rowptr ? rowptr[nv] : 0;
    if (grad) {
        memset(grad, 0, sizeof(double) * (size_t)(nv * d));
        if (gscale) memset(gscale, 0, sizeof(double) * (size_t)(nv * d));
    }
    if (hess) {
        memset(hess, 0, sizeof(double) * (size_t)(nnzb * d * d));
        if (hscale) memset(hscale, 0, sizeof(double) * (size_t)(nnzb * d * d));
    }
    int64_t total = 0;
    for (int t = 0; t < n_terms; ++t) total += n_elem[t];
    double *fvals = malloc(sizeof(double) * (size_t)(total > 0 ? total : 1));
    if (!fvals) return -4;
    int64_t fi = 0;
    double abs_sum = 0.0;
    for (int t = 0; t < n_terms; ++t) {
        int ss = kind_stencil(kind[t]);
        if (ss < 0 || kind_vardim(kind[t]) != d) { free(fvals); return -1; }
        int k = ss * d;
        int shell = kind[t] == OR_SHELL_TRI || kind[t] == OR_MLP;
        int rest_stride = rest_stride_of(kind[t]);
        double *nrm = NULL;
        if (shell) { /* passive unit vertex normals of the current positions, over this term's triangles */
            nrm = malloc(sizeof(double) * (size_t)(3 * nv));
            if (!nrm) { free(fvals); return -4; }
            oracle_vertex_normals(nv, n_elem[t], stencil[t], x, nrm);
        }
        for (int64_t e = 0; e < n_elem[t]; ++e) {
            const int32_t *s = stencil[t] + ss * e;
            double xloc[KMAX];
            int touches = (row_mask == NULL);
            for (int a = 0; a < ss; ++a) {
                for (int c = 0; c < d; ++c) xloc[a * d + c] = x[(int64_t)s[a] * d + c];
                if (row_mask && row_mask[s[a]]) touches = 1;
            }
            if (!touches && !(mode & OR_ENERGY)) continue; /* contributes to no requested output */
            const double *rs = rest_stride ? rest[t] + rest_stride * e : NULL;
            double aux[9];
            if (shell)
                for (int a = 0; a < 3; ++a)
                    for (int c = 0; c < 3; ++c) aux[3 * a + c] = nrm[3 * (int64_t)s[a] + c];
            int want_deriv = touches && (mode & (OR_GRAD | OR_HESS));
            hd r;
            if (eval_elem(kind[t], want_deriv ? k : 0, params[t], rs, aux, xloc, &r) != 0) {
                free(nrm);
                free(fvals);
                return -1;
            }
            fvals[fi++] = r.v;
            abs_sum += fabs(r.v);
            if (!want_deriv) continue;
            if ((mode & OR_GRAD) && grad) {
                double gmax = 0.0;
                for (int i = 0; i < k; ++i) gmax = fabs(r.g[i]) > gmax ? fabs(r.g[i]) : gmax;
                for (int a = 0; a < ss; ++a) {
                    if (row_mask && !row_mask[s[a]]) continue;
                    for (int c = 0; c < d; ++c) {
                        grad[(int64_t)s[a] * d + c] += r.g[a * d + c];
                        if (gscale) gscale[(int64_t)s[a] * d + c] += gmax;
                    }
                }
            }
            if ((mode & OR_HESS) && hess) {
                double Hl[KMAX * KMAX], Hp[KMAX * KMAX];
                for (int i = 0; i < k; ++i)
                    for (int j = 0; j < k; ++j) Hl[i * k + j] = r.h[i][j];
                if (mode & OR_SPD) oracle_spd_project(k, Hl, spd_eps, Hp);
                else memcpy(Hp, Hl, sizeof(double) * k * k);
                /* the entry scale: the element's largest Hessian entry, before or after the clamp (the
                   clamp's eigen-decomposition errs relative to the matrix it decomposes; an element whose
                   Hessian clamps to zero would otherwise be measured against its own rounding noise) */
                double hmax = 0.0;
                for (int i = 0; i < k * k; ++i) {
                    hmax = fabs(Hp[i]) > hmax ? fabs(Hp[i]) : hmax;
                    hmax = fabs(Hl[i]) > hmax ? fabs(Hl[i]) : hmax;
                }
                for (int a = 0; a < ss; ++a) {
                    if (row_mask && !row_mask[s[a]]) continue;
                    for (int b = 0; b < ss; ++b) {
                        int64_t blk = find_block(rowptr, colidx, s[a], s[b]);
                        if (blk < 0) { free(nrm); free(fvals); return -5; }
                        for (int i = 0; i < d; ++i)
                            for (int j = 0; j < d; ++j) {
                                hess[blk * d * d + i * d + j] += Hp[(a * d + i) * k + (b * d + j)];
                                if (hscale) hscale[blk * d * d + i * d + j] += hmax;
                            }
                    }
                }
            }
        }
    }
    if (energy) *energy = oracle_neumaier_sum(fi, fvals);
    if (esum_abs) *esum_abs = abs_sum;
    free(fvals);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* The same evaluation spread over threads (CPU baseline timing).             */
/* ------------------------------------------------------------------------- */
/* Phase 1 evaluates the elements in parallel into per-element storage (the same element code as
 * oracle_eval). Phase 2 sums every block row in one thread, from the elements touching its vertex in the
 * serial order (terms in add order, elements ascending, stencil slots ascending), starting from zero: each
 * output entry is the same sequence of additions as in oracle_eval, so the results are bit-identical to
 * it in the same build. The energy is the same Neumaier sum over the element energies in order. */
int oracle_eval_par(int64_t nv, int var_dim, int n_terms, const int *kind, const int64_t *n_elem,
                    const int32_t *const *stencil, const double *const *rest, const double *const *params,
                    const double *x, int mode, double spd_eps, const int32_t *rowptr, const int32_t *colidx,
                    int threads, double *energy, double *esum_abs, double *grad, double *hess) {
    const int d = var_dim;
    if (n_terms <= 0 || n_terms > 16) return -1;
    int64_t eoff[17], goff[17], hoff[17];
    int ks[16], sss[16];
    eoff[0] = goff[0] = hoff[0] = 0;
    for (int t = 0; t < n_terms; ++t) {
        sss[t] = kind_stencil(kind[t]);
        if (sss[t] < 0 || kind_vardim(kind[t]) != d) return -1;
        ks[t] = sss[t] * d;
        eoff[t + 1] = eoff[t] + n_elem[t];
        goff[t + 1] = goff[t] + ((mode & OR_GRAD) ? n_elem[t] * ks[t] : 0);
        hoff[t + 1] = hoff[t] + ((mode & OR_HESS) ? n_elem[t] * ks[t] * ks[t] : 0);
    }
    const int64_t total = eoff[n_terms];
    const int want_deriv = (mode & (OR_GRAD | OR_HESS)) != 0;
    double *fvals = malloc(sizeof(double) * (size_t)(total > 0 ? total : 1));
    double *gl = malloc(sizeof(double) * (size_t)(goff[n_terms] > 0 ? goff[n_terms] : 1));
    double *hl = malloc(sizeof(double) * (size_t)(hoff[n_terms] > 0 ? hoff[n_terms] : 1));
    double *nrm = malloc(sizeof(double) * (size_t)(3 * nv * n_terms > 0 ? 3 * nv * n_terms : 1));
    int err = 0;
    if (!fvals || !gl || !hl || !nrm) err = -4;
    for (int t = 0; !err && t < n_terms; ++t)
        if (kind[t] == OR_SHELL_TRI || kind[t] == OR_MLP)
            oracle_vertex_normals(nv, n_elem[t], stencil[t], x, nrm + 3 * nv * t);
#pragma omp parallel for schedule(dynamic, 256) num_threads(threads) if (!err)
    for (int64_t i = 0; i < total; ++i) {
        int t = 0;
        while (i >= eoff[t + 1]) ++t;
        const int64_t e = i - eoff[t];
        const int ss = sss[t], k = ks[t];
        const int32_t *s = stencil[t] + ss * e;
        double xloc[KMAX], aux[9];
        for (int a = 0; a < ss; ++a)
            for (int c = 0; c < d; ++c) xloc[a * d + c] = x[(int64_t)s[a] * d + c];
        if (kind[t] == OR_SHELL_TRI || kind[t] == OR_MLP)
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) aux[3 * a + c] = nrm[3 * nv * t + 3 * (int64_t)s[a] + c];
        const int rsd = rest_stride_of(kind[t]);
        hd r;
        if (eval_elem(kind[t], want_deriv ? k : 0, params[t], rsd ? rest[t] + rsd * e : NULL, aux, xloc, &r) != 0) {
#pragma omp atomic write
            err = -1;
            continue;
        }
        fvals[i] = r.v;
        if (mode & OR_GRAD)
            for (int q = 0; q < k; ++q) gl[goff[t] + e * k + q] = r.g[q];
        if (mode & OR_HESS) {
            double Hl[KMAX * KMAX];
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b) Hl[a * k + b] = r.h[a][b];
            double *Hp = hl + hoff[t] + e * k * k;
            if (mode & OR_SPD) oracle_spd_project(k, Hl, spd_eps, Hp);
            else memcpy(Hp, Hl, sizeof(double) * k * k);
        }
    }
    /* vertex -> (element, slot) incidence in the serial order */
    int64_t *iptr = NULL, *inc = NULL;
    if (!err && want_deriv) {
        iptr = calloc((size_t)nv + 1, sizeof(int64_t));
        int64_t slots = 0;
        for (int t = 0; t < n_terms; ++t) slots += n_elem[t] * sss[t];
        inc = malloc(sizeof(int64_t) * (size_t)(slots > 0 ? slots : 1));
        if (!iptr || !inc) err = -4;
        for (int t = 0; !err && t < n_terms; ++t)
            for (int64_t j = 0; j < n_elem[t] * sss[t]; ++j) iptr[stencil[t][j] + 1]++;
        for (int64_t v = 0; !err && v < nv; ++v) iptr[v + 1] += iptr[v];
        int64_t *fill = err ? NULL : malloc(sizeof(int64_t) * (size_t)(nv > 0 ? nv : 1));
        if (!err && !fill) err = -4;
        if (!err) {
            memcpy(fill, iptr, sizeof(int64_t) * (size_t)nv);
            for (int t = 0; t < n_terms; ++t)
                for (int64_t e = 0; e < n_elem[t]; ++e)
                    for (int a = 0; a < sss[t]; ++a)
                        inc[fill[stencil[t][sss[t] * e + a]]++] = ((eoff[t] + e) << 4) | a;
        }
        free(fill);
    }
    if (!err && (mode & OR_GRAD) && grad) memset(grad, 0, sizeof(double) * (size_t)(nv * d));
    if (!err && (mode & OR_HESS) && hess) memset(hess, 0, sizeof(double) * (size_t)(rowptr[nv] * d * d));
    if (!err && want_deriv) {
#pragma omp parallel for schedule(dynamic, 512) num_threads(threads)
        for (int64_t v = 0; v < nv; ++v) {
            for (int64_t q = iptr[v]; q < iptr[v + 1]; ++q) {
                const int64_t i = inc[q] >> 4;
                const int a = (int)(inc[q] & 15);
                int t = 0;
                while (i >= eoff[t + 1]) ++t;
                const int64_t e = i - eoff[t];
                const int ss = sss[t], k = ks[t];
                const int32_t *s = stencil[t] + ss * e;
                if ((mode & OR_GRAD) && grad)
                    for (int c = 0; c < d; ++c) grad[v * d + c] += gl[goff[t] + e * k + a * d + c];
                if ((mode & OR_HESS) && hess) {
                    const double *Hp = hl + hoff[t] + e * k * k;
                    for (int b = 0; b < ss; ++b) {
                        int64_t blk = find_block(rowptr, colidx, (int32_t)v, s[b]);
                        if (blk < 0) {
#pragma omp atomic write
                            err = -5;
                            continue;
                        }
                        for (int ii = 0; ii < d; ++ii)
                            for (int jj = 0; jj < d; ++jj)
                                hess[blk * d * d + ii * d + jj] += Hp[(a * d + ii) * k + (b * d + jj)];
                    }
                }
            }
        }
    }
    if (!err) {
        if (energy) *energy = oracle_neumaier_sum(total, fvals);
        if (esum_abs) {
            double abs_sum = 0.0;
            for (int64_t i = 0; i < total; ++i) abs_sum += fabs(fvals[i]);
            *esum_abs = abs_sum;
        }
    }
    free(fvals);
    free(gl);
    free(hl);
    free(nrm);
    free(iptr);
    free(inc);
    return err;
}

/* ------------------------------------------------------------------------- */
/* Residual terms and the global sparse Jacobian (Sec. 4.1 Eq. 3, Sec. 6.1).  */
/* ------------------------------------------------------------------------- */
int oracle_kind_nres(int kind) {
    switch (kind) {
    case OR_RES_POSITION: return 3;
    case OR_RES_EDGE: return 1;
    default: return 0;
    }
}

static int res_rest_stride(int kind) { return kind == OR_RES_POSITION ? 4 : (kind == OR_RES_EDGE ? 1 : 0); }

int oracle_residual(int kind, const double *params, const double *rest, const double *xloc, double *r, double *J) {
    int ss = kind_stencil(kind), vd = kind_vardim(kind), m = oracle_kind_nres(kind);
    if (ss < 0 || vd < 0 || m == 0 || m > 3) return -1;
    int k = ss * vd;
    hd res[3];
    res_elem(kind, k, params, rest, xloc, res);
    for (int i = 0; i < m; ++i) {
        if (r) r[i] = res[i].v;
        if (J)
            for (int a = 0; a < k; ++a) J[i * k + a] = res[i].g[a];
    }
    return 0;
}

int oracle_jacobian(int64_t nv, int var_dim, int n_terms, const int *kind, const int64_t *n_elem,
                    const int32_t *const *stencil, const double *const *rest, const double *const *params,
                    const double *x, double *r, int32_t *rowptr, int32_t *colidx, double *vals) {
    const int d = var_dim;
    int64_t row = 0, nz = 0;
    rowptr[0] = 0;
    for (int t = 0; t < n_terms; ++t) {
        int m = oracle_kind_nres(kind[t]);
        if (m == 0) continue;
        int ss = kind_stencil(kind[t]);
        if (ss < 0 || kind_vardim(kind[t]) != d) return -1;
        int k = ss * d;
        for (int64_t e = 0; e < n_elem[t]; ++e) {
            const int32_t *s = stencil[t] + ss * e;
            double xloc[KMAX], rr[3], J[3 * KMAX];
            for (int a = 0; a < ss; ++a) {
                if (s[a] < 0 || s[a] >= nv) return -1;
                for (int c = 0; c < d; ++c) xloc[a * d + c] = x[(int64_t)s[a] * d + c];
            }
            const double *rs = rest[t] ? rest[t] + res_rest_stride(kind[t]) * e : NULL;
            if (oracle_residual(kind[t], params[t], rs, xloc, rr, J) != 0) return -1;
            /* columns of the element: stencil DOFs, ascending global index */
            int64_t col[KMAX];
            int loc[KMAX];
            for (int i = 0; i < k; ++i) {
                col[i] = (int64_t)s[i / d] * d + i % d;
                loc[i] = i;
            }
            for (int i = 1; i < k; ++i)
                for (int j = i; j > 0 && col[loc[j - 1]] > col[loc[j]]; --j) {
                    int tmp = loc[j];
                    loc[j] = loc[j - 1];
                    loc[j - 1] = tmp;
                }
            for (int i = 0; i < m; ++i) {
                if (r) r[row] = rr[i];
                for (int j = 0; j < k; ++j) {
                    if (colidx) colidx[nz] = (int32_t)col[loc[j]];
                    if (vals) vals[nz] = J[i * k + loc[j]];
                    ++nz;
                }
                rowptr[++row] = (int32_t)nz;
            }
        }
    }
    return 0;
}
