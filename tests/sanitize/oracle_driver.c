/* Sanitizer harness of the CPU oracle (built with gcc under AddressSanitizer + UndefinedBehaviorSanitizer by
 * tests/test_sanitize.py): every entry point of oracle.h on a small rolled grid, every element kind, the
 * serial and threaded evaluations (which must agree bitwise), the residual Jacobian, the shell features and
 * the network. Exits non-zero on a failed call or a violated check. Test infrastructure only. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            exit(2);                                                          \
        }                                                                     \
    } while (0)

enum { N = 12, NV = N * N, NT = 2 * (N - 1) * (N - 1) };

static void *xcalloc(size_t n, size_t s) {
    void *p = calloc(n ? n : 1, s);
    CHECK(p != NULL);
    return p;
}

int main(void) {
    int32_t tris[3 * NT];
    double rest[3 * NV], x[3 * NV];
    int t = 0;
    for (int j = 0; j + 1 < N; ++j)
        for (int i = 0; i + 1 < N; ++i) {
            const int32_t v00 = j * N + i, v10 = v00 + 1, v01 = v00 + N, v11 = v01 + 1;
            const int32_t f[6] = {v00, v10, v11, v00, v11, v01};
            memcpy(tris + 3 * t, f, sizeof f);
            t += 2;
        }
    const double h = 1.0 / (N - 1), R = 1.0 / 3.14159265358979;
    for (int v = 0; v < NV; ++v) {
        const double s = (v % N) * h, u = (v / N) * h;
        rest[3 * v] = s, rest[3 * v + 1] = u, rest[3 * v + 2] = 0.0;
        const double w = 1e-3 * h * sin(12.9898 * v + 78.233);
        x[3 * v] = R * sin(s / R) + w, x[3 * v + 1] = u - w, x[3 * v + 2] = R * (1.0 - cos(s / R)) + 0.5 * w;
    }
    /* topology */
    int64_t ne = 0, nd = 0;
    int32_t *edges = xcalloc(6 * NT, 4), *enf = xcalloc(3 * NT, 4), *dia = xcalloc(12 * NT, 4),
            *dfc = xcalloc(6 * NT, 4);
    CHECK(oracle_topology(NV, NT, tris, &ne, edges, enf, &nd, dia, dfc) == 0);
    CHECK(ne == 3 * (N - 1) * (N - 1) + 2 * (N - 1) && nd > 0);
    /* rest data */
    double *tri_rest = xcalloc(5 * NT, 8), *dminv = xcalloc(4 * NT, 8), *area = xcalloc(NT, 8);
    CHECK(oracle_rest_tri(NT, tris, rest, dminv, area) == 0);
    for (int f = 0; f < NT; ++f) {
        memcpy(tri_rest + 5 * f, dminv + 4 * f, 4 * sizeof(double));
        tri_rest[5 * f + 4] = area[f];
    }
    double *abar = xcalloc(nd, 8), *th0 = xcalloc(nd, 8), *dia_rest = xcalloc(2 * nd, 8);
    CHECK(oracle_rest_diamond(nd, dia, dfc, tris, rest, abar, th0) == 0);
    for (int64_t e = 0; e < nd; ++e) dia_rest[2 * e] = abar[e], dia_rest[2 * e + 1] = th0[e];
    /* pattern, two-phase */
    const int kinds[2] = {OR_STVK, OR_BENDING};
    const int64_t nel[2] = {NT, nd};
    const int ss[2] = {3, 4};
    const int32_t *st[2] = {tris, dia};
    const double *rs[2] = {tri_rest, dia_rest};
    const double prm0[4] = {1.0, 1.2, 0, 0}, prm1[4] = {0.8, 1.0, 0, 0};
    const double *prm[2] = {prm0, prm1};
    int32_t *rowptr = xcalloc(NV + 1, 4);
    int64_t nnzb = 0;
    CHECK(oracle_pattern(NV, 2, nel, ss, st, rowptr, NULL, &nnzb) == 0);
    int32_t *colidx = xcalloc(nnzb, 4);
    CHECK(oracle_pattern(NV, 2, nel, ss, st, rowptr, colidx, &nnzb) == 0);
    CHECK(rowptr[NV] == nnzb);
    /* evaluation: serial with scales and a row mask, and threaded (bitwise equal to serial) */
    double e1 = 0, ea = 0, e2 = 0, ea2 = 0;
    double *g = xcalloc(3 * NV, 8), *gs = xcalloc(3 * NV, 8), *H = xcalloc(9 * nnzb, 8), *hs = xcalloc(9 * nnzb, 8);
    double *g2 = xcalloc(3 * NV, 8), *H2 = xcalloc(9 * nnzb, 8);
    char mask[NV];
    for (int v = 0; v < NV; ++v) mask[v] = (char)(v % 7 == 0);
    const int mode = OR_ENERGY | OR_GRAD | OR_HESS | OR_SPD;
    CHECK(oracle_eval(NV, 3, 2, kinds, nel, st, rs, prm, x, mode, 0.0, mask, rowptr, colidx, &e1, &ea, g, gs, H, hs) == 0);
    CHECK(oracle_eval(NV, 3, 2, kinds, nel, st, rs, prm, x, mode, 1e-3, NULL, rowptr, colidx, &e1, &ea, g, gs, H, hs) == 0);
    CHECK(oracle_eval(NV, 3, 2, kinds, nel, st, rs, prm, x, mode, 0.0, NULL, rowptr, colidx, &e1, &ea, g, gs, H, hs) == 0);
    CHECK(oracle_eval_par(NV, 3, 2, kinds, nel, st, rs, prm, x, mode, 0.0, rowptr, colidx, 3, &e2, &ea2, g2, H2) == 0);
    CHECK(e1 == e2 && memcmp(g, g2, 3 * NV * sizeof(double)) == 0 && memcmp(H, H2, 9 * nnzb * sizeof(double)) == 0);
    double gsum[3] = {0, 0, 0};
    for (int v = 0; v < NV; ++v)
        for (int c = 0; c < 3; ++c) gsum[c] += g[3 * v + c];
    for (int c = 0; c < 3; ++c) CHECK(fabs(gsum[c]) < 1e-9);   /* translation invariance */
    /* every element kind */
    double f, ge[12], He[144];
    const double xl[12] = {0.1, 0.0, 0.02, 1.05, 0.1, -0.03, 0.2, 0.95, 0.05, 0.9, -0.8, 0.1};
    const double r5[5] = {1.0, 0.0, 0.0, 1.0, 0.5}, r2[2] = {0.5, 0.1}, r1[1] = {1.1}, r4[4] = {2.0, 0.1, 0.0, 0.1};
    const double pr[4] = {1.0, 1.0, 1.0, 0.0}, ax[9] = {0, 0, 1, 0, 0.1, 0.99, 0.1, 0, 0.99};
    CHECK(oracle_element(OR_EDGE_SQLEN, pr, NULL, NULL, xl, 7, 0.0, &f, ge, He) == 0);
    CHECK(oracle_element(OR_TRI_AREA, pr, NULL, NULL, xl, 15, 0.0, &f, ge, He) == 0);
    CHECK(oracle_element(OR_DIRICHLET, pr, r5, NULL, xl, 7, 0.0, &f, ge, He) == 0);
    CHECK(oracle_element(OR_STVK, pr, r5, NULL, xl, 15, 0.0, &f, ge, He) == 0);
    CHECK(oracle_element(OR_BENDING, pr, r2, NULL, xl, 15, 0.0, &f, ge, He) == 0);
    CHECK(oracle_element(OR_SYMDIR, pr, r5, NULL, xl, 15, 0.0, &f, ge, He) == 0);
    CHECK(oracle_element(OR_SPRING, pr, r1, NULL, xl, 15, 0.0, &f, ge, He) == 0);
    CHECK(oracle_element(OR_INERTIA, pr, r4, NULL, xl, 15, 0.0, &f, ge, He) == 0);
    CHECK(oracle_element(OR_RES_POSITION, pr, r4, NULL, xl, 7, 0.0, &f, ge, He) == 0);
    CHECK(oracle_element(OR_RES_EDGE, pr, r1, NULL, xl, 7, 0.0, &f, ge, He) == 0);
    const double r8[8] = {1.0, 0.0, 0.0, 1.0, 0.5, 0.0, 0.0, 0.0};
    CHECK(oracle_element(OR_SHELL_TRI, pr, r8, ax, xl, 15, 0.0, &f, ge, He) == 0);
    /* a 4-unit network: [H, s_out, s_in(6), W1(4x6), b1(4), W2(4x4), b2(4), w3(4), b3] */
    enum { HH = 4, NP = 2 + 6 + HH * 6 + HH + HH * HH + HH + HH + 1 };
    double net[NP];
    net[0] = HH, net[1] = 0.7;
    for (int i = 2; i < NP; ++i) net[i] = 0.3 * sin(1.7 * i);
    CHECK(oracle_element(OR_MLP, net, r8, ax, xl, 15, 0.0, &f, ge, He) == 0);
    /* eigen-clamp, compensated sum */
    double A[81], out[81];
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j) A[9 * i + j] = A[9 * j + i] = sin(1.0 + i + 3.0 * j) + sin(1.0 + j + 3.0 * i);
    CHECK(oracle_spd_project(9, A, 0.0, out) == 0);
    const double vals[4] = {1e16, 1.0, -1e16, 1.0};
    CHECK(oracle_neumaier_sum(4, vals) == 2.0);
    /* shell features, density and network batch */
    double *nrm = xcalloc(3 * NV, 8), *r8s = xcalloc(8 * NT, 8), *z = xcalloc(6 * NT, 8), *W = xcalloc(NT, 8),
           *dW = xcalloc(6 * NT, 8), *psi = xcalloc(NT, 8), *dpsi = xcalloc(6 * NT, 8), *d2 = xcalloc(36 * NT, 8);
    CHECK(oracle_vertex_normals(NV, NT, tris, x, nrm) == 0);
    CHECK(oracle_rest_shell(NV, NT, tris, rest, r8s) == 0);
    CHECK(oracle_shell_features(NV, NT, tris, r8s, x, z) == 0);
    CHECK(oracle_shell_density(NT, z, pr, W, dW) == 0);
    CHECK(oracle_mlp_eval(NT, z, net, psi, dpsi, d2) == 0);
    /* residual terms and the Jacobian */
    const int rk[2] = {OR_RES_EDGE, OR_RES_POSITION};
    double *elen = xcalloc(ne, 8), *vres = xcalloc(4 * NV, 8);
    for (int64_t e = 0; e < ne; ++e) {
        double s2 = 0;
        for (int c = 0; c < 3; ++c) {
            const double dv = rest[3 * edges[2 * e] + c] - rest[3 * edges[2 * e + 1] + c];
            s2 += dv * dv;
        }
        elen[e] = sqrt(s2);
    }
    int32_t *vid = xcalloc(NV, 4);
    for (int v = 0; v < NV; ++v) {
        vid[v] = v;
        vres[4 * v] = (v % 5 == 0) ? 2.0 : 0.0;
        for (int c = 0; c < 3; ++c) vres[4 * v + 1 + c] = rest[3 * v + c];
    }
    const int64_t rn[2] = {ne, NV};
    const int32_t *rst[2] = {edges, vid};
    const double *rrs[2] = {elen, vres};
    const double rp0[4] = {3.0, 0, 0, 0};
    const double *rpm[2] = {rp0, rp0};
    const int64_t m = ne + 3 * NV;
    double *res = xcalloc(m, 8);
    int32_t *jrp = xcalloc(m + 1, 4);
    CHECK(oracle_jacobian(NV, 3, 2, rk, rn, rst, rrs, rpm, x, res, jrp, NULL, NULL) == 0);
    int32_t *jci = xcalloc(jrp[m], 4);
    double *jv = xcalloc(jrp[m], 8);
    CHECK(oracle_jacobian(NV, 3, 2, rk, rn, rst, rrs, rpm, x, res, jrp, jci, jv) == 0);
    printf("oracle checks passed: %d triangles, %lld diamonds, %lld blocks, energy %.12e\n", NT, (long long)nd,
           (long long)nnzb, e1);
    free(edges), free(enf), free(dia), free(dfc), free(tri_rest), free(dminv), free(area), free(abar), free(th0);
    free(dia_rest), free(rowptr), free(colidx), free(g), free(gs), free(H), free(hs), free(g2), free(H2);
    free(nrm), free(r8s), free(z), free(W), free(dW), free(psi), free(dpsi), free(d2), free(elen), free(vres);
    free(vid), free(res), free(jrp), free(jci), free(jv);
    return 0;
}
