/*
 * Plain FP64 CPU oracle for per-element second-order forward-mode AD on
 * triangle meshes and its sparse assembly.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The HIP product path
 * never calls it, links it or shares code with it.
 *
 * What it computes (Sec. 4.1, Eq. 1-2): F(x) = sum_j f_j(S_j x),
 * g = sum_j S_j^T grad f_j, H = sum_j S_j^T P(hess f_j) S_j, where each f_j
 * is differentiated by dense hyper-dual arithmetic over the element's stencil
 * DOFs (Sec. 5.1, Sec. 6.2) and P is the per-term eigenvalue clamp of
 * Sec. 7.1 (identity when projection is off). Element order is input order,
 * terms in the order given; sums are serial; the energy uses Neumaier
 * compensated summation.
 *
 * Every call returns 0 on success, a negative code on bad input.
 */
#ifndef MAD_ORACLE_H
#define MAD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* term kinds (same numbering as the product library's catalogue) */
enum {
    OR_EDGE_SQLEN = 1,   /* Listing 1: |x0 - x1|^2 over an edge, VarDim 3, k = 6 */
    OR_TRI_AREA = 2,     /* Sec. 7.6: triangle area, VarDim 3, k = 9 */
    OR_DIRICHLET = 3,    /* scalar Dirichlet energy 0.5 A |grad u|^2, VarDim 1, k = 3 */
    OR_STVK = 4,         /* StVK membrane, VarDim 3, k = 9 */
    OR_BENDING = 5,      /* Sec. 7.7 dihedral bending over an edge diamond, VarDim 3, k = 12 */
    OR_SYMDIR = 6,       /* Sec. 7.2 symmetric Dirichlet, VarDim 2, k = 6 */
    OR_MLP = 7,          /* learned per-triangle density A psi(z), VarDim 3, k = 9 */
    OR_SHELL_TRI = 8,    /* analytic per-triangle shell density A W(z), VarDim 3, k = 9 */
    OR_SPRING = 9,       /* Sec. 7.1 mass-spring edge: w k/2 l^2 (|x0 - x1|^2 / l^2 - 1)^2, VarDim 3, k = 6 */
    OR_INERTIA = 10,     /* Sec. 7.1 per-vertex inertia and gravity: m/2 |x - xhat|^2 - w m g.x, VarDim 3, k = 3 */
    /* residual terms (Sec. 4.1, Eq. 3): r_j in R^m; as scalar terms they contribute 1/2 |r_j|^2 with the
     * Gauss-Newton matrix J_j^T J_j in place of the Hessian */
    OR_RES_POSITION = 11, /* vertex: r = sqrt(w) (x - x_t), m = 3, rest {w, x_t}, VarDim 3, k = 3 */
    OR_RES_EDGE = 12      /* edge: r = sqrt(k_s) (|x0 - x1| - l), m = 1, rest {l}, params {k_s}, k = 6 */
};

/* eval mode bits */
enum { OR_ENERGY = 1, OR_GRAD = 2, OR_HESS = 4, OR_SPD = 8 };

/* ---- topology (Sec. 6: edges of the triangle mesh, edge diamonds) ---- */
/* edges: unique undirected edges sorted by (min, max); out arrays sized 3*nt.
 * edge_nf[e] = number of incident faces. diamonds (interior edges, exactly two
 * incident faces): (v0, v1, v2, v3) with f1 the lower face index, (v0, v1) the
 * edge as directed in f1, v2 opposite in f1, v3 opposite in f2. Returns 0 or
 * -1 on an out-of-range vertex index or degenerate face. */
int oracle_topology(int64_t nv, int64_t nt, const int32_t *tris,
                    int64_t *n_edges, int32_t *edges, int32_t *edge_nf,
                    int64_t *n_diamonds, int32_t *diamonds, int32_t *diamond_faces);

/* ---- rest data ---- */
/* per triangle: Dm^{-1} (2x2 row-major) of the rest triangle in its own 2D
 * frame, and rest area. Returns -2 if a rest triangle has zero area. */
int oracle_rest_tri(int64_t nt, const int32_t *tris, const double *rest,
                    double *dminv, double *area);
/* per diamond: mean rest area of its two faces and rest dihedral angle. */
int oracle_rest_diamond(int64_t nd, const int32_t *diamonds, const int32_t *diamond_faces,
                        const int32_t *tris, const double *rest, double *abar, double *theta0);

/* ---- pattern (Sec. 6.1) ---- */
/* Block pattern over vertices: {(i,i)} U {(s_a, s_b)} for every element of
 * every term. Two-phase: call with colidx == NULL to get *nnzb, then again
 * with colidx sized nnzb. rowptr has nv+1 entries. Returns -3 on int32 overflow. */
int oracle_pattern(int64_t nv, int n_terms, const int64_t *n_elem, const int *stencil_size,
                   const int32_t *const *stencils, int32_t *rowptr, int32_t *colidx, int64_t *nnzb);

/* ---- one element (Sec. 6.2) ---- */
/* xloc: the stencil DOFs (k = stencil * var_dim values), rest: per-element rest
 * data of the kind, aux: the three unit vertex normals (kinds OR_SHELL_TRI and
 * OR_MLP, else unused), params: the term's constants. Outputs f, g[k], H[k*k]. */
int oracle_element(int kind, const double *params, const double *rest, const double *aux, const double *xloc,
                   int mode, double spd_eps, double *f, double *g, double *H);

/* ---- evaluation + assembly (Eq. 1-2) ---- */
/* x: [nv*var_dim]. For each term t: kind[t], n_elem[t], stencil[t]
 * ([n_elem][ss]), rest[t] (per-element rest data), params[t].
 * row_mask (nullable, char[nv]): if given, derivatives are assembled only into
 * masked block rows / gradient entries (elements touching no masked vertex
 * are evaluated passively for the energy, or skipped when mode has no
 * OR_ENERGY bit).
 * Outputs (nullable when not requested): energy[1], esum_abs[1] (sum |f_j|),
 * grad[nv*var_dim], gscale[nv*var_dim], hess[nnzb*var_dim^2], hscale[same].
 * gscale / hscale accumulate, for each entry, the max-abs entry of every
 * element gradient / element Hessian that adds into it. */
int oracle_eval(int64_t nv, int var_dim, int n_terms, const int *kind, const int64_t *n_elem,
                const int32_t *const *stencil, const double *const *rest,
                const double *const *params, const double *x, int mode, double spd_eps,
                const char *row_mask, const int32_t *rowptr, const int32_t *colidx,
                double *energy, double *esum_abs, double *grad, double *gscale,
                double *hess, double *hscale);

/* The same evaluation over `threads` OpenMP threads (no row mask, no scales): elements in parallel, then
 * each block row summed by one thread in the serial order, so the outputs are bit-identical to
 * oracle_eval in the same build. Used to time the oracle on all host cores. */
int oracle_eval_par(int64_t nv, int var_dim, int n_terms, const int *kind, const int64_t *n_elem,
                    const int32_t *const *stencil, const double *const *rest, const double *const *params,
                    const double *x, int mode, double spd_eps, const int32_t *rowptr, const int32_t *colidx,
                    int threads, double *energy, double *esum_abs, double *grad, double *hess);

/* ---- per-triangle shell features and densities (project-defined; no paper counterpart) ----
 * z = (E00, E11, E01, II00 - rII00, II11 - rII11, II01 - rII01) with F = Ds Dm^{-1},
 * E = (F^T F - I)/2, N = [n_b - n_a, n_c - n_a] Dm^{-1} from passive unit vertex normals,
 * II = -(N^T F + F^T N)/2. Kind OR_SHELL_TRI: f = A W(z), params (mu, lambda, k_b),
 * W = mu (E00^2 + E11^2 + 2 E01^2) + lambda/2 (E00 + E11)^2 + k_b/2 (dII00^2 + dII11^2 + 2 dII01^2).
 * Kind OR_MLP: f = A psi(z), params [H, s_out, s_in(6), W1(Hx6), b1(H), W2(HxH), b2(H), w3(H), b3],
 * psi(z) = s_out (w3 . sp(W2 sp(W1 (s_in*z) + b1) + b2) + b3), sp = softplus, H <= 64.
 * Rest data of both kinds, per triangle: [Dm^{-1} (4), rest area, rest II (3)]. */
int oracle_vertex_normals(int64_t nv, int64_t nt, const int32_t *tris, const double *x, double *out);
int oracle_rest_shell(int64_t nv, int64_t nt, const int32_t *tris, const double *rest, double *out);
int oracle_shell_features(int64_t nv, int64_t nt, const int32_t *tris, const double *rest8, const double *x,
                          double *z);
int oracle_shell_density(int64_t n, const double *z, const double *params, double *W, double *dW);
int oracle_mlp_eval(int64_t n, const double *z, const double *params, double *psi, double *dpsi, double *d2psi);

/* symmetric eigen-clamp of an n x n matrix (cyclic Jacobi, Sec. 7.1 filtering) */
int oracle_spd_project(int n, const double *A, double eps, double *out);

/* Neumaier compensated sum (the energy reduction of Sec. 5.5) */
double oracle_neumaier_sum(int64_t n, const double *v);

/* ---- residual terms and the sparse Jacobian (Sec. 4.1 Eq. 3, Sec. 6.1) ---- */
/* residual count m of a kind (0 for scalar kinds) */
int oracle_kind_nres(int kind);
/* one element: residuals r[m] and the local Jacobian J[m][k] (row-major, stencil DOF order) */
int oracle_residual(int kind, const double *params, const double *rest, const double *xloc, double *r, double *J);
/* Global residual and Jacobian (Eq. 3): rows in term order, then element order (element e of term t owns
 * rows roff_t + e m_t ... + m_t - 1); each row's columns are the element's stencil DOFs v*var_dim + c,
 * ascending. Scalar terms own no rows. r[m_total], rowptr[m_total + 1], colidx / vals [nnz]. Pass
 * colidx = vals = NULL to get rowptr (and so nnz = rowptr[m_total]) only. */
int oracle_jacobian(int64_t nv, int var_dim, int n_terms, const int *kind, const int64_t *n_elem,
                    const int32_t *const *stencil, const double *const *rest, const double *const *params,
                    const double *x, double *r, int32_t *rowptr, int32_t *colidx, double *vals);

#ifdef __cplusplus
}
#endif
#endif
