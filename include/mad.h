/*
 * mad.h -- C ABI of the locality-aware mesh AD library for MI355X (gfx950).
 *
 * The library evaluates objectives of the partially separable form of
 * Sec. 4.1, Eq. 1, F(x) = sum_j f_j(S_j x), over the elements of a triangle
 * mesh, differentiates every local term by second-order forward-mode AD over
 * the element's stencil (Sec. 5.1, Sec. 6.2), and assembles the global
 * gradient and the sparse block-CSR Hessian of Eq. 2 on the GPU, with the
 * block pattern built once from connectivity (Sec. 6.1). Each term's local
 * Hessian can be filtered by clamping its eigenvalues from below before
 * assembly (Sec. 7.1).
 *
 * The paper's user lambdas cannot cross a C ABI; terms come from a fixed
 * catalogue (mad_term_kind) with a per-term parameter block.
 *
 * Conventions
 *  - Every call returns a mad_status; 0 is success. On failure
 *    mad_last_error() (thread-local) describes the cause. Argument and mesh
 *    validation is synchronous and happens before any device work.
 *  - Pointers named *_host are host memory; *_dev are device memory of the
 *    current HIP device; stream is a hipStream_t (NULL = default stream).
 *  - The caller owns every *_dev buffer it passes (DOFs and outputs). The
 *    library owns the mesh topology, patches, pattern and its scratch.
 *  - DOFs are vertex-major and interleaved: x[v * var_dim + c].
 *  - Hessian values are stored per block, row-major inside each
 *    var_dim x var_dim block, blocks in CSR order: hess[b * d * d + i * d + j].
 *    Block rows/columns use the caller's vertex numbering, columns sorted
 *    ascending, every diagonal block present.
 *  - A problem must not be used from two host threads at once.
 */
#ifndef MAD_H
#define MAD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mad_mesh mad_mesh;
typedef struct mad_problem mad_problem;
typedef struct mad_mlp mad_mlp;

typedef enum mad_status {
    MAD_OK = 0,
    MAD_E_INVALID_ARG = -1,     /* null pointer, bad size, bad enum value */
    MAD_E_BAD_MESH = -2,        /* vertex index out of range, repeated vertex in a face */
    MAD_E_DEGENERATE_REST = -3, /* a rest triangle of a term has zero area */
    MAD_E_OVERFLOW = -4,        /* block count or stencil incidence exceeds int32 */
    MAD_E_OOM = -5,             /* device or host allocation failed */
    MAD_E_HIP = -6,             /* a HIP runtime call or kernel launch failed */
    MAD_E_STATE = -7,           /* call out of order (e.g. eval before finalize) */
    MAD_E_UNSUPPORTED = -8,     /* kind/var_dim/precision combination not provided */
    MAD_E_CAPACITY = -9,        /* a pattern update would exceed the reserved room, or an evaluation would
                                   exceed the static scratch of mad_problem_eval_static */
    MAD_E_INTERNAL = -10        /* a device-side consistency check failed during an evaluation (reported by
                                   mad_problem_status; the outputs of the evaluations since the previous
                                   status call are not valid) */
} mad_status;

/* Term catalogue. Stencil, VarDim and the params block of each kind:
 *  MAD_EDGE_SQLEN  edge (2 vertices), VarDim 3: |x0 - x1|^2 (Listing 1). params unused.
 *  MAD_TRI_AREA    face (3 vertices), VarDim 3: triangle area (Sec. 7.6). params unused.
 *  MAD_DIRICHLET   face, VarDim 1: 0.5 * A * |grad u|^2 of a piecewise-linear scalar u over the
 *                  rest triangle (A = rest area). params unused. Needs rest positions.
 *  MAD_STVK        face, VarDim 3: A * (mu tr(E^2) + lambda/2 tr(E)^2), E = (F^T F - I)/2,
 *                  F = Ds Dm^{-1}. params = {mu, lambda}. Needs rest positions.
 *  MAD_BENDING     interior-edge diamond (4 vertices), VarDim 3 (Sec. 7.7):
 *                  k_b (A/3) (theta - theta_rest)^2 h^2, A = mean rest area of the two faces.
 *                  params = {k_b, h}. Needs rest positions. Boundary edges (one face) and
 *                  non-manifold edges (three or more faces) carry no bending term.
 *  MAD_SYMDIR      face, VarDim 2 (Sec. 7.2): A (|J|_F^2 + |J^{-1}|_F^2). params unused.
 *                  Needs rest positions.
 * The last two kinds are project-defined (the paper has no learned component). Both read the
 * per-triangle features z = (E00, E11, E01, II00 - rII00, II11 - rII11, II01 - rII01): E the
 * Green strain as above, II = -(N^T F + F^T N)/2 with N = [n_b - n_a, n_c - n_a] Dm^{-1} from the
 * area-weighted unit vertex normals of the current positions (recomputed every evaluation, not
 * differentiated), rII the same form on the rest mesh. Both need rest positions.
 *  MAD_MLP         face, VarDim 3: A psi(z), psi the network of a mad_mlp; added with
 *                  mad_problem_add_mlp_term, not mad_problem_add_term.
 *  MAD_SHELL_TRI   face, VarDim 3: A W(z), W = mu (E00^2 + E11^2 + 2 E01^2) + lambda/2 (E00 + E11)^2
 *                  + k_b/2 (dII00^2 + dII11^2 + 2 dII01^2). params = {mu, lambda, k_b}. The
 *                  analytic density the network is trained on (its fallback, and the reference its
 *                  error is measured against).
 * Mass-spring cloth (Sec. 7.1: implicit Euler, E = 1/2 |x - xhat|_M^2 + h^2 P(x)):
 *  MAD_SPRING      edge, VarDim 3: w (k/2) l^2 (|x0 - x1|^2 / l^2 - 1)^2, l the rest length.
 *                  params = {k, w} (w = h^2, the potential's weight). Needs rest positions.
 *  MAD_INERTIA     vertex (1 vertex), VarDim 3: (m/2) |x - xhat|^2 - w m g.x, params = {w, g_x,
 *                  g_y, g_z}. Per-vertex m and xhat come from a caller-owned device array read at
 *                  every evaluation; added with mad_problem_add_vertex_term.
 * Residual terms (Sec. 4.1, Eq. 3): each element returns a small residual vector r_j; the residuals
 * and the sparse Jacobian are read with mad_problem_jacobian. In mad_problem_eval / _hvp they act as
 * the scalar 1/2 |r_j|^2 whose gradient is J_j^T r_j and whose Hessian slot receives the Gauss-Newton
 * matrix J_j^T J_j (so the assembled "Hessian" of a residual-only problem is J^T J).
 *  MAD_RES_POSITION vertex, VarDim 3, 3 residuals: sqrt(w) (x - x_t), the paper's ActiveT<3>
 *                  positional constraint; per-vertex {w, x_t} (w >= 0; w = 0 leaves a vertex free)
 *                  from a caller-owned device array [n_verts][4]; added with
 *                  mad_problem_add_vertex_term. params unused.
 *  MAD_RES_EDGE    edge, VarDim 3, 1 residual: sqrt(k) (|x0 - x1| - l), l the rest length (a
 *                  least-squares spring). params = {k}. Needs rest positions.
 */
typedef enum mad_term_kind {
    MAD_EDGE_SQLEN = 1,
    MAD_TRI_AREA = 2,
    MAD_DIRICHLET = 3,
    MAD_STVK = 4,
    MAD_BENDING = 5,
    MAD_SYMDIR = 6,
    MAD_MLP = 7,
    MAD_SHELL_TRI = 8,
    MAD_SPRING = 9,
    MAD_INERTIA = 10,
    MAD_RES_POSITION = 11,
    MAD_RES_EDGE = 12
} mad_term_kind;

/* evaluation mode bits (Sec. 6.2: passive, gradient-only, full Hessian; Sec. 7.1 filtering) */
typedef enum mad_mode {
    MAD_ENERGY = 1,  /* write the FP64 energy (always computed) */
    MAD_GRAD = 2,    /* assemble the gradient */
    MAD_HESS = 4,    /* assemble the block-CSR Hessian */
    MAD_SPD = 8      /* clamp each term's local Hessian eigenvalues to >= spd_eps before assembly */
} mad_mode;

typedef enum mad_precision {
    MAD_F64 = 0,  /* derivative arithmetic and outputs in FP64 */
    MAD_F32 = 1   /* derivative arithmetic and outputs in FP32; primal values, energy in FP64 */
} mad_precision;

typedef enum mad_scatter {
    MAD_SCATTER_AUTO = 0,    /* library default (MAD_SCATTER_PATCH) */
    MAD_SCATTER_ATOMIC = 1,  /* one kernel per term; every element adds its gradient and Hessian
                                entries with device-wide atomics into pre-zeroed outputs (Sec. 5.5) */
    MAD_SCATTER_PATCH = 2,   /* one fused kernel over all terms, one workgroup per patch: x staged
                                in LDS, element contributions summed in LDS, then every entry written
                                once: by its patch if no other patch touches it, else by a gather
                                kernel summing the patches' partials in a fixed order. No global
                                atomics and no zero fill of the outputs. */
    MAD_SCATTER_COLOR = 3    /* the coloring alternative of Sec. 5.5: each term's elements greedily
                                colored so that no two elements of a color share a vertex, one launch
                                per color and term, each element adding its entries into pre-zeroed
                                outputs with plain read-add-writes (race-free within a color, colors in
                                sequence); no atomics, bitwise reproducible */
} mad_scatter;

typedef struct mad_options {
    int32_t scatter;         /* mad_scatter; 0 = default (MAD_SCATTER_PATCH) */
    int32_t patch_faces;     /* target faces per patch (Sec. 7.1 patch study); 0 = by term mix: 256 when
                                every term is a spring, inertia, edge-length or residual term, else 512 */
    double spd_eps;          /* eigenvalue floor of MAD_SPD; default 0 (PSD) */
    double degenerate_q;     /* MAD_F32: elements whose triangle quality 4 sqrt(3) A / sum(l^2)
                                falls below this are evaluated and projected in FP64; 0 = 1e-2 */
    int32_t lock_spins;      /* bound on each wait for the per-workgroup LDS lock of the patch kernels (spin
                                iterations); 0 = the default 4,194,304; MAD_LOCK_NO_WAIT gives up at once.
                                A wait that reaches its bound does not add its Hessian blocks (it never adds
                                without the lock) and raises the internal-error flag, so mad_problem_status
                                returns MAD_E_INTERNAL; the kernels still run to completion */
    int32_t wg_waves;        /* tile of the patch kernels: waves (64 lanes) per workgroup, 0 = 4 (default), 4
                                or 8 (MAD_F32 only; MAD_F64 keeps 4). With 8, a workgroup of terms other than
                                the light ones (springs, inertia, edge lengths, residuals) has the CU's LDS to
                                itself (148 KB: larger patches); light terms keep 76 KB per workgroup */
    int32_t reserved[6];     /* must be zero */
} mad_options;

enum { MAD_LOCK_NO_WAIT = -1 };  /* mad_options.lock_spins: every lock wait gives up at once */

/* library version (major * 10000 + minor * 100 + patch) */
int32_t mad_version(void);

/* description of the last failure on this thread ("" if none) */
const char *mad_last_error(void);

/* Fill *opt with the defaults. */
int32_t mad_options_default(mad_options *opt);

/* Ingest a triangle mesh (Sec. 6: triangle surface mesh, possibly non-manifold, possibly with
 * disconnected components). tris_host: [n_tris][3] vertex indices, copied. comp_vert_offsets:
 * NULL, or [n_comp + 1] ascending vertex offsets partitioning the vertices into disjoint
 * components (batched meshes); energies are then also reported per component. Builds the edge
 * list and the interior-edge diamonds: (v0, v1) the edge as directed in the lower-indexed face,
 * v2 that face's opposite vertex, v3 the other face's opposite vertex. */
int32_t mad_mesh_create(int64_t n_verts, int64_t n_tris, const int32_t *tris_host, int32_t n_comp,
                        const int64_t *comp_vert_offsets, mad_mesh **out);

/* Sizes of an ingested mesh (any output pointer may be NULL). */
int32_t mad_mesh_info(const mad_mesh *mesh, int64_t *n_verts, int64_t *n_tris, int64_t *n_edges,
                      int64_t *n_diamonds);

/* Copy the diamonds ([n_diamonds][4]) to host memory. */
int32_t mad_mesh_copy_diamonds(const mad_mesh *mesh, int32_t *diamonds_host);

int32_t mad_mesh_destroy(mad_mesh *mesh);

/* Create a problem over a mesh: var_dim DOFs per vertex (1, 2 or 3), precision mad_precision.
 * opt may be NULL (defaults). The mesh must outlive the problem. */
int32_t mad_problem_create(const mad_mesh *mesh, int32_t var_dim, int32_t precision,
                           const mad_options *opt, mad_problem **out);

/* Add a local term (Sec. 4.2, add_term). params_host: n_params doubles (see mad_term_kind).
 * rest_pos_host: [n_verts][3] rest positions for kinds that need them (copied; rest-frame data
 * is computed here). Returns MAD_E_DEGENERATE_REST if a rest triangle has zero area. */
int32_t mad_problem_add_term(mad_problem *prob, int32_t kind, const double *params_host, int32_t n_params,
                             const double *rest_pos_host);

/* Add a per-vertex term (Sec. 7.1, the per-vertex energies of the mass-spring example; Sec. 4.2,
 * the positional residual): one element per mesh vertex. kind: MAD_INERTIA (vdata_dev: {m, xhat_x,
 * xhat_y, xhat_z} per vertex) or MAD_RES_POSITION ({w, x_t}). vdata_dev: device FP64 [n_verts][4], on
 * the problem's device, owned by the caller; it is read (not copied) at every evaluation, so it must
 * stay valid while the problem is evaluated, and the caller may rewrite it between evaluations (e.g.
 * xhat = x^n + h v^n every time step). Every vertex must lie on a triangle (MAD_E_UNSUPPORTED
 * otherwise). */
int32_t mad_problem_add_vertex_term(mad_problem *prob, int32_t kind, const double *params_host, int32_t n_params,
                                    const double *vdata_dev);

/* Build patches, upload element data and build the block pattern on the GPU (Sec. 6.1), once.
 * Starts with the layout of the options; with the patch scatter the launch is persistent unless every
 * term is a spring, inertia, edge-length or residual term (those run one workgroup per patch).
 * Synchronises the stream. */
int32_t mad_problem_finalize(mad_problem *prob, void *stream);

/* Dynamic sparsity (Sec. 6.3): before mad_problem_finalize, reserve room for interaction pairs. The
 * pattern is then kept in two device buffers (double buffering: an insertion writes the inactive one and
 * makes it active), each with capacity for the initial blocks plus 2 * max_pairs; one insertion call takes
 * at most max_pairs pairs. No allocation happens at insertion time. max_pairs >= 0; 0 turns it off. */
int32_t mad_problem_reserve_pairs(mad_problem *prob, int64_t max_pairs);

/* Insert the blocks of new interaction pairs into the Hessian pattern, on the GPU (Sec. 6.3 and the CSR
 * update of the appendix). pairs_dev: device int32 [n_pairs][2] vertex pairs. A pair (a, b), a != b, adds
 * the blocks (a, b) and (b, a); a pair naming one vertex twice, a repeated pair or one already in the
 * pattern adds nothing. Rows stay sorted, so the new pattern is unique whatever the order of the pairs.
 * Blocks are renumbered (a block's index may change, its row and column do not; the library follows its
 * own references): re-read the pattern and size hess buffers for the new nnzb (mad_problem_pattern_info)
 * before the next evaluation, which writes zeros into blocks no term touches. *n_added (host, may be
 * NULL): blocks added. Synchronises the stream (the new block count is read back).
 * Errors: MAD_E_STATE before finalize or without a reserve; MAD_E_INVALID_ARG if n_pairs exceeds the
 * reserved max_pairs or a pair names a vertex out of range; MAD_E_CAPACITY if the pattern would outgrow
 * the reserve. On an error the pattern is unchanged. */
int32_t mad_problem_insert_pairs(mad_problem *prob, const int32_t *pairs_dev, int64_t n_pairs, int64_t *n_added,
                                 void *stream);

/* Residual terms and the sparse Jacobian (Sec. 4.1 Eq. 3, Sec. 6.1). The global residual stacks the
 * residual terms in the order they were added, each term's elements in their original order (element e
 * of a term with m_t residuals owns rows row_off_t + e m_t ... + m_t - 1: the row ownership P_j of
 * Eq. 3); scalar terms own no rows. Each row holds the element's stencil DOFs v * var_dim + c in
 * ascending order (scalar entries: the Jacobian is m x n_verts * var_dim).
 * mad_problem_jacobian_info: *m rows and *nnz entries. MAD_E_STATE before finalize or without residual
 * terms; MAD_E_OVERFLOW beyond int32 indexing. */
int32_t mad_problem_jacobian_info(const mad_problem *prob, int64_t *m, int64_t *nnz);

/* The Jacobian's CSR pattern into rowptr_dev [m + 1] and colidx_dev [nnz] (device int32). Fixed by the
 * stencils: computed once, valid for every evaluation. Synchronises the stream. */
int32_t mad_problem_copy_jacobian_pattern(const mad_problem *prob, int32_t *rowptr_dev, int32_t *colidx_dev,
                                          void *stream);

/* Evaluate the residuals r_dev [m] (FP64) and the Jacobian values vals_dev [nnz] (FP32 for MAD_F32, FP64
 * for MAD_F64) at x_dev [n_verts * var_dim], in the pattern above. Every entry is written by the element
 * that owns its row (no atomics); non-finite values raise the flag mad_problem_status reports.
 * Asynchronous on stream. J^T J and J^T r are what mad_problem_eval assembles for residual terms. */
int32_t mad_problem_jacobian(mad_problem *prob, const double *x_dev, double *r_dev, void *vals_dev, void *stream);

/* Pattern sizes: block rows (= n_verts), nnzb blocks, block_dim (= var_dim). */
int32_t mad_problem_pattern_info(const mad_problem *prob, int64_t *n_block_rows, int64_t *nnzb,
                                 int32_t *block_dim);

/* Number of doubles written to energy_dev by mad_problem_eval: 1, or 1 + n_comp for a mesh
 * created with components (entry 0 is the total, entry 1 + c component c). */
int32_t mad_problem_energy_count(const mad_problem *prob, int32_t *count);

/* Copy the pattern: rowptr_dev [n_block_rows + 1], colidx_dev [nnzb] (device int32). */
int32_t mad_problem_copy_pattern(const mad_problem *prob, int32_t *rowptr_dev, int32_t *colidx_dev,
                                 void *stream);

/* Evaluate every term at x_dev ([n_verts * var_dim] FP64) and assemble (Eq. 1-2).
 * mode: OR of mad_mode bits. energy_dev: [energy_count] FP64 (may be NULL without MAD_ENERGY).
 * grad_dev: [n_verts * var_dim], hess_dev: [nnzb * var_dim^2], both FP64 for MAD_F64 and FP32
 * for MAD_F32 (may be NULL when not requested). Outputs are overwritten, not accumulated.
 * Asynchronous on stream: no host synchronisation. The energy is a deterministic FP64 sum. */
int32_t mad_problem_eval(mad_problem *prob, const double *x_dev, uint32_t mode, double *energy_dev,
                         void *grad_dev, void *hess_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops with a
 * fixed memory budget): mad_problem_eval with the same arguments, outputs and errors, that allocates
 * nothing. Every buffer the evaluation writes and reads back within itself (per-patch energies, queue
 * counters, halo partials of entries several patches share, the queue of FP32 elements redone in FP64,
 * vertex normals, network outputs) is taken from a static device array of 64 MiB that each GPU holds
 * from the library's load until the process ends, instead of from the problem's buffers. The problem
 * must live on the current device (MAD_E_INVALID_ARG otherwise). MAD_E_CAPACITY, before any launch, if
 * the problem needs more than 64 MiB of it (at the default patches the elastic shell of a 724 x 724 vertex
 * grid, 1M triangles, needs 36 MB; the 1024 x 1024 one, 72 MB, does not fit); the FP64 redo queue takes what is left, and an evaluation that queues more elements
 * than that is reported by mad_problem_status as MAD_E_INTERNAL. The array keeps the last call's
 * contents; each call initialises what it reads. Calls on one GPU share its array: calls that overlap
 * on one GPU (other streams, other threads) race and must be ordered by the caller. Per-stage profiling
 * (mad_problem_set_profiling) does not record these calls. Asynchronous on stream. */
int32_t mad_problem_eval_static(mad_problem *prob, const double *x_dev, uint32_t mode, double *energy_dev,
                                void *grad_dev, void *hess_dev, void *stream);

/* Matrix-free Hessian-vector product (Sec. 5.5, Sec. 6.2 matrix-free mode): y = H(x) v with
 * H = sum_j S_j^T P(hess f_j) S_j (P the eigenvalue clamp when mode has MAD_SPD, else the
 * identity), each element's Hessian applied to its slice of v in LDS and the products summed, no
 * Hessian assembled. v_dev: [n_verts * var_dim] FP64; y_dev: [n_verts * var_dim], FP64 for MAD_F64,
 * FP32 for MAD_F32, overwritten. mode may add MAD_ENERGY (energy_dev) and MAD_GRAD (grad_dev) from
 * the same pass; MAD_HESS is not allowed. Asynchronous on stream. */
int32_t mad_problem_hvp(mad_problem *prob, const double *x_dev, const double *v_dev, uint32_t mode,
                        double *energy_dev, void *grad_dev, void *y_dev, void *stream);

/* Synchronise the stream and report whether any evaluation since the last call produced a
 * non-finite element energy or derivative (*nonfinite = 1) and how many elements took the FP64
 * fallback (*fp64_fallbacks); both counters are reset. Returns MAD_E_INTERNAL (after filling both
 * outputs and resetting the counters) if a device-side check failed in one of those evaluations: a
 * wait for the LDS lock of a patch kernel reached its bound (mad_options.lock_spins), or an element
 * redone in FP64 found a block missing from the pattern; mad_last_error() names which. The outputs
 * of those evaluations are then not valid. */
int32_t mad_problem_status(mad_problem *prob, int32_t *nonfinite, int64_t *fp64_fallbacks, void *stream);

/* Per-stage timing (profiling aid). enable = 1 starts recording HIP events on the eval stream
 * around each stage of every mad_problem_eval (zero fill, network pass, element kernels, energy)
 * and clears earlier records; enable = 0 stops recording. Recording adds no synchronisation. */
int32_t mad_problem_set_profiling(mad_problem *prob, int32_t enable);

/* Synchronise with the recorded events and report, summed over the evaluations recorded since
 * profiling was enabled, with S = max(n_terms, 2): ms_out[0] zero fills; ms_out[1] the vertex
 * normals and network passes of shell-feature terms (0 without them); with MAD_SCATTER_ATOMIC
 * ms_out[2 + t] the kernel of term t (in add order); with MAD_SCATTER_PATCH ms_out[2] the fused
 * kernel and ms_out[3] the gather of shared entries plus the FP64 redo of queued FP32 elements;
 * ms_out[2 + S] the energy reduction. *n_stages = S + 3, *n_evals = evaluations. ms_out must hold
 * at least 12 doubles. Records are kept (call set_profiling(1) to clear). */
int32_t mad_problem_profile(mad_problem *prob, double *ms_out, int32_t *n_stages, int64_t *n_evals);

/* Current evaluation layout (any output may be NULL): scatter strategy, effective patch target
 * (after shrinking to fit the LDS budget), persistent launch (0/1/2), number of patches and the tile
 * (waves per workgroup of the patch kernels). */
int32_t mad_problem_layout(const mad_problem *prob, int32_t *scatter, int32_t *patch_faces,
                           int32_t *persistent, int32_t *n_patches, int32_t *wg_waves);

/* Rebuild the evaluation layout of a finalized problem: scatter (mad_scatter), patch_faces target
 * (1 .. 2^20; shrunk until the largest patch fits the LDS budget of the tile), persistent = 1 for one
 * grid sized to the device whose workgroups take patches from a queue (patches in index order within
 * four size classes, the largest first; 2: strictly largest first; patch scatter only), 0 for one
 * workgroup per patch; wg_waves: the tile as in mad_options (0 keeps the current one). The block pattern
 * and the outputs' layout do not change. Synchronises the stream. On failure the problem is left
 * unusable (MAD_E_STATE on eval). */
int32_t mad_problem_set_layout(mad_problem *prob, int32_t scatter, int32_t patch_faces, int32_t persistent,
                               int32_t wg_waves, void *stream);

enum { MAD_TUNE_FORCE = 1 };  /* mad_problem_autotune: re-time even if this problem was tuned before */

/* Choose the layout by timing (batched scheduling and the patch-size study, Sec. 7.1): builds each
 * candidate layout (patch scatter with patch targets 128, 256, 512, 1024, each with and without the
 * persistent launch, each with the 4- and (MAD_F32) 8-wave tile; the atomic and the colored scatter), times
 * `reps` evaluations of `mode` on the caller's x_dev and outputs (arguments as for mad_problem_eval;
 * their contents are overwritten), and keeps the one with the lowest median time: every candidate
 * writes the same outputs from the same inputs, so the fastest is also the one with the highest
 * algorithmic bytes per second. The choice is cached by a fingerprint of the device, the
 * connectivity, the terms, the precision and the mode, for the process and, when the environment
 * variable MAD_TUNE_CACHE names a file, in that file across processes (one line per fingerprint); a
 * later call on an identical problem applies it without timing unless flags has MAD_TUNE_FORCE.
 * Synchronises the stream. On failure the problem is left unusable. */
int32_t mad_problem_autotune(mad_problem *prob, const double *x_dev, uint32_t mode, double *energy_dev,
                             void *grad_dev, void *hess_dev, int32_t reps, int32_t flags, void *stream);

/* The last autotune's timings as JSON (candidates with their median ms, and the choice). Copies at
 * most cap - 1 bytes plus a terminating zero into buf (may be NULL); *len = full length. */
int32_t mad_problem_tune_report(const mad_problem *prob, char *buf, int64_t cap, int64_t *len);

int32_t mad_problem_destroy(mad_problem *prob);

/* ---- learned per-triangle density (project-defined) ------------------------------------------
 * psi(z) = s_out (w3 . sp(W2 sp(W1 (s_in * z) + b1) + b2) + b3), sp(a) = log(1 + e^a), hidden
 * width 64. Trainable parameters, packed in this order, row-major (4673 floats):
 * W1 [64][6], b1 [64], W2 [64][64], b2 [64], w3 [64], b3. The library keeps an FP32 master copy
 * (trained) and a BF16 copy (round to nearest even) that evaluation uses: layer 2 runs on the
 * matrix cores with BF16 weights and FP32 accumulation. */
enum { MAD_MLP_HIDDEN = 64, MAD_MLP_PARAMS = 4673 };

/* Create a network on the current device. hidden must be 64. params_host: MAD_MLP_PARAMS floats
 * (copied); s_in_host: 6 input scales; s_out: output scale. */
int32_t mad_mlp_create(int32_t hidden, const float *params_host, const float *s_in_host, float s_out,
                       mad_mlp **out);

/* Replace the parameters (FP32 master and BF16 copy); resets Adam's moments and step count. */
int32_t mad_mlp_set_params(mad_mlp *mlp, const float *params_host);

/* Copy the parameters to host memory: which = 0 the FP32 master, 1 the BF16 copy widened to FP32. */
int32_t mad_mlp_get_params(const mad_mlp *mlp, int32_t which, float *params_host);

/* Training loss and gradient over a batch, on the stream (no host synchronisation):
 *   loss = mean_b (psi(z_b) - W_b)^2 / c_e + lam_g mean_b sum_i (dpsi/dz_i(z_b) - dW_bi)^2 / c_g[i]
 * (c_g_host: 6 per-feature normalisers, copied) over the samples idx_dev[base .. base + count) (idx_dev NULL: samples base .. base + count) of
 * z_dev [N][6], W_dev [N], dW_dev [N][6] (device FP32). Uses the FP32 master parameters.
 * grad_dev: MAD_MLP_PARAMS floats, loss_dev: 1 float (device). Deterministic: per-wave partial
 * sums are reduced in a fixed order. count must be >= 1. */
int32_t mad_mlp_loss_grad(mad_mlp *mlp, const float *z_dev, const float *W_dev, const float *dW_dev,
                          const int32_t *idx_dev, int64_t base, int64_t count, float c_e, const float *c_g_host,
                          float lam_g, float *grad_dev, float *loss_dev, void *stream);

/* One Adam step (Kingma and Ba) on the FP32 master with the gradient grad_dev (device), step
 * count incremented first on the device; refreshes the BF16 copy. */
int32_t mad_mlp_adam_step(mad_mlp *mlp, const float *grad_dev, float lr, float beta1, float beta2, float eps,
                          void *stream);

/* One pass over the samples in the order perm_dev [n] (device int32, a permutation the caller
 * draws): minibatches of `batch` consecutive entries (the last may be shorter), each a loss_grad
 * followed by an Adam step. loss_hist_dev (nullable): one float per minibatch. No host sync. */
int32_t mad_mlp_train_epoch(mad_mlp *mlp, const float *z_dev, const float *W_dev, const float *dW_dev,
                            const int32_t *perm_dev, int64_t n, int32_t batch, float c_e, const float *c_g_host,
                            float lam_g, float lr, float beta1, float beta2, float eps, float *loss_hist_dev,
                            void *stream);

int32_t mad_mlp_destroy(mad_mlp *mlp);

/* Add a learned-density term (MAD_MLP) over every triangle. The network must live on the
 * problem's device and outlive the problem; each evaluation reads its current BF16 parameters.
 * rest_pos_host: [n_verts][3] rest positions (copied). */
int32_t mad_problem_add_mlp_term(mad_problem *prob, const mad_mlp *mlp, const double *rest_pos_host);

#ifdef __cplusplus
}
#endif

#endif /* MAD_H */
