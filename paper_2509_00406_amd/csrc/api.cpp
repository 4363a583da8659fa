// C ABI entry points (include/mad.h). Validation is synchronous and precedes
// any device work; evaluation is asynchronous on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>

#include "mad_internal.hpp"

namespace mad {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

}  // namespace mad

using namespace mad;

namespace mad {

int check_eval_args(const mad_problem* p, const double* x, uint32_t mode, const double* energy, const void* grad,
                    const void* hess) {
    if (!p) return fail(MAD_E_INVALID_ARG, "problem is NULL");
    if (!p->finalized) return fail(MAD_E_STATE, "eval before finalize");
    if (!x) return fail(MAD_E_INVALID_ARG, "x is NULL");
    if (mode & ~15u) return fail(MAD_E_INVALID_ARG, "unknown mode bits");
    if ((mode & MAD_ENERGY) && !energy) return fail(MAD_E_INVALID_ARG, "energy output is NULL");
    if ((mode & MAD_GRAD) && !grad) return fail(MAD_E_INVALID_ARG, "gradient output is NULL");
    if ((mode & MAD_HESS) && !hess) return fail(MAD_E_INVALID_ARG, "Hessian output is NULL");
    if ((mode & MAD_SPD) && !(mode & MAD_HESS)) return fail(MAD_E_INVALID_ARG, "MAD_SPD needs MAD_HESS");
    return MAD_OK;
}

}  // namespace mad

extern "C" {

int32_t mad_version(void) { return 100; }

const char* mad_last_error(void) { return g_last_error.c_str(); }

int32_t mad_options_default(mad_options* opt) {
    if (!opt) return fail(MAD_E_INVALID_ARG, "opt is NULL");
    std::memset(opt, 0, sizeof(*opt));
    opt->scatter = MAD_SCATTER_PATCH;
    opt->patch_faces = 0;
    opt->spd_eps = 0.0;
    opt->degenerate_q = 1e-2;
    return MAD_OK;
}

int32_t mad_mesh_create(int64_t n_verts, int64_t n_tris, const int32_t* tris_host, int32_t n_comp,
                        const int64_t* comp_vert_offsets, mad_mesh** out) {
    if (!out) return fail(MAD_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n_verts <= 0 || n_tris < 0) return fail(MAD_E_INVALID_ARG, "n_verts must be > 0 and n_tris >= 0");
    if (n_tris > 0 && !tris_host) return fail(MAD_E_INVALID_ARG, "tris_host is NULL");
    if (n_verts >= INT32_MAX || n_tris >= INT32_MAX / 3) return fail(MAD_E_OVERFLOW, "mesh too large for int32 indices");
    if (n_comp < 0 || (n_comp > 0 && !comp_vert_offsets)) return fail(MAD_E_INVALID_ARG, "bad component offsets");
    if (n_comp > 0) {
        if (comp_vert_offsets[0] != 0 || comp_vert_offsets[n_comp] != n_verts)
            return fail(MAD_E_INVALID_ARG, "component offsets must start at 0 and end at n_verts");
        for (int32_t c = 0; c < n_comp; ++c)
            if (comp_vert_offsets[c + 1] <= comp_vert_offsets[c])
                return fail(MAD_E_INVALID_ARG, "component offsets must be strictly increasing");
    }
    mad_mesh* m = new (std::nothrow) mad_mesh();
    if (!m) return fail(MAD_E_OOM, "mesh");
    m->nv = n_verts;
    m->nt = n_tris;
    m->tris.assign(tris_host, tris_host + 3 * n_tris);
    for (int64_t f = 0; f < n_tris; ++f) {
        const int32_t* t = &m->tris[3 * f];
        for (int c = 0; c < 3; ++c)
            if (t[c] < 0 || t[c] >= n_verts) {
                delete m;
                return fail(MAD_E_BAD_MESH, "face " + std::to_string(f) + " has a vertex index out of range");
            }
        if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2]) {
            delete m;
            return fail(MAD_E_BAD_MESH, "face " + std::to_string(f) + " repeats a vertex");
        }
    }
    if (n_comp > 0) {
        m->comp_off.assign(comp_vert_offsets, comp_vert_offsets + n_comp + 1);
        m->batched = true;
        // a face must not straddle components
        for (int64_t f = 0; f < n_tris; ++f) {
            const int32_t* t = &m->tris[3 * f];
            auto comp = [&](int32_t v) {
                return std::upper_bound(m->comp_off.begin(), m->comp_off.end(), (int64_t)v) - m->comp_off.begin();
            };
            if (comp(t[0]) != comp(t[1]) || comp(t[0]) != comp(t[2])) {
                delete m;
                return fail(MAD_E_BAD_MESH, "face " + std::to_string(f) + " spans two components");
            }
        }
    } else {
        m->comp_off = {0, n_verts};
    }
    int rc = build_topology(*m);
    if (rc != MAD_OK) {
        delete m;
        return rc;
    }
    *out = m;
    return MAD_OK;
}

int32_t mad_mesh_info(const mad_mesh* m, int64_t* nv, int64_t* nt, int64_t* ne, int64_t* nd) {
    if (!m) return fail(MAD_E_INVALID_ARG, "mesh is NULL");
    if (nv) *nv = m->nv;
    if (nt) *nt = m->nt;
    if (ne) *ne = m->ne();
    if (nd) *nd = m->nd();
    return MAD_OK;
}

int32_t mad_mesh_copy_diamonds(const mad_mesh* m, int32_t* out) {
    if (!m || (!out && m->nd() > 0)) return fail(MAD_E_INVALID_ARG, "NULL argument");
    std::copy(m->diamonds.begin(), m->diamonds.end(), out);
    return MAD_OK;
}

int32_t mad_mesh_destroy(mad_mesh* m) {
    delete m;
    return MAD_OK;
}

int32_t mad_problem_create(const mad_mesh* mesh, int32_t var_dim, int32_t precision, const mad_options* opt,
                           mad_problem** out) {
    if (!out) return fail(MAD_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!mesh) return fail(MAD_E_INVALID_ARG, "mesh is NULL");
    if (var_dim < 1 || var_dim > 3) return fail(MAD_E_INVALID_ARG, "var_dim must be 1, 2 or 3");
    if (precision != MAD_F64 && precision != MAD_F32) return fail(MAD_E_INVALID_ARG, "bad precision");
    mad_options o;
    mad_options_default(&o);
    if (opt) {
        for (int i = 0; i < 6; ++i)
            if (opt->reserved[i] != 0) return fail(MAD_E_INVALID_ARG, "reserved option fields must be zero");
        if (opt->wg_waves != 0 && opt->wg_waves != 4 && opt->wg_waves != 8)
            return fail(MAD_E_INVALID_ARG, "wg_waves must be 0, 4 or 8");
        o.wg_waves = opt->wg_waves;
        if (opt->scatter != MAD_SCATTER_AUTO && opt->scatter != MAD_SCATTER_ATOMIC && opt->scatter != MAD_SCATTER_PATCH &&
            opt->scatter != MAD_SCATTER_COLOR)
            return fail(MAD_E_INVALID_ARG, "bad scatter mode");
        o.scatter = opt->scatter == MAD_SCATTER_AUTO ? MAD_SCATTER_PATCH : opt->scatter;
        if (opt->patch_faces < 0 || opt->patch_faces > (1 << 20)) return fail(MAD_E_INVALID_ARG, "bad patch_faces");
        if (!(opt->spd_eps >= 0.0) || !std::isfinite(opt->spd_eps)) return fail(MAD_E_INVALID_ARG, "spd_eps must be >= 0");
        if (!(opt->degenerate_q >= 0.0) || opt->degenerate_q > 1.0) return fail(MAD_E_INVALID_ARG, "degenerate_q in [0, 1]");
        if (opt->patch_faces > 0) o.patch_faces = opt->patch_faces;
        o.spd_eps = opt->spd_eps;
        if (opt->degenerate_q > 0.0) o.degenerate_q = opt->degenerate_q;
        if (opt->lock_spins < MAD_LOCK_NO_WAIT) return fail(MAD_E_INVALID_ARG, "lock_spins must be >= -1");
        o.lock_spins = opt->lock_spins;
    }
    mad_problem* p = new (std::nothrow) mad_problem();
    if (!p) return fail(MAD_E_OOM, "problem");
    p->mesh = mesh;
    p->d = var_dim;
    p->prec = precision;
    p->opt = o;
    p->scatter = o.scatter;
    p->wg_waves = (o.wg_waves == 8 && precision == MAD_F32) ? 8 : 4;
    *out = p;
    return MAD_OK;
}

static int32_t add_term(mad_problem* p, int32_t kind, const double* params, int32_t n_params, const double* rest_pos,
                        const mad_mlp* mlp, const double* vdata = nullptr) {
    if (!p) return fail(MAD_E_INVALID_ARG, "problem is NULL");
    if (p->finalized) return fail(MAD_E_STATE, "add_term after finalize");
    const int ns = kind_stencil(kind);
    if (ns < 0) return fail(MAD_E_INVALID_ARG, "unknown term kind");
    if (kind_vardim(kind) != p->d) return fail(MAD_E_UNSUPPORTED, "term kind does not match the problem's var_dim");
    if (n_params < 0 || n_params > 4 || (n_params > 0 && !params)) return fail(MAD_E_INVALID_ARG, "bad params");
    if (p->terms.size() >= 8) return fail(MAD_E_UNSUPPORTED, "at most 8 terms");
    const int nrest = kind_nrest(kind);
    if (nrest > 0 && !rest_pos) return fail(MAD_E_INVALID_ARG, "this term kind needs rest positions");
    const mad_mesh& m = *p->mesh;
    Term t;
    t.kind = kind;
    t.ns = ns;
    t.d = p->d;
    t.nrest = nrest;
    for (int i = 0; i < n_params; ++i) {
        if (!std::isfinite(params[i])) return fail(MAD_E_INVALID_ARG, "non-finite parameter");
        t.prm[i] = params[i];
    }
    int rc = MAD_OK;
    switch (kind) {
    case MAD_EDGE_SQLEN:
        t.n = m.ne();
        t.stencil = m.edges;
        break;
    case MAD_TRI_AREA:
        t.n = m.nt;
        t.stencil = m.tris;
        break;
    case MAD_DIRICHLET: case MAD_STVK: case MAD_SYMDIR:
        t.n = m.nt;
        t.stencil = m.tris;
        rc = rest_tri(m, rest_pos, t.rest);
        break;
    case MAD_BENDING:
        t.n = m.nd();
        t.stencil = m.diamonds;
        rc = rest_diamond(m, rest_pos, t.rest);
        break;
    case MAD_MLP: case MAD_SHELL_TRI:
        t.n = m.nt;
        t.stencil = m.tris;
        t.mlp = mlp;
        rc = rest_shell(m, rest_pos, t.rest);
        break;
    case MAD_SPRING:
        t.n = m.ne();
        t.stencil = m.edges;
        rc = rest_spring(m, rest_pos, t.rest);
        break;
    case MAD_RES_EDGE:
        t.n = m.ne();
        t.stencil = m.edges;
        rc = rest_edge_length(m, rest_pos, t.rest);
        break;
    case MAD_INERTIA: case MAD_RES_POSITION:
        for (int64_t v = 0; v < m.nv; ++v)
            if (m.vert_face0[v] < 0) return fail(MAD_E_UNSUPPORTED, "vertex " + std::to_string(v) + " lies on no triangle");
        t.n = m.nv;
        t.stencil.resize((size_t)m.nv);
        std::iota(t.stencil.begin(), t.stencil.end(), 0);
        t.vdata = vdata;
        break;
    }
    if (rc != MAD_OK) return rc;
    if (kind == MAD_MLP || kind == MAD_SHELL_TRI) p->shell = true;
    if (!(kind == MAD_EDGE_SQLEN || kind == MAD_SPRING || kind == MAD_INERTIA || kind == MAD_RES_EDGE ||
          kind == MAD_RES_POSITION))
        p->light = false;
    p->terms.push_back(std::move(t));
    return MAD_OK;
}

int32_t mad_problem_add_term(mad_problem* p, int32_t kind, const double* params, int32_t n_params,
                             const double* rest_pos) {
    if (kind == MAD_MLP) return fail(MAD_E_INVALID_ARG, "learned-density terms are added with mad_problem_add_mlp_term");
    if (kind == MAD_INERTIA || kind == MAD_RES_POSITION)
        return fail(MAD_E_INVALID_ARG, "vertex terms are added with mad_problem_add_vertex_term");
    return add_term(p, kind, params, n_params, rest_pos, nullptr);
}

int32_t mad_problem_add_vertex_term(mad_problem* p, int32_t kind, const double* params, int32_t n_params,
                                    const double* vdata) {
    if (!p || !vdata) return fail(MAD_E_INVALID_ARG, "NULL argument");
    if (kind != MAD_INERTIA && kind != MAD_RES_POSITION) return fail(MAD_E_INVALID_ARG, "not a vertex term kind");
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, vdata) != hipSuccess || at.type != hipMemoryTypeDevice)
        return fail(MAD_E_INVALID_ARG, "vdata must be device memory");
    int dev = 0;
    MAD_HIP_TRY(hipGetDevice(&dev));
    if (at.device != dev) return fail(MAD_E_INVALID_ARG, "vdata lives on another device");
    return add_term(p, kind, params, n_params, nullptr, nullptr, vdata);
}

int32_t mad_problem_add_mlp_term(mad_problem* p, const mad_mlp* mlp, const double* rest_pos) {
    if (!p || !mlp) return fail(MAD_E_INVALID_ARG, "NULL argument");
    int dev = 0;
    MAD_HIP_TRY(hipGetDevice(&dev));
    if (dev != mlp->device) return fail(MAD_E_INVALID_ARG, "the network lives on another device");
    return add_term(p, MAD_MLP, nullptr, 0, rest_pos, mlp);
}

// Two pattern buffers with room for the reserved pairs' blocks, the first holding the built pattern, and
// the scratch of the update (no allocation later, at insertion time).
static int alloc_dynamic(mad_problem* p, hipStream_t s) {
    const int64_t nv = p->mesh->nv;
    const int64_t cap = p->nnzb + 2 * p->pair_reserve;
    if (cap > INT32_MAX) return fail(MAD_E_OVERFLOW, "reserved block count exceeds int32");
    p->nnzb_cap = cap;
    auto dev = [&](void** q, size_t bytes) -> int {
        if (hipMalloc(q, std::max<size_t>(bytes, 16)) != hipSuccess) return fail(MAD_E_OOM, "pattern reserve");
        p->owned.push_back(*q);
        return MAD_OK;
    };
    int32_t* colidx_a = nullptr;
    int rc;
    if ((rc = dev((void**)&colidx_a, sizeof(int32_t) * cap)) != MAD_OK) return rc;
    MAD_HIP_TRY(hipMemcpyAsync(colidx_a, p->d_colidx, sizeof(int32_t) * p->nnzb, hipMemcpyDeviceToDevice, s));
    MAD_HIP_TRY(hipStreamSynchronize(s));
    for (auto it = p->owned.begin(); it != p->owned.end(); ++it)
        if (*it == (void*)p->d_colidx) {
            (void)hipFree(*it);
            p->owned.erase(it);
            break;
        }
    p->d_colidx = colidx_a;
    DynBuffers& B = p->dyn;
    const int64_t nb = (std::max<int64_t>(nv, 1) + 2047) / 2048 + 4;
    if ((rc = dev((void**)&p->d_rowptr_b, sizeof(int32_t) * (nv + 1))) != MAD_OK ||
        (rc = dev((void**)&p->d_colidx_b, sizeof(int32_t) * cap)) != MAD_OK ||
        (rc = dev((void**)&p->d_extra_blocks, sizeof(int32_t) * 2 * p->pair_reserve)) != MAD_OK ||
        (rc = dev((void**)&B.cnt, sizeof(int32_t) * (nv + 1))) != MAD_OK ||
        (rc = dev((void**)&B.fill, sizeof(int32_t) * (nv + 1))) != MAD_OK ||
        (rc = dev((void**)&B.coff, sizeof(int32_t) * (nv + 1))) != MAD_OK ||
        (rc = dev((void**)&B.stage, sizeof(int32_t) * 2 * p->pair_reserve)) != MAD_OK ||
        (rc = dev((void**)&B.nnew, sizeof(int32_t) * (nv + 1))) != MAD_OK ||
        (rc = dev((void**)&B.rowcnt, sizeof(int32_t) * (nv + 1))) != MAD_OK ||
        (rc = dev((void**)&B.noff, sizeof(int32_t) * (nv + 1))) != MAD_OK ||
        (rc = dev((void**)&B.map, sizeof(int32_t) * cap)) != MAD_OK ||
        (rc = dev((void**)&B.flags, sizeof(int32_t) * 4)) != MAD_OK ||
        (rc = dev((void**)&B.rp64, sizeof(int64_t) * (nv + 1))) != MAD_OK ||
        (rc = dev((void**)&B.scan_tmp, sizeof(int64_t) * (nb + 1))) != MAD_OK)
        return rc;
    return MAD_OK;
}

int32_t mad_problem_reserve_pairs(mad_problem* p, int64_t max_pairs) {
    if (!p) return fail(MAD_E_INVALID_ARG, "problem is NULL");
    if (p->finalized) return fail(MAD_E_STATE, "reserve before finalize");
    if (max_pairs < 0 || max_pairs > INT32_MAX / 4) return fail(MAD_E_INVALID_ARG, "max_pairs out of range");
    p->pair_reserve = max_pairs;
    return MAD_OK;
}

int32_t mad_problem_insert_pairs(mad_problem* p, const int32_t* pairs, int64_t n_pairs, int64_t* n_added,
                                 void* stream) {
    if (!p) return fail(MAD_E_INVALID_ARG, "problem is NULL");
    if (!p->finalized) return fail(MAD_E_STATE, "insert before finalize");
    if (p->pair_reserve == 0) return fail(MAD_E_STATE, "no pair reserve (mad_problem_reserve_pairs)");
    if (n_pairs < 0 || n_pairs > p->pair_reserve) return fail(MAD_E_INVALID_ARG, "n_pairs exceeds the reserve");
    if (n_pairs > 0 && !pairs) return fail(MAD_E_INVALID_ARG, "pairs is NULL");
    if (n_added) *n_added = 0;
    return insert_pairs_device(p, pairs, n_pairs, n_added, (hipStream_t)stream);
}

int32_t mad_problem_finalize(mad_problem* p, void* stream) {
    if (!p) return fail(MAD_E_INVALID_ARG, "problem is NULL");
    if (p->finalized) return fail(MAD_E_STATE, "already finalized");
    if (p->terms.empty()) return fail(MAD_E_STATE, "no terms");
    hipStream_t s = (hipStream_t)stream;
    const mad_mesh& m = *p->mesh;
    MAD_HIP_TRY(hipGetDevice(&p->device));
    MAD_HIP_TRY(hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device));
    MAD_HIP_TRY(hipMalloc((void**)&p->d_flags, sizeof(int32_t) * 4));
    p->owned.push_back(p->d_flags);
    MAD_HIP_TRY(hipMalloc((void**)&p->d_fallbacks, sizeof(unsigned long long)));
    p->owned.push_back(p->d_fallbacks);
    MAD_HIP_TRY(launch_fill(p->d_flags, 4, 4, s));
    MAD_HIP_TRY(launch_fill(p->d_fallbacks, 1, 8, s));
    int rc;
    if (p->shell) {
        // triangles of each vertex in ascending order (the normals' fixed summation order)
        std::vector<int32_t> ptr((size_t)m.nv + 1, 0), vf((size_t)m.nt * 3);
        for (int64_t f = 0; f < m.nt; ++f)
            for (int a = 0; a < 3; ++a) ptr[m.tris[3 * f + a] + 1]++;
        for (int64_t v = 0; v < m.nv; ++v) ptr[v + 1] += ptr[v];
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
        for (int64_t f = 0; f < m.nt; ++f)
            for (int a = 0; a < 3; ++a) vf[fill[m.tris[3 * f + a]]++] = (int32_t)f;
        auto up = [&](void** dst, const void* src, size_t bytes) -> int {
            MAD_HIP_TRY(hipMalloc(dst, std::max<size_t>(bytes, 16)));
            p->owned.push_back(*dst);
            if (bytes) MAD_HIP_TRY(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
            return MAD_OK;
        };
        if ((rc = up((void**)&p->d_tris, m.tris.data(), m.tris.size() * 4)) != MAD_OK) return rc;
        if ((rc = up((void**)&p->d_vf_ptr, ptr.data(), ptr.size() * 4)) != MAD_OK) return rc;
        if ((rc = up((void**)&p->d_vf, vf.data(), vf.size() * 4)) != MAD_OK) return rc;
        MAD_HIP_TRY(hipMalloc((void**)&p->d_normals, sizeof(double) * 3 * (size_t)std::max<int64_t>(m.nv, 1)));
        p->owned.push_back(p->d_normals);
    }
    // element order first (the pattern is built from the device stencils), then the pattern, then
    // the scatter structures that index into it
    // default patch target: smaller patches for cheap elements (more workgroups to hide their latency)
    if (p->opt.patch_faces == 0) p->opt.patch_faces = p->light ? 256 : 512;
    // default launch: the persistent grid for the patch scatter of heavy elements (a workgroup's
    // flush of one patch overlaps its next patch's work); one workgroup per patch for light terms
    const int persistent = (p->scatter == MAD_SCATTER_PATCH && !p->light) ? 1 : 0;
    if ((rc = build_layout(p, p->opt.patch_faces, p->scatter, persistent, s)) != MAD_OK) return rc;
    std::vector<PatternTerm> pts;
    for (auto& t : p->terms) pts.push_back({t.d_stencil, t.n, t.ns});
    if ((rc = build_pattern_device(m.nv, pts, &p->d_rowptr, &p->d_colidx, &p->nnzb, p->owned, s)) != MAD_OK) return rc;
    p->h_rowptr.resize((size_t)m.nv + 1);
    p->h_colidx.resize((size_t)std::max<int64_t>(p->nnzb, 1));
    MAD_HIP_TRY(hipMemcpyAsync(p->h_rowptr.data(), p->d_rowptr, p->h_rowptr.size() * 4, hipMemcpyDeviceToHost, s));
    MAD_HIP_TRY(hipMemcpyAsync(p->h_colidx.data(), p->d_colidx, (size_t)p->nnzb * 4, hipMemcpyDeviceToHost, s));
    MAD_HIP_TRY(hipStreamSynchronize(s));
    p->h_colidx.resize((size_t)p->nnzb);
    if (p->pair_reserve > 0 && (rc = alloc_dynamic(p, s)) != MAD_OK) return rc;
    if ((rc = build_scatter(p, s)) != MAD_OK) return rc;
    int32_t hflags[4];
    MAD_HIP_TRY(hipMemcpyAsync(hflags, p->d_flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
    MAD_HIP_TRY(hipStreamSynchronize(s));
    if (hflags[1] != 0) return fail(MAD_E_INTERNAL, "element block missing from the pattern");
    p->finalized = true;
    return MAD_OK;
}

// residual terms: the launch description and the global sizes (rows by term, then element)
static int jac_launch(const mad_problem* p, JacLaunch& L, int64_t* m_out, int64_t* nnz_out) {
    L = JacLaunch{};
    L.prec = p->prec;
    int64_t m = 0, nnz = 0;
    for (const auto& t : p->terms) {
        const int nr = kind_nres(t.kind);
        if (nr == 0) continue;
        JacTerm& J = L.terms[L.n_terms++];
        J.kind = t.kind;
        J.n = t.n;
        J.stencil = t.d_jstencil;
        J.rest = t.d_jrest;
        J.vdata = t.vdata;
        std::memcpy(J.prm, t.prm, sizeof(t.prm));
        J.row_off = m;
        J.nz_off = nnz;
        m += t.n * nr;
        nnz += t.n * nr * t.ns * t.d;
    }
    if (m == 0) return fail(MAD_E_STATE, "the problem has no residual terms");
    if (nnz > INT32_MAX || m > INT32_MAX) return fail(MAD_E_OVERFLOW, "Jacobian exceeds int32 indexing");
    L.flags = p->d_flags;
    *m_out = m;
    *nnz_out = nnz;
    return MAD_OK;
}

int32_t mad_problem_jacobian_info(const mad_problem* p, int64_t* m, int64_t* nnz) {
    if (!p || !m || !nnz) return fail(MAD_E_INVALID_ARG, "NULL argument");
    if (!p->finalized) return fail(MAD_E_STATE, "not finalized");
    JacLaunch L;
    return jac_launch(p, L, m, nnz);
}

int32_t mad_problem_copy_jacobian_pattern(const mad_problem* p, int32_t* rowptr, int32_t* colidx, void* stream) {
    if (!p || !rowptr || !colidx) return fail(MAD_E_INVALID_ARG, "NULL argument");
    if (!p->finalized) return fail(MAD_E_STATE, "not finalized");
    JacLaunch L;
    int64_t m = 0, nnz = 0;
    int rc = jac_launch(p, L, &m, &nnz);
    if (rc != MAD_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    L.pattern = 1;
    L.rowptr = rowptr;
    L.colidx = colidx;
    MAD_HIP_TRY(launch_jacobian(L, s));
    const int32_t last = (int32_t)nnz;
    MAD_HIP_TRY(hipMemcpyAsync(rowptr + m, &last, sizeof(int32_t), hipMemcpyHostToDevice, s));
    MAD_HIP_TRY(hipStreamSynchronize(s));
    return MAD_OK;
}

int32_t mad_problem_jacobian(mad_problem* p, const double* x, double* r, void* vals, void* stream) {
    if (!p || !x || !r || !vals) return fail(MAD_E_INVALID_ARG, "NULL argument");
    if (!p->finalized) return fail(MAD_E_STATE, "not finalized");
    JacLaunch L;
    int64_t m = 0, nnz = 0;
    int rc = jac_launch(p, L, &m, &nnz);
    if (rc != MAD_OK) return rc;
    L.x = x;
    L.r = r;
    L.vals = vals;
    MAD_HIP_TRY(launch_jacobian(L, (hipStream_t)stream));
    return MAD_OK;
}

int32_t mad_problem_pattern_info(const mad_problem* p, int64_t* rows, int64_t* nnzb, int32_t* bd) {
    if (!p) return fail(MAD_E_INVALID_ARG, "problem is NULL");
    if (!p->finalized) return fail(MAD_E_STATE, "not finalized");
    if (rows) *rows = p->mesh->nv;
    if (nnzb) *nnzb = p->nnzb;
    if (bd) *bd = p->d;
    return MAD_OK;
}

int32_t mad_problem_energy_count(const mad_problem* p, int32_t* count) {
    if (!p || !count) return fail(MAD_E_INVALID_ARG, "NULL argument");
    *count = p->mesh->batched ? 1 + (int32_t)(p->mesh->comp_off.size() - 1) : 1;
    return MAD_OK;
}

int32_t mad_problem_copy_pattern(const mad_problem* p, int32_t* rowptr, int32_t* colidx, void* stream) {
    if (!p || !rowptr || !colidx) return fail(MAD_E_INVALID_ARG, "NULL argument");
    if (!p->finalized) return fail(MAD_E_STATE, "not finalized");
    hipStream_t s = (hipStream_t)stream;
    MAD_HIP_TRY(hipMemcpyAsync(rowptr, p->d_rowptr, sizeof(int32_t) * (p->mesh->nv + 1), hipMemcpyDeviceToDevice, s));
    MAD_HIP_TRY(hipMemcpyAsync(colidx, p->d_colidx, sizeof(int32_t) * p->nnzb, hipMemcpyDeviceToDevice, s));
    return MAD_OK;
}

int32_t mad_problem_eval(mad_problem* p, const double* x, uint32_t mode, double* energy, void* grad, void* hess,
                         void* stream) {
    const int rc = check_eval_args(p, x, mode, energy, grad, hess);
    if (rc != MAD_OK) return rc;
    return eval_problem(p, x, mode, energy, grad, hess, (hipStream_t)stream);
}

int32_t mad_problem_hvp(mad_problem* p, const double* x, const double* v, uint32_t mode, double* energy, void* grad,
                        void* y, void* stream) {
    if (!p) return fail(MAD_E_INVALID_ARG, "problem is NULL");
    if (!p->finalized) return fail(MAD_E_STATE, "hvp before finalize");
    if (!x || !v || !y) return fail(MAD_E_INVALID_ARG, "x, v and y must not be NULL");
    if (mode & ~(uint32_t)(MAD_ENERGY | MAD_GRAD | MAD_SPD))
        return fail(MAD_E_INVALID_ARG, "hvp mode takes MAD_ENERGY, MAD_GRAD and MAD_SPD only");
    if ((mode & MAD_ENERGY) && !energy) return fail(MAD_E_INVALID_ARG, "energy output is NULL");
    if ((mode & MAD_GRAD) && !grad) return fail(MAD_E_INVALID_ARG, "gradient output is NULL");
    return eval_problem(p, x, mode, energy, grad, nullptr, (hipStream_t)stream, v, y);
}

int32_t mad_problem_set_profiling(mad_problem* p, int32_t enable) {
    if (!p) return fail(MAD_E_INVALID_ARG, "problem is NULL");
    p->profiling = enable != 0;
    if (p->profiling) p->prof_count = 0;
    return MAD_OK;
}

int32_t mad_problem_profile(mad_problem* p, double* ms, int32_t* n_stages, int64_t* n_evals) {
    if (!p || !ms) return fail(MAD_E_INVALID_ARG, "NULL argument");
    const int ns = (int)std::max<size_t>(p->terms.size(), 2) + 3;
    for (int i = 0; i < 12; ++i) ms[i] = 0.0;
    for (int64_t k = 0; k < p->prof_count; ++k) {
        auto& row = p->prof_events[(size_t)k];
        MAD_HIP_TRY(hipEventSynchronize(row[ns]));
        for (int st = 0; st < ns; ++st) {
            float t = 0.f;
            MAD_HIP_TRY(hipEventElapsedTime(&t, row[st], row[st + 1]));
            ms[st] += t;
        }
    }
    if (n_stages) *n_stages = ns;
    if (n_evals) *n_evals = p->prof_count;
    return MAD_OK;
}

int32_t mad_problem_status(mad_problem* p, int32_t* nonfinite, int64_t* fallbacks, void* stream) {
    if (!p) return fail(MAD_E_INVALID_ARG, "problem is NULL");
    if (!p->finalized) return fail(MAD_E_STATE, "not finalized");
    hipStream_t s = (hipStream_t)stream;
    int32_t hf[4];
    unsigned long long hb = 0;
    MAD_HIP_TRY(hipMemcpyAsync(hf, p->d_flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    MAD_HIP_TRY(hipMemcpyAsync(&hb, p->d_fallbacks, sizeof(hb), hipMemcpyDeviceToHost, s));
    MAD_HIP_TRY(hipStreamSynchronize(s));
    MAD_HIP_TRY(launch_fill(p->d_flags, 4, 4, s));
    MAD_HIP_TRY(launch_fill(p->d_fallbacks, 1, 8, s));
    MAD_HIP_TRY(hipStreamSynchronize(s));
    if (nonfinite) *nonfinite = hf[0] != 0;
    if (fallbacks) *fallbacks = (int64_t)hb;
    if (hf[1] != 0) {
        std::string what;
        if (hf[1] & kFlagLockTimeout) what += " a wait for the LDS lock of a patch kernel reached its bound;";
        if (hf[1] & kFlagRedoBlockMissing) what += " an element redone in FP64 found a block missing from the pattern;";
        if (hf[1] & kFlagSlotMissing) what += " an element block is missing from the pattern;";
        if (hf[1] & kFlagQueueOverflow) what += " the FP64 redo queue of the static scratch overflowed;";
        return fail(MAD_E_INTERNAL, "device-side check failed (flags " + std::to_string(hf[1]) + "):" + what +
                                        " the outputs since the previous status call are not valid");
    }
    return MAD_OK;
}

int32_t mad_problem_destroy(mad_problem* p) {
    if (!p) return MAD_OK;
    for (auto& row : p->prof_events)
        for (hipEvent_t e : row) (void)hipEventDestroy(e);
    for (void* q : p->layout_owned) (void)hipFree(q);
    for (void* q : p->owned) (void)hipFree(q);
    delete p;
    return MAD_OK;
}

}  // extern "C"
