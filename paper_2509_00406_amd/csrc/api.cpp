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

extern "C" {

int32_t mad_version(void) { return 100; }

const char* mad_last_error(void) { return g_last_error.c_str(); }

int32_t mad_options_default(mad_options* opt) {
    if (!opt) return fail(MAD_E_INVALID_ARG, "opt is NULL");
    std::memset(opt, 0, sizeof(*opt));
    opt->scatter = MAD_SCATTER_PATCH;
    opt->patch_faces = 512;
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
        for (int i = 0; i < 8; ++i)
            if (opt->reserved[i] != 0) return fail(MAD_E_INVALID_ARG, "reserved option fields must be zero");
        if (opt->scatter != MAD_SCATTER_AUTO && opt->scatter != MAD_SCATTER_ATOMIC && opt->scatter != MAD_SCATTER_PATCH)
            return fail(MAD_E_INVALID_ARG, "bad scatter mode");
        o.scatter = opt->scatter == MAD_SCATTER_AUTO ? MAD_SCATTER_PATCH : opt->scatter;
        if (opt->patch_faces < 0 || opt->patch_faces > (1 << 20)) return fail(MAD_E_INVALID_ARG, "bad patch_faces");
        if (!(opt->spd_eps >= 0.0) || !std::isfinite(opt->spd_eps)) return fail(MAD_E_INVALID_ARG, "spd_eps must be >= 0");
        if (!(opt->degenerate_q >= 0.0) || opt->degenerate_q > 1.0) return fail(MAD_E_INVALID_ARG, "degenerate_q in [0, 1]");
        if (opt->patch_faces > 0) o.patch_faces = opt->patch_faces;
        o.spd_eps = opt->spd_eps;
        if (opt->degenerate_q > 0.0) o.degenerate_q = opt->degenerate_q;
    }
    mad_problem* p = new (std::nothrow) mad_problem();
    if (!p) return fail(MAD_E_OOM, "problem");
    p->mesh = mesh;
    p->d = var_dim;
    p->prec = precision;
    p->opt = o;
    p->scatter = o.scatter;
    *out = p;
    return MAD_OK;
}

int32_t mad_problem_add_term(mad_problem* p, int32_t kind, const double* params, int32_t n_params,
                             const double* rest_pos) {
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
    }
    if (rc != MAD_OK) return rc;
    p->terms.push_back(std::move(t));
    return MAD_OK;
}

static int upload(mad_problem* p, void** dst, const void* src, size_t bytes, hipStream_t s) {
    MAD_HIP_TRY(hipMalloc(dst, std::max<size_t>(bytes, 16)));
    p->owned.push_back(*dst);
    if (bytes) MAD_HIP_TRY(hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, s));
    return MAD_OK;
}

// Patch order of every term's elements: faces by their patch, diamonds by their lower face,
// edges by their first face; inside a patch, by that face's index.
static void order_terms(mad_problem* p) {
    const mad_mesh& m = *p->mesh;
    const int32_t np = p->patches.n;
    for (auto& t : p->terms) {
        std::vector<int32_t> ep((size_t)t.n), key((size_t)t.n);
        for (int64_t e = 0; e < t.n; ++e) {
            int32_t f;
            if (t.kind == MAD_BENDING) f = m.diamond_faces[2 * e];
            else if (t.kind == MAD_EDGE_SQLEN) f = m.edge_face0[e];
            else f = (int32_t)e;
            ep[e] = p->patches.face_patch[f];
            key[e] = f;
        }
        t.perm.resize((size_t)t.n);
        std::iota(t.perm.begin(), t.perm.end(), 0);
        std::stable_sort(t.perm.begin(), t.perm.end(), [&](int32_t a, int32_t b) {
            if (ep[a] != ep[b]) return ep[a] < ep[b];
            return key[a] < key[b];
        });
        t.elem_ptr.assign((size_t)np + 1, 0);
        for (int64_t e = 0; e < t.n; ++e) t.elem_ptr[ep[e] + 1]++;
        for (int32_t q = 0; q < np; ++q) t.elem_ptr[q + 1] += t.elem_ptr[q];
    }
}

// largest per-patch vertex and upper-block counts of the current patching
static void patch_extent(const mad_problem* p, int32_t* max_lv, int32_t* max_lb) {
    const int64_t nv = p->mesh->nv;
    int32_t mv = 0, mb = 0;
    std::vector<int32_t> verts;
    std::vector<int64_t> keys;
    for (int32_t q = 0; q < p->patches.n; ++q) {
        verts.clear();
        keys.clear();
        for (const auto& t : p->terms)
            for (int32_t i = t.elem_ptr[q]; i < t.elem_ptr[q + 1]; ++i) {
                const int32_t* st = &t.stencil[(int64_t)t.perm[i] * t.ns];
                for (int a = 0; a < t.ns; ++a) {
                    verts.push_back(st[a]);
                    for (int b = a; b < t.ns; ++b)
                        keys.push_back((int64_t)std::min(st[a], st[b]) * nv + std::max(st[a], st[b]));
                }
            }
        std::sort(verts.begin(), verts.end());
        std::sort(keys.begin(), keys.end());
        mv = std::max(mv, (int32_t)(std::unique(verts.begin(), verts.end()) - verts.begin()));
        mb = std::max(mb, (int32_t)(std::unique(keys.begin(), keys.end()) - keys.begin()));
    }
    *max_lv = mv;
    *max_lb = mb;
}

static constexpr size_t kLdsBudget = 60 * 1024;  // dynamic LDS per workgroup; 2 workgroups per CU

int32_t mad_problem_finalize(mad_problem* p, void* stream) {
    if (!p) return fail(MAD_E_INVALID_ARG, "problem is NULL");
    if (p->finalized) return fail(MAD_E_STATE, "already finalized");
    if (p->terms.empty()) return fail(MAD_E_STATE, "no terms");
    hipStream_t s = (hipStream_t)stream;
    const mad_mesh& m = *p->mesh;
    MAD_HIP_TRY(hipGetDevice(&p->device));
    int target = p->opt.patch_faces;
    build_patches(m, target, p->patches);
    order_terms(p);
    if (p->scatter == MAD_SCATTER_PATCH) {
        // shrink the patch target until the largest patch's LDS working set fits the budget
        for (;;) {
            int32_t mv, mb;
            patch_extent(p, &mv, &mb);
            p->lds_bytes = patch_lds_bytes(p->d, p->prec, 3, mv, mb);
            if (p->lds_bytes <= kLdsBudget) break;
            if (target <= 1) return fail(MAD_E_UNSUPPORTED, "a single element exceeds the LDS budget");
            target = std::max(1, (int)(target * 0.75));
            build_patches(m, target, p->patches);
            order_terms(p);
        }
        p->opt.patch_faces = target;
    }
    const int32_t np = p->patches.n;
    int rc;
    for (auto& t : p->terms) {
        std::vector<int32_t> st((size_t)t.n * t.ns);
        std::vector<double> rs((size_t)t.n * t.nrest);
        for (int64_t i = 0; i < t.n; ++i) {
            const int32_t e = t.perm[i];
            for (int a = 0; a < t.ns; ++a) st[i * t.ns + a] = t.stencil[(int64_t)e * t.ns + a];
            for (int k = 0; k < t.nrest; ++k) rs[(int64_t)k * t.n + i] = t.rest[(int64_t)e * t.nrest + k];
        }
        if ((rc = upload(p, (void**)&t.d_stencil, st.data(), st.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = upload(p, (void**)&t.d_rest, rs.data(), rs.size() * 8, s)) != MAD_OK) return rc;
        if ((rc = upload(p, (void**)&t.d_elem_ptr, t.elem_ptr.data(), t.elem_ptr.size() * 4, s)) != MAD_OK) return rc;
    }
    if ((rc = upload(p, (void**)&p->d_comp_patch_ptr, p->patches.comp_patch_ptr.data(),
                     p->patches.comp_patch_ptr.size() * 4, s)) != MAD_OK)
        return rc;
    MAD_HIP_TRY(hipMalloc((void**)&p->d_partial, sizeof(double) * std::max<size_t>(1, (size_t)np * p->terms.size())));
    p->owned.push_back(p->d_partial);
    MAD_HIP_TRY(hipMalloc((void**)&p->d_flags, sizeof(int32_t) * 4));
    p->owned.push_back(p->d_flags);
    MAD_HIP_TRY(hipMalloc((void**)&p->d_fallbacks, sizeof(unsigned long long)));
    p->owned.push_back(p->d_fallbacks);
    MAD_HIP_TRY(launch_fill(p->d_flags, 4, 4, s));
    MAD_HIP_TRY(launch_fill(p->d_fallbacks, 1, 8, s));
    std::vector<PatternTerm> pts;
    for (auto& t : p->terms) pts.push_back({t.d_stencil, t.n, t.ns});
    if ((rc = build_pattern_device(m.nv, pts, &p->d_rowptr, &p->d_colidx, &p->nnzb, p->owned, s)) != MAD_OK) return rc;
    if (p->scatter == MAD_SCATTER_ATOMIC) {
        for (auto& t : p->terms) {
            MAD_HIP_TRY(hipMalloc((void**)&t.d_slots, sizeof(int32_t) * std::max<int64_t>(1, t.n * t.ns * t.ns)));
            p->owned.push_back(t.d_slots);
            MAD_HIP_TRY(launch_slots(t.d_stencil, t.n, t.ns, p->d_rowptr, p->d_colidx, t.d_slots, p->d_flags, s));
        }
    } else {
        std::vector<int32_t> rowptr((size_t)m.nv + 1), colidx((size_t)std::max<int64_t>(p->nnzb, 1));
        MAD_HIP_TRY(hipMemcpyAsync(rowptr.data(), p->d_rowptr, rowptr.size() * 4, hipMemcpyDeviceToHost, s));
        MAD_HIP_TRY(hipMemcpyAsync(colidx.data(), p->d_colidx, (size_t)p->nnzb * 4, hipMemcpyDeviceToHost, s));
        MAD_HIP_TRY(hipStreamSynchronize(s));
        colidx.resize((size_t)p->nnzb);
        PatchLocal L;
        if ((rc = build_patch_local(*p, rowptr, colidx, L)) != MAD_OK) return rc;
        p->max_lv = L.max_lv;
        p->max_lb = L.max_lb;
        p->lds_bytes = patch_lds_bytes(p->d, p->prec, 3, L.max_lv, L.max_lb);
        if ((rc = upload(p, (void**)&p->d_lv_ptr, L.lv_ptr.data(), L.lv_ptr.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = upload(p, (void**)&p->d_lv_global, L.lv_global.data(), L.lv_global.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = upload(p, (void**)&p->d_lv_halo, L.lv_halo.data(), L.lv_halo.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = upload(p, (void**)&p->d_lb_ptr, L.lb_ptr.data(), L.lb_ptr.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = upload(p, (void**)&p->d_lb_gidx, L.lb_gidx.data(), L.lb_gidx.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = upload(p, (void**)&p->d_lb_gidxT, L.lb_gidxT.data(), L.lb_gidxT.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = upload(p, (void**)&p->d_lb_halo, L.lb_halo.data(), L.lb_halo.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = upload(p, (void**)&p->d_gv_ptr, L.gv_ptr.data(), L.gv_ptr.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = upload(p, (void**)&p->d_gv_src, L.gv_src.data(), L.gv_src.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = upload(p, (void**)&p->d_gv_vert, L.gv_vert.data(), L.gv_vert.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = upload(p, (void**)&p->d_gb_ptr, L.gb_ptr.data(), L.gb_ptr.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = upload(p, (void**)&p->d_gb_src, L.gb_src.data(), L.gb_src.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = upload(p, (void**)&p->d_gb_gidx, L.gb_gidx.data(), L.gb_gidx.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = upload(p, (void**)&p->d_gb_gidxT, L.gb_gidxT.data(), L.gb_gidxT.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = upload(p, (void**)&p->d_orphan_vert, L.orphan_vert.data(), L.orphan_vert.size() * 4, s)) != MAD_OK)
            return rc;
        if ((rc = upload(p, (void**)&p->d_orphan_block, L.orphan_block.data(), L.orphan_block.size() * 4, s)) != MAD_OK)
            return rc;
        p->n_gv = (int32_t)L.gv_vert.size();
        p->n_gb = (int32_t)L.gb_gidx.size();
        p->n_orphan_vert = (int32_t)L.orphan_vert.size();
        p->n_orphan_block = (int32_t)L.orphan_block.size();
        const size_t eb = p->prec == MAD_F32 ? 4 : 8;
        const size_t nhv = L.gv_src.size(), nhb = L.gb_src.size();
        MAD_HIP_TRY(hipMalloc(&p->d_halo_g, std::max<size_t>(16, nhv * p->d * eb)));
        p->owned.push_back(p->d_halo_g);
        MAD_HIP_TRY(hipMalloc(&p->d_halo_h, std::max<size_t>(16, nhb * p->d * p->d * eb)));
        p->owned.push_back(p->d_halo_h);
        for (size_t ti = 0; ti < p->terms.size(); ++ti) {
            auto& t = p->terms[ti];
            if ((rc = upload(p, (void**)&t.d_lvert, L.lvert[ti].data(), L.lvert[ti].size() * 2, s)) != MAD_OK) return rc;
            if ((rc = upload(p, (void**)&t.d_lslot, L.lslot[ti].data(), L.lslot[ti].size() * 2, s)) != MAD_OK) return rc;
        }
        if (p->prec == MAD_F32) {
            // queue for FP32 elements redone in FP64: room for every element
            int64_t total = 0;
            for (auto& t : p->terms) {
                if (t.n >= (1ll << 29)) return fail(MAD_E_OVERFLOW, "more than 2^29 elements in one term");
                total += t.n;
            }
            if (total >= INT32_MAX) return fail(MAD_E_OVERFLOW, "more than 2^31 elements");
            p->fb_cap = (int32_t)std::max<int64_t>(total, 1);
            MAD_HIP_TRY(hipMalloc((void**)&p->d_fb_list, sizeof(uint32_t) * (size_t)p->fb_cap));
            p->owned.push_back(p->d_fb_list);
            MAD_HIP_TRY(hipMalloc((void**)&p->d_fb_count, sizeof(int32_t) * 4));
            p->owned.push_back(p->d_fb_count);
        }
    }
    int32_t hflags[4];
    MAD_HIP_TRY(hipMemcpyAsync(hflags, p->d_flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
    MAD_HIP_TRY(hipStreamSynchronize(s));
    if (hflags[1] != 0) return fail(MAD_E_HIP, "internal error: element block missing from the pattern");
    // host copies of element data are no longer needed
    for (auto& t : p->terms) {
        std::vector<int32_t>().swap(t.stencil);
        std::vector<double>().swap(t.rest);
        std::vector<int32_t>().swap(t.perm);
    }
    p->finalized = true;
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
    if (!p) return fail(MAD_E_INVALID_ARG, "problem is NULL");
    if (!p->finalized) return fail(MAD_E_STATE, "eval before finalize");
    if (!x) return fail(MAD_E_INVALID_ARG, "x is NULL");
    if (mode & ~15u) return fail(MAD_E_INVALID_ARG, "unknown mode bits");
    if ((mode & MAD_ENERGY) && !energy) return fail(MAD_E_INVALID_ARG, "energy output is NULL");
    if ((mode & MAD_GRAD) && !grad) return fail(MAD_E_INVALID_ARG, "gradient output is NULL");
    if ((mode & MAD_HESS) && !hess) return fail(MAD_E_INVALID_ARG, "Hessian output is NULL");
    if ((mode & MAD_SPD) && !(mode & MAD_HESS)) return fail(MAD_E_INVALID_ARG, "MAD_SPD needs MAD_HESS");
    hipStream_t s = (hipStream_t)stream;
    const mad_mesh& m = *p->mesh;
    const int d = p->d;
    const int eb = p->prec == MAD_F32 ? 4 : 8;
    std::vector<hipEvent_t>* ev = nullptr;
    if (p->profiling) {
        const size_t need = std::max<size_t>(p->terms.size(), 2) + 3;
        if ((size_t)p->prof_count >= p->prof_events.size()) {
            std::vector<hipEvent_t> row(need, nullptr);
            for (auto& e : row) MAD_HIP_TRY(hipEventCreate(&e));
            p->prof_events.push_back(std::move(row));
        }
        ev = &p->prof_events[(size_t)p->prof_count++];
        MAD_HIP_TRY(hipEventRecord((*ev)[0], s));
    }
    const bool fallback_pass = p->scatter == MAD_SCATTER_PATCH && p->prec == MAD_F32 && (mode & MAD_SPD);
    // the atomic scatter adds into zeroed outputs; the patch scatter writes every entry exactly once
    if (p->scatter == MAD_SCATTER_ATOMIC) {
        if (mode & MAD_GRAD) MAD_HIP_TRY(launch_fill(grad, m.nv * d, eb, s));
        if (mode & MAD_HESS) MAD_HIP_TRY(launch_fill(hess, p->nnzb * d * d, eb, s));
    }
    if (fallback_pass) MAD_HIP_TRY(launch_fill(p->d_fb_count, 1, 4, s));
    if (ev) MAD_HIP_TRY(hipEventRecord((*ev)[1], s));
    const int kmode = (mode & MAD_HESS) ? ((mode & MAD_SPD) ? 3 : 2) : ((mode & MAD_GRAD) ? 1 : 0);
    const int np = p->patches.n;
    int n_partial_terms = (int)p->terms.size();
    if (p->scatter == MAD_SCATTER_PATCH) {
        PatchLaunch L{};
        L.prec = p->prec;
        L.mode = kmode;
        L.want_grad = (mode & MAD_GRAD) ? 1 : 0;
        L.var_dim = d;
        L.n_terms = (int)p->terms.size();
        L.n_patch = np;
        L.lds_bytes = patch_lds_bytes(d, p->prec, kmode, p->max_lv, p->max_lb);
        L.x = x;
        L.grad = grad;
        L.hess = hess;
        L.lv_ptr = p->d_lv_ptr;
        L.lv_global = p->d_lv_global;
        L.lv_halo = p->d_lv_halo;
        L.lb_ptr = p->d_lb_ptr;
        L.lb_gidx = p->d_lb_gidx;
        L.lb_gidxT = p->d_lb_gidxT;
        L.lb_halo = p->d_lb_halo;
        L.halo_g = p->d_halo_g;
        L.halo_h = p->d_halo_h;
        L.partial = p->d_partial;
        L.flags = p->d_flags;
        L.fallbacks = p->d_fallbacks;
        L.fb_list = p->d_fb_list;
        L.fb_count = p->d_fb_count;
        L.fb_cap = p->fb_cap;
        L.eps = p->opt.spd_eps;
        L.qmin = p->opt.degenerate_q;
        for (size_t ti = 0; ti < p->terms.size(); ++ti) {
            const Term& t = p->terms[ti];
            PatchTermArgs& A = L.terms[ti];
            A.kind = t.kind;
            A.n = t.n;
            A.rest = t.d_rest;
            A.lvert = t.d_lvert;
            A.lslot = t.d_lslot;
            A.elem_ptr = t.d_elem_ptr;
            std::memcpy(A.prm, t.prm, sizeof(A.prm));
        }
        MAD_HIP_TRY(launch_eval_patch(L, s));
        if (ev) MAD_HIP_TRY(hipEventRecord((*ev)[2], s));
        GatherLaunch G{};
        G.prec = p->prec;
        G.var_dim = d;
        G.want_grad = (mode & MAD_GRAD) ? 1 : 0;
        G.want_hess = (mode & MAD_HESS) ? 1 : 0;
        G.grad = grad;
        G.hess = hess;
        G.halo_g = p->d_halo_g;
        G.halo_h = p->d_halo_h;
        G.gv_ptr = p->d_gv_ptr;
        G.gv_src = p->d_gv_src;
        G.gv_vert = p->d_gv_vert;
        G.gb_ptr = p->d_gb_ptr;
        G.gb_src = p->d_gb_src;
        G.gb_gidx = p->d_gb_gidx;
        G.gb_gidxT = p->d_gb_gidxT;
        G.orphan_vert = p->d_orphan_vert;
        G.orphan_block = p->d_orphan_block;
        G.n_gv = p->n_gv;
        G.n_gb = p->n_gb;
        G.n_orphan_vert = p->n_orphan_vert;
        G.n_orphan_block = p->n_orphan_block;
        MAD_HIP_TRY(launch_gather(G, s));
        if (fallback_pass) {
            FallbackLaunch F{};
            F.var_dim = d;
            F.want_grad = L.want_grad;
            F.x = x;
            F.grad = grad;
            F.hess = hess;
            F.rowptr = p->d_rowptr;
            F.colidx = p->d_colidx;
            F.fb_list = p->d_fb_list;
            F.fb_count = p->d_fb_count;
            F.fb_cap = p->fb_cap;
            F.flags = p->d_flags;
            F.eps = p->opt.spd_eps;
            for (size_t ti = 0; ti < p->terms.size(); ++ti) {
                const Term& t = p->terms[ti];
                F.terms[ti].kind = t.kind;
                F.terms[ti].n = t.n;
                F.terms[ti].stencil = t.d_stencil;
                F.terms[ti].rest = t.d_rest;
                std::memcpy(F.terms[ti].prm, t.prm, sizeof(t.prm));
            }
            MAD_HIP_TRY(launch_fallback(F, s));
        }
        if (ev)
            for (size_t k = 3; k < ev->size() - 1; ++k) MAD_HIP_TRY(hipEventRecord((*ev)[k], s));
        n_partial_terms = 1;
    }
    for (size_t ti = 0; p->scatter == MAD_SCATTER_ATOMIC && ti < p->terms.size(); ++ti) {
        const Term& t = p->terms[ti];
        EvalLaunch L{};
        L.kind = t.kind;
        L.prec = p->prec;
        L.mode = kmode;
        L.want_grad = (mode & MAD_GRAD) ? 1 : 0;
        L.n_patch = np;
        L.x = x;
        L.stencil = t.d_stencil;
        L.rest = t.d_rest;
        L.n = t.n;
        L.elem_ptr = t.d_elem_ptr;
        L.slots = t.d_slots;
        L.grad = grad;
        L.hess = hess;
        L.partial = p->d_partial + ti * (size_t)np;
        L.flags = p->d_flags;
        L.fallbacks = p->d_fallbacks;
        std::memcpy(L.prm, t.prm, sizeof(L.prm));
        L.eps = p->opt.spd_eps;
        L.qmin = p->opt.degenerate_q;
        MAD_HIP_TRY(launch_eval(L, s));
        if (ev) MAD_HIP_TRY(hipEventRecord((*ev)[2 + ti], s));
    }
    if (mode & MAD_ENERGY) {
        const int ncomp = (int)m.comp_off.size() - 1;
        MAD_HIP_TRY(launch_energy_reduce(p->d_partial, n_partial_terms, np, p->d_comp_patch_ptr,
                                         std::max(ncomp, 1), m.batched, energy, s));
    }
    if (ev) MAD_HIP_TRY(hipEventRecord(ev->back(), s));
    return MAD_OK;
}

int32_t mad_problem_set_profiling(mad_problem* p, int32_t enable) {
    if (!p) return fail(MAD_E_INVALID_ARG, "problem is NULL");
    p->profiling = enable != 0;
    if (p->profiling) p->prof_count = 0;
    return MAD_OK;
}

int32_t mad_problem_profile(mad_problem* p, double* ms, int32_t* n_stages, int64_t* n_evals) {
    if (!p || !ms) return fail(MAD_E_INVALID_ARG, "NULL argument");
    const int ns = (int)std::max<size_t>(p->terms.size(), 2) + 2;
    for (int i = 0; i < 10; ++i) ms[i] = 0.0;
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
    return MAD_OK;
}

int32_t mad_problem_destroy(mad_problem* p) {
    if (!p) return MAD_OK;
    for (auto& row : p->prof_events)
        for (hipEvent_t e : row) (void)hipEventDestroy(e);
    for (void* q : p->owned) (void)hipFree(q);
    delete p;
    return MAD_OK;
}

}  // extern "C"
