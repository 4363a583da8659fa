// Evaluation layout of a problem: patches, the patch order of every term's
// elements, and the structures of the chosen scatter strategy. Built at
// finalize and rebuilt by the autotuner; the block pattern is independent of it.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <thread>

#include "mad_internal.hpp"

namespace mad {

// allocate and fill from host memory; waits for the copy (the source is often a temporary)
static int upload_layout(mad_problem* p, void** dst, const void* src, size_t bytes, hipStream_t s) {
    MAD_HIP_TRY(hipMalloc(dst, std::max<size_t>(bytes, 16)));
    p->layout_owned.push_back(*dst);
    if (bytes) {
        MAD_HIP_TRY(hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, s));
        MAD_HIP_TRY(hipStreamSynchronize(s));
    }
    return MAD_OK;
}

static int alloc_layout(mad_problem* p, void** dst, size_t bytes) {
    MAD_HIP_TRY(hipMalloc(dst, std::max<size_t>(bytes, 16)));
    p->layout_owned.push_back(*dst);
    return MAD_OK;
}

static void free_layout(mad_problem* p) {
    for (void* q : p->layout_owned) (void)hipFree(q);
    p->layout_owned.clear();
    for (auto& t : p->terms) {
        t.d_stencil = nullptr;
        t.d_rest = nullptr;
        t.d_elem_ptr = nullptr;
        t.d_slots = nullptr;
        t.d_lvert = nullptr;
        t.d_lslot = nullptr;
        t.d_lseg = nullptr;
        t.d_psi = nullptr;
        t.d_xh = nullptr;
        t.d_jstencil = nullptr;
        t.d_jrest = nullptr;
        t.d_slot_map = nullptr;
    }
    p->d_color_comp_ptr = nullptr;
    p->d_lv_ptr = p->d_lv_global = p->d_lv_halo = nullptr;
    p->d_lb_ptr = p->d_lb_gidx = p->d_lb_gidxT = p->d_lb_halo = nullptr;
    p->n_lb = 0;
    p->d_gv_ptr = p->d_gv_src = p->d_gv_vert = nullptr;
    p->d_gb_ptr = p->d_gb_src = p->d_gb_gidx = p->d_gb_gidxT = nullptr;
    p->d_orphan_vert = p->d_orphan_block = nullptr;
    p->d_halo_g = p->d_halo_h = p->d_halo_y = nullptr;
    p->n_halo_v = p->n_halo_b = 0;
    p->d_fb_list = nullptr;
    p->d_fb_count = nullptr;
    p->d_work_order = p->d_work_counter = nullptr;
    p->d_partial = nullptr;
    p->d_comp_energy = nullptr;
    p->d_comp_patch_ptr = nullptr;
}

// Build the patches and the element order (host), then upload the element arrays. If the pattern
// already exists, also build the structures of the scatter strategy.
size_t lds_budget(const mad_problem* p) {
    return (p->wg_waves == 8 && p->prec == MAD_F32 && !p->light) ? kLdsBudgetWide : kLdsBudget;
}

int build_layout(mad_problem* p, int target, int scatter, int persistent, hipStream_t s, int wg_waves) {
    const mad_mesh& m = *p->mesh;
    MAD_HIP_TRY(hipStreamSynchronize(s));
    free_layout(p);
    p->scatter = scatter;
    p->persistent = scatter == MAD_SCATTER_PATCH ? persistent : 0;
    if (wg_waves != 0) p->wg_waves = (wg_waves == 8 && p->prec == MAD_F32) ? 8 : 4;
    // the fit below needs only which elements each patch holds: the colour order comes after it
    build_patches(m, target, p->patches);
    order_terms(p);
    if (scatter == MAD_SCATTER_PATCH) {
        // shrink the patch target until the largest patch's LDS working set fits the budget and
        // every patch has at most kMaxPatchUnits work units
        for (;;) {
            int32_t mv, mb;
            patch_extent(p, &mv, &mb);
            p->lds_bytes = patch_lds_bytes(p->d, p->prec, 3, mv, mb);
            int32_t mu = 0;
            for (int32_t q = 0; q < p->patches.n; ++q) {
                int32_t u = 0;
                for (const auto& t : p->terms) u += (t.elem_ptr[q + 1] - t.elem_ptr[q] + 63) / 64;
                mu = std::max(mu, u);
            }
            if (p->lds_bytes <= lds_budget(p) && mu <= kMaxPatchUnits) break;
            if (target <= 1) return fail(MAD_E_UNSUPPORTED, "a single element exceeds the LDS budget");
            target = std::max(1, (int)(target * 0.75));
            build_patches(m, target, p->patches);
            order_terms(p);
        }
    }
    for (auto& t : p->terms) color_within_patches(t, m.nv);
    std::vector<int32_t> comp_slot_ptr;
    p->n_color_slots = 0;
    if (scatter == MAD_SCATTER_COLOR) color_order(p, comp_slot_ptr);
    p->opt.patch_faces = target;
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
        if ((rc = upload_layout(p, (void**)&t.d_stencil, st.data(), st.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = upload_layout(p, (void**)&t.d_rest, rs.data(), rs.size() * 8, s)) != MAD_OK) return rc;
        if ((rc = upload_layout(p, (void**)&t.d_elem_ptr, t.elem_ptr.data(), t.elem_ptr.size() * 4, s)) != MAD_OK)
            return rc;
        if (kind_nres(t.kind) > 0) {
            // the Jacobian kernel runs in element order, so that each element's rows are written next to its
            // neighbours' (the evaluation kernels run in patch order)
            std::vector<double> rj((size_t)t.n * t.nrest);
            for (int64_t e = 0; e < t.n; ++e)
                for (int k = 0; k < t.nrest; ++k) rj[(int64_t)k * t.n + e] = t.rest[(int64_t)e * t.nrest + k];
            if ((rc = upload_layout(p, (void**)&t.d_jstencil, t.stencil.data(), t.stencil.size() * 4, s)) != MAD_OK)
                return rc;
            if ((rc = upload_layout(p, (void**)&t.d_jrest, rj.data(), rj.size() * 8, s)) != MAD_OK) return rc;
        }
        if (scatter == MAD_SCATTER_COLOR &&
            (rc = upload_layout(p, (void**)&t.d_slot_map, t.slot_map.data(), t.slot_map.size() * 4, s)) != MAD_OK)
            return rc;
        if (t.kind == MAD_MLP) {
            const size_t n = (size_t)std::max<int64_t>(t.n, 1);
            if ((rc = alloc_layout(p, (void**)&t.d_psi, sizeof(float) * (size_t)kPsi * n)) != MAD_OK) return rc;
            if ((rc = alloc_layout(p, (void**)&t.d_xh, sizeof(float) * 6 * n)) != MAD_OK) return rc;
        }
    }
    if ((rc = upload_layout(p, (void**)&p->d_comp_patch_ptr, p->patches.comp_patch_ptr.data(),
                            p->patches.comp_patch_ptr.size() * 4, s)) != MAD_OK)
        return rc;
    if (scatter == MAD_SCATTER_COLOR &&
        (rc = upload_layout(p, (void**)&p->d_color_comp_ptr, comp_slot_ptr.data(), comp_slot_ptr.size() * 4, s)) !=
            MAD_OK)
        return rc;
    const size_t n_partial = std::max<size_t>({(size_t)1, (size_t)np * p->terms.size(), (size_t)p->n_color_slots});
    if ((rc = alloc_layout(p, (void**)&p->d_partial, sizeof(double) * n_partial)) != MAD_OK) return rc;
    if ((rc = alloc_layout(p, (void**)&p->d_comp_energy,
                           sizeof(double) * std::max<size_t>(1, p->patches.comp_patch_ptr.size()))) != MAD_OK)
        return rc;
    // work order of the persistent launch. persistent == 1: patches in index order, which is spatial
    // order (neighbouring patches share halo vertices and output cache lines, so they run close in time),
    // grouped into four size classes with the largest class first (no large patch starts last).
    // persistent == 2: strictly by decreasing element count.
    {
        std::vector<int64_t> cnt((size_t)np, 0);
        for (auto& t : p->terms)
            for (int32_t q = 0; q < np; ++q) cnt[q] += t.elem_ptr[q + 1] - t.elem_ptr[q];
        const int64_t cmax = np > 0 ? *std::max_element(cnt.begin(), cnt.end()) : 0;
        std::vector<int32_t> order((size_t)np);
        std::iota(order.begin(), order.end(), 0);
        if (persistent == 2) {
            std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cnt[a] > cnt[b]; });
        } else {
            auto cls = [&](int32_t q) { return (cnt[q] * 4) / (cmax + 1); };
            std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cls(a) > cls(b); });
        }
        if ((rc = upload_layout(p, (void**)&p->d_work_order, order.data(), order.size() * 4, s)) != MAD_OK) return rc;
        if ((rc = alloc_layout(p, (void**)&p->d_work_counter, 16)) != MAD_OK) return rc;
    }
    MAD_HIP_TRY(hipStreamSynchronize(s));
    if (p->h_rowptr.empty()) return MAD_OK;   // pattern not built yet (first layout, inside finalize)
    return build_scatter(p, s);
}

// Structures of the scatter strategy for the current element order; needs the pattern.
int build_scatter(mad_problem* p, hipStream_t s) {
    int rc;
    if (p->host_pattern_stale) {
        // pairs were inserted since the host copy was taken: refresh it; the rebuilt structures cover
        // the inserted blocks (as blocks no element touches), so the extra list starts over
        p->h_rowptr.resize((size_t)p->mesh->nv + 1);
        p->h_colidx.resize((size_t)std::max<int64_t>(p->nnzb, 1));
        MAD_HIP_TRY(hipMemcpyAsync(p->h_rowptr.data(), p->d_rowptr, p->h_rowptr.size() * 4, hipMemcpyDeviceToHost, s));
        MAD_HIP_TRY(hipMemcpyAsync(p->h_colidx.data(), p->d_colidx, (size_t)p->nnzb * 4, hipMemcpyDeviceToHost, s));
        MAD_HIP_TRY(hipStreamSynchronize(s));
        p->h_colidx.resize((size_t)p->nnzb);
        p->host_pattern_stale = false;
    }
    p->n_extra = 0;
    if (p->scatter != MAD_SCATTER_PATCH) {   // atomic and colored: the global block of every element pair
        for (auto& t : p->terms) {
            if ((rc = alloc_layout(p, (void**)&t.d_slots, sizeof(int32_t) * std::max<int64_t>(1, t.n * t.ns * t.ns))) !=
                MAD_OK)
                return rc;
            MAD_HIP_TRY(launch_slots(t.d_stencil, t.n, t.ns, p->d_rowptr, p->d_colidx, t.d_slots, p->d_flags, s));
        }
        MAD_HIP_TRY(hipStreamSynchronize(s));
        return MAD_OK;
    }
    PatchLocal L;
    if ((rc = build_patch_local(*p, p->h_rowptr, p->h_colidx, L)) != MAD_OK) return rc;
    p->max_lv = L.max_lv;
    p->max_lb = L.max_lb;
    p->lds_bytes = patch_lds_bytes(p->d, p->prec, 3, L.max_lv, L.max_lb);
    struct Up {
        void** dst;
        const std::vector<int32_t>* v;
    } ups[] = {{(void**)&p->d_lv_ptr, &L.lv_ptr},       {(void**)&p->d_lv_global, &L.lv_global},
               {(void**)&p->d_lv_halo, &L.lv_halo},     {(void**)&p->d_lb_ptr, &L.lb_ptr},
               {(void**)&p->d_lb_gidx, &L.lb_gidx},     {(void**)&p->d_lb_gidxT, &L.lb_gidxT},
               {(void**)&p->d_lb_halo, &L.lb_halo},     {(void**)&p->d_gv_ptr, &L.gv_ptr},
               {(void**)&p->d_gv_src, &L.gv_src},       {(void**)&p->d_gv_vert, &L.gv_vert},
               {(void**)&p->d_gb_ptr, &L.gb_ptr},       {(void**)&p->d_gb_src, &L.gb_src},
               {(void**)&p->d_gb_gidx, &L.gb_gidx},     {(void**)&p->d_gb_gidxT, &L.gb_gidxT},
               {(void**)&p->d_orphan_vert, &L.orphan_vert}, {(void**)&p->d_orphan_block, &L.orphan_block}};
    for (auto& u : ups)
        if ((rc = upload_layout(p, u.dst, u.v->data(), u.v->size() * 4, s)) != MAD_OK) return rc;
    p->n_lb = (int64_t)L.lb_gidx.size();
    p->n_gv = (int32_t)L.gv_vert.size();
    p->n_gb = (int32_t)L.gb_gidx.size();
    p->n_orphan_vert = (int32_t)L.orphan_vert.size();
    p->n_orphan_block = (int32_t)L.orphan_block.size();
    const size_t eb = p->prec == MAD_F32 ? 4 : 8;
    p->n_halo_v = (int64_t)L.gv_src.size();
    p->n_halo_b = (int64_t)L.gb_src.size();
    if ((rc = alloc_layout(p, &p->d_halo_g, L.gv_src.size() * p->d * eb)) != MAD_OK) return rc;
    if ((rc = alloc_layout(p, &p->d_halo_h, L.gb_src.size() * p->d * p->d * eb)) != MAD_OK) return rc;
    if ((rc = alloc_layout(p, &p->d_halo_y, L.gv_src.size() * p->d * eb)) != MAD_OK) return rc;
    for (size_t ti = 0; ti < p->terms.size(); ++ti) {
        auto& t = p->terms[ti];
        if ((rc = upload_layout(p, (void**)&t.d_lvert, L.lvert[ti].data(), L.lvert[ti].size() * 2, s)) != MAD_OK)
            return rc;
        if ((rc = upload_layout(p, (void**)&t.d_lslot, L.lslot[ti].data(), L.lslot[ti].size() * 2, s)) != MAD_OK)
            return rc;
        std::vector<uint8_t> seg;
        unit_segments(t, (int32_t)p->patches.n, p->mesh->nv, seg);
        if ((rc = upload_layout(p, (void**)&t.d_lseg, seg.data(), seg.size(), s)) != MAD_OK) return rc;
    }
    if (p->prec == MAD_F32) {
        // queue for FP32 elements redone in FP64: room for every element
        int64_t total = 0;
        for (auto& t : p->terms) {
            if (t.n >= (1ll << 28)) return fail(MAD_E_OVERFLOW, "more than 2^28 elements in one term");
            total += t.n;
        }
        if (total >= INT32_MAX) return fail(MAD_E_OVERFLOW, "more than 2^31 elements");
        p->fb_cap = (int32_t)std::max<int64_t>(total, 1);
        if ((rc = alloc_layout(p, (void**)&p->d_fb_list, sizeof(uint32_t) * (size_t)p->fb_cap)) != MAD_OK) return rc;
        if ((rc = alloc_layout(p, (void**)&p->d_fb_count, 16)) != MAD_OK) return rc;
    }
    MAD_HIP_TRY(hipStreamSynchronize(s));
    return MAD_OK;
}

}  // namespace mad
