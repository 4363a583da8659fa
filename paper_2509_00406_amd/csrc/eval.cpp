// One evaluation of a finalized problem on a stream (Sec. 5.5 and Sec. 6.2):
// zero what the strategy needs zeroed, launch the element kernels, gather the
// shared entries, redo the queued FP32 elements in FP64, reduce the energy.
// Called by mad_problem_eval after validation and by the autotuner.
#include <algorithm>
#include <cstring>

#include "mad_internal.hpp"

namespace mad {

EvalScratch own_scratch(const mad_problem* p) {
    EvalScratch sc;
    sc.partial = p->d_partial;
    sc.comp_energy = p->d_comp_energy;
    sc.work_counter = p->d_work_counter;
    sc.fb_count = p->d_fb_count;
    sc.fb_list = p->d_fb_list;
    sc.fb_cap = p->fb_cap;
    sc.halo_g = p->d_halo_g;
    sc.halo_h = p->d_halo_h;
    sc.halo_y = p->d_halo_y;
    sc.normals = p->d_normals;
    for (size_t ti = 0; ti < p->terms.size() && ti < 8; ++ti) {
        sc.psi[ti] = p->terms[ti].d_psi;
        sc.xh[ti] = p->terms[ti].d_xh;
    }
    return sc;
}

int eval_problem(mad_problem* p, const double* x, uint32_t mode, double* energy, void* grad, void* hess,
                 hipStream_t s, const double* v, void* y, const EvalScratch* scp) {
    const EvalScratch sc = scp ? *scp : own_scratch(p);
    const bool hvp = v != nullptr;
    const mad_mesh& m = *p->mesh;
    const int d = p->d;
    const int eb = p->prec == MAD_F32 ? 4 : 8;
    std::vector<hipEvent_t>* ev = nullptr;
    if (p->profiling) {
        const size_t need = std::max<size_t>(p->terms.size(), 2) + 4;
        if ((size_t)p->prof_count >= p->prof_events.size()) {
            std::vector<hipEvent_t> row(need, nullptr);
            for (auto& e : row) MAD_HIP_TRY(hipEventCreate(&e));
            p->prof_events.push_back(std::move(row));
        }
        ev = &p->prof_events[(size_t)p->prof_count++];
        MAD_HIP_TRY(hipEventRecord((*ev)[0], s));
    }
    const bool fallback_pass = p->scatter == MAD_SCATTER_PATCH && p->prec == MAD_F32 && (mode & MAD_SPD);
    // the atomic and colored scatters add into zeroed outputs; the patch scatter writes every entry exactly once
    if (p->scatter != MAD_SCATTER_PATCH) {
        if (mode & MAD_GRAD) MAD_HIP_TRY(launch_fill(grad, m.nv * d, eb, s));
        if (mode & MAD_HESS) MAD_HIP_TRY(launch_fill(hess, p->nnzb * d * d, eb, s));
        if (hvp) MAD_HIP_TRY(launch_fill(y, m.nv * d, eb, s));
    }
    // the FP64 redo queue's count and the persistent queue's head, cleared by one small kernel
    MAD_HIP_TRY(launch_zero_counters(fallback_pass ? sc.fb_count : nullptr,
                                     (p->scatter == MAD_SCATTER_PATCH && p->persistent) ? sc.work_counter : nullptr, s));
    if (ev) MAD_HIP_TRY(hipEventRecord((*ev)[1], s));
    // learned and analytic shell densities: vertex normals of x, then the network pass per MLP term
    if (p->shell) MAD_HIP_TRY(launch_vertex_normals(x, m.nv, p->d_vf_ptr, p->d_vf, p->d_tris, sc.normals, s));
    for (size_t ti = 0; ti < p->terms.size(); ++ti) {
        const Term& t = p->terms[ti];
        if (t.kind != MAD_MLP) continue;
        MlpHeadLaunch H{};
        H.x = x;
        H.normals = sc.normals;
        H.stencil = t.d_stencil;
        H.rest = t.d_rest;
        H.n = t.n;
        H.wbf = t.mlp->d_wbf;
        for (int i = 0; i < 6; ++i) H.s_in[i] = t.mlp->s_in[i];
        H.s_out = t.mlp->s_out;
        H.xh = sc.xh[ti];
        H.psi = sc.psi[ti];
        H.n_cu = p->n_cu;
        MAD_HIP_TRY(launch_mlp_head(H, s));
    }
    if (ev) MAD_HIP_TRY(hipEventRecord((*ev)[2], s));
    const int kmode = (hvp || (mode & MAD_HESS)) ? ((mode & MAD_SPD) ? 3 : 2) : ((mode & MAD_GRAD) ? 1 : 0);
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
        L.lds_bytes = patch_lds_bytes(d, p->prec, kmode, p->max_lv, p->max_lb, hvp);
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
        L.halo_g = sc.halo_g;
        L.halo_h = sc.halo_h;
        L.partial = sc.partial;
        L.flags = p->d_flags;
        L.fallbacks = p->d_fallbacks;
        L.fb_list = sc.fb_list;
        L.fb_count = sc.fb_count;
        L.fb_cap = sc.fb_cap;
        L.eps = p->opt.spd_eps;
        L.qmin = p->opt.degenerate_q;
        L.lock_spins = p->opt.lock_spins == MAD_LOCK_NO_WAIT ? 0
                       : (p->opt.lock_spins > 0 ? p->opt.lock_spins : kDefaultLockSpins);
        L.persistent = p->persistent;
        L.block = (p->wg_waves == 8 && p->prec == MAD_F32) ? 512 : 256;
        L.work_order = p->d_work_order;
        L.work_counter = sc.work_counter;
        L.n_cu = p->n_cu;
        L.normals = sc.normals;
        L.shell = p->shell ? 1 : 0;
        L.light = p->light ? 1 : 0;
        L.hvp = hvp ? 1 : 0;
        L.v = v;
        L.y = y;
        L.halo_y = sc.halo_y;
        {
            // relative element cost by kind (reduced dual size, eigen-problem size, network outputs)
            auto cost = [](int kind) {
                switch (kind) {
                case MAD_BENDING: return 6;
                case MAD_MLP: return 4;
                case MAD_STVK: case MAD_SHELL_TRI: return 3;
                case MAD_SYMDIR: return 2;
                default: return 1;
                }
            };
            const int nt = (int)p->terms.size();
            for (int k = 0; k < nt; ++k) L.term_order[k] = k;
            std::stable_sort(L.term_order, L.term_order + nt,
                             [&](int a, int b) { return cost(p->terms[a].kind) > cost(p->terms[b].kind); });
        }
        for (size_t ti = 0; ti < p->terms.size(); ++ti) {
            const Term& t = p->terms[ti];
            PatchTermArgs& A = L.terms[ti];
            A.kind = t.kind;
            A.n = t.n;
            A.rest = t.d_rest;
            A.lvert = t.d_lvert;
            A.lslot = t.d_lslot;
            A.lseg = t.d_lseg;
            A.elem_ptr = t.d_elem_ptr;
            A.psi = sc.psi[ti];
            A.vdata = t.vdata;
            std::memcpy(A.prm, t.prm, sizeof(A.prm));
        }
        MAD_HIP_TRY(launch_eval_patch(L, s));
        if (ev) MAD_HIP_TRY(hipEventRecord((*ev)[3], s));
        GatherLaunch G{};
        G.prec = p->prec;
        G.var_dim = d;
        G.want_grad = (mode & MAD_GRAD) ? 1 : 0;
        G.want_hess = (mode & MAD_HESS) ? 1 : 0;
        G.grad = grad;
        G.hess = hess;
        G.halo_g = sc.halo_g;
        G.halo_h = sc.halo_h;
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
        if ((mode & MAD_HESS) && p->n_extra > 0)   // blocks of inserted pairs that no term touches
            MAD_HIP_TRY(launch_zero_blocks(hess, p->d_extra_blocks, p->n_extra, d * d, (int)eb, s));
        if (hvp) {   // the product's shared entries, through the same gather lists
            G.want_grad = 1;
            G.want_hess = 0;
            G.grad = y;
            G.halo_g = sc.halo_y;
            MAD_HIP_TRY(launch_gather(G, s));
        }
        if (fallback_pass) {
            FallbackLaunch F{};
            F.var_dim = d;
            F.want_grad = L.want_grad;
            F.x = x;
            F.grad = grad;
            F.hess = hess;
            F.rowptr = p->d_rowptr;
            F.colidx = p->d_colidx;
            F.fb_list = sc.fb_list;
            F.fb_count = sc.fb_count;
            F.fb_cap = sc.fb_cap;
            F.flags = p->d_flags;
            F.eps = p->opt.spd_eps;
            F.normals = sc.normals;
            F.hvp = hvp ? 1 : 0;
            F.v = v;
            F.y = y;
            for (size_t ti = 0; ti < p->terms.size(); ++ti) {
                const Term& t = p->terms[ti];
                F.terms[ti].kind = t.kind;
                F.terms[ti].n = t.n;
                F.terms[ti].stencil = t.d_stencil;
                F.terms[ti].rest = t.d_rest;
                F.terms[ti].psi = sc.psi[ti];
                F.terms[ti].vdata = t.vdata;
                std::memcpy(F.terms[ti].prm, t.prm, sizeof(t.prm));
            }
            MAD_HIP_TRY(launch_fallback(F, s));
        }
        if (ev)
            for (size_t k = 4; k < ev->size() - 1; ++k) MAD_HIP_TRY(hipEventRecord((*ev)[k], s));
        n_partial_terms = 1;
    }
    for (size_t ti = 0; p->scatter != MAD_SCATTER_PATCH && ti < p->terms.size(); ++ti) {
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
        L.partial = sc.partial + ti * (size_t)np;
        L.flags = p->d_flags;
        L.fallbacks = p->d_fallbacks;
        std::memcpy(L.prm, t.prm, sizeof(L.prm));
        L.eps = p->opt.spd_eps;
        L.qmin = p->opt.degenerate_q;
        L.normals = sc.normals;
        L.psi = sc.psi[ti];
        L.vdata = t.vdata;
        L.hvp = hvp ? 1 : 0;
        L.v = v;
        L.y = y;
        if (p->scatter == MAD_SCATTER_COLOR) {
            // one launch per color: no two elements of a launch share a vertex, so plain adds cannot race
            L.plain = 1;
            L.partial = sc.partial;
            L.slot_map = t.d_slot_map;
            for (size_t c = 0; c + 1 < t.color_chunk_ptr.size(); ++c) {
                L.chunk0 = t.color_chunk_ptr[c];
                L.n_patch = t.color_chunk_ptr[c + 1] - t.color_chunk_ptr[c];
                MAD_HIP_TRY(launch_eval(L, s));
            }
        } else {
            MAD_HIP_TRY(launch_eval(L, s));
        }
        if (ev) MAD_HIP_TRY(hipEventRecord((*ev)[3 + ti], s));
    }
    if (mode & MAD_ENERGY) {
        const int ncomp = (int)m.comp_off.size() - 1;
        if (p->scatter == MAD_SCATTER_COLOR)
            MAD_HIP_TRY(launch_energy_reduce(sc.partial, 1, (int)p->n_color_slots, p->d_color_comp_ptr,
                                             std::max(ncomp, 1), m.batched, energy, sc.comp_energy, s));
        else
            MAD_HIP_TRY(launch_energy_reduce(sc.partial, n_partial_terms, np, p->d_comp_patch_ptr,
                                             std::max(ncomp, 1), m.batched, energy, sc.comp_energy, s));
    }
    if (ev) MAD_HIP_TRY(hipEventRecord(ev->back(), s));
    return MAD_OK;
}

}  // namespace mad
