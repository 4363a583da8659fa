// Patch-local index structures for the LDS-accumulating assembly.
//
// For every patch: the sorted list of vertices its elements touch (x is
// staged into LDS from this list, gradient entries are flushed through it)
// and the sorted list of upper-triangle blocks (r <= c) its elements add to
// (the workgroup accumulates them in LDS and writes each once). An entry is
// "exclusive" when no other patch touches it: it is written with a plain
// store; a shared entry is written to a halo slot of its own and summed
// afterwards, in a fixed order, by a gather kernel.
//
// Per element, the stencil becomes patch-local vertex indices (u16) and, for
// each unordered stencil pair s <= t, a local block index (low 14 bits) with
// two flag bits: bit 14 = the element's (s, t) block lands transposed in the
// stored (min, max) block; bit 15 = s != t name the same vertex (a degenerate
// stencil), so both (s, t) and (t, s) add into that diagonal block.
#include <algorithm>
#include <array>
#include <atomic>
#include <thread>

#include "mad_internal.hpp"

namespace mad {

static int32_t find_block(const std::vector<int32_t>& rowptr, const std::vector<int32_t>& colidx, int32_t r,
                          int32_t c) {
    auto b = colidx.begin() + rowptr[r], e = colidx.begin() + rowptr[r + 1];
    auto it = std::lower_bound(b, e, c);
    return (it != e && *it == c) ? (int32_t)(it - colidx.begin()) : -1;
}

int build_patch_local(mad_problem& P, const std::vector<int32_t>& rowptr, const std::vector<int32_t>& colidx,
                      PatchLocal& L) {
    const int32_t np = P.patches.n;
    const int nt = (int)P.terms.size();
    const int64_t nv = P.mesh->nv;
    std::vector<std::vector<int32_t>> pv((size_t)np), pb_g((size_t)np), pb_gt((size_t)np);
    // per term, per element (patch order): local maps
    L.lvert.assign(nt, {});
    L.lslot.assign(nt, {});
    for (int t = 0; t < nt; ++t) {
        const Term& T = P.terms[t];
        L.lvert[t].assign((size_t)T.n * T.ns, 0);
        L.lslot[t].assign((size_t)T.n * (T.ns * (T.ns + 1) / 2), 0);
    }
    std::atomic<int> err{0};
    // Per patch: its vertices, numbered in ascending global order (local index), and its upper blocks,
    // numbered in ascending (row, column) order. The local numbers come from a table per thread: the
    // vertex map loc[global vertex] and, for patches of at most kDenseLocal vertices, a dense table
    // tab[local row * nloc + local column] of the block numbers; both are reset after each patch, so a
    // patch costs time in proportion to its elements. Larger patches (a caller's large patch target)
    // sort and binary-search instead.
    constexpr int32_t kDenseLocal = 1024;
    auto work = [&](int32_t p0, int32_t p1) {
        std::vector<int32_t> verts, keys, loc((size_t)nv, -1), tab;
        std::vector<int64_t> lkeys;
        for (int32_t p = p0; p < p1; ++p) {
            verts.clear();
            for (int t = 0; t < nt; ++t) {
                const Term& T = P.terms[t];
                for (int32_t i = T.elem_ptr[p]; i < T.elem_ptr[p + 1]; ++i) {
                    const int32_t* st = &T.stencil[(int64_t)T.perm[i] * T.ns];
                    for (int a = 0; a < T.ns; ++a)
                        if (loc[st[a]] < 0) {
                            loc[st[a]] = 0;
                            verts.push_back(st[a]);
                        }
                }
            }
            std::sort(verts.begin(), verts.end());
            const int32_t nloc = (int32_t)verts.size();
            for (int32_t k = 0; k < nloc; ++k) loc[verts[k]] = k;
            const bool dense = nloc <= kDenseLocal;
            keys.clear();
            lkeys.clear();
            if (dense) {
                if (tab.size() < (size_t)nloc * nloc) tab.assign((size_t)nloc * nloc, 0);
                for (int t = 0; t < nt; ++t) {
                    const Term& T = P.terms[t];
                    for (int32_t i = T.elem_ptr[p]; i < T.elem_ptr[p + 1]; ++i) {
                        const int32_t* st = &T.stencil[(int64_t)T.perm[i] * T.ns];
                        for (int a = 0; a < T.ns; ++a)
                            for (int b = a; b < T.ns; ++b) {
                                const int32_t la = loc[st[a]], lb = loc[st[b]];
                                const int32_t key = std::min(la, lb) * nloc + std::max(la, lb);
                                if (tab[key] == 0) {
                                    tab[key] = -1;
                                    keys.push_back(key);
                                }
                            }
                    }
                }
                std::sort(keys.begin(), keys.end());
                for (size_t k = 0; k < keys.size(); ++k) tab[keys[k]] = (int32_t)k + 1;
            } else {
                for (int t = 0; t < nt; ++t) {
                    const Term& T = P.terms[t];
                    for (int32_t i = T.elem_ptr[p]; i < T.elem_ptr[p + 1]; ++i) {
                        const int32_t* st = &T.stencil[(int64_t)T.perm[i] * T.ns];
                        for (int a = 0; a < T.ns; ++a)
                            for (int b = a; b < T.ns; ++b) {
                                const int64_t la = loc[st[a]], lb = loc[st[b]];
                                lkeys.push_back(std::min(la, lb) * nloc + std::max(la, lb));
                            }
                    }
                }
                std::sort(lkeys.begin(), lkeys.end());
                lkeys.erase(std::unique(lkeys.begin(), lkeys.end()), lkeys.end());
            }
            const size_t nkeys = dense ? keys.size() : lkeys.size();
            auto key_at = [&](size_t k) { return dense ? (int64_t)keys[k] : lkeys[k]; };
            if (nkeys > (1u << 14) || nloc > (1 << 16)) {
                err.fetch_or(1);
            } else {
                pv[p] = verts;
                // global indices of the patch's upper blocks and of their transposes
                pb_g[p].resize(nkeys);
                pb_gt[p].resize(nkeys);
                for (size_t k = 0; k < nkeys; ++k) {
                    const int64_t key = key_at(k);
                    const int32_t r = verts[(size_t)(key / nloc)], c = verts[(size_t)(key % nloc)];
                    pb_g[p][k] = find_block(rowptr, colidx, r, c);
                    pb_gt[p][k] = find_block(rowptr, colidx, c, r);
                    if (pb_g[p][k] < 0 || pb_gt[p][k] < 0) err.fetch_or(2);
                }
                for (int t = 0; t < nt; ++t) {
                    const Term& T = P.terms[t];
                    for (int32_t i = T.elem_ptr[p]; i < T.elem_ptr[p + 1]; ++i) {
                        const int32_t* st = &T.stencil[(int64_t)T.perm[i] * T.ns];
                        int k = 0;
                        for (int a = 0; a < T.ns; ++a) {
                            const int32_t la = loc[st[a]];
                            L.lvert[t][(size_t)a * T.n + i] = (uint16_t)la;
                            for (int b = a; b < T.ns; ++b, ++k) {
                                const int32_t lb = loc[st[b]];
                                const int64_t key = (int64_t)std::min(la, lb) * nloc + std::max(la, lb);
                                const uint32_t idx =
                                    dense ? (uint32_t)(tab[(size_t)key] - 1)
                                          : (uint32_t)(std::lower_bound(lkeys.begin(), lkeys.end(), key) - lkeys.begin());
                                uint32_t flag = 0;
                                if (a != b && st[a] == st[b]) flag = 2u;
                                else if (st[a] > st[b]) flag = 1u;
                                L.lslot[t][(size_t)k * T.n + i] = (uint16_t)(idx | (flag << 14));
                            }
                        }
                    }
                }
            }
            for (int32_t v : verts) loc[v] = -1;
            if (dense)
                for (int32_t key : keys) tab[key] = 0;
        }
    };
    const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int w = 0; w < nth; ++w) {
        const int32_t p0 = (int32_t)((int64_t)np * w / nth), p1 = (int32_t)((int64_t)np * (w + 1) / nth);
        th.emplace_back(work, p0, p1);
    }
    for (auto& x : th) x.join();
    if (err.load() & 2) return fail(MAD_E_HIP, "internal error: patch block missing from the pattern");
    if (err.load()) return fail(MAD_E_UNSUPPORTED, "a patch touches more than 16384 blocks; use smaller patches");

    // concatenate (threads over patch ranges) and count each entry's patches, for exclusivity
    L.lv_ptr.assign((size_t)np + 1, 0);
    L.lb_ptr.assign((size_t)np + 1, 0);
    for (int32_t p = 0; p < np; ++p) {
        L.lv_ptr[p + 1] = L.lv_ptr[p] + (int32_t)pv[p].size();
        L.lb_ptr[p + 1] = L.lb_ptr[p] + (int32_t)pb_g[p].size();
    }
    L.lv_global.resize((size_t)L.lv_ptr[np]);
    L.lv_halo.resize((size_t)L.lv_ptr[np]);
    L.lb_gidx.resize((size_t)L.lb_ptr[np]);
    L.lb_gidxT.resize((size_t)L.lb_ptr[np]);
    L.lb_halo.resize((size_t)L.lb_ptr[np]);
    std::vector<int32_t> vcount((size_t)nv, 0), bcount(colidx.size(), 0);
    {
        auto copy = [&](int32_t p0, int32_t p1) {
            for (int32_t p = p0; p < p1; ++p) {
                for (size_t k = 0; k < pv[p].size(); ++k) {
                    L.lv_global[L.lv_ptr[p] + k] = pv[p][k];
                    __atomic_fetch_add(&vcount[pv[p][k]], 1, __ATOMIC_RELAXED);
                }
                for (size_t k = 0; k < pb_g[p].size(); ++k) {
                    L.lb_gidx[L.lb_ptr[p] + k] = pb_g[p][k];
                    L.lb_gidxT[L.lb_ptr[p] + k] = pb_gt[p][k];
                    __atomic_fetch_add(&bcount[pb_g[p][k]], 1, __ATOMIC_RELAXED);
                }
                std::vector<int32_t>().swap(pv[p]);
                std::vector<int32_t>().swap(pb_g[p]);
                std::vector<int32_t>().swap(pb_gt[p]);
            }
        };
        std::vector<std::thread> cth;
        for (int w = 0; w < nth; ++w)
            cth.emplace_back(copy, (int32_t)((int64_t)np * w / nth), (int32_t)((int64_t)np * (w + 1) / nth));
        for (auto& x : cth) x.join();
    }
    // halo slots, assigned patch by patch (each patch writes its shared partials contiguously)
    int32_t nhv = 0, nhb = 0;
    for (size_t k = 0; k < L.lv_global.size(); ++k) L.lv_halo[k] = vcount[L.lv_global[k]] == 1 ? -1 : nhv++;
    for (size_t k = 0; k < L.lb_gidx.size(); ++k) L.lb_halo[k] = bcount[L.lb_gidx[k]] == 1 ? -1 : nhb++;
    // gather lists: every shared entry in ascending order with its halo slots in patch order (a counting
    // sort: entries numbered in ascending order, then the patch-ordered slots dealt out to them)
    {
        for (int64_t v = 0; v < nv; ++v)
            if (vcount[v] == 0) L.orphan_vert.push_back((int32_t)v);
        L.gv_ptr.assign(1, 0);
        for (int64_t v = 0; v < nv; ++v)
            if (vcount[v] > 1) {
                L.gv_vert.push_back((int32_t)v);
                L.gv_ptr.push_back(L.gv_ptr.back() + vcount[v]);
                vcount[v] = (int32_t)L.gv_vert.size() - 1;   // from here on: the vertex's gather entry
            }
        L.gv_src.resize((size_t)L.gv_ptr.back());
        std::vector<int32_t> fill(L.gv_vert.size(), 0);
        for (size_t k = 0; k < L.lv_global.size(); ++k)
            if (L.lv_halo[k] >= 0) {
                const int32_t e = vcount[L.lv_global[k]];
                L.gv_src[(size_t)L.gv_ptr[e] + fill[e]++] = L.lv_halo[k];
            }
        L.gb_ptr.assign(1, 0);
        for (size_t b = 0; b < bcount.size(); ++b)
            if (bcount[b] > 1) {
                L.gb_gidx.push_back((int32_t)b);
                L.gb_ptr.push_back(L.gb_ptr.back() + bcount[b]);
                bcount[b] = (int32_t)L.gb_gidx.size() - 1;   // from here on: the block's gather entry
            }
        L.gb_src.resize((size_t)L.gb_ptr.back());
        L.gb_gidxT.resize(L.gb_gidx.size());
        fill.assign(L.gb_gidx.size(), 0);
        for (size_t k = 0; k < L.lb_gidx.size(); ++k)
            if (L.lb_halo[k] >= 0) {
                const int32_t e = bcount[L.lb_gidx[k]];
                L.gb_src[(size_t)L.gb_ptr[e] + fill[e]++] = L.lb_halo[k];
                L.gb_gidxT[e] = L.lb_gidxT[k];
            }
        // blocks no patch writes: blocks (r, c) and (c, r) are both written through the upper one
        std::vector<uint8_t> covered(colidx.size(), 0);
        for (size_t k = 0; k < L.lb_gidx.size(); ++k) covered[L.lb_gidx[k]] = covered[L.lb_gidxT[k]] = 1;
        for (size_t b = 0; b < colidx.size(); ++b)
            if (!covered[b]) L.orphan_block.push_back((int32_t)b);
    }
    L.max_lv = 0;
    L.max_lb = 0;
    for (int32_t p = 0; p < np; ++p) {
        L.max_lv = std::max(L.max_lv, L.lv_ptr[p + 1] - L.lv_ptr[p]);
        L.max_lb = std::max(L.max_lb, L.lb_ptr[p + 1] - L.lb_ptr[p]);
    }
    return MAD_OK;
}

}  // namespace mad
