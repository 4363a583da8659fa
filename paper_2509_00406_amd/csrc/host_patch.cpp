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
    auto work = [&](int32_t p0, int32_t p1) {
        std::vector<int32_t> verts;
        std::vector<int64_t> keys;
        for (int32_t p = p0; p < p1; ++p) {
            verts.clear();
            keys.clear();
            for (int t = 0; t < nt; ++t) {
                const Term& T = P.terms[t];
                for (int32_t i = T.elem_ptr[p]; i < T.elem_ptr[p + 1]; ++i) {
                    const int32_t* st = &T.stencil[(int64_t)T.perm[i] * T.ns];
                    for (int a = 0; a < T.ns; ++a) {
                        verts.push_back(st[a]);
                        for (int b = a; b < T.ns; ++b) {
                            const int64_t r = std::min(st[a], st[b]), c = std::max(st[a], st[b]);
                            keys.push_back(r * nv + c);
                        }
                    }
                }
            }
            std::sort(verts.begin(), verts.end());
            verts.erase(std::unique(verts.begin(), verts.end()), verts.end());
            std::sort(keys.begin(), keys.end());
            keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
            if (keys.size() > (1u << 14) || verts.size() > (1u << 16)) {
                err.fetch_or(1);
                continue;
            }
            pv[p] = verts;
            // global indices of the patch's upper blocks and of their transposes
            pb_g[p].resize(keys.size());
            pb_gt[p].resize(keys.size());
            for (size_t k = 0; k < keys.size(); ++k) {
                const int32_t r = (int32_t)(keys[k] / nv), c = (int32_t)(keys[k] % nv);
                pb_g[p][k] = find_block(rowptr, colidx, r, c);
                pb_gt[p][k] = find_block(rowptr, colidx, c, r);
                if (pb_g[p][k] < 0 || pb_gt[p][k] < 0) err.fetch_or(2);
            }
            for (int t = 0; t < nt; ++t) {
                const Term& T = P.terms[t];
                const int npair = T.ns * (T.ns + 1) / 2;
                for (int32_t i = T.elem_ptr[p]; i < T.elem_ptr[p + 1]; ++i) {
                    const int32_t* st = &T.stencil[(int64_t)T.perm[i] * T.ns];
                    int k = 0;
                    for (int a = 0; a < T.ns; ++a) {
                        L.lvert[t][(size_t)a * T.n + i] =
                            (uint16_t)(std::lower_bound(verts.begin(), verts.end(), st[a]) - verts.begin());
                        for (int b = a; b < T.ns; ++b, ++k) {
                            const int64_t r = std::min(st[a], st[b]), c = std::max(st[a], st[b]);
                            const uint32_t idx =
                                (uint32_t)(std::lower_bound(keys.begin(), keys.end(), r * nv + c) - keys.begin());
                            uint32_t flag = 0;
                            if (a != b && st[a] == st[b]) flag = 2u;
                            else if (st[a] > st[b]) flag = 1u;
                            L.lslot[t][(size_t)k * T.n + i] = (uint16_t)(idx | (flag << 14));
                        }
                    }
                    (void)npair;
                }
            }
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

    // concatenate, resolve global block indices, count patch occurrences for exclusivity
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
    for (int32_t p = 0; p < np; ++p) {
        for (size_t k = 0; k < pv[p].size(); ++k) {
            L.lv_global[L.lv_ptr[p] + k] = pv[p][k];
            vcount[pv[p][k]]++;
        }
        for (size_t k = 0; k < pb_g[p].size(); ++k) {
            L.lb_gidx[L.lb_ptr[p] + k] = pb_g[p][k];
            L.lb_gidxT[L.lb_ptr[p] + k] = pb_gt[p][k];
            bcount[pb_g[p][k]]++;
        }
    }
    // halo slots, assigned patch by patch (each patch writes its shared partials contiguously)
    int32_t nhv = 0, nhb = 0;
    for (size_t k = 0; k < L.lv_global.size(); ++k) L.lv_halo[k] = vcount[L.lv_global[k]] == 1 ? -1 : nhv++;
    for (size_t k = 0; k < L.lb_gidx.size(); ++k) L.lb_halo[k] = bcount[L.lb_gidx[k]] == 1 ? -1 : nhb++;
    // gather lists: for every shared entry its halo slots, in patch order
    {
        std::vector<int32_t> first((size_t)nv, -1);
        std::vector<std::pair<int32_t, int32_t>> vs;   // (vertex, slot)
        for (size_t k = 0; k < L.lv_global.size(); ++k)
            if (L.lv_halo[k] >= 0) vs.push_back({L.lv_global[k], L.lv_halo[k]});
        std::stable_sort(vs.begin(), vs.end(), [](auto& a, auto& b) { return a.first < b.first; });
        L.gv_ptr.assign(1, 0);
        for (size_t i = 0; i < vs.size();) {
            size_t j = i;
            while (j < vs.size() && vs[j].first == vs[i].first) L.gv_src.push_back(vs[j++].second);
            L.gv_vert.push_back(vs[i].first);
            L.gv_ptr.push_back((int32_t)L.gv_src.size());
            i = j;
        }
        std::vector<std::array<int32_t, 3>> bs;         // (block, transposed block, slot)
        for (size_t k = 0; k < L.lb_gidx.size(); ++k)
            if (L.lb_halo[k] >= 0) bs.push_back({L.lb_gidx[k], L.lb_gidxT[k], L.lb_halo[k]});
        std::stable_sort(bs.begin(), bs.end(), [](auto& a, auto& b) { return a[0] < b[0]; });
        L.gb_ptr.assign(1, 0);
        for (size_t i = 0; i < bs.size();) {
            size_t j = i;
            while (j < bs.size() && bs[j][0] == bs[i][0]) L.gb_src.push_back(bs[j++][2]);
            L.gb_gidx.push_back(bs[i][0]);
            L.gb_gidxT.push_back(bs[i][1]);
            L.gb_ptr.push_back((int32_t)L.gb_src.size());
            i = j;
        }
        for (int64_t v = 0; v < nv; ++v)
            if (vcount[v] == 0) L.orphan_vert.push_back((int32_t)v);
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
