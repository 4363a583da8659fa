// Host steps of the evaluation layout that need no device: the patch order of every term's elements,
// the colour order inside patches, the largest patch's LDS working set and the segments of the patch
// kernel's work units. Threaded over patches; layout.cpp uploads the results.
#include <algorithm>
#include <functional>
#include <numeric>
#include <thread>

#include "mad_internal.hpp"

namespace mad {

// Inside each patch, greedy-colour the term's elements so that no two elements of a colour share a
// vertex, and store them colour by colour (stable), so that the elements a wave evaluates together
// rarely add into the same LDS accumulators.
void color_within_patches(Term& t, int64_t nv) {
    const int32_t np = (int32_t)t.elem_ptr.size() - 1;
    // patches are independent: split them over threads, each with its own vertex bit array
    auto work = [&](int32_t q0, int32_t q1) {
        std::vector<uint64_t> busy_at((size_t)nv, 0);
        std::vector<int32_t> color, order, seg;
        for (int32_t q = q0; q < q1; ++q) {
            const int32_t b = t.elem_ptr[q], e = t.elem_ptr[q + 1];
            if (e - b < 2) continue;
            color.assign((size_t)(e - b), 0);
            for (int32_t i = b; i < e; ++i) {
                const int32_t* st = &t.stencil[(int64_t)t.perm[i] * t.ns];
                uint64_t busy = 0;
                for (int a = 0; a < t.ns; ++a) busy |= busy_at[st[a]];
                int c = 0;
                while (c < 63 && ((busy >> c) & 1ull)) ++c;
                color[i - b] = c;
                for (int a = 0; a < t.ns; ++a) busy_at[st[a]] |= 1ull << c;
            }
            for (int32_t i = b; i < e; ++i) {
                const int32_t* st = &t.stencil[(int64_t)t.perm[i] * t.ns];
                for (int a = 0; a < t.ns; ++a) busy_at[st[a]] = 0;
            }
            order.resize((size_t)(e - b));
            std::iota(order.begin(), order.end(), 0);
            std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return color[x] < color[y]; });
            seg.assign(t.perm.begin() + b, t.perm.begin() + e);
            for (int32_t i = 0; i < e - b; ++i) t.perm[b + i] = seg[order[i]];
        }
    };
    const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int w = 1; w < nth; ++w)
        pool.emplace_back(work, (int32_t)((int64_t)np * w / nth), (int32_t)((int64_t)np * (w + 1) / nth));
    work(0, (int32_t)((int64_t)np / nth));
    for (auto& th : pool) th.join();
}

// Patch order of every term's elements: faces by their patch, diamonds by their lower face, edges
// by their first face, vertices by their lowest face; inside a patch by that face's index. Two
// stable counting sorts (by face, then by patch): linear in the element count. The colour order
// inside each patch (color_within_patches) is applied once the patches are final.
void order_terms(mad_problem* p) {
    const mad_mesh& m = *p->mesh;
    const int32_t np = p->patches.n;
    auto one = [&](Term& t) {
        std::vector<int32_t> key((size_t)t.n);
        for (int64_t e = 0; e < t.n; ++e) {
            if (t.kind == MAD_BENDING) key[e] = m.diamond_faces[2 * e];
            else if (t.kind == MAD_EDGE_SQLEN || t.kind == MAD_SPRING || t.kind == MAD_RES_EDGE) key[e] = m.edge_face0[e];
            else if (t.kind == MAD_INERTIA || t.kind == MAD_RES_POSITION) key[e] = m.vert_face0[t.stencil[e]];
            else key[e] = (int32_t)e;
        }
        // by face
        std::vector<int32_t> cnt((size_t)m.nt + 1, 0), byface((size_t)t.n);
        for (int64_t e = 0; e < t.n; ++e) cnt[key[e] + 1]++;
        for (int64_t f = 0; f < m.nt; ++f) cnt[f + 1] += cnt[f];
        for (int64_t e = 0; e < t.n; ++e) byface[cnt[key[e]]++] = (int32_t)e;
        // then by patch (stable)
        t.elem_ptr.assign((size_t)np + 1, 0);
        for (int64_t e = 0; e < t.n; ++e) t.elem_ptr[p->patches.face_patch[key[e]] + 1]++;
        for (int32_t q = 0; q < np; ++q) t.elem_ptr[q + 1] += t.elem_ptr[q];
        std::vector<int32_t> fill(t.elem_ptr.begin(), t.elem_ptr.end() - 1);
        t.perm.resize((size_t)t.n);
        for (int32_t e : byface) t.perm[fill[p->patches.face_patch[key[e]]]++] = e;
    };
    // terms are independent: one thread each
    std::vector<std::thread> pool;
    for (size_t i = 1; i < p->terms.size(); ++i) pool.emplace_back(one, std::ref(p->terms[i]));
    if (!p->terms.empty()) one(p->terms[0]);
    for (auto& th : pool) th.join();
}

// largest per-patch vertex and upper-block counts of the current patching (patches split over threads)
void patch_extent(const mad_problem* p, int32_t* max_lv, int32_t* max_lb) {
    const int64_t nv = p->mesh->nv;
    const int32_t np = p->patches.n;
    const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<int32_t> mv_t((size_t)nth, 0), mb_t((size_t)nth, 0);
    // Per patch: distinct vertices through a per-thread vertex map (first-seen local numbers), distinct upper
    // blocks through a dense table of local (row, column) pairs for patches of at most kDenseLocal vertices
    // (sorted keys beyond); both are reset after each patch, so a patch costs time in proportion to its elements.
    constexpr int32_t kDenseLocal = 1024;
    auto work = [&](int th) {
        std::vector<int32_t> loc((size_t)nv, -1), verts, marked;
        std::vector<uint8_t> tab;
        std::vector<int64_t> keys;
        int32_t mv = 0, mb = 0;
        for (int32_t q = th; q < np; q += nth) {
            verts.clear();
            for (const auto& t : p->terms)
                for (int32_t i = t.elem_ptr[q]; i < t.elem_ptr[q + 1]; ++i) {
                    const int32_t* st = &t.stencil[(int64_t)t.perm[i] * t.ns];
                    for (int a = 0; a < t.ns; ++a)
                        if (loc[st[a]] < 0) {
                            loc[st[a]] = (int32_t)verts.size();
                            verts.push_back(st[a]);
                        }
                }
            const int32_t nloc = (int32_t)verts.size();
            int32_t nblocks = 0;
            if (nloc <= kDenseLocal) {
                if (tab.size() < (size_t)nloc * nloc) tab.assign((size_t)nloc * nloc, 0);
                marked.clear();
                for (const auto& t : p->terms)
                    for (int32_t i = t.elem_ptr[q]; i < t.elem_ptr[q + 1]; ++i) {
                        const int32_t* st = &t.stencil[(int64_t)t.perm[i] * t.ns];
                        for (int a = 0; a < t.ns; ++a)
                            for (int b = a; b < t.ns; ++b) {
                                // a block is (min, max) of its global vertices; first-seen local numbers do
                                // not follow global order, so the pair is ordered by the global indices
                                const int32_t r = std::min(st[a], st[b]), c = std::max(st[a], st[b]);
                                const int32_t key = loc[r] * nloc + loc[c];
                                if (!tab[key]) {
                                    tab[key] = 1;
                                    marked.push_back(key);
                                }
                            }
                    }
                nblocks = (int32_t)marked.size();
                for (int32_t key : marked) tab[key] = 0;
            } else {
                keys.clear();
                for (const auto& t : p->terms)
                    for (int32_t i = t.elem_ptr[q]; i < t.elem_ptr[q + 1]; ++i) {
                        const int32_t* st = &t.stencil[(int64_t)t.perm[i] * t.ns];
                        for (int a = 0; a < t.ns; ++a)
                            for (int b = a; b < t.ns; ++b)
                                keys.push_back((int64_t)std::min(st[a], st[b]) * nv + std::max(st[a], st[b]));
                    }
                std::sort(keys.begin(), keys.end());
                nblocks = (int32_t)(std::unique(keys.begin(), keys.end()) - keys.begin());
            }
            for (int32_t v : verts) loc[v] = -1;
            mv = std::max(mv, nloc);
            mb = std::max(mb, nblocks);
        }
        mv_t[th] = mv;
        mb_t[th] = mb;
    };
    std::vector<std::thread> pool;
    for (int th = 1; th < nth; ++th) pool.emplace_back(work, th);
    work(0);
    for (auto& th : pool) th.join();
    *max_lv = *std::max_element(mv_t.begin(), mv_t.end());
    *max_lb = *std::max_element(mb_t.begin(), mb_t.end());
}

// Segments of the patch kernel's work units (the 64 consecutive elements of one term in one patch
// that one wave evaluates together): inside a unit, greedily, each element takes the lowest segment
// in which no earlier element of the unit shares a vertex with it. Elements of one segment touch
// disjoint gradient entries and Hessian blocks, so a wave can add a segment's contributions with
// plain LDS read-add-writes. The colour order inside each patch keeps most units at one or two
// segments.
void unit_segments(const Term& t, int32_t np, int64_t nv, std::vector<uint8_t>& seg) {
    seg.assign((size_t)std::max<int64_t>(t.n, 1), 0);
    // units are independent: patches split over threads, each with its own vertex bit array
    auto work = [&](int32_t q0, int32_t q1) {
        std::vector<uint64_t> used((size_t)nv, 0);   // segments of the current unit using the vertex
        for (int32_t q = q0; q < q1; ++q)
            for (int32_t u0 = t.elem_ptr[q]; u0 < t.elem_ptr[q + 1]; u0 += 64) {
                const int32_t u1 = std::min(u0 + 64, t.elem_ptr[q + 1]);
                for (int32_t i = u0; i < u1; ++i) {
                    const int32_t* st = &t.stencil[(int64_t)t.perm[i] * t.ns];
                    uint64_t busy = 0;
                    for (int a = 0; a < t.ns; ++a) busy |= used[st[a]];
                    int sg = 0;
                    while ((busy >> sg) & 1ull) ++sg;   // at most 63: a unit has 64 elements
                    seg[i] = (uint8_t)sg;
                    for (int a = 0; a < t.ns; ++a) used[st[a]] |= 1ull << sg;
                }
                for (int32_t i = u0; i < u1; ++i) {
                    const int32_t* st = &t.stencil[(int64_t)t.perm[i] * t.ns];
                    for (int a = 0; a < t.ns; ++a) used[st[a]] = 0;
                }
            }
    };
    const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int w = 1; w < nth; ++w)
        pool.emplace_back(work, (int32_t)((int64_t)np * w / nth), (int32_t)((int64_t)np * (w + 1) / nth));
    work(0, (int32_t)((int64_t)np / nth));
    for (auto& th : pool) th.join();
}

// Colored scatter (the coloring alternative of Sec. 5.5). Each term's elements are colored greedily in
// their current (patch) order: an element takes the lowest color that no earlier element sharing one of its
// vertices holds (per-vertex bit sets of used colors, widened when a color beyond them is needed), so no two
// elements of a color share a vertex and so no gradient entry or Hessian block. The elements are then
// sorted by (color, component), keeping the patch order inside, and cut into chunks of at most kColorChunk
// elements of one color and one component: a launch per color covers that color's chunks. Each chunk's
// energy goes to a slot; slots are numbered by component, then term, color and chunk, so the energy
// reduction sums each component's slots as one contiguous range, always in the same order.
void color_order(mad_problem* p, std::vector<int32_t>& comp_slot_ptr) {
    const mad_mesh& m = *p->mesh;
    const int64_t nv = m.nv;
    const int ncomp = (int)std::max<size_t>(m.comp_off.size(), 2) - 1;
    auto comp_of = [&](int32_t v) -> int32_t {
        if (ncomp == 1) return 0;
        return (int32_t)(std::upper_bound(m.comp_off.begin(), m.comp_off.end(), (int64_t)v) - m.comp_off.begin() - 1);
    };
    const int nt = (int)p->terms.size();
    std::vector<std::vector<int32_t>> chunk_comp((size_t)nt);
    for (int ti = 0; ti < nt; ++ti) {
        Term& t = p->terms[ti];
        const int64_t n = t.n;
        std::vector<int32_t> color((size_t)std::max<int64_t>(n, 1), 0);
        int words = 1;
        std::vector<uint64_t> used((size_t)nv * words, 0);
        int32_t n_colors = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int32_t* st = &t.stencil[(int64_t)t.perm[i] * t.ns];
            int c = -1;
            for (int w = 0; w < words && c < 0; ++w) {
                uint64_t busy = 0;
                for (int a = 0; a < t.ns; ++a) busy |= used[(size_t)st[a] * words + w];
                if (~busy != 0ull) c = 64 * w + __builtin_ctzll(~busy);
            }
            if (c < 0) {
                // every color in the sets is taken around this element: widen the sets by one word
                std::vector<uint64_t> wider((size_t)nv * (words + 1), 0);
                for (int64_t v = 0; v < nv; ++v)
                    for (int w = 0; w < words; ++w) wider[(size_t)v * (words + 1) + w] = used[(size_t)v * words + w];
                used.swap(wider);
                c = 64 * words;
                ++words;
            }
            color[(size_t)i] = c;
            n_colors = std::max(n_colors, c + 1);
            for (int a = 0; a < t.ns; ++a) used[(size_t)st[a] * words + c / 64] |= 1ull << (c % 64);
        }
        // stable counting sort by (color, component)
        const int64_t nkeys = (int64_t)n_colors * ncomp;
        std::vector<int64_t> cnt((size_t)nkeys + 1, 0);
        std::vector<int32_t> key((size_t)std::max<int64_t>(n, 1));
        for (int64_t i = 0; i < n; ++i) {
            key[(size_t)i] = color[(size_t)i] * ncomp + comp_of(t.stencil[(int64_t)t.perm[i] * t.ns]);
            cnt[(size_t)key[(size_t)i] + 1]++;
        }
        for (int64_t k = 0; k < nkeys; ++k) cnt[(size_t)k + 1] += cnt[(size_t)k];
        std::vector<int32_t> perm((size_t)n);
        {
            std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
            for (int64_t i = 0; i < n; ++i) perm[(size_t)fill[(size_t)key[(size_t)i]]++] = t.perm[i];
        }
        t.perm.swap(perm);
        // chunks: runs of at most kColorChunk elements inside one (color, component) group
        t.elem_ptr.assign(1, 0);
        t.color_chunk_ptr.assign((size_t)n_colors + 1, 0);
        chunk_comp[ti].clear();
        for (int32_t c = 0; c < n_colors; ++c) {
            t.color_chunk_ptr[c] = (int32_t)chunk_comp[ti].size();
            for (int q = 0; q < ncomp; ++q) {
                const int64_t b = cnt[(size_t)c * ncomp + q], e = cnt[(size_t)c * ncomp + q + 1];
                for (int64_t s0 = b; s0 < e; s0 += kColorChunk) {
                    t.elem_ptr.push_back((int32_t)std::min<int64_t>(e, s0 + kColorChunk));
                    chunk_comp[ti].push_back(q);
                }
            }
        }
        t.color_chunk_ptr[n_colors] = (int32_t)chunk_comp[ti].size();
    }
    // energy slots: by component, then term, then chunk (chunks are in color order within a term)
    comp_slot_ptr.assign((size_t)ncomp + 1, 0);
    for (int ti = 0; ti < nt; ++ti)
        for (int32_t q : chunk_comp[ti]) comp_slot_ptr[(size_t)q + 1]++;
    for (int q = 0; q < ncomp; ++q) comp_slot_ptr[(size_t)q + 1] += comp_slot_ptr[(size_t)q];
    std::vector<int32_t> next(comp_slot_ptr.begin(), comp_slot_ptr.end() - 1);
    for (int ti = 0; ti < nt; ++ti) {
        Term& t = p->terms[ti];
        t.slot_map.resize(chunk_comp[ti].size());
        for (size_t k = 0; k < chunk_comp[ti].size(); ++k) t.slot_map[k] = next[(size_t)chunk_comp[ti][k]]++;
    }
    p->n_color_slots = comp_slot_ptr[(size_t)ncomp];
}

}  // namespace mad
