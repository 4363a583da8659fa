// Sanitizer harness of the library's host runtime (built with g++ under AddressSanitizer +
// UndefinedBehaviorSanitizer and, separately, ThreadSanitizer by tests/test_sanitize.py): mesh topology,
// patching, the patch order and colour order of the elements, the LDS working-set count, the work-unit
// segments and the patch-local index structures of the LDS assembly, on generated meshes (grids,
// disjoint components, a high-valence fan, non-manifold edges). Beyond running them clean, it checks
// the structural invariants the patch kernel relies on, and exits non-zero on the first violation.
// Test infrastructure: not part of the library.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <string>
#include <vector>

#include "mad_internal.hpp"

namespace mad {
// the library's error reporting lives with the C ABI (api.cpp), which this harness does not link
static std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}
}  // namespace mad

using namespace mad;

#define CHECK(cond)                                                                 \
    do {                                                                            \
        if (!(cond)) {                                                              \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            std::exit(2);                                                           \
        }                                                                           \
    } while (0)

struct MeshIn {
    std::string name;
    int64_t nv = 0;
    std::vector<int32_t> tris;
    std::vector<int64_t> comp;   // empty: one component
};

static void add_grid(MeshIn& m, int n) {
    const int32_t base = (int32_t)m.nv;
    for (int j = 0; j + 1 < n; ++j)
        for (int i = 0; i + 1 < n; ++i) {
            const int32_t v00 = base + j * n + i, v10 = v00 + 1, v01 = v00 + n, v11 = v01 + 1;
            m.tris.insert(m.tris.end(), {v00, v10, v11, v00, v11, v01});
        }
    m.nv += (int64_t)n * n;
}

static std::vector<MeshIn> meshes() {
    std::vector<MeshIn> out;
    {
        MeshIn m{"grid 48x48"};
        add_grid(m, 48);
        out.push_back(m);
    }
    {
        MeshIn m{"5 components"};
        m.comp.push_back(0);
        for (int n : {7, 12, 5, 20, 9}) {
            add_grid(m, n);
            m.comp.push_back(m.nv);
        }
        out.push_back(m);
    }
    {
        // a closed fan: centre 0, rim 1..k, plus a cap vertex k+1 (valence k at both poles)
        MeshIn m{"fan of valence 300"};
        const int k = 300;
        for (int i = 0; i < k; ++i) {
            const int32_t a = 1 + i, b = 1 + (i + 1) % k;
            m.tris.insert(m.tris.end(), {0, a, b, k + 1, b, a});
        }
        m.nv = k + 2;
        out.push_back(m);
    }
    {
        // three faces on one edge (non-manifold), an isolated vertex, a boundary strip
        MeshIn m{"non-manifold"};
        m.tris = {0, 1, 2, 1, 0, 3, 0, 1, 4, 2, 1, 5, 5, 1, 6};
        m.nv = 8;
        out.push_back(m);
    }
    return out;
}

static void check_problem(const MeshIn& in, int target) {
    mad_mesh mesh;
    mesh.nv = in.nv;
    mesh.nt = (int64_t)in.tris.size() / 3;
    mesh.tris = in.tris;
    if (in.comp.empty()) {
        mesh.comp_off = {0, in.nv};
    } else {
        mesh.comp_off = in.comp;
        mesh.batched = true;
    }
    CHECK(build_topology(mesh) == MAD_OK);
    mad_problem P;
    P.mesh = &mesh;
    P.d = 3;
    P.prec = MAD_F32;
    auto add = [&](int kind, const int32_t* st, int64_t n) {
        Term t;
        t.kind = kind;
        t.ns = kind_stencil(kind);
        t.d = 3;
        t.n = n;
        t.stencil.assign(st, st + n * t.ns);
        P.terms.push_back(std::move(t));
    };
    add(MAD_STVK, mesh.tris.data(), mesh.nt);
    add(MAD_BENDING, mesh.diamonds.data(), mesh.nd());
    add(MAD_SPRING, mesh.edges.data(), mesh.ne());
    std::vector<int32_t> verts;
    for (int64_t v = 0; v < mesh.nv; ++v)
        if (mesh.vert_face0[v] >= 0) verts.push_back((int32_t)v);
    add(MAD_INERTIA, verts.data(), (int64_t)verts.size());

    build_patches(mesh, target, P.patches);
    const int32_t np = P.patches.n;
    CHECK(np >= 1);
    for (int64_t f = 0; f < mesh.nt; ++f) CHECK(P.patches.face_patch[f] >= 0 && P.patches.face_patch[f] < np);
    order_terms(&P);
    int32_t mv = 0, mb = 0;
    patch_extent(&P, &mv, &mb);
    for (auto& t : P.terms) color_within_patches(t, mesh.nv);
    // every element exactly once, in its patch's range
    for (const Term& t : P.terms) {
        CHECK((int32_t)t.elem_ptr.size() == np + 1 && t.elem_ptr[np] == t.n);
        std::vector<int32_t> seen(t.perm.begin(), t.perm.end());
        std::sort(seen.begin(), seen.end());
        for (int64_t i = 0; i < t.n; ++i) CHECK(seen[i] == i);
    }
    // pattern by brute force: the diagonal plus every stencil pair
    std::vector<std::set<int32_t>> rows((size_t)mesh.nv);
    for (int64_t v = 0; v < mesh.nv; ++v) rows[v].insert((int32_t)v);
    for (const Term& t : P.terms)
        for (int64_t e = 0; e < t.n; ++e)
            for (int a = 0; a < t.ns; ++a)
                for (int b = 0; b < t.ns; ++b) rows[t.stencil[e * t.ns + a]].insert(t.stencil[e * t.ns + b]);
    std::vector<int32_t> rowptr(1, 0), colidx;
    for (auto& r : rows) {
        colidx.insert(colidx.end(), r.begin(), r.end());
        rowptr.push_back((int32_t)colidx.size());
    }
    PatchLocal L;
    CHECK(build_patch_local(P, rowptr, colidx, L) == MAD_OK);
    CHECK(L.max_lv == mv && L.max_lb == mb);
    // patch-local maps point back at the stencil and the right blocks
    for (size_t ti = 0; ti < P.terms.size(); ++ti) {
        const Term& t = P.terms[ti];
        std::vector<uint8_t> seg;
        unit_segments(t, np, mesh.nv, seg);
        for (int32_t p = 0; p < np; ++p) {
            const int32_t lv0 = L.lv_ptr[p], lb0 = L.lb_ptr[p];
            for (int32_t i = t.elem_ptr[p]; i < t.elem_ptr[p + 1]; ++i) {
                const int32_t* st = &t.stencil[(int64_t)t.perm[i] * t.ns];
                int k = 0;
                for (int a = 0; a < t.ns; ++a) {
                    const int lv = L.lvert[ti][(size_t)a * t.n + i];
                    CHECK(lv0 + lv < L.lv_ptr[p + 1] && L.lv_global[lv0 + lv] == st[a]);
                    for (int b = a; b < t.ns; ++b, ++k) {
                        const uint16_t w = L.lslot[ti][(size_t)k * t.n + i];
                        const int lb = w & 0x3fff;
                        CHECK(lb0 + lb < L.lb_ptr[p + 1]);
                        const int32_t r = std::min(st[a], st[b]), c = std::max(st[a], st[b]);
                        const int32_t g = L.lb_gidx[lb0 + lb];
                        CHECK(colidx[g] == c && g >= rowptr[r] && g < rowptr[r + 1]);
                    }
                }
            }
            // elements of one segment inside a 64-element unit share no vertex
            for (int32_t u0 = t.elem_ptr[p]; u0 < t.elem_ptr[p + 1]; u0 += 64) {
                const int32_t u1 = std::min(u0 + 64, t.elem_ptr[p + 1]);
                for (int32_t i = u0; i < u1; ++i)
                    for (int32_t j = i + 1; j < u1; ++j) {
                        if (seg[i] != seg[j]) continue;
                        const int32_t* si = &t.stencil[(int64_t)t.perm[i] * t.ns];
                        const int32_t* sj = &t.stencil[(int64_t)t.perm[j] * t.ns];
                        for (int a = 0; a < t.ns; ++a)
                            for (int b = 0; b < t.ns; ++b) CHECK(si[a] != sj[b]);
                    }
            }
        }
    }
    // colored scatter: each color's elements share no vertex, chunks hold one color and one component, and the
    // energy slots number every chunk once, each component's slots contiguous
    {
        std::vector<int32_t> comp_slot_ptr;
        color_order(&P, comp_slot_ptr);
        const int ncomp = (int)mesh.comp_off.size() - 1;
        auto comp_of = [&](int32_t v) {
            return (int)(std::upper_bound(mesh.comp_off.begin(), mesh.comp_off.end(), (int64_t)v) -
                         mesh.comp_off.begin() - 1);
        };
        CHECK((int)comp_slot_ptr.size() == ncomp + 1 && comp_slot_ptr[ncomp] == P.n_color_slots);
        std::vector<int32_t> slot_uses((size_t)P.n_color_slots, 0);
        for (const Term& t : P.terms) {
            std::vector<int32_t> seen(t.perm.begin(), t.perm.end());
            std::sort(seen.begin(), seen.end());
            for (int64_t i = 0; i < t.n; ++i) CHECK(seen[i] == i);
            const int ncol = (int)t.color_chunk_ptr.size() - 1;
            std::vector<int32_t> stamp((size_t)mesh.nv, -1);
            for (int c = 0; c < ncol; ++c) {
                for (int32_t k = t.color_chunk_ptr[c]; k < t.color_chunk_ptr[c + 1]; ++k) {
                    const int q = comp_of(t.stencil[(int64_t)t.perm[t.elem_ptr[k]] * t.ns]);
                    const int32_t slot = t.slot_map[k];
                    CHECK(slot >= comp_slot_ptr[q] && slot < comp_slot_ptr[q + 1]);
                    slot_uses[slot]++;
                    CHECK(t.elem_ptr[k + 1] - t.elem_ptr[k] <= kColorChunk && t.elem_ptr[k + 1] > t.elem_ptr[k]);
                    for (int32_t i = t.elem_ptr[k]; i < t.elem_ptr[k + 1]; ++i) {
                        const int32_t* st = &t.stencil[(int64_t)t.perm[i] * t.ns];
                        CHECK(comp_of(st[0]) == q);
                        for (int a = 0; a < t.ns; ++a) {
                            // a vertex appears at most once per color (an element may not repeat a vertex either)
                            CHECK(stamp[st[a]] != c);
                            stamp[st[a]] = c;
                        }
                    }
                }
            }
            CHECK(t.elem_ptr.back() == t.n);
        }
        for (int32_t u : slot_uses) CHECK(u == 1);
        std::printf("  colored: %lld energy slots; colors per term:", (long long)P.n_color_slots);
        for (const Term& t : P.terms) std::printf(" %zu", t.color_chunk_ptr.size() - 1);
        std::printf("\n");
    }
    // every shared vertex is gathered from at least two halo slots, every slot exactly once
    std::vector<int32_t> slot_uses(L.gv_src.size(), 0);
    for (size_t v = 0; v + 1 < L.gv_ptr.size(); ++v) {
        CHECK(L.gv_ptr[v + 1] - L.gv_ptr[v] >= 2);
        for (int32_t j = L.gv_ptr[v]; j < L.gv_ptr[v + 1]; ++j) slot_uses[L.gv_src[j]]++;
    }
    for (int32_t u : slot_uses) CHECK(u == 1);
    std::printf("%s, patch target %d: %d patches, max %d vertices / %d blocks per patch, %zu shared vertices, "
                "%zu shared blocks\n",
                in.name.c_str(), target, np, mv, mb, L.gv_vert.size(), L.gb_gidx.size());
}

int main() {
    for (const MeshIn& m : meshes())
        for (int target : {1, 7, 64, 384, 3000}) check_problem(m, target);
    std::printf("host runtime checks passed\n");
    return 0;
}
