// Host-side setup, run once per mesh / problem (timings of the paper exclude
// it, Sec. 7): edge topology and edge diamonds, rest-frame data of each
// term, and the locality-ordered patches that element arrays are laid out by.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <numeric>
#include <thread>

#include "mad_internal.hpp"

namespace mad {

int kind_stencil(int kind) {
    switch (kind) {
    case MAD_INERTIA: case MAD_RES_POSITION: return 1;
    case MAD_EDGE_SQLEN: case MAD_SPRING: case MAD_RES_EDGE: return 2;
    case MAD_TRI_AREA: case MAD_DIRICHLET: case MAD_STVK: case MAD_SYMDIR: case MAD_MLP: case MAD_SHELL_TRI: return 3;
    case MAD_BENDING: return 4;
    default: return -1;
    }
}
int kind_vardim(int kind) {
    switch (kind) {
    case MAD_DIRICHLET: return 1;
    case MAD_SYMDIR: return 2;
    case MAD_EDGE_SQLEN: case MAD_TRI_AREA: case MAD_STVK: case MAD_BENDING: case MAD_MLP: case MAD_SHELL_TRI:
    case MAD_SPRING: case MAD_INERTIA: case MAD_RES_POSITION: case MAD_RES_EDGE: return 3;
    default: return -1;
    }
}
int kind_nres(int kind) {
    switch (kind) {
    case MAD_RES_POSITION: return 3;
    case MAD_RES_EDGE: return 1;
    default: return 0;
    }
}
int kind_nrest(int kind) {
    switch (kind) {
    case MAD_DIRICHLET: case MAD_STVK: case MAD_SYMDIR: return 5;
    case MAD_BENDING: case MAD_SPRING: return 2;
    case MAD_RES_EDGE: return 1;
    case MAD_MLP: case MAD_SHELL_TRI: return 8;
    default: return 0;
    }
}

// Edges sorted by (min, max) vertex; per edge the incident faces in ascending order.
// An edge with exactly two incident faces yields a diamond (v0, v1, v2, v3): (v0, v1) as the
// edge is directed in the lower-indexed face f1, v2 opposite in f1, v3 opposite in f2.
int build_topology(mad_mesh& m) {
    // edge-sides as corner ids c = 3 f + k: the side from tris[c] to the next corner of face f,
    // opposite the remaining corner. Every step is split over threads; the results do not depend on
    // their number.
    const int64_t nr = 3 * m.nt, nv = m.nv;
    const int32_t* T = m.tris.data();
    auto to = [&](int64_t c) { return T[c - c % 3 + (c % 3 + 1) % 3]; };
    auto opp = [&](int64_t c) { return T[c - c % 3 + (c % 3 + 2) % 3]; };
    const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto parallel = [&](int64_t n, auto&& fn) {   // fn(i0, i1) over nth contiguous ranges of [0, n)
        std::vector<std::thread> pool;
        for (int w = 1; w < nth; ++w) pool.emplace_back(fn, n * w / nth, n * (w + 1) / nth);
        fn((int64_t)0, n / nth);
        for (auto& th : pool) th.join();
    };
    // each side's (lo, hi) vertex pair, and the sides bucketed by lo
    std::vector<int32_t> side_lo((size_t)nr), side_hi((size_t)nr), cnt((size_t)nv + 1, 0);
    parallel(nr, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c) {
            const int32_t a = T[c], b = to(c);
            side_lo[c] = std::min(a, b);
            side_hi[c] = std::max(a, b);
            __atomic_fetch_add(&cnt[(size_t)side_lo[c] + 1], 1, __ATOMIC_RELAXED);
        }
    });
    std::vector<int64_t> start((size_t)nv + 1, 0);
    for (int64_t v = 0; v < nv; ++v) start[v + 1] = start[v] + cnt[v + 1];
    std::vector<int64_t> cursor(start.begin(), start.end() - 1);
    std::vector<int32_t> rec((size_t)nr);
    parallel(nr, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c)
            rec[(size_t)__atomic_fetch_add(&cursor[side_lo[c]], 1, __ATOMIC_RELAXED)] = (int32_t)c;
    });
    // inside each bucket by (hi, side): an insertion sort (a vertex's bucket holds a handful of sides);
    // then per vertex the count of its edges (runs of equal hi), diamonds (runs of two) and face links
    std::vector<int64_t> ne_v((size_t)nv + 1, 0), nd_v((size_t)nv + 1, 0), nl_v((size_t)nv + 1, 0);
    parallel(nv, [&](int64_t v0, int64_t v1) {
        for (int64_t v = v0; v < v1; ++v) {
            const int64_t b = start[v], e = start[v + 1];
            for (int64_t a = b + 1; a < e; ++a) {
                const int32_t x = rec[(size_t)a];
                const int32_t hx = side_hi[x];
                int64_t k = a;
                while (k > b && (side_hi[rec[(size_t)k - 1]] > hx || (side_hi[rec[(size_t)k - 1]] == hx && rec[(size_t)k - 1] > x))) {
                    rec[(size_t)k] = rec[(size_t)k - 1];
                    --k;
                }
                rec[(size_t)k] = x;
            }
            int64_t ne = 0, nd = 0, nl = 0;
            for (int64_t i = b; i < e;) {
                int64_t j = i;
                while (j < e && side_hi[rec[(size_t)j]] == side_hi[rec[(size_t)i]]) ++j;
                ++ne;
                if (j - i == 2) ++nd;
                for (int64_t a = i; a < j; ++a)
                    for (int64_t c = a + 1; c < j; ++c)
                        if (rec[(size_t)a] / 3 != rec[(size_t)c] / 3) ++nl;
                i = j;
            }
            ne_v[v + 1] = ne;
            nd_v[v + 1] = nd;
            nl_v[v + 1] = nl;
        }
    });
    for (int64_t v = 0; v < nv; ++v) {
        ne_v[v + 1] += ne_v[v];
        nd_v[v + 1] += nd_v[v];
        nl_v[v + 1] += nl_v[v];
    }
    const int64_t ne = ne_v[nv], nd = nd_v[nv], nl = nl_v[nv];
    m.edges.assign((size_t)ne * 2, 0);
    m.edge_nf.assign((size_t)ne, 0);
    m.edge_face0.assign((size_t)ne, 0);
    m.diamonds.assign((size_t)nd * 4, 0);
    m.diamond_faces.assign((size_t)nd * 2, 0);
    std::vector<int32_t> links((size_t)nl * 2);
    // edges sorted by (lo, hi); per edge its sides in ascending face order: the first face is the lowest. An
    // edge with exactly two sides is a diamond, directed as in its lower face
    parallel(nv, [&](int64_t v0, int64_t v1) {
        for (int64_t v = v0; v < v1; ++v) {
            int64_t oe = ne_v[v], od = nd_v[v], ol = nl_v[v];
            const int64_t b = start[v], e = start[v + 1];
            for (int64_t i = b; i < e;) {
                const int32_t ci = rec[(size_t)i];
                int64_t j = i;
                while (j < e && side_hi[rec[(size_t)j]] == side_hi[ci]) ++j;
                m.edges[2 * oe] = (int32_t)v;
                m.edges[2 * oe + 1] = side_hi[ci];
                m.edge_nf[oe] = (int32_t)(j - i);
                m.edge_face0[oe] = ci / 3;
                ++oe;
                if (j - i == 2) {
                    const int32_t cj = rec[(size_t)i + 1];
                    m.diamonds[4 * od] = T[ci];
                    m.diamonds[4 * od + 1] = to(ci);
                    m.diamonds[4 * od + 2] = opp(ci);
                    m.diamonds[4 * od + 3] = opp(cj);
                    m.diamond_faces[2 * od] = ci / 3;
                    m.diamond_faces[2 * od + 1] = cj / 3;
                    ++od;
                }
                for (int64_t a = i; a < j; ++a)
                    for (int64_t c = a + 1; c < j; ++c)
                        if (rec[(size_t)a] / 3 != rec[(size_t)c] / 3) {
                            links[2 * ol] = rec[(size_t)a] / 3;
                            links[2 * ol + 1] = rec[(size_t)c] / 3;
                            ++ol;
                        }
                i = j;
            }
        }
    });
    // face adjacency CSR (rows sorted)
    std::vector<int32_t> deg((size_t)m.nt, 0);
    parallel(nl, [&](int64_t l0, int64_t l1) {
        for (int64_t l = l0; l < l1; ++l) {
            __atomic_fetch_add(&deg[links[2 * l]], 1, __ATOMIC_RELAXED);
            __atomic_fetch_add(&deg[links[2 * l + 1]], 1, __ATOMIC_RELAXED);
        }
    });
    m.fadj_ptr.assign((size_t)m.nt + 1, 0);
    for (int64_t f = 0; f < m.nt; ++f) m.fadj_ptr[f + 1] = m.fadj_ptr[f] + deg[f];
    m.fadj.assign((size_t)m.fadj_ptr[m.nt], 0);
    std::vector<int32_t> cur(m.fadj_ptr.begin(), m.fadj_ptr.end() - 1);
    parallel(nl, [&](int64_t l0, int64_t l1) {
        for (int64_t l = l0; l < l1; ++l) {
            const int32_t f = links[2 * l], g = links[2 * l + 1];
            m.fadj[__atomic_fetch_add(&cur[f], 1, __ATOMIC_RELAXED)] = g;
            m.fadj[__atomic_fetch_add(&cur[g], 1, __ATOMIC_RELAXED)] = f;
        }
    });
    parallel(m.nt, [&](int64_t f0, int64_t f1) {
        for (int64_t f = f0; f < f1; ++f) std::sort(m.fadj.begin() + m.fadj_ptr[f], m.fadj.begin() + m.fadj_ptr[f + 1]);
    });
    // lowest face of every vertex (places a vertex term's element in that face's patch)
    m.vert_face0.assign((size_t)m.nv, -1);
    for (int64_t f = m.nt - 1; f >= 0; --f)
        for (int a = 0; a < 3; ++a) m.vert_face0[m.tris[3 * f + a]] = (int32_t)f;
    return MAD_OK;
}

// Rest triangle in its own 2D frame: Dm = [[|e1|, e1.e2/|e1|], [0, |e1 x e2|/|e1|]].
static bool rest_frame(const double* X0, const double* X1, const double* X2, double* mi, double* area) {
    const double e1[3] = {X1[0] - X0[0], X1[1] - X0[1], X1[2] - X0[2]};
    const double e2[3] = {X2[0] - X0[0], X2[1] - X0[1], X2[2] - X0[2]};
    const double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double l1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    const double cn = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    if (!(l1 > 0.0) || !(cn > 0.0) || !std::isfinite(cn)) return false;
    const double a = l1, b = (e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2]) / l1, d = cn / l1;
    // inverse of the upper-triangular [[a, b], [0, d]]
    mi[0] = 1.0 / a;
    mi[1] = -b / (a * d);
    mi[2] = 0.0;
    mi[3] = 1.0 / d;
    *area = 0.5 * cn;
    return true;
}

int rest_tri(const mad_mesh& m, const double* X, std::vector<double>& out) {
    out.assign((size_t)m.nt * 5, 0.0);
    for (int64_t f = 0; f < m.nt; ++f) {
        const int32_t* t = &m.tris[3 * f];
        if (!rest_frame(X + 3 * (int64_t)t[0], X + 3 * (int64_t)t[1], X + 3 * (int64_t)t[2], &out[5 * f], &out[5 * f + 4]))
            return fail(MAD_E_DEGENERATE_REST, "rest triangle " + std::to_string(f) + " has zero area");
    }
    return MAD_OK;
}

// Rest data of the shell-feature terms: Dm^{-1} (4), rest area, and the rest second form
// rII = -(N^T F + F^T N)/2 of the rest mesh with its own area-weighted unit vertex normals
// (F = rest Ds Dm^{-1}, N = [n_b - n_a, n_c - n_a] Dm^{-1}).
int rest_shell(const mad_mesh& m, const double* X, std::vector<double>& out) {
    out.assign((size_t)m.nt * 8, 0.0);
    std::vector<double> nrm((size_t)m.nv * 3, 0.0);
    for (int64_t f = 0; f < m.nt; ++f) {
        const int32_t* t = &m.tris[3 * f];
        const double *a = X + 3 * (int64_t)t[0], *b = X + 3 * (int64_t)t[1], *c = X + 3 * (int64_t)t[2];
        const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        for (int v = 0; v < 3; ++v)
            for (int d = 0; d < 3; ++d) nrm[3 * (size_t)t[v] + d] += n[d];
    }
    for (int64_t v = 0; v < m.nv; ++v) {
        double* n = &nrm[3 * v];
        const double l = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (l > 0.0)
            for (int d = 0; d < 3; ++d) n[d] /= l;
    }
    for (int64_t f = 0; f < m.nt; ++f) {
        const int32_t* t = &m.tris[3 * f];
        double* o = &out[8 * f];
        if (!rest_frame(X + 3 * (int64_t)t[0], X + 3 * (int64_t)t[1], X + 3 * (int64_t)t[2], o, o + 4))
            return fail(MAD_E_DEGENERATE_REST, "rest triangle " + std::to_string(f) + " has zero area");
        double F[3][2], N[3][2];
        for (int i = 0; i < 3; ++i) {
            const double d1 = X[3 * (int64_t)t[1] + i] - X[3 * (int64_t)t[0] + i];
            const double d2 = X[3 * (int64_t)t[2] + i] - X[3 * (int64_t)t[0] + i];
            const double n1 = nrm[3 * (size_t)t[1] + i] - nrm[3 * (size_t)t[0] + i];
            const double n2 = nrm[3 * (size_t)t[2] + i] - nrm[3 * (size_t)t[0] + i];
            for (int j = 0; j < 2; ++j) {
                F[i][j] = d1 * o[j] + d2 * o[2 + j];
                N[i][j] = n1 * o[j] + n2 * o[2 + j];
            }
        }
        double ii00 = 0, ii11 = 0, ii01 = 0;
        for (int i = 0; i < 3; ++i) {
            ii00 += F[i][0] * N[i][0];
            ii11 += F[i][1] * N[i][1];
            ii01 += F[i][1] * N[i][0] + F[i][0] * N[i][1];
        }
        o[5] = -ii00;
        o[6] = -ii11;
        o[7] = -0.5 * ii01;
    }
    return MAD_OK;
}

// rest dihedral of a diamond: atan2(-|e| (n1 . b), n1 . n2) with e = X1 - X0, n1 = e x (X2 - X0),
// n2 = (X3 - X0) x e, b = X3 - X0 (the same angle as atan2(((n1 x n2) . e)/|e|, n1 . n2))
static double dihedral(const double* X0, const double* X1, const double* X2, const double* X3) {
    double e[3], a[3], b[3];
    for (int k = 0; k < 3; ++k) {
        e[k] = X1[k] - X0[k];
        a[k] = X2[k] - X0[k];
        b[k] = X3[k] - X0[k];
    }
    const double n1[3] = {e[1] * a[2] - e[2] * a[1], e[2] * a[0] - e[0] * a[2], e[0] * a[1] - e[1] * a[0]};
    const double n2[3] = {b[1] * e[2] - b[2] * e[1], b[2] * e[0] - b[0] * e[2], b[0] * e[1] - b[1] * e[0]};
    const double c = n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2];
    const double s = -std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]) * (n1[0] * b[0] + n1[1] * b[1] + n1[2] * b[2]);
    return std::atan2(s, c);
}

int rest_diamond(const mad_mesh& m, const double* X, std::vector<double>& out) {
    const int64_t nd = m.nd();
    out.assign((size_t)nd * 2, 0.0);
    for (int64_t e = 0; e < nd; ++e) {
        double mi[4], a1, a2;
        const int32_t* t1 = &m.tris[3 * (int64_t)m.diamond_faces[2 * e]];
        const int32_t* t2 = &m.tris[3 * (int64_t)m.diamond_faces[2 * e + 1]];
        if (!rest_frame(X + 3 * (int64_t)t1[0], X + 3 * (int64_t)t1[1], X + 3 * (int64_t)t1[2], mi, &a1) ||
            !rest_frame(X + 3 * (int64_t)t2[0], X + 3 * (int64_t)t2[1], X + 3 * (int64_t)t2[2], mi, &a2))
            return fail(MAD_E_DEGENERATE_REST, "rest face of diamond " + std::to_string(e) + " has zero area");
        out[2 * e] = 0.5 * (a1 + a2);
        const int32_t* d = &m.diamonds[4 * e];
        out[2 * e + 1] = dihedral(X + 3 * (int64_t)d[0], X + 3 * (int64_t)d[1], X + 3 * (int64_t)d[2], X + 3 * (int64_t)d[3]);
    }
    return MAD_OK;
}

// Springs (Sec. 7.1): per edge the rest squared length l^2 and its reciprocal.
int rest_spring(const mad_mesh& m, const double* X, std::vector<double>& out) {
    const int64_t ne = m.ne();
    out.assign((size_t)ne * 2, 0.0);
    for (int64_t e = 0; e < ne; ++e) {
        const double* a = X + 3 * (int64_t)m.edges[2 * e];
        const double* b = X + 3 * (int64_t)m.edges[2 * e + 1];
        const double l2 = (a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) + (a[2] - b[2]) * (a[2] - b[2]);
        if (!(l2 > 0.0) || !std::isfinite(l2))
            return fail(MAD_E_DEGENERATE_REST, "rest edge " + std::to_string(e) + " has zero length");
        out[2 * e] = l2;
        out[2 * e + 1] = 1.0 / l2;
    }
    return MAD_OK;
}

// Edge-length residuals: per edge the rest length l.
int rest_edge_length(const mad_mesh& m, const double* X, std::vector<double>& out) {
    std::vector<double> sq;
    int rc = rest_spring(m, X, sq);
    if (rc != MAD_OK) return rc;
    const int64_t ne = m.ne();
    out.assign((size_t)ne, 0.0);
    for (int64_t e = 0; e < ne; ++e) out[e] = std::sqrt(sq[2 * e]);
    return MAD_OK;
}

// Patches: faces grouped into connected pieces of about target_faces by breadth-first growth
// over face adjacency. A new patch is seeded from the previous patch's unvisited frontier (so
// consecutive patches are neighbours), otherwise from the lowest unassigned face. Growth never
// crosses a component boundary, so every patch lies in one component; patches are numbered
// component by component.
void build_patches(const mad_mesh& m, int target, Patches& P) {
    const int64_t nt = m.nt;
    P.face_patch.assign((size_t)nt, -1);
    const int64_t ncomp = (int64_t)m.comp_off.size() - 1;
    // component of each face = component of its first vertex
    std::vector<int32_t> fcomp((size_t)nt, 0);
    if (ncomp > 1) {
        for (int64_t f = 0; f < nt; ++f) {
            const int64_t v = m.tris[3 * f];
            fcomp[f] = (int32_t)(std::upper_bound(m.comp_off.begin(), m.comp_off.end(), v) - m.comp_off.begin() - 1);
        }
    }
    // faces ordered by component, then index: seeds are taken in this order
    std::vector<int32_t> order((size_t)nt);
    std::iota(order.begin(), order.end(), 0);
    if (ncomp > 1)
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return fcomp[a] < fcomp[b]; });
    int32_t np = 0;
    size_t scan = 0;
    std::deque<int32_t> q;
    std::vector<int32_t> frontier;
    std::vector<int32_t> patch_comp;
    while (true) {
        int32_t seed = -1;
        for (int32_t f : frontier)
            if (P.face_patch[f] < 0) {
                seed = f;
                break;
            }
        if (seed < 0) {
            while (scan < order.size() && P.face_patch[order[scan]] >= 0) ++scan;
            if (scan == order.size()) break;
            seed = order[scan];
        }
        const int32_t pid = np++;
        patch_comp.push_back(fcomp[seed]);
        int32_t count = 0;
        q.clear();
        q.push_back(seed);
        P.face_patch[seed] = pid;
        std::vector<int32_t> next_frontier;
        while (!q.empty()) {
            const int32_t f = q.front();
            q.pop_front();
            ++count;
            for (int32_t k = m.fadj_ptr[f]; k < m.fadj_ptr[f + 1]; ++k) {
                const int32_t g = m.fadj[k];
                if (P.face_patch[g] >= 0) continue;
                if (count + (int32_t)q.size() < target) {
                    P.face_patch[g] = pid;
                    q.push_back(g);
                } else {
                    next_frontier.push_back(g);
                }
            }
        }
        frontier.swap(next_frontier);
    }
    P.n = np;
    P.comp_patch_ptr.assign((size_t)std::max<int64_t>(ncomp, 1) + 1, 0);
    for (int32_t p = 0; p < np; ++p) P.comp_patch_ptr[patch_comp[p] + 1]++;
    for (size_t c = 1; c < P.comp_patch_ptr.size(); ++c) P.comp_patch_ptr[c] += P.comp_patch_ptr[c - 1];
    // patches were created component by component only if seeds never jumped back; renumber so
    // that patches of component c form one contiguous range
    std::vector<int32_t> newid((size_t)np);
    std::vector<int32_t> fill(P.comp_patch_ptr.begin(), P.comp_patch_ptr.end() - 1);
    for (int32_t p = 0; p < np; ++p) newid[p] = fill[patch_comp[p]]++;
    for (int64_t f = 0; f < nt; ++f) P.face_patch[f] = newid[P.face_patch[f]];
}

}  // namespace mad
