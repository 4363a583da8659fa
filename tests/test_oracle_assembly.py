"""Pins of the oracle's topology, pattern, assembly and energy reduction:
brute-force sets and dense sums on tiny meshes, closed-form grid counts, the
cotangent Laplacian on a whole mesh, finite differences of the global energy
and an exact (fsum) reference for the compensated sum."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_00406_amd import meshgen

RNG = np.random.default_rng(777)


def grid_counts(n):
    V = n * n
    T = 2 * (n - 1) ** 2
    E = 2 * n * (n - 1) + (n - 1) ** 2
    Ebd = 4 * (n - 1)
    Eint = (3 * T - Ebd) // 2
    return V, T, E, Eint


# ------------------------------------------------------------------ topology
def test_topology_two_triangles_diamond_order():
    tris = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    topo = O.topology(tris, 4)
    assert topo.edges.tolist() == [[0, 1], [0, 2], [0, 3], [1, 2], [2, 3]]
    assert topo.edge_nf.tolist() == [1, 2, 1, 1, 1]
    # shared edge (0,2): f1 = face 0 traverses it as 2 -> 0, opposite 1; face 1 opposite 3
    assert topo.diamonds.tolist() == [[2, 0, 1, 3]]
    assert topo.diamond_faces.tolist() == [[0, 1]]


def test_topology_nonmanifold_and_isolated():
    tris, pos = meshgen.tiny_meshes()["nonmanifold"]
    topo = O.topology(tris, pos.shape[0])
    e01 = [i for i, e in enumerate(topo.edges.tolist()) if e == [0, 1]][0]
    assert topo.edge_nf[e01] == 3
    assert topo.diamonds.shape[0] == 0        # no edge has exactly two faces


def test_topology_octahedron_closed():
    tris, pos = meshgen.tiny_meshes()["octahedron"]
    topo = O.topology(tris, 6)
    assert topo.edges.shape[0] == 12 and np.all(topo.edge_nf == 2)
    assert topo.diamonds.shape[0] == 12
    # every diamond's wings lie on opposite sides: flat rest dihedral of a convex solid is nonzero
    rd = O.rest_diamond(topo, tris, pos)
    assert np.allclose(np.abs(rd[:, 1]), math.pi - math.acos(-1 / 3), atol=1e-12)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 8, 16])
def test_topology_grid_counts(n):
    tris, pos = meshgen.grid(n)
    V, T, E, Eint = grid_counts(n)
    topo = O.topology(tris, V)
    assert tris.shape[0] == T and topo.edges.shape[0] == E and topo.diamonds.shape[0] == Eint
    # flat grid: every rest dihedral is zero
    assert np.all(O.rest_diamond(topo, tris, pos)[:, 1] == 0.0)


def test_topology_rejects_bad_indices():
    with pytest.raises(RuntimeError):
        O.topology(np.array([[0, 1, 5]], np.int32), 4)
    with pytest.raises(RuntimeError):
        O.topology(np.array([[0, 1, 1]], np.int32), 4)


def test_rest_tri_rejects_degenerate():
    with pytest.raises(RuntimeError):
        O.rest_tri(np.array([[0, 1, 2]], np.int32), np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0.0]]))


# ------------------------------------------------------------------ pattern
def brute_pattern(nv, stencils):
    s = {(i, i) for i in range(nv)}
    for st in stencils:
        for el in st:
            for a in el:
                for b in el:
                    s.add((int(a), int(b)))
    return sorted(s)


@pytest.mark.parametrize("name", ["two_tris", "octahedron", "nonmanifold", "grid3", "grid5"])
def test_pattern_brute_force(name):
    tris, pos = meshgen.tiny_meshes()[name]
    nv = pos.shape[0]
    topo = O.topology(tris, nv)
    sts = [tris, topo.diamonds]
    rowptr, colidx = O.pattern(nv, sts)
    pairs = [(r, int(c)) for r in range(nv) for c in colidx[rowptr[r]:rowptr[r + 1]]]
    assert pairs == brute_pattern(nv, sts)


@pytest.mark.parametrize("n", [4, 8, 16, 64])
def test_pattern_grid_closed_form(n):
    tris, pos = meshgen.grid(n)
    V, T, E, Eint = grid_counts(n)
    topo = O.topology(tris, V)
    rp, ci = O.pattern(V, [tris])
    assert rp[-1] == V + 2 * E
    rp, ci = O.pattern(V, [tris, topo.diamonds])
    assert rp[-1] == V + 2 * E + 2 * Eint
    if n == 64:
        assert rp[-1] == 51724
        assert O.pattern(V, [tris])[0][-1] == 28162


# ------------------------------------------------------------------ assembly
def dense_assembly(P: O.Problem, x, mode):
    """Eq. 2 written densely: H = sum_j S_j^T H_j S_j, g = sum_j S_j^T g_j."""
    d = P.d
    n = P.nv * d
    Hd = np.zeros((n, n))
    gd = np.zeros(n)
    fs = []
    for t in P.terms:
        ss = t.stencil.shape[1]
        for e in range(t.stencil.shape[0]):
            s = t.stencil[e]
            idx = np.concatenate([np.arange(v * d, v * d + d) for v in s])
            rest = None if t.rest is None else t.rest[e]
            f, g, H = O.element(t.kind, x.reshape(-1)[idx], rest, t.params, mode=mode)
            S = np.zeros((ss * d, n))
            S[np.arange(ss * d), idx] = 1.0
            gd += S.T @ g
            Hd += S.T @ H @ S
            fs.append(f)
    return math.fsum(fs), gd, Hd


def to_dense(P: O.Problem, hess):
    d = P.d
    Hd = np.zeros((P.nv * d, P.nv * d))
    for r in range(P.nv):
        for b in range(P.rowptr[r], P.rowptr[r + 1]):
            c = P.colidx[b]
            Hd[r * d:r * d + d, c * d:c * d + d] = hess[b]
    return Hd


def shell_problem(name, spd):
    tris, pos = meshgen.tiny_meshes()[name]
    P = O.Problem(tris, pos, pos.shape[0], 3)
    P.add_term(O.STVK, (0.9, 1.1))
    P.add_term(O.BENDING, (0.8, 1.0))
    x = pos + 0.15 * RNG.normal(size=pos.shape)
    return P, x


@pytest.mark.parametrize("name", ["two_tris", "octahedron", "grid3", "nonmanifold"])
@pytest.mark.parametrize("spd", [False, True])
def test_assembly_equals_dense_sum(name, spd):
    P, x = shell_problem(name, spd)
    mode = O.ENERGY | O.GRAD | O.HESS | (O.SPD if spd else 0)
    r = P.eval(x, mode)
    f, g, H = dense_assembly(P, x, mode)
    Hs = to_dense(P, r.hess)
    scale = np.abs(H).max()
    assert r.energy == pytest.approx(f, rel=1e-14)
    assert np.allclose(r.grad, g, atol=1e-14 * np.abs(g).max())
    assert np.allclose(Hs, H, atol=1e-14 * scale)
    assert np.allclose(Hs, Hs.T, atol=1e-13 * scale)
    if spd:
        assert np.linalg.eigvalsh(Hs).min() > -1e-12 * scale


def test_global_gradient_is_fd_of_global_energy():
    P, x = shell_problem("octahedron", False)
    r = P.eval(x)
    def F(v):
        return P.eval(v.reshape(x.shape), O.ENERGY).energy
    h = 1e-4
    g = np.zeros(x.size)
    for i in range(x.size):
        xp = x.ravel().copy(); xm = x.ravel().copy()
        xp[i] += h; xm[i] -= h
        xp2 = x.ravel().copy(); xm2 = x.ravel().copy()
        xp2[i] += h / 2; xm2[i] -= h / 2
        d1 = (F(xp) - F(xm)) / (2 * h)
        d2 = (F(xp2) - F(xm2)) / h
        g[i] = (4 * d2 - d1) / 3
    assert np.allclose(r.grad, g, atol=1e-7 * np.abs(g).max())


def cot_laplacian(tris, pos):
    nv = pos.shape[0]
    L = np.zeros((nv, nv))
    for t in tris:
        for c in range(3):
            a, b = t[(c + 1) % 3], t[(c + 2) % 3]
            u, v = pos[a] - pos[t[c]], pos[b] - pos[t[c]]
            w = 0.5 * (u @ v) / np.linalg.norm(np.cross(u, v))
            L[a, b] -= w; L[b, a] -= w
            L[a, a] += w; L[b, b] += w
    return L


def test_dirichlet_assembly_is_cotangent_laplacian():
    inp = meshgen.dirichlet_grid(n=12)
    P = O.Problem(inp.tris, inp.rest, inp.n_verts, 1)
    P.add_term(O.DIRICHLET)
    r = P.eval(inp.x)
    L = cot_laplacian(inp.tris, inp.rest)
    H = to_dense(P, r.hess)
    u = inp.x.ravel()
    assert np.allclose(H, L, atol=1e-13 * np.abs(L).max())
    assert np.allclose(r.grad, L @ u, atol=1e-12 * np.abs(L @ u).max())
    assert r.energy == pytest.approx(0.5 * u @ L @ u, rel=1e-12)
    assert abs(r.grad.sum()) < 1e-12 * np.abs(r.grad).max() * inp.n_verts


def test_row_mask_restricts_assembly():
    P, x = shell_problem("grid5", True)
    mode = O.ENERGY | O.GRAD | O.HESS | O.SPD
    full = P.eval(x, mode)
    mask = np.zeros(P.nv, bool)
    mask[[3, 7, 12]] = True
    part = P.eval(x, mode, row_mask=mask)
    assert part.energy == full.energy
    for r in range(P.nv):
        blk = slice(P.rowptr[r], P.rowptr[r + 1])
        if mask[r]:
            assert np.array_equal(part.hess[blk], full.hess[blk])
            assert np.array_equal(part.grad[3 * r:3 * r + 3], full.grad[3 * r:3 * r + 3])
        else:
            assert np.all(part.hess[blk] == 0)


# ------------------------------------------------------------------ energy reduction
def test_neumaier_matches_exact_sum():
    for scale in (1.0, 1e8):
        v = RNG.normal(size=100000) * np.exp(RNG.uniform(-20, 20, size=100000)) * scale
        v = np.concatenate([v, -v[:50000] * (1 + 1e-9)])
        exact = math.fsum(v)
        assert abs(O.neumaier_sum(v) - exact) <= 2 ** -52 * abs(exact) + 1e-300
    assert O.neumaier_sum(np.array([1e100, 1.0, -1e100])) == 1.0


# ---------------------------------------------------------------- Hessian-vector products
def test_hvp_is_directional_derivative_of_gradient():
    # H(x) v = d/de g(x + e v) at e = 0: central differences of the oracle's own gradient
    from paper_2509_00406_amd import meshgen
    inp = meshgen.shell_cylinder(n=7, seed=17)
    P = O.Problem(inp.tris, inp.rest, inp.n_verts, 3)
    P.add_term(O.STVK, (1.0, 0.7))
    P.add_term(O.BENDING, (0.9, 1.0))
    x = inp.x.ravel().copy()
    v = np.random.default_rng(4).normal(size=x.size)
    y, ys = P.hvp(x, v)

    def g(t):
        return P.eval(x + t * v, O.GRAD).grad
    h = 1e-4
    fd = (4 * (g(h / 2) - g(-h / 2)) / h - (g(h) - g(-h)) / (2 * h)) / 3
    assert np.max(np.abs(y - fd)) < 1e-6 * np.max(np.abs(y))
    # linear in v, and symmetric: u.(H v) = v.(H u)
    u = np.random.default_rng(5).normal(size=x.size)
    yu, _ = P.hvp(x, u)
    yuv, _ = P.hvp(x, 2.0 * v - 3.0 * u)
    assert np.allclose(yuv, 2.0 * y - 3.0 * yu, rtol=1e-12, atol=1e-12 * np.max(np.abs(y)))
    assert abs(u @ y - v @ yu) < 1e-11 * np.sqrt((u @ u) * (v @ v)) * np.max(np.abs(ys))
    assert np.all(ys >= np.abs(y) * (1 - 1e-12))


def test_hvp_spd_is_psd_and_dense_product():
    # with the clamp, v.(H v) >= 0 for every v; and the product equals the dense assembled matrix's
    tris, pos = meshgen.tiny_meshes()["grid3"]
    x = pos + np.random.default_rng(6).normal(scale=0.2, size=pos.shape)
    P = O.Problem(tris, pos, pos.shape[0], 3)
    P.add_term(O.STVK, (1.0, 1.0))
    P.add_term(O.BENDING, (1.0, 1.0))
    P.build_pattern()
    r = P.eval(x, O.HESS | O.SPD)
    n = pos.shape[0]
    Hd = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for b in range(P.rowptr[i], P.rowptr[i + 1]):
            j = P.colidx[b]
            Hd[3 * i:3 * i + 3, 3 * j:3 * j + 3] = r.hess[b]
    rng = np.random.default_rng(7)
    for _ in range(5):
        v = rng.normal(size=3 * n)
        y, _ = P.hvp(x, v, spd=True)
        assert np.allclose(y, Hd @ v, rtol=0, atol=1e-12 * np.max(np.abs(Hd)) * np.max(np.abs(v)) * 9)
        assert v @ y >= -1e-10 * np.max(np.abs(Hd)) * (v @ v)
