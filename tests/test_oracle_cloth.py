"""Pins of the oracle's mass-spring cloth terms (Sec. 7.1): the spring of an edge and the
per-vertex inertia plus gravity, checked against their closed-form derivatives, the closed-form
eigen-decomposition of a spring's Hessian (what the filtering must produce), and a dense assembly
of the whole time-step energy written out here from those closed forms."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_00406_amd import meshgen


def spring_closed(x0, x1, l, k, w):
    """f, g (6), H (6x6) of w (k/2) l^2 (|d|^2/l^2 - 1)^2, d = x0 - x1, by hand:
    df/dd = 2 w k q d, d2f/dd2 = 2 w k (q I + 2 d d^T / l^2), q = |d|^2/l^2 - 1."""
    d = np.asarray(x0, float) - np.asarray(x1, float)
    q = d @ d / l ** 2 - 1.0
    f = w * 0.5 * k * l ** 2 * q * q
    gd = 2 * w * k * q * d
    B = 2 * w * k * (q * np.eye(3) + 2 * np.outer(d, d) / l ** 2)
    g = np.concatenate([gd, -gd])
    H = np.block([[B, -B], [-B, B]])
    return f, g, H


def spring_filtered(x0, x1, l, k, w, eps):
    """The clamped spring Hessian from its known eigen-structure: H = [[B, -B], [-B, B]] has the
    eigenvalues 2 mu of B on the vectors (b, -b)/sqrt2 and 0 on the translations (e, e)/sqrt2; B
    has mu_par = 2wk(3|d|^2/l^2 - 1) along d and mu_perp = 2wk(|d|^2/l^2 - 1) across it."""
    d = np.asarray(x0, float) - np.asarray(x1, float)
    s = d @ d / l ** 2
    dh = d / np.linalg.norm(d)
    Pp = np.outer(dh, dh)
    mu_par, mu_perp = 2 * w * k * (3 * s - 1), 2 * w * k * (s - 1)
    Bc = max(2 * mu_par, eps) * Pp + max(2 * mu_perp, eps) * (np.eye(3) - Pp)
    minus = 0.5 * np.array([[1.0, -1.0], [-1.0, 1.0]])
    plus = 0.5 * np.array([[1.0, 1.0], [1.0, 1.0]])
    return np.kron(minus, Bc) + np.kron(plus, max(0.0, eps) * np.eye(3))


@pytest.mark.parametrize("stretch", [0.7, 0.95, 1.0, 1.2, 1.8])
def test_spring_matches_closed_form(stretch):
    rng = np.random.default_rng(int(stretch * 100))
    for _ in range(5):
        l = rng.uniform(0.1, 2.0)
        dirn = rng.normal(size=3)
        dirn /= np.linalg.norm(dirn)
        x1 = rng.normal(size=3)
        x0 = x1 + stretch * l * dirn
        k, w = rng.uniform(0.5, 3.0), rng.uniform(0.1, 2.0)
        f, g, H = O.element(O.SPRING, np.concatenate([x0, x1]), rest=[l], params=[k, w])
        fr, gr, Hr = spring_closed(x0, x1, l, k, w)
        sc = max(1.0, np.abs(Hr).max())
        assert abs(f - fr) <= 1e-13 * max(1.0, abs(fr))
        assert np.abs(g - gr).max() <= 1e-13 * max(1.0, np.abs(gr).max())
        assert np.abs(H - Hr).max() <= 1e-12 * sc


@pytest.mark.parametrize("stretch", [0.6, 0.9, 1.1, 1.5])
@pytest.mark.parametrize("eps", [0.0, 1e-3, 0.5])
def test_spring_filtering_matches_eigen_structure(stretch, eps):
    # compressed springs (stretch < 1) have negative transverse eigenvalues: the filtering must lift
    # exactly those (and the translations, when eps > 0) and leave the rest
    rng = np.random.default_rng(7)
    l = 0.8
    dirn = np.array([0.3, -0.5, 0.81])
    dirn /= np.linalg.norm(dirn)
    x1 = rng.normal(size=3)
    x0 = x1 + stretch * l * dirn
    k, w = 2.0, 0.7
    _, _, Hp = O.element(O.SPRING, np.concatenate([x0, x1]), rest=[l], params=[k, w],
                         mode=O.ENERGY | O.GRAD | O.HESS | O.SPD, spd_eps=eps)
    ref = spring_filtered(x0, x1, l, k, w, eps)
    assert np.abs(Hp - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    lam = np.linalg.eigvalsh(Hp)
    assert lam.min() >= eps - 1e-12


def test_inertia_matches_closed_form():
    rng = np.random.default_rng(11)
    for _ in range(10):
        x = rng.normal(size=3)
        m = rng.uniform(0.1, 3.0)
        xh = rng.normal(size=3)
        w = rng.uniform(0.01, 1.0)
        gv = rng.normal(size=3)
        f, g, H = O.element(O.INERTIA, x, rest=[m, *xh], params=[w, *gv])
        assert abs(f - (0.5 * m * np.sum((x - xh) ** 2) - w * m * gv @ x)) <= 1e-13 * max(1.0, abs(f))
        assert np.abs(g - (m * (x - xh) - w * m * gv)).max() <= 1e-13 * max(1.0, np.abs(g).max())
        assert np.abs(H - m * np.eye(3)).max() <= 1e-14 * m
        # the filter leaves an SPD m I alone below m and lifts it to eps above
        _, _, Hp = O.element(O.INERTIA, x, rest=[m, *xh], params=[w, *gv], mode=O.ENERGY | O.HESS | O.SPD,
                             spd_eps=0.5 * m)
        assert np.abs(Hp - m * np.eye(3)).max() <= 1e-14 * m
        _, _, Hp = O.element(O.INERTIA, x, rest=[m, *xh], params=[w, *gv], mode=O.ENERGY | O.HESS | O.SPD,
                             spd_eps=2 * m)
        assert np.abs(Hp - 2 * m * np.eye(3)).max() <= 1e-14 * m


def dense_step(inp, spd, eps=0.0):
    """The whole time-step energy, gradient and dense Hessian written out from the closed forms:
    springs over the mesh edges (listed here from the triangles) plus inertia and gravity."""
    tris, X, x = inp.tris, inp.rest, inp.x
    nv = x.shape[0]
    k, w = inp.meta["spring_params"]
    wg, gx, gy, gz = inp.meta["inertia_params"]
    vd = inp.meta["vdata"]
    edges = set()
    for t in tris:
        for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            edges.add((min(a, b), max(a, b)))
    E = 0.0
    g = np.zeros(3 * nv)
    H = np.zeros((3 * nv, 3 * nv))
    for i, j in sorted(edges):
        l = np.linalg.norm(X[i] - X[j])
        f, ge, He = spring_closed(x[i], x[j], l, k, w)
        if spd:
            He = spring_filtered(x[i], x[j], l, k, w, eps)
        E += f
        idx = np.r_[3 * i:3 * i + 3, 3 * j:3 * j + 3]
        g[idx] += ge
        H[np.ix_(idx, idx)] += He
    grav = np.array([gx, gy, gz])
    for v in range(nv):
        m, xh = vd[v, 0], vd[v, 1:]
        E += 0.5 * m * np.sum((x[v] - xh) ** 2) - wg * m * grav @ x[v]
        g[3 * v:3 * v + 3] += m * (x[v] - xh) - wg * m * grav
        H[3 * v:3 * v + 3, 3 * v:3 * v + 3] += max(m, eps if spd else m) * np.eye(3)
    return E, g, H


def oracle_step(inp, mode, eps=0.0):
    P = O.Problem(inp.tris, inp.rest, inp.n_verts, 3)
    P.add_term(O.SPRING, inp.meta["spring_params"])
    P.add_term(O.INERTIA, inp.meta["inertia_params"], vertex_data=inp.meta["vdata"])
    return P, P.eval(inp.x, mode, spd_eps=eps)


def densify(P, hess):
    nv = P.nv
    D = np.zeros((3 * nv, 3 * nv))
    for r in range(nv):
        for b in range(P.rowptr[r], P.rowptr[r + 1]):
            c = P.colidx[b]
            D[3 * r:3 * r + 3, 3 * c:3 * c + 3] = hess[b]
    return D


@pytest.mark.parametrize("spd,eps", [(False, 0.0), (True, 0.0), (True, 1e-9)])
def test_cloth_step_assembly_matches_dense_closed_form(spd, eps):
    inp = meshgen.cloth(n=7, seed=17)
    P, r = oracle_step(inp, O.ENERGY | O.GRAD | O.HESS | (O.SPD if spd else 0), eps)
    E, g, H = dense_step(inp, spd, eps)
    assert abs(r.energy - E) <= 1e-13 * r.esum_abs
    assert np.abs(r.grad - g).max() <= 1e-13 * np.abs(g).max()
    D = densify(P, r.hess)
    assert np.abs(D - H).max() <= 1e-12 * np.abs(H).max()
    if spd:
        # every element's filtered Hessian is PSD, so the sum is too
        assert np.linalg.eigvalsh(D).min() >= -1e-12 * np.abs(H).max()


def test_cloth_workload_has_compressed_and_stretched_springs():
    inp = meshgen.cloth(n=40, seed=6001)
    P, r = oracle_step(inp, O.ENERGY | O.HESS)
    e = P.topo.edges
    d = inp.x[e[:, 0]] - inp.x[e[:, 1]]
    l = np.linalg.norm(inp.rest[e[:, 0]] - inp.rest[e[:, 1]], axis=1)
    q = np.sum(d * d, axis=1) / l ** 2 - 1
    assert 0.2 < np.mean(q < 0) < 0.8
    # without filtering the assembled step Hessian is indefinite on this state
    D = densify(P, r.hess)
    assert np.linalg.eigvalsh(D).min() < 0
