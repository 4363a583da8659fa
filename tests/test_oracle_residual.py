"""Pins of the oracle's residual terms and sparse Jacobian (Sec. 4.1 Eq. 3, Sec. 6.1): the positional
residual of the paper's vector-term example and an edge-length residual against closed forms and finite
differences, the Gauss-Newton scalar form (1/2 |r|^2, J^T r, J^T J), and the assembled Jacobian
against a dense stacking of the local Jacobians written out here; J^T J and J^T r of the assembled
Jacobian equal the assembled Gauss-Newton matrix and gradient."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_00406_amd import meshgen


def test_position_residual_closed_form():
    rng = np.random.default_rng(1)
    for _ in range(10):
        x, xt, w = rng.normal(size=3), rng.normal(size=3), rng.uniform(0.1, 4.0)
        r, J = O.residual(O.RES_POSITION, x, [w, *xt])
        assert np.allclose(r, np.sqrt(w) * (x - xt), rtol=1e-15, atol=1e-15)
        assert np.allclose(J, np.sqrt(w) * np.eye(3), rtol=1e-15, atol=0)


def test_edge_residual_closed_form_and_fd():
    rng = np.random.default_rng(2)
    for _ in range(10):
        x = rng.normal(size=6)
        l, k = rng.uniform(0.2, 2.0), rng.uniform(0.5, 3.0)
        r, J = O.residual(O.RES_EDGE, x, [l], (k,))
        d = x[:3] - x[3:]
        n = np.linalg.norm(d)
        assert r[0] == pytest.approx(np.sqrt(k) * (n - l), rel=1e-14)
        assert np.allclose(J[0], np.sqrt(k) * np.concatenate([d / n, -d / n]), rtol=1e-13, atol=1e-15)
        # Richardson central differences of the residual
        for i in range(6):
            def rr(hh):
                y = x.copy()
                y[i] += hh
                return O.residual(O.RES_EDGE, y, [l], (k,))[0][0]
            h = 1e-4
            d1 = (rr(h) - rr(-h)) / (2 * h)
            d2 = (rr(h / 2) - rr(-h / 2)) / h
            assert (4 * d2 - d1) / 3 == pytest.approx(J[0, i], rel=1e-8, abs=1e-10)


@pytest.mark.parametrize("kind", [O.RES_POSITION, O.RES_EDGE])
def test_residual_kind_as_scalar_term_is_gauss_newton(kind):
    rng = np.random.default_rng(3)
    k = O.STENCIL[kind] * 3
    x = rng.normal(size=k)
    rest = [1.3, *rng.normal(size=3)] if kind == O.RES_POSITION else [0.7]
    prm = (2.0,)
    r, J = O.residual(kind, x, rest, prm)
    f, g, H = O.element(kind, x, rest, prm)
    assert f == pytest.approx(0.5 * r @ r, rel=1e-14)
    assert np.allclose(g, J.T @ r, rtol=1e-13, atol=1e-15)
    assert np.allclose(H, J.T @ J, rtol=1e-13, atol=1e-15)


def residual_problem(n=9, seed=5):
    tris, rest = meshgen.grid(n)
    rng = np.random.default_rng(seed)
    x = rest + 0.05 * rng.normal(size=rest.shape)
    vd = np.zeros((n * n, 4))
    vd[:, 0] = rng.uniform(0.0, 2.0, n * n) * (rng.random(n * n) < 0.3)   # a subset constrained
    vd[:, 1:] = rest + 0.1 * rng.normal(size=rest.shape)
    P = O.Problem(tris, rest, n * n, 3)
    P.add_term(O.RES_EDGE, (3.0,))
    P.add_term(O.RES_POSITION, (), vertex_data=vd)
    P.add_term(O.STVK, (1.0, 1.0))          # a scalar term owns no Jacobian rows
    return P, x, vd


def test_assembled_jacobian_is_the_stacked_local_jacobians():
    P, x, vd = residual_problem()
    r, rp, ci, vals = P.jacobian(x)
    nv = P.nv
    Jd = np.zeros((len(r), 3 * nv))
    Jd[np.repeat(np.arange(len(r)), np.diff(rp)), ci] = vals
    # written out: rows by term, then element; each local Jacobian into its stencil's columns
    Jref = np.zeros_like(Jd)
    rref = np.zeros(len(r))
    row = 0
    X = P.rest_pos
    for e, (a, b) in enumerate(P.topo.edges):
        rr, J = O.residual(O.RES_EDGE, np.concatenate([x[a], x[b]]), [np.linalg.norm(X[a] - X[b])], (3.0,))
        rref[row] = rr[0]
        Jref[row, 3 * a:3 * a + 3] = J[0, :3]
        Jref[row, 3 * b:3 * b + 3] = J[0, 3:]
        row += 1
    for v in range(nv):
        rr, J = O.residual(O.RES_POSITION, x[v], vd[v])
        rref[row:row + 3] = rr
        Jref[row:row + 3, 3 * v:3 * v + 3] = J
        row += 3
    assert row == len(r)
    assert np.allclose(r, rref, rtol=1e-15, atol=1e-15)
    assert np.allclose(Jd, Jref, rtol=1e-15, atol=1e-15)
    for i in range(len(r)):
        assert np.all(np.diff(ci[rp[i]:rp[i + 1]]) > 0)


def test_jtj_and_jtr_equal_the_gauss_newton_assembly():
    P, x, vd = residual_problem()
    P.terms = P.terms[:2]                    # residual terms only
    P.rowptr = None
    r, rp, ci, vals = P.jacobian(x)
    nv = P.nv
    Jd = np.zeros((len(r), 3 * nv))
    Jd[np.repeat(np.arange(len(r)), np.diff(rp)), ci] = vals
    res = P.eval(x, O.ENERGY | O.GRAD | O.HESS)
    D = np.zeros((3 * nv, 3 * nv))
    for i in range(nv):
        for b in range(P.rowptr[i], P.rowptr[i + 1]):
            j = P.colidx[b]
            D[3 * i:3 * i + 3, 3 * j:3 * j + 3] = res.hess[b]
    JtJ = Jd.T @ Jd
    assert np.max(np.abs(D - JtJ)) <= 1e-13 * np.max(np.abs(JtJ))
    assert np.max(np.abs(res.grad - Jd.T @ r)) <= 1e-13 * np.max(np.abs(Jd.T @ r))
    assert res.energy == pytest.approx(0.5 * r @ r, rel=1e-13)
