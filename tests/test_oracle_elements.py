"""Pins of the oracle's element derivatives against facts independent of it:
closed forms printed in the paper, textbook stiffness matrices, finite
differences and invariances. A dropped chain-rule term, a wrong sign or a
transposed operand in the hyper-dual arithmetic or in an energy fails here."""
import math

import numpy as np
import pytest

from oracle import oracle as O

RNG = np.random.default_rng(12345)


def fd_grad(fun, x, h):
    """Richardson-extrapolated central differences of a scalar function."""
    g = np.zeros_like(x)
    for i in range(x.size):
        def d(step):
            xp = x.copy(); xm = x.copy()
            xp[i] += step; xm[i] -= step
            return (fun(xp) - fun(xm)) / (2 * step)
        g[i] = (4 * d(h / 2) - d(h)) / 3
    return g


def fd_jac(fun, x, h):
    cols = []
    for i in range(x.size):
        def d(step):
            xp = x.copy(); xm = x.copy()
            xp[i] += step; xm[i] -= step
            return (fun(xp) - fun(xm)) / (2 * step)
        cols.append((4 * d(h / 2) - d(h)) / 3)
    return np.stack(cols, axis=1)


def check_fd(kind, xloc, rest=None, params=None, rtol=2e-7):
    f, g, H = O.element(kind, xloc, rest, params)
    fg = lambda x: O.element(kind, x, rest, params, mode=O.ENERGY)[0]
    gg = lambda x: O.element(kind, x, rest, params, mode=O.ENERGY | O.GRAD)[1]
    h = 1e-3 * max(1e-3, float(np.max(np.abs(xloc))))
    g_fd = fd_grad(fg, np.array(xloc, float), h)
    H_fd = fd_jac(gg, np.array(xloc, float), h)
    assert np.max(np.abs(g - g_fd)) <= rtol * max(1e-300, np.max(np.abs(g))) + 1e-12 * abs(f)
    assert np.max(np.abs(H - H_fd)) <= rtol * max(1e-300, np.max(np.abs(H)))
    assert np.allclose(H, H.T, rtol=0, atol=1e-14 * np.max(np.abs(H)))
    return f, g, H


def rest_of_tri(X):
    tris = np.array([[0, 1, 2]], np.int32)
    return O.rest_tri(tris, np.asarray(X, float).reshape(3, 3))[0]


# ------------------------------------------------------------------ Listing 1: squared edge length
def test_edge_sqlen_closed_form():
    x = RNG.normal(size=6)
    f, g, H = O.element(O.EDGE_SQLEN, x)
    d = x[:3] - x[3:]
    assert f == pytest.approx(d @ d, rel=1e-15)
    assert np.allclose(g, np.concatenate([2 * d, -2 * d]), rtol=1e-15, atol=0)
    I = np.eye(3)
    assert np.array_equal(H, np.block([[2 * I, -2 * I], [-2 * I, 2 * I]]))


# ------------------------------------------------------------------ Sec. 7.6: triangle area and its printed gradient
def test_area_gradient_matches_paper_closed_form():
    for _ in range(5):
        x = RNG.normal(size=(3, 3))
        f, g, H = O.element(O.TRI_AREA, x.ravel())
        n = np.cross(x[1] - x[0], x[2] - x[0])
        area = 0.5 * np.linalg.norm(n)
        nh = n / np.linalg.norm(n)
        assert f == pytest.approx(area, rel=1e-14)
        # dA/dx_i = 0.5 (x_j - x_k) x n, cyclic (i, j, k)
        for i in range(3):
            j, k = (i + 1) % 3, (i + 2) % 3
            assert np.allclose(g[3 * i:3 * i + 3], 0.5 * np.cross(x[j] - x[k], nh), rtol=1e-12, atol=1e-14)
        check_fd(O.TRI_AREA, x.ravel())


# ------------------------------------------------------------------ scalar Dirichlet energy == cotangent stiffness
def cot_stiffness(P):
    """Textbook P1 stiffness: K[a][b] = -cot(angle at c)/2, K[a][a] = -sum_b K[a][b]."""
    K = np.zeros((3, 3))
    for c in range(3):
        a, b = (c + 1) % 3, (c + 2) % 3
        u, v = P[a] - P[c], P[b] - P[c]
        cot = (u @ v) / np.linalg.norm(np.cross(u, v))
        K[a, b] -= 0.5 * cot
        K[b, a] -= 0.5 * cot
    for a in range(3):
        K[a, a] = -(K[a].sum() - K[a, a])
    return K


def test_dirichlet_is_cotangent_stiffness():
    for _ in range(10):
        P = np.zeros((3, 3))
        P[:, :2] = RNG.normal(size=(3, 2))
        if abs(np.cross(P[1] - P[0], P[2] - P[0])[2]) < 0.1:
            continue
        u = RNG.normal(size=3)
        rest = rest_of_tri(P)
        f, g, H = O.element(O.DIRICHLET, u, rest)
        K = cot_stiffness(P)
        assert np.allclose(H, K, rtol=1e-12, atol=1e-12 * np.abs(K).max())
        assert np.allclose(g, K @ u, rtol=1e-12, atol=1e-12 * np.abs(K).max())
        assert f == pytest.approx(0.5 * u @ K @ u, rel=1e-12)


def test_dirichlet_constant_field_and_linear_field():
    P = np.array([[0.1, 0.2, 0], [1.3, 0.1, 0], [0.4, 0.9, 0]])
    rest = rest_of_tri(P)
    f, g, _ = O.element(O.DIRICHLET, np.full(3, 2.5), rest)
    assert f == 0.0 and np.all(g == 0.0)
    # u = a.p gives |grad u|^2 = |a|^2, energy = 0.5 * area * |a|^2
    a = np.array([0.7, -1.9])
    u = P[:, :2] @ a
    area = 0.5 * abs(np.cross(P[1] - P[0], P[2] - P[0])[2])
    f, _, _ = O.element(O.DIRICHLET, u, rest)
    assert f == pytest.approx(0.5 * area * (a @ a), rel=1e-13)


# ------------------------------------------------------------------ StVK membrane
STVK_PRM = [0.8, 1.7]


def cst_stiffness(P, lam, mu):
    """Constant-strain-triangle plane-stress stiffness K = A B^T D B (Voigt, engineering shear)."""
    x, y = P[:, 0], P[:, 1]
    A2 = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0])
    b = np.array([y[1] - y[2], y[2] - y[0], y[0] - y[1]]) / A2
    c = np.array([x[2] - x[1], x[0] - x[2], x[1] - x[0]]) / A2
    B = np.zeros((3, 6))
    for i in range(3):
        B[0, 2 * i] = b[i]
        B[1, 2 * i + 1] = c[i]
        B[2, 2 * i] = c[i]
        B[2, 2 * i + 1] = b[i]
    D = np.array([[lam + 2 * mu, lam, 0], [lam, lam + 2 * mu, 0], [0, 0, mu]])
    return 0.5 * abs(A2) * B.T @ D @ B


def test_stvk_rest_hessian_is_linear_elastic_cst():
    mu, lam = STVK_PRM
    for _ in range(5):
        P = np.zeros((3, 3))
        P[:, :2] = RNG.normal(size=(3, 2))
        if np.cross(P[1] - P[0], P[2] - P[0])[2] < 0.2:
            continue
        rest = rest_of_tri(P)
        f, g, H = O.element(O.STVK, P.ravel(), rest, STVK_PRM)
        assert abs(f) < 1e-28 and np.max(np.abs(g)) < 1e-13
        K = cst_stiffness(P, lam, mu)
        idx = [0, 1, 3, 4, 6, 7]   # in-plane DOFs
        assert np.allclose(H[np.ix_(idx, idx)], K, rtol=1e-11, atol=1e-11 * np.abs(K).max())
        z = [2, 5, 8]
        assert np.max(np.abs(H[z, :])) < 1e-12 * np.abs(K).max()


def random_rotation():
    q, r = np.linalg.qr(RNG.normal(size=(3, 3)))
    q = q @ np.diag(np.sign(np.diag(r)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_stvk_rigid_motion_zero_and_invariances():
    P = np.array([[0, 0, 0], [1.1, 0.1, 0], [0.3, 0.9, 0.2]])
    rest = rest_of_tri(P)
    R = random_rotation()
    t = RNG.normal(size=3)
    f, g, _ = O.element(O.STVK, (P @ R.T + t).ravel(), rest, STVK_PRM)
    assert abs(f) < 1e-26 and np.max(np.abs(g)) < 1e-12
    x = P + 0.2 * RNG.normal(size=(3, 3))
    f0, g0, H0 = check_fd(O.STVK, x.ravel(), rest, STVK_PRM)
    f1, g1, H1 = O.element(O.STVK, (x @ R.T + t).ravel(), rest, STVK_PRM)
    assert f1 == pytest.approx(f0, rel=1e-12)
    Rb = np.kron(np.eye(3), R)
    assert np.allclose(g1, Rb @ g0, atol=1e-12 * np.abs(g0).max())
    assert np.allclose(H1, Rb @ H0 @ Rb.T, atol=1e-11 * np.abs(H0).max())
    gg = g0.reshape(3, 3)
    assert np.allclose(gg.sum(0), 0, atol=1e-13 * np.abs(g0).max())          # translation
    assert np.allclose(np.cross(x, gg).sum(0), 0, atol=1e-12 * np.abs(g0).max())  # rotation


def test_stvk_uniform_stretch_energy():
    # F = s * I (in-plane) gives E = (s^2 - 1)/2 I, psi = mu * 2 e^2 + lam/2 * (2e)^2
    P = np.array([[0, 0, 0], [1.0, 0.2, 0], [0.1, 0.8, 0]])
    rest = rest_of_tri(P)
    s = 1.3
    mu, lam = STVK_PRM
    e = 0.5 * (s * s - 1)
    area = 0.5 * np.cross(P[1] - P[0], P[2] - P[0])[2]
    f, _, _ = O.element(O.STVK, (s * P).ravel(), rest, STVK_PRM)
    assert f == pytest.approx(area * (mu * 2 * e * e + 0.5 * lam * (2 * e) ** 2), rel=1e-13)


# ------------------------------------------------------------------ Sec. 7.7: dihedral bending
BEND_PRM = [1.3, 0.7]


def hinge(phi, rot=None, t=None):
    x0 = np.array([0.0, 0, 0]); x1 = np.array([1.0, 0, 0])
    x2 = np.array([0.3, 1.0, 0])
    x3 = np.array([0.6, -math.cos(phi), -math.sin(phi)])
    X = np.stack([x0, x1, x2, x3])
    if rot is not None:
        X = X @ rot.T
    if t is not None:
        X = X + t
    return X


def theta_acos(X):
    """Independent signed dihedral: angle between face normals via acos, sign
    from the orientation of n1 x n2 along the hinge edge."""
    e = X[1] - X[0]
    n1 = np.cross(e, X[2] - X[0]); n2 = np.cross(X[3] - X[0], e)
    c = np.clip(n1 @ n2 / np.linalg.norm(n1) / np.linalg.norm(n2), -1, 1)
    return math.copysign(math.acos(c), np.cross(n1, n2) @ e)


@pytest.mark.parametrize("phi", [-2.5, -0.7, -0.01, 0.0, 0.3, 1.2, 2.9])
def test_bending_hinge_angle_closed_form(phi):
    abar, th0 = 1.5, 0.2
    kb, ht = BEND_PRM
    R = random_rotation()
    X = hinge(phi, R, RNG.normal(size=3))
    f, g, H = O.element(O.BENDING, X.ravel(), [abar, th0], BEND_PRM)
    assert f == pytest.approx(kb * abar / 3 * (phi - th0) ** 2 * ht * ht, rel=1e-12)
    # rest data: the rest dihedral of the oracle equals the construction angle
    tris = np.array([[0, 1, 2], [1, 0, 3]], np.int32)
    topo = O.topology(tris, 4)
    assert topo.diamonds.tolist() == [[0, 1, 2, 3]]
    rd = O.rest_diamond(topo, tris, X)
    assert rd[0, 1] == pytest.approx(phi, abs=1e-13)
    A1 = 0.5 * np.linalg.norm(np.cross(X[1] - X[0], X[2] - X[0]))
    A2 = 0.5 * np.linalg.norm(np.cross(X[1] - X[0], X[3] - X[0]))
    assert rd[0, 0] == pytest.approx(0.5 * (A1 + A2), rel=1e-14)


def test_bending_wing_gradient_and_rank_one_at_rest_angle():
    kb, ht = BEND_PRM
    abar = 0.9
    R = random_rotation()
    X = hinge(0.8, R, RNG.normal(size=3))
    th = theta_acos(X)
    c = kb * abar / 3 * ht * ht
    # at theta == theta': zero energy, zero gradient, H = 2 c grad(theta) grad(theta)^T
    f, g, H = O.element(O.BENDING, X.ravel(), [abar, th], BEND_PRM)
    assert abs(f) < 1e-28 and np.max(np.abs(g)) < 1e-13
    gth = fd_grad(lambda x: theta_acos(x.reshape(4, 3)), X.ravel(), 1e-4)
    assert np.allclose(H, 2 * c * np.outer(gth, gth), atol=1e-8 * np.abs(H).max())
    # wing vertices: d theta / d x_wing = -n_hat / h (face unit normal over the wing's height)
    e = X[1] - X[0]
    for wing, n in ((2, np.cross(e, X[2] - X[0])), (3, np.cross(X[3] - X[0], e))):
        hgt = np.linalg.norm(n) / np.linalg.norm(e)
        assert np.allclose(gth[3 * wing:3 * wing + 3], -n / np.linalg.norm(n) / hgt, atol=1e-8)
    # away from the rest angle: gradient = 2 c (theta - theta') grad(theta)
    f, g, H = O.element(O.BENDING, X.ravel(), [abar, th - 0.25], BEND_PRM)
    assert np.allclose(g, 2 * c * 0.25 * gth, atol=1e-8 * np.abs(g).max())


def test_bending_fd_and_invariances():
    for _ in range(4):
        X = hinge(RNG.uniform(-2, 2), random_rotation()) + 0.1 * RNG.normal(size=(4, 3))
        rest = [0.7, 0.3]
        f, g, H = check_fd(O.BENDING, X.ravel(), rest, BEND_PRM, rtol=1e-6)
        gg = g.reshape(4, 3)
        assert np.allclose(gg.sum(0), 0, atol=1e-12 * np.abs(g).max())
        assert np.allclose(np.cross(X, gg).sum(0), 0, atol=1e-12 * np.abs(g).max())
        T = np.kron(np.ones(4), np.eye(3)).T   # translations
        assert np.max(np.abs(H @ T)) < 1e-11 * np.abs(H).max()


# ------------------------------------------------------------------ Sec. 7.2: symmetric Dirichlet
def test_symdir_identity_map_and_fd():
    P = np.array([[0.1, 0.0, 0], [1.2, 0.3, 0], [0.2, 0.9, 0]])
    rest = rest_of_tri(P)
    area = 0.5 * np.cross(P[1] - P[0], P[2] - P[0])[2]
    f, g, H = O.element(O.SYMDIR, P[:, :2].ravel(), rest)
    assert f == pytest.approx(4 * area, rel=1e-13)
    assert np.max(np.abs(g)) < 1e-12
    assert np.linalg.eigvalsh(H).min() > -1e-12 * np.abs(H).max()
    # J = diag(2, 1/2) scaled map: |J|^2 = 4.25, |J^-1|^2 = 4.25
    uv = P[:, :2] @ np.diag([2.0, 0.5])
    f, g, H = check_fd(O.SYMDIR, uv.ravel(), rest)
    assert f == pytest.approx(area * 8.5, rel=1e-13)
    uv = P[:, :2] + 0.2 * RNG.normal(size=(3, 2))
    f, g, H = check_fd(O.SYMDIR, uv.ravel(), rest)
    gg = g.reshape(3, 2)
    assert np.allclose(gg.sum(0), 0, atol=1e-12 * np.abs(g).max())
    th = 0.7
    Rm = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    f2, _, _ = O.element(O.SYMDIR, (uv @ Rm.T + [3, -1]).ravel(), rest)
    assert f2 == pytest.approx(f, rel=1e-12)


def test_stvk_fd_large_deformation():
    P = np.array([[0, 0, 0], [1.0, 0.1, 0], [0.2, 0.9, 0]])
    rest = rest_of_tri(P)
    for _ in range(4):
        x = P + 0.4 * RNG.normal(size=(3, 3))
        check_fd(O.STVK, x.ravel(), rest, STVK_PRM)


# ------------------------------------------------------------------ Sec. 7.1 filtering: eigen-clamp
def eigh_clamp(A, eps):
    w, V = np.linalg.eigh(0.5 * (A + A.T))
    return (V * np.maximum(w, eps)) @ V.T


@pytest.mark.parametrize("n", [2, 3, 6, 9, 12])
def test_spd_projection_matches_lapack(n):
    for eps in (0.0, 1e-3):
        A = RNG.normal(size=(n, n))
        A = A + A.T
        P = O.spd_project(A, eps)
        Pl = eigh_clamp(A, eps)
        assert np.allclose(P, Pl, atol=1e-13 * np.abs(A).max())
        assert np.linalg.eigvalsh(P).min() >= eps - 1e-12 * np.abs(A).max()
        assert np.allclose(O.spd_project(P, eps), P, atol=1e-13 * np.abs(A).max())


def test_spd_projection_leaves_psd_unchanged_and_handles_repeated_eigs():
    B = RNG.normal(size=(9, 5))
    A = B @ B.T                                   # PSD, rank 5 (4 zero eigenvalues)
    assert np.allclose(O.spd_project(A, 0.0), A, atol=1e-13 * np.abs(A).max())
    Q, _ = np.linalg.qr(RNG.normal(size=(12, 12)))
    A = Q @ np.diag([-2, -2, -2, 1, 1, 1, 0, 0, 3, 3, -1e-9, 5.0]) @ Q.T
    assert np.allclose(O.spd_project(A, 0.0), eigh_clamp(A, 0.0), atol=1e-13 * 5)
    assert np.all(O.spd_project(np.zeros((4, 4)), 0.0) == 0)


def test_element_spd_mode_equals_projection_of_raw_hessian():
    X = hinge(1.0) + 0.05 * RNG.normal(size=(4, 3))
    _, _, H = O.element(O.BENDING, X.ravel(), [0.5, -0.4], BEND_PRM)
    _, _, Hp = O.element(O.BENDING, X.ravel(), [0.5, -0.4], BEND_PRM, mode=O.ENERGY | O.GRAD | O.HESS | O.SPD)
    assert np.linalg.eigvalsh(H).min() < 0          # the raw bending Hessian is indefinite here
    assert np.allclose(Hp, eigh_clamp(H, 0.0), atol=1e-13 * np.abs(H).max())
