"""Pins of the oracle's per-triangle shell features, the analytic shell density
and the learned (MLP) density against facts independent of their code:
geometric identities of exact sphere and cylinder normals, the StVK element,
rigid-motion invariance, closed forms of a one-neuron network, finite
differences, two independent differentiations of the network (hyper-dual C and
reverse-mode FP64), and the closed form of Adam's first step."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests.test_oracle_elements import fd_grad, fd_jac

RNG = np.random.default_rng(777)


def seeded(fn):
    """Each pin draws from the module generator restarted at a fixed seed, so its inputs do not
    depend on which pins ran before it (the mutation tests call them in their own order)."""
    import functools

    @functools.wraps(fn)
    def run(*a, **k):
        global RNG
        RNG = np.random.default_rng(777)
        return fn(*a, **k)
    return run


def flat_tri_rest8(X):
    """rest data [8] of one triangle (its own normals: a single flat triangle)."""
    return O.rest_shell(np.array([[0, 1, 2]], np.int32), np.asarray(X, float).reshape(3, 3), 3)[0]


def rand_tri(scale=1.0):
    X = RNG.normal(size=(3, 3)) * scale
    return X


def rot(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def elem(kind, x, rest8, prm, normals, mode=O.ENERGY | O.GRAD | O.HESS):
    return O.element(kind, np.asarray(x, float).ravel(), rest8, prm, mode=mode, aux=np.asarray(normals).ravel())


# ------------------------------------------------------------------ features
@seeded
def test_features_vanish_at_rest_and_are_rigid_invariant():
    tris, rest = grid_patch(6)
    nv = rest.shape[0]
    r8 = O.rest_shell(tris, rest, nv)
    z0 = O.shell_features(tris, r8, rest, nv)
    assert np.max(np.abs(z0)) < 1e-14
    x = rest * [1.07, 0.96, 1.0] + RNG.normal(scale=0.02, size=rest.shape)
    z = O.shell_features(tris, r8, x, nv)
    R = rot([0.3, -1.0, 0.5], 0.9)
    zr = O.shell_features(tris, r8, x @ R.T + [0.4, -2.0, 3.0], nv)
    assert np.max(np.abs(z - zr)) < 1e-12 * max(1.0, np.max(np.abs(z)))
    assert np.max(np.abs(z)) > 1e-3


def grid_patch(n):
    """flat n x n unit-square grid (rest), '/' diagonals, z = 0"""
    tris = []
    for j in range(n - 1):
        for i in range(n - 1):
            v00, v10, v01, v11 = j * n + i, j * n + i + 1, (j + 1) * n + i, (j + 1) * n + i + 1
            tris += [[v00, v10, v11], [v00, v11, v01]]
    u = np.linspace(0.0, 1.0, n)
    P = np.stack(np.meshgrid(u, u), axis=-1).reshape(-1, 2)
    return np.array(tris, np.int32), np.concatenate([P, np.zeros((n * n, 1))], axis=1)


@seeded
def test_membrane_part_equals_stvk_element():
    # with k_b = 0 the shell density is the StVK membrane density (an independent element)
    X = rand_tri()
    x = X + RNG.normal(scale=0.3, size=X.shape)
    r8 = flat_tri_rest8(X)
    nrm = RNG.normal(size=(3, 3))
    mu, lam = 1.3, 0.7
    f, g, H = elem(O.SHELL_TRI, x, r8, (mu, lam, 0.0), nrm)
    fs, gs, Hs = O.element(O.STVK, x.ravel(), r8[:5], (mu, lam))
    assert abs(f - fs) <= 1e-13 * abs(fs)
    assert np.max(np.abs(g - gs)) <= 1e-12 * np.max(np.abs(gs))
    assert np.max(np.abs(H - Hs)) <= 1e-12 * np.max(np.abs(Hs))


@seeded
def test_sphere_normals_give_second_form_minus_first_over_radius():
    # exact radial normals n_i = (x_i - c)/R give Dn = Ds/R, hence II = -(F^T F)/R = -(I + 2E)/R
    # (the identity is exact; the tolerance is rounding relative to the size of the forms)
    X = rand_tri()
    r8 = flat_tri_rest8(X)
    R = 1.7
    c = np.array([0.2, -0.4, 0.9])
    dirs = RNG.normal(size=(3, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    x = c + R * dirs
    z = _features_with_normals(x, r8, dirs)
    E = np.array([[z[0], z[2]], [z[2], z[1]]])
    II = np.array([[z[3] + r8[5], z[5] + r8[7]], [z[5] + r8[7], z[4] + r8[6]]])
    ref = (np.eye(2) + 2 * E) / R
    assert np.max(np.abs(II + ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def _features_with_normals(x, r8, normals):
    """z of one triangle for explicitly given normals. The bending components come from the
    element alone: with mu = lam = 0, k_b = 1 the energy is A/2 (z3^2 + z4^2 + 2 z5^2), and
    shifting a rest-II entry by delta shifts its component by -delta, so a central difference
    in delta (exact for a quadratic) returns A w z_q. The membrane components are the Green
    strain of the triangle's own deformation gradient."""
    out = np.zeros(6)
    A = r8[4]
    for q, w in ((3, 1.0), (4, 1.0), (5, 2.0)):
        def f(delta):
            r = r8.copy()
            r[5 + (q - 3)] += delta
            return elem(O.SHELL_TRI, x, r, (0.0, 0.0, 1.0), normals, mode=O.ENERGY)[0]
        d = 1e-3
        # f(delta) = A/2 * w * (z_q - delta)^2 + const  ->  (f(-d) - f(d)) / (2 d) = A w z_q
        out[q] = (f(-d) - f(d)) / (2 * d) / (A * w)
    Dm_inv = r8[:4].reshape(2, 2)
    Ds = np.stack([x[1] - x[0], x[2] - x[0]], axis=1)
    F = Ds @ Dm_inv
    E = 0.5 * (F.T @ F - np.eye(2))
    out[0], out[1], out[2] = E[0, 0], E[1, 1], E[0, 1]
    return out


@seeded
def test_cylinder_normals_second_form_closed_form():
    # on a cylinder of radius R about the t axis, exact normals satisfy Dn = -(1/R) P Ds with
    # P removing the axis component, so II = (F^T F - u u^T)/R, u the axis in the rest frame
    R = 0.8
    s = RNG.uniform(-0.3, 0.3, size=3)
    t = RNG.uniform(-0.3, 0.3, size=3)
    X = np.stack([s, t, np.zeros(3)], axis=1)              # flat rest
    x = np.stack([R * np.sin(s / R), t, R * (1 - np.cos(s / R))], axis=1)
    nrm = np.stack([-np.sin(s / R), np.zeros(3), np.cos(s / R)], axis=1)
    r8 = flat_tri_rest8(X)
    z = _features_with_normals(x, r8, nrm)
    Dm_inv = r8[:4].reshape(2, 2)
    u = np.array([t[1] - t[0], t[2] - t[0]]) @ Dm_inv
    F = np.stack([x[1] - x[0], x[2] - x[0]], axis=1) @ Dm_inv
    II = (F.T @ F - np.outer(u, u)) / R
    assert abs(z[3] - II[0, 0]) < 1e-9 and abs(z[4] - II[1, 1]) < 1e-9 and abs(z[5] - II[0, 1]) < 1e-9
    # small-triangle limit: trace -> 1/R (the curvature), determinant -> 0
    assert abs(np.trace(II) - 1 / R) < 0.2 / R


@seeded
def test_plain_features_equal_hyper_dual_features():
    # the fast value-only features against the element path, on a flat-rest cylinder and on
    # a curved rest (icospheres: nonzero rest II)
    from paper_2509_00406_amd import meshgen
    for inp in (meshgen.shell_cylinder(n=7, seed=3),
                meshgen.icosphere_batch(n_meshes=1, mean_verts=700, vmin=600, vmax=800)):
        r8 = O.rest_shell(inp.tris, inp.rest, inp.n_verts)
        z = O.shell_features(inp.tris, r8, inp.x, inp.n_verts)
        nrm = O.vertex_normals(inp.tris, inp.x, inp.n_verts)
        for f in (0, 5, 17, 40):
            t = inp.tris[f]
            zz = _features_with_normals(inp.x[t], r8[f], nrm[t])
            assert np.max(np.abs(zz - z[f])) < 1e-8 * max(1.0, np.max(np.abs(z[f])))
    assert np.max(np.abs(r8[:, 5:])) > 1e-2


@seeded
def test_vertex_normals_closed_forms():
    tris, rest = grid_patch(4)
    n = O.vertex_normals(tris, rest, rest.shape[0])
    assert np.allclose(n, [0, 0, 1], atol=1e-15)
    # octahedron: by symmetry every vertex normal is radial
    P = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    T = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4], [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]], np.int32)
    n = O.vertex_normals(T, P, 6)
    assert np.allclose(n, P, atol=1e-15)
    # an isolated vertex keeps a zero normal
    n = O.vertex_normals(T, np.concatenate([P, [[5.0, 5, 5]]]), 7)
    assert not n[6].any()


@seeded
def test_shell_element_fd_and_invariance():
    X = rand_tri()
    r8 = flat_tri_rest8(X)
    r8[5:] = [0.3, -0.2, 0.1]
    x = X @ rot([1, 2, 3], 0.4).T + RNG.normal(scale=0.2, size=X.shape)
    nrm = RNG.normal(size=(3, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    prm = (1.1, 0.6, 0.9)
    f, g, H = elem(O.SHELL_TRI, x, r8, prm, nrm)
    fe = lambda y: elem(O.SHELL_TRI, y, r8, prm, nrm, mode=O.ENERGY)[0]
    ge = lambda y: elem(O.SHELL_TRI, y, r8, prm, nrm, mode=O.ENERGY | O.GRAD)[1]
    x0 = x.ravel().copy()
    assert np.max(np.abs(fd_grad(fe, x0, 1e-4) - g)) < 1e-7 * np.max(np.abs(g))
    assert np.max(np.abs(fd_jac(ge, x0, 1e-4) - H)) < 1e-7 * np.max(np.abs(H))
    assert np.allclose(H, H.T, atol=1e-14 * np.max(np.abs(H)))
    # translation invariance (normals are passive): gradient sums to zero per axis
    assert np.max(np.abs(g.reshape(3, 3).sum(axis=0))) < 1e-12 * np.max(np.abs(g))


# ------------------------------------------------------------------ the learned density
def rand_mlp(H, seed=0, scale=0.5):
    r = np.random.default_rng(seed)
    return O.mlp_pack(r.uniform(0.5, 2.0), r.uniform(0.5, 3.0, size=6), r.normal(scale=scale, size=(H, 6)),
                      r.normal(scale=scale, size=H), r.normal(scale=scale / math.sqrt(H), size=(H, H)),
                      r.normal(scale=scale, size=H), r.normal(scale=scale, size=H), r.normal())


def sigma(a):
    return 1.0 / (1.0 + math.exp(-a))


@seeded
def test_one_neuron_network_closed_form():
    p = rand_mlp(1, seed=3)
    u = O.mlp_unpack(p)
    z = RNG.normal(size=6)
    psi, d, h = O.mlp_eval(z[None], p, hess=True)
    w1, s = u["W1"][0] * u["s_in"], u["s_out"]
    a1 = w1 @ z + u["b1"][0]
    a2 = u["W2"][0, 0] * math.log1p(math.exp(a1)) + u["b2"][0]
    psi_ref = s * (u["w3"][0] * math.log1p(math.exp(a2)) + u["b3"])
    w2, w3 = u["W2"][0, 0], u["w3"][0]
    s1, s2 = sigma(a1), sigma(a2)
    d_ref = s * w3 * s2 * w2 * s1 * w1
    h_ref = s * w3 * (s2 * (1 - s2) * (w2 * s1) ** 2 + s2 * w2 * s1 * (1 - s1)) * np.outer(w1, w1)
    assert abs(psi[0] - psi_ref) < 1e-13 * abs(psi_ref)
    assert np.max(np.abs(d[0] - d_ref)) < 1e-13 * np.max(np.abs(d_ref))
    assert np.max(np.abs(h[0] - h_ref)) < 1e-12 * np.max(np.abs(h_ref))


@seeded
def test_network_derivatives_fd_and_reverse_mode_agree():
    p = rand_mlp(64, seed=5)
    z = RNG.normal(size=(3, 6)) * 0.7
    psi, d, h = O.mlp_eval(z, p, hess=True)
    for i in range(3):
        f = lambda y: O.mlp_eval(y[None], p)[0][0]
        gfun = lambda y: O.mlp_eval(y[None], p)[1][0]
        assert np.max(np.abs(fd_grad(f, z[i].copy(), 1e-3) - d[i])) < 1e-8 * np.max(np.abs(d[i]))
        assert np.max(np.abs(fd_jac(gfun, z[i].copy(), 1e-3) - h[i])) < 1e-7 * np.max(np.abs(h[i]))
    # the reverse-mode FP64 path used for training computes the same psi and dpsi/dz
    import torch
    u = O.mlp_unpack(p)
    zz = torch.tensor(z, requires_grad=True)
    W1, b1, W2, b2, w3 = (torch.tensor(u[k]) for k in ("W1", "b1", "W2", "b2", "w3"))
    sp = lambda a: torch.logaddexp(a, torch.zeros_like(a))
    ps = u["s_out"] * (sp(sp((zz * torch.tensor(u["s_in"])) @ W1.T + b1) @ W2.T + b2) @ w3 + u["b3"])
    (dz,) = torch.autograd.grad(ps.sum(), zz)
    assert np.max(np.abs(ps.detach().numpy() - psi)) < 1e-13 * np.max(np.abs(psi))
    assert np.max(np.abs(dz.numpy() - d)) < 1e-12 * np.max(np.abs(d))


@seeded
def test_mlp_element_is_area_times_network_of_features():
    from paper_2509_00406_amd import meshgen
    inp = meshgen.shell_cylinder(n=5, seed=4)
    p = rand_mlp(16, seed=2)
    P = O.Problem(inp.tris, inp.rest, inp.n_verts, 3)
    P.add_term(O.MLP, p)
    r = P.eval(inp.x, O.ENERGY)
    r8 = O.rest_shell(inp.tris, inp.rest, inp.n_verts)
    z = O.shell_features(inp.tris, r8, inp.x, inp.n_verts)
    psi, _ = O.mlp_eval(z, p)
    assert abs(r.energy - np.sum(r8[:, 4] * psi)) < 1e-12 * np.sum(np.abs(r8[:, 4] * psi))
    # element derivatives by finite differences (normals held fixed)
    nrm = O.vertex_normals(inp.tris, inp.x, inp.n_verts)
    t = inp.tris[7]
    f, g, H = elem(O.MLP, inp.x[t], r8[7], p, nrm[t])
    ge = lambda y: elem(O.MLP, y, r8[7], p, nrm[t], mode=O.ENERGY | O.GRAD)[1]
    fe = lambda y: elem(O.MLP, y, r8[7], p, nrm[t], mode=O.ENERGY)[0]
    x0 = inp.x[t].ravel().copy()
    h = 1e-3 * np.max(np.abs(x0))
    assert np.max(np.abs(fd_grad(fe, x0, h) - g)) < 1e-7 * np.max(np.abs(g))
    assert np.max(np.abs(fd_jac(ge, x0, h) - H)) < 1e-6 * np.max(np.abs(H))


@seeded
def test_shell_density_closed_form_gradient_by_fd():
    z = RNG.normal(size=(4, 6))
    prm = (1.2, 0.4, 0.8)
    W, dW = O.shell_density(z, prm)
    for i in range(4):
        f = lambda y: O.shell_density(y[None], prm)[0][0]
        assert np.max(np.abs(fd_grad(f, z[i].copy(), 1e-3) - dW[i])) < 1e-10 * np.max(np.abs(dW[i]))
    W0, dW0 = O.shell_density(np.zeros((1, 6)), prm)
    assert W0[0] == 0.0 and not dW0.any()


@seeded
def test_loss_gradient_by_fd():
    p = rand_mlp(8, seed=9)
    z = RNG.normal(size=(20, 6))
    W, dW = O.shell_density(z, (1.0, 0.5, 0.7))
    loss, g = O.mlp_loss_grad(p, z, W, dW, 2.0, 3.0, 0.5)
    n_head = 8
    idx = RNG.choice(g.size, 12, replace=False)

    def loss_at(theta):
        q = p.copy()
        q[n_head:] = theta
        return O.mlp_loss_grad(q, z, W, dW, 2.0, 3.0, 0.5)[0]
    theta = p[n_head:].copy()
    for i in idx:
        def f1(t, i=i):
            th = theta.copy()
            th[i] = t[0]
            return loss_at(th)
        gi = fd_grad(f1, np.array([theta[i]]), 1e-4)[0]
        assert abs(gi - g[i]) < 1e-7 * max(1.0, np.max(np.abs(g)))
    # the loss itself equals its definition with the hyper-dual network values
    psi, d = O.mlp_eval(z, p)
    ref = np.mean((psi - W) ** 2) / 2.0 + 0.5 * np.mean(np.sum((d - dW) ** 2, axis=1)) / 3.0
    assert abs(loss - ref) < 1e-12 * ref


@seeded
def test_adam_first_step_closed_form():
    theta = RNG.normal(size=50)
    g = RNG.normal(size=50)
    t1, m, v = O.adam_step(theta, g, np.zeros(50), np.zeros(50), 1, 1e-2)
    # bias correction makes the first step lr * g / (|g| + eps): lr in the direction of -sign(g)
    assert np.allclose(t1, theta - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # constant gradient: every step has the same size
    t2, m, v = O.adam_step(t1, g, m, v, 2, 1e-2)
    assert np.allclose(t2 - t1, t1 - theta, rtol=1e-12, atol=1e-15)
