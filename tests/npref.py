"""Independent vectorised FP64 energies (numpy) for full-size energy checks.

The oracle evaluates elements one by one through hyper-duals, which takes
minutes for millions of elements in passive mode; these plain formulas give
the total energy of the large workloads in seconds. They are a second,
separately written statement of the same energies (pinned against the
oracle on small meshes in test_npref.py), not a copy of either path.
"""
from __future__ import annotations

import math

import numpy as np


def rest_frames(tris, rest):
    """Per-triangle inverse rest shape matrix (2x2) in the triangle's own frame, and rest area."""
    a, b, c = rest[tris[:, 0]], rest[tris[:, 1]], rest[tris[:, 2]]
    e1, e2 = b - a, c - a
    n = np.cross(e1, e2)
    l1 = np.linalg.norm(e1, axis=1)
    nn = np.linalg.norm(n, axis=1)
    Dm = np.zeros((tris.shape[0], 2, 2))
    Dm[:, 0, 0] = l1
    Dm[:, 0, 1] = np.einsum("ij,ij->i", e1, e2) / l1
    Dm[:, 1, 1] = nn / l1
    return np.linalg.inv(Dm), 0.5 * nn


def stvk_energies(tris, rest, x, mu, lam):
    Minv, area = rest_frames(tris, rest)
    Ds = np.stack([x[tris[:, 1]] - x[tris[:, 0]], x[tris[:, 2]] - x[tris[:, 0]]], axis=2)   # [T,3,2]
    F = Ds @ Minv
    E = 0.5 * (np.transpose(F, (0, 2, 1)) @ F - np.eye(2))
    tr = E[:, 0, 0] + E[:, 1, 1]
    tr2 = np.einsum("tij,tji->t", E, E)
    return area * (mu * tr2 + 0.5 * lam * tr * tr)


def dihedral(x, d):
    x0, x1, x2, x3 = (x[d[:, k]] for k in range(4))
    e = x1 - x0
    n1 = np.cross(e, x2 - x0)
    n2 = np.cross(x3 - x0, e)
    y = np.einsum("ij,ij->i", np.cross(n1, n2), e) / np.linalg.norm(e, axis=1)
    return np.arctan2(y, np.einsum("ij,ij->i", n1, n2))


def bending_energies(tris, rest, x, diamonds, diamond_faces, kb, ht):
    _, area = rest_frames(tris, rest)
    abar = 0.5 * (area[diamond_faces[:, 0]] + area[diamond_faces[:, 1]])
    th0 = dihedral(rest, diamonds)
    th = dihedral(x, diamonds)
    return kb * abar / 3.0 * (th - th0) ** 2 * ht * ht


def shell_energy(tris, rest, x, diamonds, diamond_faces, stvk_prm, bend_prm):
    fs = stvk_energies(tris, rest, x, *stvk_prm)
    fb = bending_energies(tris, rest, x, diamonds, diamond_faces, *bend_prm)
    return math.fsum(fs) + math.fsum(fb), float(np.abs(fs).sum() + np.abs(fb).sum())


def cloth_energy(tris, rest, x, vdata, spring_params, inertia_params):
    """Mass-spring time-step energy (Sec. 7.1): springs over the unique mesh edges plus inertia and
    gravity per vertex. Returns (total, sum of |element energies|)."""
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]]).astype(np.int64)
    e.sort(axis=1)
    nv = rest.shape[0]
    e = np.unique(e[:, 0] * nv + e[:, 1])
    i, j = e // nv, e % nv
    k, w = spring_params
    l2 = np.sum((rest[i] - rest[j]) ** 2, axis=1)
    d = x[i] - x[j]
    q = np.sum(d * d, axis=1) / l2 - 1.0
    fs = w * 0.5 * k * l2 * q * q
    wg, gx, gy, gz = inertia_params
    m, xh = vdata[:, 0], vdata[:, 1:]
    fv = 0.5 * m * np.sum((x - xh) ** 2, axis=1) - wg * m * (x @ np.array([gx, gy, gz]))
    return math.fsum(fs) + math.fsum(fv), float(np.sum(np.abs(fs)) + np.sum(np.abs(fv)))


def component_of_triangles(tris, comp_offsets):
    """Component index of every triangle (meshes of disjoint components)."""
    return np.searchsorted(np.asarray(comp_offsets), tris[:, 0], side="right") - 1


def shell_energy_by_component(tris, rest, x, diamonds, diamond_faces, stvk_prm, bend_prm, comp_offsets):
    """Per-component totals and |element|-sums of the StVK + bending energy (component of a diamond = that
    of its first face). Returns (energies [C], abs sums [C])."""
    fs = stvk_energies(tris, rest, x, *stvk_prm)
    fb = bending_energies(tris, rest, x, diamonds, diamond_faces, *bend_prm)
    ct = component_of_triangles(tris, comp_offsets)
    cd = ct[diamond_faces[:, 0]]
    nc = len(comp_offsets) - 1
    e = np.zeros(nc)
    s = np.zeros(nc)
    order_t = np.argsort(ct, kind="stable")
    order_d = np.argsort(cd, kind="stable")
    bt = np.searchsorted(ct[order_t], np.arange(nc + 1))
    bd = np.searchsorted(cd[order_d], np.arange(nc + 1))
    for c in range(nc):
        a = fs[order_t[bt[c]:bt[c + 1]]]
        b = fb[order_d[bd[c]:bd[c + 1]]]
        e[c] = math.fsum(a) + math.fsum(b)
        s[c] = float(np.abs(a).sum() + np.abs(b).sum())
    return e, s


def symdir_energies(tris, rest, uv):
    """Symmetric Dirichlet A (|J|_F^2 + |J^-1|_F^2) per triangle, J the 2x2 map from the planar rest
    triangle (its first two coordinates) to the UV triangle."""
    p = rest[:, :2]
    Dm = np.stack([p[tris[:, 1]] - p[tris[:, 0]], p[tris[:, 2]] - p[tris[:, 0]]], axis=2)   # [T,2,2]
    Ds = np.stack([uv[tris[:, 1]] - uv[tris[:, 0]], uv[tris[:, 2]] - uv[tris[:, 0]]], axis=2)
    J = Ds @ np.linalg.inv(Dm)
    Ji = np.linalg.inv(J)
    area = 0.5 * np.abs(np.linalg.det(Dm))
    return area * (np.sum(J * J, axis=(1, 2)) + np.sum(Ji * Ji, axis=(1, 2)))


def symdir_energy(tris, rest, uv):
    f = symdir_energies(tris, rest, uv)
    return math.fsum(f), float(np.abs(f).sum())


def unit_vertex_normals(tris, x):
    """Area-weighted unit vertex normals: normalised sums of the incident face cross products."""
    n = np.cross(x[tris[:, 1]] - x[tris[:, 0]], x[tris[:, 2]] - x[tris[:, 0]])
    acc = np.zeros_like(x)
    for a in range(3):
        np.add.at(acc, tris[:, a], n)
    ln = np.linalg.norm(acc, axis=1, keepdims=True)
    return np.divide(acc, ln, out=np.zeros_like(acc), where=ln > 0)


def shell_features(tris, rest, x):
    """Per-triangle features (E00, E11, E01, dII00, dII11, dII01) and rest areas: Green strain of
    F = Ds Dm^-1 in the triangle's rest frame, II = -(N^T F + F^T N)/2 with N = [n_b - n_a, n_c - n_a] Dm^-1
    from the unit vertex normals, minus the same form on the rest mesh."""
    Minv, area = rest_frames(tris, rest)

    def second_form(pos):
        nrm = unit_vertex_normals(tris, pos)
        F = np.stack([pos[tris[:, 1]] - pos[tris[:, 0]], pos[tris[:, 2]] - pos[tris[:, 0]]], axis=2) @ Minv
        N = np.stack([nrm[tris[:, 1]] - nrm[tris[:, 0]], nrm[tris[:, 2]] - nrm[tris[:, 0]]], axis=2) @ Minv
        NF = np.transpose(N, (0, 2, 1)) @ F
        return F, -0.5 * (NF + np.transpose(NF, (0, 2, 1)))

    F, II = second_form(x)
    _, II0 = second_form(rest)
    E = 0.5 * (np.transpose(F, (0, 2, 1)) @ F - np.eye(2))
    dII = II - II0
    z = np.stack([E[:, 0, 0], E[:, 1, 1], E[:, 0, 1], dII[:, 0, 0], dII[:, 1, 1], dII[:, 0, 1]], axis=1)
    return z, area


def mlp_energy(tris, rest, x, theta, s_in, s_out, hidden=64):
    """Learned density sum_t A_t psi(z_t), psi(z) = s_out (w3 . sp(W2 sp(W1 (s_in z) + b1) + b2) + b3),
    sp(a) = log(1 + e^a), with the packed parameters theta (W1, b1, W2, b2, w3, b3) in FP64."""
    t = np.asarray(theta, np.float64)
    H = hidden
    W1, b1 = t[:6 * H].reshape(H, 6), t[6 * H:7 * H]
    W2, b2 = t[7 * H:7 * H + H * H].reshape(H, H), t[7 * H + H * H:8 * H + H * H]
    w3, b3 = t[8 * H + H * H:9 * H + H * H], t[9 * H + H * H]
    z, area = shell_features(tris, rest, x)
    h1 = np.logaddexp(0.0, (z * np.asarray(s_in, np.float64)) @ W1.T + b1)
    h2 = np.logaddexp(0.0, h1 @ W2.T + b2)
    f = area * (float(s_out) * (h2 @ w3 + b3))
    return math.fsum(f), float(np.abs(f).sum())
