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
