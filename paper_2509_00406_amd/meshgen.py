"""Seeded synthetic inputs: triangle meshes, rest positions and DOF vectors.

This module only draws inputs. It holds none of the method's arithmetic (no
topology, no rest-frame data, no energies or derivatives): both the HIP path
and the CPU oracle receive exactly these arrays and derive everything else on
their own.

The paper measures on meshes that are not available here (its cow, brain,
parameterisation and polyvector meshes), so every workload is synthetic with
the shapes and sizes of the evaluated scenes:

* ``grid``            n x n vertex grid on the unit square, every square split
                      along the same "/" diagonal, counter-clockwise faces.
* ``dirichlet_grid``  jittered planar grid + a random scalar field (a scalar
                      Dirichlet energy workload; 64 x 64 vertices by default).
* ``shell_cylinder``  flat rest grid rolled into a half cylinder plus Gaussian
                      displacement noise (the elastic-shell workload of the
                      paper's shell simulation, Sec. 7.7, at 1024 x 1024).
* ``warped_grid``     flat rest grid with UVs moved by a sum of 8 seeded
                      sinusoids (parameterisation workload, Sec. 7.2).
* ``icosphere_batch`` hundreds of geodesic icospheres of lognormal size as
                      disjoint components of one mesh (the many-body shell
                      scene of Sec. 7.7).
* ``cloth``           mass-spring cloth time step (Sec. 7.1, Table 1 sizes
                      10^2 ... 1000^2 vertices): flat rest grid, a current
                      state moved by smooth seeded waves (springs both
                      stretched and compressed), smooth velocities, uniform
                      lumped masses and gravity.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class MeshInput:
    """A triangle mesh with rest positions and a DOF vector.

    tris      int32 [T, 3]  counter-clockwise vertex indices
    rest      float64 [V, 3] rest positions (z = 0 for planar rests)
    x         float64 [V, var_dim] current DOFs (positions, a scalar field or UVs)
    comp_offsets int64 [C+1] vertex offsets of disjoint components (batched meshes)
    """

    tris: np.ndarray
    rest: np.ndarray
    x: np.ndarray
    var_dim: int
    comp_offsets: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n_verts(self) -> int:
        return int(self.rest.shape[0])

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])


def grid(n: int) -> tuple[np.ndarray, np.ndarray]:
    """n x n vertex grid on [0,1]^2; vertex (i, j) has index j*n + i.

    Square (i, j) is split into (v00, v10, v11) and (v00, v11, v01), both
    counter-clockwise. Returns (tris int32 [2(n-1)^2, 3], pos float64 [n^2, 3]).
    """
    if n < 2:
        raise ValueError("grid needs n >= 2")
    h = 1.0 / (n - 1)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    pos = np.zeros((n * n, 3), dtype=np.float64)
    pos[:, 0] = (ii.ravel()) * h
    pos[:, 1] = (jj.ravel()) * h
    i = np.arange(n - 1)
    j = np.arange(n - 1)
    I, J = np.meshgrid(i, j, indexing="xy")
    v00 = (J * n + I).ravel()
    v10 = v00 + 1
    v01 = v00 + n
    v11 = v01 + 1
    tris = np.empty((2 * (n - 1) * (n - 1), 3), dtype=np.int32)
    tris[0::2, 0] = v00
    tris[0::2, 1] = v10
    tris[0::2, 2] = v11
    tris[1::2, 0] = v00
    tris[1::2, 1] = v11
    tris[1::2, 2] = v01
    return tris, pos


def dirichlet_grid(n: int = 64, jitter_seed: int = 1001, field_seed: int = 1002,
                   jitter: float = 0.2) -> MeshInput:
    """Jittered planar grid with a scalar field u ~ N(0, 1) per vertex.

    Every vertex moves by U[-jitter*h, jitter*h] per in-plane coordinate; with
    jitter = 0.2 every triangle keeps a positive area of at least 0.1 h^2.
    """
    tris, pos = grid(n)
    h = 1.0 / (n - 1)
    rng = np.random.default_rng(jitter_seed)
    pos[:, :2] += rng.uniform(-jitter * h, jitter * h, size=(pos.shape[0], 2))
    u = np.random.default_rng(field_seed).standard_normal((pos.shape[0], 1))
    return MeshInput(tris, pos, u, 1, meta=dict(workload="dirichlet_grid", n=n,
                                                 jitter_seed=jitter_seed, field_seed=field_seed))


def roll_cylinder(pos: np.ndarray, radius: float) -> np.ndarray:
    """Map the planar point (s, t, 0) to (R sin(s/R), t, R (1 - cos(s/R)))."""
    s = pos[:, 0]
    t = pos[:, 1]
    out = np.empty_like(pos)
    out[:, 0] = radius * np.sin(s / radius)
    out[:, 1] = t
    out[:, 2] = radius * (1.0 - np.cos(s / radius))
    return out


def shell_cylinder(n: int = 1024, seed: int = 2001, noise: str = "relative",
                   radius: float = 1.0 / math.pi) -> MeshInput:
    """Flat n x n rest grid rolled into a half cylinder, plus N(0, sigma^2) noise.

    noise = "relative": sigma = 1e-3 * h (small-strain shell, the default).
    noise = "absolute": sigma = 1e-3 (about one edge length at n = 1024; yields
    near-degenerate and inverted elements; used as a stress input).
    """
    tris, rest = grid(n)
    h = 1.0 / (n - 1)
    x = roll_cylinder(rest, radius)
    if noise == "relative":
        sigma = 1e-3 * h
    elif noise == "absolute":
        sigma = 1e-3
    else:
        raise ValueError(noise)
    x += np.random.default_rng(seed).normal(0.0, sigma, size=x.shape)
    return MeshInput(tris, rest, x, 3, meta=dict(workload="shell_cylinder", n=n, seed=seed,
                                                   noise=noise, sigma=sigma, radius=radius))


def warped_grid(n: int = 1001, seed: int = 3001, n_waves: int = 8,
                total_amplitude: float = 0.1) -> MeshInput:
    """Flat n x n rest grid; UV = p + sum_k a_k sin(2 pi f_k . p + phi_k).

    a_k = (total_amplitude / n_waves) (cos b_k, sin b_k), f_k = r_k (cos g_k, sin g_k)
    with r_k ~ U[0.5, 1], b_k, g_k, phi_k ~ U[0, 2 pi). The warp's Lipschitz
    constant stays below 1, so no UV triangle flips (checked by signed area).
    """
    tris, rest = grid(n)
    rng = np.random.default_rng(seed)
    beta = rng.uniform(0.0, 2 * math.pi, n_waves)
    gamma = rng.uniform(0.0, 2 * math.pi, n_waves)
    phi = rng.uniform(0.0, 2 * math.pi, n_waves)
    rho = rng.uniform(0.5, 1.0, n_waves)
    amp = total_amplitude / n_waves
    p = rest[:, :2]
    uv = p.copy()
    for k in range(n_waves):
        a = amp * np.array([math.cos(beta[k]), math.sin(beta[k])])
        f = rho[k] * np.array([math.cos(gamma[k]), math.sin(gamma[k])])
        uv += np.outer(np.sin(2 * math.pi * (p @ f) + phi[k]), a)
    a_, b_, c_ = uv[tris[:, 0]], uv[tris[:, 1]], uv[tris[:, 2]]
    signed2 = (b_[:, 0] - a_[:, 0]) * (c_[:, 1] - a_[:, 1]) - (b_[:, 1] - a_[:, 1]) * (c_[:, 0] - a_[:, 0])
    if not np.all(signed2 > 0):
        raise RuntimeError("warp flipped a triangle")
    return MeshInput(tris, rest, uv, 2, meta=dict(workload="warped_grid", n=n, seed=seed))


def _waves(p: np.ndarray, rng, n_waves: int, amplitude: float, dim: int) -> np.ndarray:
    """sum_k a_k sin(2 pi f_k . p + phi_k): a_k ~ amplitude/n_waves * unit vector in R^dim,
    f_k = r_k (cos g_k, sin g_k), r_k ~ U[0.5, 2], over the 2D points p."""
    out = np.zeros((p.shape[0], dim))
    for _ in range(n_waves):
        a = rng.normal(size=dim)
        a *= amplitude / n_waves / np.linalg.norm(a)
        g, r, phi = rng.uniform(0, 2 * math.pi), rng.uniform(0.5, 2.0), rng.uniform(0, 2 * math.pi)
        f = r * np.array([math.cos(g), math.sin(g)])
        out += np.outer(np.sin(2 * math.pi * (p @ f) + phi), a)
    return out


def cloth(n: int = 1000, seed: int = 6001, h: float = 1.0 / 60.0, k: float = 1.0e3,
          gravity=(0.0, 0.0, -9.81), density: float = 1.0) -> MeshInput:
    """One implicit-Euler step of a mass-spring cloth (Sec. 7.1) on an n x n grid.

    rest: the flat unit-square grid (springs = mesh edges, rest lengths from it).
    x (the current iterate x^n): rest + smooth waves of amplitude 0.02 in all three
    coordinates, so some springs are stretched and others compressed (compressed springs
    have negative Hessian eigenvalues, which the filtering clamps). v^n: smooth waves of
    amplitude 0.5. Lumped mass m = density / n^2 per vertex; spring stiffness k = 1e3 makes the
    springs dominate the inertia, so the unfiltered step Hessian is indefinite. meta holds the per-vertex
    data vdata = (m, xhat) with xhat = x^n + h v^n, the spring params (k, h^2) and the
    inertia params (h^2, g).
    """
    tris, rest = grid(n)
    rng = np.random.default_rng(seed)
    x = rest + _waves(rest[:, :2], rng, 6, 0.02, 3)
    v = _waves(rest[:, :2], rng, 6, 0.5, 3)
    m = np.full(n * n, density / (n * n))
    vdata = np.empty((n * n, 4))
    vdata[:, 0] = m
    vdata[:, 1:] = x + h * v
    w = h * h
    return MeshInput(tris, rest, x, 3, meta=dict(workload="cloth", n=n, seed=seed, h=h, k=k, vdata=vdata,
                                                   spring_params=(k, w), inertia_params=(w, *gravity)))


# --- geodesic icospheres -------------------------------------------------------------------------

_ICO_FACES = np.array([
    [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
    [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
    [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
    [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)


def _ico_corners() -> np.ndarray:
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def icosphere(freq: int) -> tuple[np.ndarray, np.ndarray]:
    """Class-I geodesic sphere of frequency ``freq`` on the unit sphere.

    V = 10 f^2 + 2, T = 20 f^2, counter-clockwise seen from outside. Lattice
    points shared by neighbouring icosahedron faces get one index via a
    canonical key (corner id, or edge + position from the lower corner, or
    face interior).
    """
    f = int(freq)
    if f < 1:
        raise ValueError("freq >= 1")
    corners = _ico_corners()
    keys: dict = {}
    pts: list = []
    tris: list = []

    def vid(face: int, i: int, j: int) -> int:
        # lattice point p = A + (i/f)(B-A) + (j/f)(C-A), i + j <= f
        a, b, c = _ICO_FACES[face]
        wa, wb, wc = f - i - j, i, j
        nz = [(w, cid) for w, cid in ((wa, a), (wb, b), (wc, c)) if w > 0]
        if len(nz) == 1:
            key = ("v", int(nz[0][1]))
        elif len(nz) == 2:
            (w0, c0), (w1, c1) = sorted(nz, key=lambda t: t[1])
            key = ("e", int(c0), int(c1), int(w1))
        else:
            key = ("f", face, i, j)
        idx = keys.get(key)
        if idx is None:
            idx = len(pts)
            keys[key] = idx
            p = (wa * corners[a] + wb * corners[b] + wc * corners[c]) / f
            pts.append(p / np.linalg.norm(p))
        return idx

    for face in range(20):
        for j in range(f):
            for i in range(f - j):
                v0 = vid(face, i, j)
                v1 = vid(face, i + 1, j)
                v2 = vid(face, i, j + 1)
                tris.append((v0, v1, v2))
                if i + j + 1 < f:
                    v3 = vid(face, i + 1, j + 1)
                    tris.append((v1, v3, v2))
    pos = np.asarray(pts, dtype=np.float64)
    t = np.asarray(tris, dtype=np.int32)
    # orient outward
    a, b, c = pos[t[:, 0]], pos[t[:, 1]], pos[t[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", nrm, a + b + c) < 0
    t[flip] = t[flip][:, [0, 2, 1]]
    return t, pos


def icosphere_batch(n_meshes: int = 700, size_seed: int = 4001, shape_seed: int = 4002,
                    mean_verts: float = 3000.0, sigma: float = 0.5,
                    vmin: int = 500, vmax: int = 12000) -> MeshInput:
    """Disjoint geodesic icospheres of lognormal vertex count, as one mesh.

    ln V ~ N(ln(mean) - sigma^2/2, sigma^2), redrawn until inside [vmin, vmax];
    freq = clamp(round(sqrt((V-2)/10)), 8, 34). Rest: sphere of radius
    U[0.5, 1.5] centred at a per-mesh offset; current: diag(1.1, 1.1, 0.8)
    applied to the rest about the centre, plus N(0, (1e-3 * mean edge)^2).
    """
    rs = np.random.default_rng(size_seed)
    freqs = []
    mu = math.log(mean_verts) - sigma * sigma / 2.0
    while len(freqs) < n_meshes:
        v = math.exp(rs.normal(mu, sigma))
        if vmin <= v <= vmax:
            freqs.append(int(min(34, max(8, round(math.sqrt((v - 2.0) / 10.0))))))
    rg = np.random.default_rng(shape_seed)
    cache: dict = {}
    tri_parts, rest_parts, x_parts, offs = [], [], [], [0]
    for m, fq in enumerate(freqs):
        if fq not in cache:
            cache[fq] = icosphere(fq)
        t, p = cache[fq]
        radius = rg.uniform(0.5, 1.5)
        centre = np.array([3.5 * (m % 27), 3.5 * ((m // 27) % 27), 3.5 * (m // 729)], dtype=np.float64)
        rest = p * radius
        ea = rest[t[:, 1]] - rest[t[:, 0]]
        mean_edge = float(np.mean(np.linalg.norm(ea, axis=1)))
        cur = rest * np.array([1.1, 1.1, 0.8]) + rg.normal(0.0, 1e-3 * mean_edge, size=rest.shape)
        tri_parts.append(t + offs[-1])
        rest_parts.append(rest + centre)
        x_parts.append(cur + centre)
        offs.append(offs[-1] + p.shape[0])
    tris = np.concatenate(tri_parts).astype(np.int32)
    return MeshInput(tris, np.concatenate(rest_parts), np.concatenate(x_parts), 3,
                     comp_offsets=np.asarray(offs, dtype=np.int64),
                     meta=dict(workload="icosphere_batch", n_meshes=n_meshes, freqs=freqs,
                               size_seed=size_seed, shape_seed=shape_seed))


def training_shells(n_meshes: int, n: int = 32, seed: int = 5002, noise_max: float = 1e-3) -> list[MeshInput]:
    """Perturbed rolled sheets whose triangles supply training samples of the learned density.

    Each sheet: flat n x n rest grid on [0,1]^2 (grid()); deformed by rotating the sheet in its
    plane by phi ~ U[0, pi), stretching the two in-plane axes by 1 + U[-0.05, 0.05] each, rolling
    (roll_cylinder) with radius R = +-U[0.2, 2] (random sign: bending either way), and adding
    N(0, (s h)^2) noise per coordinate, s = 1e-3, or with noise_max > 1e-3, s log-uniform in
    [1e-3, noise_max] per sheet (drawn after the sheet's other parameters). The normal-based second form
    of a triangle picks up noise of about s / h: a wider s range covers the spread of the features of
    finer meshes (s / h ~ 0.7 on a 708 x 708 sheet with s = 1e-3).
    """
    rg = np.random.default_rng(seed)
    tris, rest = grid(n)
    h = 1.0 / (n - 1)
    out = []
    for _ in range(n_meshes):
        phi = rg.uniform(0.0, math.pi)
        c, s = math.cos(phi), math.sin(phi)
        st = 1.0 + rg.uniform(-0.05, 0.05, size=2)
        p = rest.copy()
        p[:, 0] = (c * rest[:, 0] - s * rest[:, 1]) * st[0]
        p[:, 1] = (s * rest[:, 0] + c * rest[:, 1]) * st[1]
        radius = rg.uniform(0.2, 2.0) * (1.0 if rg.uniform() < 0.5 else -1.0)
        x = roll_cylinder(p, radius)
        sc = 1e-3 if noise_max <= 1e-3 else math.exp(rg.uniform(math.log(1e-3), math.log(noise_max)))
        x += rg.normal(0.0, sc * h, size=x.shape)
        out.append(MeshInput(tris, rest, x, 3, meta=dict(workload="training_shell", phi=phi, stretch=st,
                                                         radius=radius)))
    return out


def tiny_meshes() -> dict[str, tuple[np.ndarray, np.ndarray]]:
    """Small hand-made meshes for brute-force checks: (tris, positions)."""
    out = {}
    out["two_tris"] = (np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32),
                       np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], dtype=np.float64))
    octa_p = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=np.float64)
    octa_t = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4],
                       [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]], dtype=np.int32)
    out["octahedron"] = (octa_t, octa_p)
    # three triangles sharing the edge (0,1): a non-manifold fan, plus an isolated vertex 5
    out["nonmanifold"] = (np.array([[0, 1, 2], [1, 0, 3], [0, 1, 4]], dtype=np.int32),
                          np.array([[0, 0, 0], [1, 0, 0], [0.5, 1, 0], [0.5, -1, 0.2],
                                    [0.5, 0.3, 1], [2, 2, 2]], dtype=np.float64))
    for n in (2, 3, 4, 5):
        out[f"grid{n}"] = grid(n)
    return out
