"""ctypes front end of the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark. The product library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

EDGE_SQLEN, TRI_AREA, DIRICHLET, STVK, BENDING, SYMDIR, MLP, SHELL_TRI = 1, 2, 3, 4, 5, 6, 7, 8
SPRING, INERTIA = 9, 10
RES_POSITION, RES_EDGE = 11, 12
ENERGY, GRAD, HESS, SPD = 1, 2, 4, 8

STENCIL = {EDGE_SQLEN: 2, TRI_AREA: 3, DIRICHLET: 3, STVK: 3, BENDING: 4, SYMDIR: 3, MLP: 3, SHELL_TRI: 3,
           SPRING: 2, INERTIA: 1, RES_POSITION: 1, RES_EDGE: 2}
VARDIM = {EDGE_SQLEN: 3, TRI_AREA: 3, DIRICHLET: 1, STVK: 3, BENDING: 3, SYMDIR: 2, MLP: 3, SHELL_TRI: 3,
          SPRING: 3, INERTIA: 3, RES_POSITION: 3, RES_EDGE: 3}
NRES = {RES_POSITION: 3, RES_EDGE: 1}   # residuals per element of the residual kinds


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, no FMA contraction, no fast-math): the parity reference. OpenMP
    is enabled for oracle_eval_par only; oracle_eval stays serial."""
    src = os.path.join(HERE, "oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(
            os.path.getmtime(src), os.path.getmtime(os.path.join(HERE, "oracle.h"))):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-ffp-contract=off", "-fopenmp", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def build_fast() -> str:
    """A timing build of the same source for the host it runs on (-O3 -march=native, the compiler's
    default FMA contraction): used only to time the oracle, never as the parity reference. Built on first
    use on each host (the file name carries a hash of the CPU model, so a copy built elsewhere is not
    reused)."""
    import hashlib
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    tag = hashlib.sha1(model.encode()).hexdigest()[:10]
    src = os.path.join(HERE, "oracle.c")
    path = os.path.join(HERE, f"liboracle_fast_{tag}.so")
    if not os.path.exists(path) or os.path.getmtime(path) < max(
            os.path.getmtime(src), os.path.getmtime(os.path.join(HERE, "oracle.h"))):
        tmp = path + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=native", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-o", tmp,
                               src, "-lm"])
        os.replace(tmp, path)
    return path


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        build()
        _lib = load(LIB_PATH)
    return _lib


def load(path: str) -> C.CDLL:
    h = C.CDLL(path)
    h.oracle_neumaier_sum.restype = C.c_double
    return h


class using:
    """Temporarily route every call of this module through another build of
    the oracle (used by the mutation test to run the pins on mutants)."""

    def __init__(self, handle: C.CDLL):
        self.handle = handle

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = self.handle
        return self.handle

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


@dataclass
class Topology:
    edges: np.ndarray          # int32 [E, 2]
    edge_nf: np.ndarray        # int32 [E]
    diamonds: np.ndarray       # int32 [D, 4]
    diamond_faces: np.ndarray  # int32 [D, 2]


def topology(tris: np.ndarray, nv: int) -> Topology:
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    nt = tris.shape[0]
    edges = np.zeros((3 * nt + 1, 2), np.int32)
    nf = np.zeros(3 * nt + 1, np.int32)
    dia = np.zeros((3 * nt + 1, 4), np.int32)
    dfc = np.zeros((3 * nt + 1, 2), np.int32)
    ne = C.c_int64()
    nd = C.c_int64()
    _check(lib().oracle_topology(C.c_int64(nv), C.c_int64(nt), _p(tris), C.byref(ne), _p(edges), _p(nf),
                                 C.byref(nd), _p(dia), _p(dfc)), "topology")
    return Topology(edges[:ne.value].copy(), nf[:ne.value].copy(), dia[:nd.value].copy(), dfc[:nd.value].copy())


def rest_tri(tris: np.ndarray, rest: np.ndarray) -> np.ndarray:
    """Per-triangle rest data [T, 5] = (Dm^{-1} row-major, area)."""
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    rest = np.ascontiguousarray(rest, dtype=np.float64)
    nt = tris.shape[0]
    mi = np.zeros((nt, 4))
    ar = np.zeros(nt)
    _check(lib().oracle_rest_tri(C.c_int64(nt), _p(tris), _p(rest), _p(mi), _p(ar)), "rest_tri")
    return np.ascontiguousarray(np.concatenate([mi, ar[:, None]], axis=1))


def rest_diamond(topo: Topology, tris: np.ndarray, rest: np.ndarray) -> np.ndarray:
    """Per-diamond rest data [D, 2] = (mean rest area of the two faces, rest dihedral)."""
    nd = topo.diamonds.shape[0]
    ab = np.zeros(nd)
    th = np.zeros(nd)
    _check(lib().oracle_rest_diamond(C.c_int64(nd), _p(topo.diamonds), _p(topo.diamond_faces),
                                     _p(np.ascontiguousarray(tris, dtype=np.int32)),
                                     _p(np.ascontiguousarray(rest, dtype=np.float64)), _p(ab), _p(th)),
           "rest_diamond")
    return np.ascontiguousarray(np.stack([ab, th], axis=1))


def pattern(nv: int, stencils: list[np.ndarray]) -> tuple[np.ndarray, np.ndarray]:
    n = len(stencils)
    sts = [np.ascontiguousarray(s, dtype=np.int32) for s in stencils]
    ne = (C.c_int64 * max(n, 1))(*[s.shape[0] for s in sts])
    ss = (C.c_int * max(n, 1))(*[s.shape[1] for s in sts])
    ptrs = (C.c_void_p * max(n, 1))(*[s.ctypes.data for s in sts])
    rowptr = np.zeros(nv + 1, np.int32)
    nnzb = C.c_int64()
    _check(lib().oracle_pattern(C.c_int64(nv), C.c_int(n), ne, ss, ptrs, _p(rowptr), None, C.byref(nnzb)), "pattern")
    colidx = np.zeros(nnzb.value, np.int32)
    _check(lib().oracle_pattern(C.c_int64(nv), C.c_int(n), ne, ss, ptrs, _p(rowptr), _p(colidx), C.byref(nnzb)),
           "pattern")
    return rowptr, colidx


def residual(kind: int, xloc, rest, params=(1.0,)):
    """One element of a residual kind: (r[m], J[m, k]) in stencil DOF order (Eq. 3's r_j and J_j)."""
    m = NRES[kind]
    k = STENCIL[kind] * VARDIM[kind]
    xl = np.ascontiguousarray(xloc, dtype=np.float64).ravel()
    rs = np.ascontiguousarray(rest, dtype=np.float64).ravel()
    pr = np.zeros(4)
    pr[:len(params)] = params
    r = np.zeros(m)
    J = np.zeros((m, k))
    _check(lib().oracle_residual(C.c_int(kind), _p(pr), _p(rs), _p(xl), _p(r), _p(J)), "residual")
    return r, J


def insert_pairs(rowptr: np.ndarray, colidx: np.ndarray, pairs: np.ndarray, nv: int):
    """Dynamic sparsity (Sec. 6.3 and the CSR update of the appendix), by its definition: the block
    pattern after new interaction pairs is the union of the old (row, column) set and, for every pair
    (a, b) with a != b, the blocks (a, b) and (b, a), stored as CSR with every row sorted. Returns
    (rowptr, colidx, old_to_new) where old_to_new[j] is the new index of old block j.
    Reading: pairs naming one vertex twice, repeated pairs and pairs already present add nothing."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    rows = np.repeat(np.arange(nv, dtype=np.int64), np.diff(rowptr))
    old = rows * nv + colidx
    pr = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    if pr.size and (pr.min() < 0 or pr.max() >= nv):
        raise ValueError("pair names a vertex out of range")
    pr = pr[pr[:, 0] != pr[:, 1]]
    new = np.concatenate([pr[:, 0] * nv + pr[:, 1], pr[:, 1] * nv + pr[:, 0]])
    keys = np.union1d(old, new)                      # sorted, unique
    r, c = keys // nv, keys % nv
    rp = np.zeros(nv + 1, dtype=np.int64)
    np.add.at(rp, r + 1, 1)
    rp = np.cumsum(rp)
    return rp.astype(np.int32), c.astype(np.int32), np.searchsorted(keys, old).astype(np.int64)


def element(kind: int, xloc, rest=None, params=None, mode: int = ENERGY | GRAD | HESS, spd_eps: float = 0.0,
            aux=None):
    """One element: returns (f, g[k], H[k, k]). aux: the three unit vertex normals of the
    shell-feature kinds (SHELL_TRI, MLP)."""
    k = STENCIL[kind] * VARDIM[kind]
    xl = np.ascontiguousarray(xloc, dtype=np.float64).ravel()
    assert xl.size == k
    rs = None if rest is None else np.ascontiguousarray(rest, dtype=np.float64).ravel()
    pr = np.ascontiguousarray(params if params is not None else [0.0, 0.0], dtype=np.float64).ravel()
    ax = None if aux is None else np.ascontiguousarray(aux, dtype=np.float64).ravel()
    f = C.c_double()
    g = np.zeros(k)
    H = np.zeros((k, k))
    _check(lib().oracle_element(C.c_int(kind), _p(pr), _p(rs), _p(ax), _p(xl), C.c_int(mode),
                                C.c_double(spd_eps), C.byref(f), _p(g), _p(H)), "element")
    return f.value, g, H


# ---- per-triangle shell features, analytic density and the learned density -----------------------
def vertex_normals(tris: np.ndarray, x: np.ndarray, nv: int) -> np.ndarray:
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros((nv, 3))
    _check(lib().oracle_vertex_normals(C.c_int64(nv), C.c_int64(tris.shape[0]), _p(tris), _p(x), _p(out)),
           "vertex_normals")
    return out


def rest_shell(tris: np.ndarray, rest: np.ndarray, nv: int) -> np.ndarray:
    """Per-triangle rest data [T, 8] = (Dm^{-1} row-major, rest area, rest II00, II11, II01)."""
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    rest = np.ascontiguousarray(rest, dtype=np.float64)
    out = np.zeros((tris.shape[0], 8))
    _check(lib().oracle_rest_shell(C.c_int64(nv), C.c_int64(tris.shape[0]), _p(tris), _p(rest), _p(out)),
           "rest_shell")
    return out


def shell_features(tris: np.ndarray, rest8: np.ndarray, x: np.ndarray, nv: int) -> np.ndarray:
    """Feature vectors z [T, 6] at positions x."""
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    z = np.zeros((tris.shape[0], 6))
    _check(lib().oracle_shell_features(C.c_int64(nv), C.c_int64(tris.shape[0]), _p(tris),
                                       _p(np.ascontiguousarray(rest8, dtype=np.float64)),
                                       _p(np.ascontiguousarray(x, dtype=np.float64)), _p(z)), "shell_features")
    return z


def shell_density(z: np.ndarray, params) -> tuple[np.ndarray, np.ndarray]:
    """Analytic density W(z) and dW/dz (params: mu, lambda, k_b)."""
    z = np.ascontiguousarray(z, dtype=np.float64).reshape(-1, 6)
    pr = np.ascontiguousarray(params, dtype=np.float64)
    W = np.zeros(z.shape[0])
    dW = np.zeros_like(z)
    _check(lib().oracle_shell_density(C.c_int64(z.shape[0]), _p(z), _p(pr), _p(W), _p(dW)), "shell_density")
    return W, dW


def mlp_eval(z: np.ndarray, params: np.ndarray, hess: bool = False):
    """psi(z), dpsi/dz [n, 6] and, if asked, d2psi/dz2 [n, 6, 6] by hyper-dual arithmetic."""
    z = np.ascontiguousarray(z, dtype=np.float64).reshape(-1, 6)
    pr = np.ascontiguousarray(params, dtype=np.float64)
    n = z.shape[0]
    psi = np.zeros(n)
    d = np.zeros((n, 6))
    h = np.zeros((n, 6, 6)) if hess else None
    _check(lib().oracle_mlp_eval(C.c_int64(n), _p(z), _p(pr), _p(psi), _p(d), _p(h)), "mlp_eval")
    return (psi, d, h) if hess else (psi, d)


MLP_PARTS = ("W1", "b1", "W2", "b2", "w3", "b3")   # trainable parameters, in packing order


def mlp_pack(s_out: float, s_in, W1, b1, W2, b2, w3, b3) -> np.ndarray:
    """The parameter block [H, s_out, s_in(6), W1(H x 6), b1, W2(H x H), b2, w3, b3]."""
    H = np.asarray(W1).shape[0]
    return np.concatenate([[float(H), float(s_out)], np.asarray(s_in, float).ravel(), np.asarray(W1, float).ravel(),
                           np.asarray(b1, float).ravel(), np.asarray(W2, float).ravel(),
                           np.asarray(b2, float).ravel(), np.asarray(w3, float).ravel(), [float(b3)]])


def mlp_unpack(params: np.ndarray) -> dict:
    p = np.asarray(params, dtype=np.float64)
    H = int(p[0])
    o = 8
    out = {"H": H, "s_out": p[1], "s_in": p[2:8]}
    for name, size in (("W1", 6 * H), ("b1", H), ("W2", H * H), ("b2", H), ("w3", H), ("b3", 1)):
        out[name] = p[o:o + size].copy()
        o += size
    out["W1"] = out["W1"].reshape(H, 6)
    out["W2"] = out["W2"].reshape(H, H)
    out["b3"] = float(out["b3"][0])
    return out


def mlp_loss_grad(params: np.ndarray, z: np.ndarray, W: np.ndarray, dW: np.ndarray, c_e: float, c_g,
                  lam_g: float) -> tuple[float, np.ndarray]:
    """Training loss and its gradient over the trainable parameters (W1, b1, W2, b2, w3, b3, in
    packing order), by reverse-mode differentiation in FP64 on the CPU:
        loss = mean_i (psi(z_i) - W_i)^2 / c_e + lam_g mean_i sum_q (dpsi/dz_q(z_i) - dW_iq)^2 / c_g[q]
    (c_g: one normaliser per feature, or a scalar for all)."""
    import torch
    u = mlp_unpack(params)
    T = {k: torch.tensor(u[k], dtype=torch.float64, requires_grad=True) for k in MLP_PARTS}
    s_in = torch.tensor(u["s_in"], dtype=torch.float64)
    zz = torch.tensor(np.asarray(z, dtype=np.float64).reshape(-1, 6), requires_grad=True)

    def sp(a):   # softplus, exactly log(1 + e^a)
        return torch.logaddexp(a, torch.zeros_like(a))
    h1 = sp((zz * s_in) @ T["W1"].T + T["b1"])
    h2 = sp(h1 @ T["W2"].T + T["b2"])
    psi = u["s_out"] * (h2 @ T["w3"] + T["b3"])
    (dpsi,) = torch.autograd.grad(psi.sum(), zz, create_graph=True)
    Wt = torch.tensor(np.asarray(W, dtype=np.float64))
    dWt = torch.tensor(np.asarray(dW, dtype=np.float64).reshape(-1, 6))
    cg = torch.tensor(np.broadcast_to(np.asarray(c_g, dtype=np.float64), (6,)).copy())
    loss = ((psi - Wt) ** 2).mean() / c_e + lam_g * (((dpsi - dWt) ** 2) / cg).sum(dim=1).mean()
    grads = torch.autograd.grad(loss, [T[k] for k in MLP_PARTS])
    return float(loss.detach()), np.concatenate([g.detach().numpy().ravel() for g in grads])


def adam_step(theta: np.ndarray, grad: np.ndarray, m: np.ndarray, v: np.ndarray, t: int, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba), step number t >= 1; returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def spd_project(A: np.ndarray, eps: float = 0.0) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    out = np.zeros_like(A)
    _check(lib().oracle_spd_project(C.c_int(n), _p(A), C.c_double(eps), _p(out)), "spd_project")
    return out


def neumaier_sum(v: np.ndarray) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().oracle_neumaier_sum(C.c_int64(v.size), _p(v))


@dataclass
class Term:
    kind: int
    stencil: np.ndarray   # int32 [n, ss]
    rest: np.ndarray | None  # float64 [n, r]
    params: np.ndarray    # float64 [>= 2]


@dataclass
class Result:
    energy: float
    esum_abs: float
    grad: np.ndarray | None
    gscale: np.ndarray | None
    hess: np.ndarray | None    # [nnzb, d, d]
    hscale: np.ndarray | None


class Problem:
    """Oracle-side problem: topology, rest data and pattern built from the same
    raw inputs (triangles + rest positions) that the product library receives."""

    def __init__(self, tris: np.ndarray, rest: np.ndarray, nv: int, var_dim: int):
        self.tris = np.ascontiguousarray(tris, dtype=np.int32)
        self.rest_pos = np.ascontiguousarray(rest, dtype=np.float64)
        self.nv = int(nv)
        self.d = int(var_dim)
        self.terms: list[Term] = []
        self._topo = None
        self.rowptr = None
        self.colidx = None

    @property
    def topo(self) -> Topology:
        if self._topo is None:
            self._topo = topology(self.tris, self.nv)
        return self._topo

    def add_term(self, kind: int, params=(0.0, 0.0), vertex_data=None):
        """vertex_data: for INERTIA, per-vertex (m, xhat_x, xhat_y, xhat_z) [nv, 4]."""
        if VARDIM[kind] != self.d:
            raise ValueError("term VarDim does not match the problem")
        prm = np.zeros(max(4, len(params)))
        prm[:len(params)] = params
        if kind in (SPRING, RES_EDGE):
            st = self.topo.edges
            rs = np.linalg.norm(self.rest_pos[st[:, 0]] - self.rest_pos[st[:, 1]], axis=1)[:, None]
        elif kind in (INERTIA, RES_POSITION):
            if vertex_data is None:
                raise ValueError("vertex terms need vertex_data [nv, 4]")
            st = np.arange(self.nv, dtype=np.int32)[:, None]
            rs = np.ascontiguousarray(vertex_data, dtype=np.float64).reshape(self.nv, 4)
        elif kind in (SHELL_TRI, MLP):
            st = self.tris
            rs = rest_shell(self.tris, self.rest_pos, self.nv)
        elif kind == BENDING:
            st = self.topo.diamonds
            rs = rest_diamond(self.topo, self.tris, self.rest_pos)
        elif kind in (DIRICHLET, STVK, SYMDIR):
            st = self.tris
            rs = rest_tri(self.tris, self.rest_pos)
        elif kind == TRI_AREA:
            st, rs = self.tris, None
        elif kind == EDGE_SQLEN:
            st, rs = self.topo.edges, None
        else:
            raise ValueError(kind)
        self.terms.append(Term(kind, np.ascontiguousarray(st, dtype=np.int32), rs, prm))
        self.rowptr = None

    def build_pattern(self):
        self.rowptr, self.colidx = pattern(self.nv, [t.stencil for t in self.terms])
        return self.rowptr, self.colidx

    def eval(self, x: np.ndarray, mode: int = ENERGY | GRAD | HESS, spd_eps: float = 0.0,
             row_mask: np.ndarray | None = None, scales: bool = True) -> Result:
        if self.rowptr is None:
            self.build_pattern()
        x = np.ascontiguousarray(x, dtype=np.float64).ravel()
        assert x.size == self.nv * self.d
        n = len(self.terms)
        kinds = (C.c_int * n)(*[t.kind for t in self.terms])
        ne = (C.c_int64 * n)(*[t.stencil.shape[0] for t in self.terms])
        st = (C.c_void_p * n)(*[t.stencil.ctypes.data for t in self.terms])
        rs = (C.c_void_p * n)(*[(t.rest.ctypes.data if t.rest is not None else None) for t in self.terms])
        pr = (C.c_void_p * n)(*[t.params.ctypes.data for t in self.terms])
        d = self.d
        nnzb = int(self.rowptr[-1])
        grad = np.zeros(self.nv * d) if mode & GRAD else None
        gscale = np.zeros(self.nv * d) if (mode & GRAD and scales) else None
        hess = np.zeros((nnzb, d, d)) if mode & HESS else None
        hscale = np.zeros((nnzb, d, d)) if (mode & HESS and scales) else None
        mask = None
        if row_mask is not None:
            mask = np.ascontiguousarray(row_mask, dtype=np.int8)
        e = C.c_double()
        ea = C.c_double()
        _check(lib().oracle_eval(C.c_int64(self.nv), C.c_int(d), C.c_int(n), kinds, ne, st, rs, pr, _p(x),
                                 C.c_int(mode), C.c_double(spd_eps), _p(mask), _p(self.rowptr), _p(self.colidx),
                                 C.byref(e), C.byref(ea), _p(grad), _p(gscale), _p(hess), _p(hscale)), "eval")
        return Result(e.value, ea.value, grad, gscale, hess, hscale)

    def eval_par(self, x: np.ndarray, mode: int = ENERGY | GRAD | HESS, spd_eps: float = 0.0,
                 threads: int = 1) -> Result:
        """oracle_eval_par: the same evaluation over `threads` OpenMP threads (bit-identical to eval in the
        same build; no row mask, no scales)."""
        if self.rowptr is None:
            self.build_pattern()
        x = np.ascontiguousarray(x, dtype=np.float64).ravel()
        assert x.size == self.nv * self.d
        n = len(self.terms)
        kinds = (C.c_int * n)(*[t.kind for t in self.terms])
        ne = (C.c_int64 * n)(*[t.stencil.shape[0] for t in self.terms])
        st = (C.c_void_p * n)(*[t.stencil.ctypes.data for t in self.terms])
        rs = (C.c_void_p * n)(*[(t.rest.ctypes.data if t.rest is not None else None) for t in self.terms])
        pr = (C.c_void_p * n)(*[t.params.ctypes.data for t in self.terms])
        d = self.d
        nnzb = int(self.rowptr[-1])
        grad = np.zeros(self.nv * d) if mode & GRAD else None
        hess = np.zeros((nnzb, d, d)) if mode & HESS else None
        e = C.c_double()
        ea = C.c_double()
        _check(lib().oracle_eval_par(C.c_int64(self.nv), C.c_int(d), C.c_int(n), kinds, ne, st, rs, pr, _p(x),
                                     C.c_int(mode), C.c_double(spd_eps), _p(self.rowptr), _p(self.colidx),
                                     C.c_int(int(threads)), C.byref(e), C.byref(ea), _p(grad), _p(hess)), "eval_par")
        return Result(e.value, ea.value, grad, None, hess, None)

    def jacobian(self, x: np.ndarray):
        """Residual vector and sparse Jacobian of the residual terms (Eq. 3), CSR with scalar entries:
        (r, rowptr, colidx, vals); rows by term, then element; columns ascending DOF indices."""
        x = np.ascontiguousarray(x, dtype=np.float64).ravel()
        n = len(self.terms)
        kinds = (C.c_int * n)(*[t.kind for t in self.terms])
        ne = (C.c_int64 * n)(*[t.stencil.shape[0] for t in self.terms])
        st = (C.c_void_p * n)(*[t.stencil.ctypes.data for t in self.terms])
        rs = (C.c_void_p * n)(*[(t.rest.ctypes.data if t.rest is not None else None) for t in self.terms])
        pr = (C.c_void_p * n)(*[t.params.ctypes.data for t in self.terms])
        m = sum(NRES.get(t.kind, 0) * t.stencil.shape[0] for t in self.terms)
        rowptr = np.zeros(m + 1, np.int32)
        args = (C.c_int64(self.nv), C.c_int(self.d), C.c_int(n), kinds, ne, st, rs, pr, _p(x))
        _check(lib().oracle_jacobian(*args, None, _p(rowptr), None, None), "jacobian")
        nnz = int(rowptr[-1])
        r = np.zeros(m)
        colidx = np.zeros(nnz, np.int32)
        vals = np.zeros(nnz)
        _check(lib().oracle_jacobian(*args, _p(r), _p(rowptr), _p(colidx), _p(vals)), "jacobian")
        return r, rowptr, colidx, vals

    def hvp(self, x: np.ndarray, v: np.ndarray, spd: bool = False, spd_eps: float = 0.0):
        """Hessian-vector product by its definition: the assembled Hessian (clamped per element when
        spd) times v, block row by block row. Returns (y, yscale) with yscale = |H| scales times |v|
        (the per-entry tolerance scale of a product: sum over the row's blocks of the oracle's
        per-entry Hessian scale times |v|)."""
        r = self.eval(x, ENERGY | HESS | (SPD if spd else 0), spd_eps=spd_eps)
        d = self.d
        v = np.asarray(v, dtype=np.float64).reshape(self.nv, d)
        y = np.zeros((self.nv, d))
        ys = np.zeros((self.nv, d))
        for i in range(self.nv):
            for b in range(self.rowptr[i], self.rowptr[i + 1]):
                j = self.colidx[b]
                y[i] += r.hess[b] @ v[j]
                ys[i] += r.hscale[b] @ np.abs(v[j])
        return y.ravel(), ys.ravel()
