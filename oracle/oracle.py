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

EDGE_SQLEN, TRI_AREA, DIRICHLET, STVK, BENDING, SYMDIR, MLP = 1, 2, 3, 4, 5, 6, 7
ENERGY, GRAD, HESS, SPD = 1, 2, 4, 8

STENCIL = {EDGE_SQLEN: 2, TRI_AREA: 3, DIRICHLET: 3, STVK: 3, BENDING: 4, SYMDIR: 3, MLP: 3}
VARDIM = {EDGE_SQLEN: 3, TRI_AREA: 3, DIRICHLET: 1, STVK: 3, BENDING: 3, SYMDIR: 2, MLP: 3}


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (serial, -O2, no fast-math)."""
    src = os.path.join(HERE, "oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(
            os.path.getmtime(src), os.path.getmtime(os.path.join(HERE, "oracle.h"))):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-ffp-contract=off", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


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


def element(kind: int, xloc, rest=None, params=None, mode: int = ENERGY | GRAD | HESS, spd_eps: float = 0.0):
    """One element: returns (f, g[k], H[k, k])."""
    k = STENCIL[kind] * VARDIM[kind]
    xl = np.ascontiguousarray(xloc, dtype=np.float64).ravel()
    assert xl.size == k
    rs = None if rest is None else np.ascontiguousarray(rest, dtype=np.float64).ravel()
    pr = np.ascontiguousarray(params if params is not None else [0.0, 0.0], dtype=np.float64).ravel()
    f = C.c_double()
    g = np.zeros(k)
    H = np.zeros((k, k))
    _check(lib().oracle_element(C.c_int(kind), _p(pr), _p(rs), _p(xl), C.c_int(mode), C.c_double(spd_eps),
                                C.byref(f), _p(g), _p(H)), "element")
    return f.value, g, H


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

    def add_term(self, kind: int, params=(0.0, 0.0)):
        if VARDIM[kind] != self.d:
            raise ValueError("term VarDim does not match the problem")
        prm = np.zeros(4)
        prm[:len(params)] = params
        if kind == BENDING:
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
