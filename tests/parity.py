"""Shared helpers of the parity tests: build the same problem on the HIP path
(through the C ABI) and on the oracle, and compare element by element.

Tolerance model: every assembled entry y is compared as
    |y - y_ref| <= rtol * scale
where scale sums, over the elements that add into the entry, the largest
magnitude in that element's local gradient (for g) or local Hessian (for H),
as the oracle reports it. An FP32 element computation commits errors of about
eps32 times its own magnitude, so this is the natural yardstick; it is never
looser than 'rtol relative to the contributing elements'. Energies compare as
|E - E_ref| <= rtol * sum_j |f_j|. rtol is 1e-12 for FP64, 1e-5 for FP32.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

RTOL = {0: 1e-12, 1: 1e-5}

KIND_MAP = {1: O.EDGE_SQLEN, 2: O.TRI_AREA, 3: O.DIRICHLET, 4: O.STVK, 5: O.BENDING, 6: O.SYMDIR}


def build_oracle(tris, rest, nv, var_dim, terms):
    P = O.Problem(tris, rest, nv, var_dim)
    for kind, prm in terms:
        P.add_term(KIND_MAP[kind], prm)
    P.build_pattern()
    return P


def build_gpu(tris, rest, nv, var_dim, terms, precision, comp_offsets=None, patch_faces=0, spd_eps=0.0,
              scatter=0):
    from paper_2509_00406_amd import mad
    mesh = mad.Mesh(tris, nv, comp_offsets)
    prob = mad.Problem(mesh, var_dim, precision, patch_faces=patch_faces, spd_eps=spd_eps, scatter=scatter)
    for kind, prm in terms:
        prob.add_term(kind, prm, rest if kind in mad.NEEDS_REST else None)
    prob.finalize()
    return mesh, prob


def worst(y, yref, scale):
    y = np.asarray(y, dtype=np.float64).ravel()
    yref = np.asarray(yref, dtype=np.float64).ravel()
    scale = np.asarray(scale, dtype=np.float64).ravel()
    err = np.abs(y - yref)
    ratio = err / np.maximum(scale, 1e-300)
    ratio[(err == 0)] = 0.0
    i = int(np.argmax(ratio)) if ratio.size else 0
    return (float(ratio[i]) if ratio.size else 0.0), i


def assert_close(name, y, yref, scale, rtol):
    r, i = worst(y, yref, scale)
    assert np.all(np.isfinite(np.asarray(y, dtype=np.float64))), f"{name}: non-finite values"
    assert r <= rtol, (f"{name}: worst |err|/scale = {r:.3e} > {rtol:.1e} at {i}: "
                       f"got {np.ravel(y)[i]!r} want {np.ravel(yref)[i]!r} scale {np.ravel(scale)[i]!r}")
    return r


def normwise(y, yref):
    y = np.asarray(y, dtype=np.float64).ravel()
    yref = np.asarray(yref, dtype=np.float64).ravel()
    den = np.max(np.abs(yref)) if yref.size else 1.0
    return float(np.max(np.abs(y - yref)) / den) if den > 0 else float(np.max(np.abs(y - yref)))
