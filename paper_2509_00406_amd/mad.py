"""Python binding of libmad.so: argument marshalling only.

Every function named ``mad_*`` mirrors the C entry point of the same name in
include/mad.h. Device buffers are torch CUDA (HIP) tensors; streams are torch
streams. Every step of the evaluation runs in the library's HIP kernels. If the
library is missing this module raises; it never falls back to another path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmad.so")

EDGE_SQLEN, TRI_AREA, DIRICHLET, STVK, BENDING, SYMDIR, MLP, SHELL_TRI = 1, 2, 3, 4, 5, 6, 7, 8
SPRING, INERTIA = 9, 10
RES_POSITION, RES_EDGE = 11, 12
ENERGY, GRAD, HESS, SPD = 1, 2, 4, 8
F64, F32 = 0, 1
SCATTER_AUTO, SCATTER_ATOMIC, SCATTER_PATCH, SCATTER_COLOR = 0, 1, 2, 3
TUNE_FORCE = 1

STATUS = {0: "MAD_OK", -1: "MAD_E_INVALID_ARG", -2: "MAD_E_BAD_MESH", -3: "MAD_E_DEGENERATE_REST",
          -4: "MAD_E_OVERFLOW", -5: "MAD_E_OOM", -6: "MAD_E_HIP", -7: "MAD_E_STATE", -8: "MAD_E_UNSUPPORTED",
          -9: "MAD_E_CAPACITY", -10: "MAD_E_INTERNAL"}
LOCK_NO_WAIT = -1
VARDIM = {EDGE_SQLEN: 3, TRI_AREA: 3, DIRICHLET: 1, STVK: 3, BENDING: 3, SYMDIR: 2, MLP: 3, SHELL_TRI: 3}
NEEDS_REST = {DIRICHLET, STVK, BENDING, SYMDIR, MLP, SHELL_TRI, SPRING, RES_EDGE}
MLP_HIDDEN, MLP_PARAMS = 64, 4673


class MadError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__(f"{what}: {STATUS.get(code, code)}: {msg}")
        self.code = code


class mad_options(C.Structure):
    _fields_ = [("scatter", C.c_int32), ("patch_faces", C.c_int32), ("spd_eps", C.c_double),
                ("degenerate_q", C.c_double), ("lock_spins", C.c_int32), ("wg_waves", C.c_int32),
                ("reserved", C.c_int32 * 6)]


_lib = None

_SIGS = {
    "mad_version": ([], C.c_int32),
    "mad_last_error": ([], C.c_char_p),
    "mad_options_default": ([C.POINTER(mad_options)], C.c_int32),
    "mad_mesh_create": ([C.c_int64, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)], C.c_int32),
    "mad_mesh_info": ([C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                       C.POINTER(C.c_int64)], C.c_int32),
    "mad_mesh_copy_diamonds": ([C.c_void_p, C.c_void_p], C.c_int32),
    "mad_mesh_destroy": ([C.c_void_p], C.c_int32),
    "mad_problem_create": ([C.c_void_p, C.c_int32, C.c_int32, C.POINTER(mad_options), C.POINTER(C.c_void_p)],
                           C.c_int32),
    "mad_problem_add_term": ([C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p], C.c_int32),
    "mad_problem_finalize": ([C.c_void_p, C.c_void_p], C.c_int32),
    "mad_problem_pattern_info": ([C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32)],
                                 C.c_int32),
    "mad_problem_energy_count": ([C.c_void_p, C.POINTER(C.c_int32)], C.c_int32),
    "mad_problem_copy_pattern": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int32),
    "mad_problem_eval": ([C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
                         C.c_int32),
    "mad_problem_eval_static": ([C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p], C.c_int32),
    "mad_problem_status": ([C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.c_void_p], C.c_int32),
    "mad_problem_hvp": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                         C.c_void_p], C.c_int32),
    "mad_problem_set_profiling": ([C.c_void_p, C.c_int32], C.c_int32),
    "mad_problem_profile": ([C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)],
                            C.c_int32),
    "mad_problem_layout": ([C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                            C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int32),
    "mad_problem_set_layout": ([C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p], C.c_int32),
    "mad_problem_autotune": ([C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                              C.c_int32, C.c_void_p], C.c_int32),
    "mad_problem_tune_report": ([C.c_void_p, C.c_char_p, C.c_int64, C.POINTER(C.c_int64)], C.c_int32),
    "mad_problem_destroy": ([C.c_void_p], C.c_int32),
    "mad_mlp_create": ([C.c_int32, C.c_void_p, C.c_void_p, C.c_float, C.POINTER(C.c_void_p)], C.c_int32),
    "mad_mlp_set_params": ([C.c_void_p, C.c_void_p], C.c_int32),
    "mad_mlp_get_params": ([C.c_void_p, C.c_int32, C.c_void_p], C.c_int32),
    "mad_mlp_loss_grad": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                           C.c_float, C.c_void_p, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int32),
    "mad_mlp_adam_step": ([C.c_void_p, C.c_void_p, C.c_float, C.c_float, C.c_float, C.c_float, C.c_void_p],
                          C.c_int32),
    "mad_mlp_train_epoch": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                             C.c_float, C.c_void_p, C.c_float, C.c_float, C.c_float, C.c_float, C.c_float,
                             C.c_void_p, C.c_void_p], C.c_int32),
    "mad_mlp_destroy": ([C.c_void_p], C.c_int32),
    "mad_problem_add_mlp_term": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int32),
    "mad_problem_add_vertex_term": ([C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p], C.c_int32),
    "mad_problem_reserve_pairs": ([C.c_void_p, C.c_int64], C.c_int32),
    "mad_problem_jacobian_info": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int32),
    "mad_problem_copy_jacobian_pattern": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int32),
    "mad_problem_jacobian": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int32),
    "mad_problem_insert_pairs": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p], C.c_int32),
}


def lib() -> C.CDLL:
    """Load libmad.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "python -m paper_2509_00406_amd.build")
        h = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(h, name)
            fn.argtypes = args
            fn.restype = res
        _lib = h
    return _lib


def exported_symbols() -> list[str]:
    return sorted(_SIGS)


def _check(rc: int, what: str):
    if rc != 0:
        raise MadError(rc, what, lib().mad_last_error().decode(errors="replace"))


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream) -> int | None:
    """torch stream -> hipStream_t; None = torch's current stream; an int is taken as a raw handle."""
    if isinstance(stream, int):
        return stream
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


# ---- thin wrappers, one per C entry point --------------------------------------------------------
def mad_version() -> int:
    return lib().mad_version()


def mad_options_default() -> mad_options:
    o = mad_options()
    _check(lib().mad_options_default(C.byref(o)), "mad_options_default")
    return o


def mad_mesh_create(n_verts: int, tris: np.ndarray, comp_offsets: np.ndarray | None = None) -> C.c_void_p:
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    h = C.c_void_p()
    co = None if comp_offsets is None else np.ascontiguousarray(comp_offsets, dtype=np.int64)
    n_comp = 0 if co is None else co.size - 1
    _check(lib().mad_mesh_create(n_verts, tris.shape[0], _ptr(tris), n_comp, _ptr(co), C.byref(h)),
           "mad_mesh_create")
    return h


def mad_mesh_info(mesh) -> tuple[int, int, int, int]:
    v = [C.c_int64() for _ in range(4)]
    _check(lib().mad_mesh_info(mesh, *[C.byref(a) for a in v]), "mad_mesh_info")
    return tuple(a.value for a in v)


def mad_mesh_copy_diamonds(mesh) -> np.ndarray:
    nd = mad_mesh_info(mesh)[3]
    out = np.zeros((nd, 4), np.int32)
    _check(lib().mad_mesh_copy_diamonds(mesh, _ptr(out)), "mad_mesh_copy_diamonds")
    return out


def mad_mesh_destroy(mesh):
    _check(lib().mad_mesh_destroy(mesh), "mad_mesh_destroy")


def mad_problem_create(mesh, var_dim: int, precision: int, opt: mad_options | None = None) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().mad_problem_create(mesh, var_dim, precision, C.byref(opt) if opt is not None else None,
                                    C.byref(h)), "mad_problem_create")
    return h


def mad_problem_add_term(prob, kind: int, params=(), rest_pos: np.ndarray | None = None):
    prm = np.ascontiguousarray(params, dtype=np.float64)
    rp = None if rest_pos is None else np.ascontiguousarray(rest_pos, dtype=np.float64)
    _check(lib().mad_problem_add_term(prob, kind, _ptr(prm) if prm.size else None, prm.size, _ptr(rp)),
           "mad_problem_add_term")


def mad_problem_add_vertex_term(prob, kind: int, params, vdata):
    """vdata: device FP64 tensor [n_verts, 4] (m, xhat), read at every evaluation (keep it alive)."""
    prm = np.ascontiguousarray(params, dtype=np.float64)
    _check(lib().mad_problem_add_vertex_term(prob, kind, _ptr(prm) if prm.size else None, prm.size, _ptr(vdata)),
           "mad_problem_add_vertex_term")


def mad_problem_reserve_pairs(prob, max_pairs: int):
    _check(lib().mad_problem_reserve_pairs(prob, max_pairs), "mad_problem_reserve_pairs")


def mad_problem_insert_pairs(prob, pairs, n_pairs: int, stream=None) -> int:
    """pairs: device int32 tensor [n_pairs, 2]. Returns the number of blocks added."""
    added = C.c_int64()
    _check(lib().mad_problem_insert_pairs(prob, _ptr(pairs), n_pairs, C.byref(added), _stream(stream)),
           "mad_problem_insert_pairs")
    return added.value


def mad_problem_jacobian_info(prob) -> tuple[int, int]:
    m, nnz = C.c_int64(), C.c_int64()
    _check(lib().mad_problem_jacobian_info(prob, C.byref(m), C.byref(nnz)), "mad_problem_jacobian_info")
    return m.value, nnz.value


def mad_problem_copy_jacobian_pattern(prob, rowptr, colidx, stream=None):
    _check(lib().mad_problem_copy_jacobian_pattern(prob, _ptr(rowptr), _ptr(colidx), _stream(stream)),
           "mad_problem_copy_jacobian_pattern")


def mad_problem_jacobian(prob, x, r, vals, stream=None):
    _check(lib().mad_problem_jacobian(prob, _ptr(x), _ptr(r), _ptr(vals), _stream(stream)), "mad_problem_jacobian")


def mad_problem_finalize(prob, stream=None):
    _check(lib().mad_problem_finalize(prob, _stream(stream)), "mad_problem_finalize")


def mad_problem_pattern_info(prob) -> tuple[int, int, int]:
    r, n, b = C.c_int64(), C.c_int64(), C.c_int32()
    _check(lib().mad_problem_pattern_info(prob, C.byref(r), C.byref(n), C.byref(b)), "mad_problem_pattern_info")
    return r.value, n.value, b.value


def mad_problem_energy_count(prob) -> int:
    c = C.c_int32()
    _check(lib().mad_problem_energy_count(prob, C.byref(c)), "mad_problem_energy_count")
    return c.value


def mad_problem_copy_pattern(prob, rowptr, colidx, stream=None):
    _check(lib().mad_problem_copy_pattern(prob, _ptr(rowptr), _ptr(colidx), _stream(stream)),
           "mad_problem_copy_pattern")


def mad_problem_eval(prob, x, mode: int, energy=None, grad=None, hess=None, stream=None):
    _check(lib().mad_problem_eval(prob, _ptr(x), mode, _ptr(energy), _ptr(grad), _ptr(hess), _stream(stream)),
           "mad_problem_eval")


def mad_problem_eval_static(prob, x, mode: int, energy=None, grad=None, hess=None, stream=None):
    _check(lib().mad_problem_eval_static(prob, _ptr(x), mode, _ptr(energy), _ptr(grad), _ptr(hess),
                                         _stream(stream)), "mad_problem_eval_static")


def mad_problem_hvp(prob, x, v, mode: int, energy=None, grad=None, y=None, stream=None):
    _check(lib().mad_problem_hvp(prob, _ptr(x), _ptr(v), mode, _ptr(energy), _ptr(grad), _ptr(y), _stream(stream)),
           "mad_problem_hvp")


def mad_problem_status(prob, stream=None) -> tuple[bool, int]:
    nf, fb = C.c_int32(), C.c_int64()
    _check(lib().mad_problem_status(prob, C.byref(nf), C.byref(fb), _stream(stream)), "mad_problem_status")
    return bool(nf.value), fb.value


def mad_problem_set_profiling(prob, enable: bool):
    _check(lib().mad_problem_set_profiling(prob, 1 if enable else 0), "mad_problem_set_profiling")


def mad_problem_profile(prob) -> tuple[list[float], int]:
    ms = (C.c_double * 12)()
    n, k = C.c_int32(), C.c_int64()
    _check(lib().mad_problem_profile(prob, ms, C.byref(n), C.byref(k)), "mad_problem_profile")
    return [ms[i] for i in range(n.value)], k.value


def mad_problem_layout(prob) -> dict:
    sc, pf, pe, n, w = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().mad_problem_layout(prob, C.byref(sc), C.byref(pf), C.byref(pe), C.byref(n), C.byref(w)),
           "mad_problem_layout")
    return {"scatter": sc.value, "patch_faces": pf.value, "persistent": pe.value, "n_patches": n.value,
            "wg_waves": w.value}


def mad_problem_set_layout(prob, scatter: int, patch_faces: int, persistent: int, wg_waves: int = 0, stream=None):
    _check(lib().mad_problem_set_layout(prob, scatter, patch_faces, persistent, wg_waves, _stream(stream)),
           "mad_problem_set_layout")


def mad_problem_autotune(prob, x, mode: int, energy=None, grad=None, hess=None, reps: int = 5, flags: int = 0,
                         stream=None):
    _check(lib().mad_problem_autotune(prob, _ptr(x), mode, _ptr(energy), _ptr(grad), _ptr(hess), reps, flags,
                                      _stream(stream)), "mad_problem_autotune")


def mad_problem_tune_report(prob) -> str:
    n = C.c_int64()
    _check(lib().mad_problem_tune_report(prob, None, 0, C.byref(n)), "mad_problem_tune_report")
    buf = C.create_string_buffer(n.value + 1)
    _check(lib().mad_problem_tune_report(prob, buf, n.value + 1, C.byref(n)), "mad_problem_tune_report")
    return buf.value.decode()


def mad_problem_destroy(prob):
    _check(lib().mad_problem_destroy(prob), "mad_problem_destroy")


def mad_mlp_create(params: np.ndarray, s_in, s_out: float) -> C.c_void_p:
    p = np.ascontiguousarray(params, dtype=np.float32).ravel()
    si = np.ascontiguousarray(s_in, dtype=np.float32).ravel()
    if p.size != MLP_PARAMS or si.size != 6:
        raise ValueError("network parameters must have 4673 entries and s_in 6")
    out = C.c_void_p()
    _check(lib().mad_mlp_create(MLP_HIDDEN, p.ctypes.data, si.ctypes.data, float(s_out), C.byref(out)),
           "mad_mlp_create")
    return out


def mad_mlp_set_params(mlp, params: np.ndarray):
    p = np.ascontiguousarray(params, dtype=np.float32).ravel()
    if p.size != MLP_PARAMS:
        raise ValueError("network parameters must have 4673 entries")
    _check(lib().mad_mlp_set_params(mlp, p.ctypes.data), "mad_mlp_set_params")


def mad_mlp_get_params(mlp, which: int = 0) -> np.ndarray:
    out = np.zeros(MLP_PARAMS, np.float32)
    _check(lib().mad_mlp_get_params(mlp, which, out.ctypes.data), "mad_mlp_get_params")
    return out


def _c_g(c_g) -> np.ndarray:
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(c_g, dtype=np.float32), (6,)))
    return a


def mad_mlp_loss_grad(mlp, z, W, dW, idx, base: int, count: int, c_e: float, c_g, lam_g: float, grad, loss,
                      stream=None):
    cg = _c_g(c_g)
    _check(lib().mad_mlp_loss_grad(mlp, _ptr(z), _ptr(W), _ptr(dW), _ptr(idx), base, count, c_e, cg.ctypes.data,
                                   lam_g, _ptr(grad), _ptr(loss), _stream(stream)), "mad_mlp_loss_grad")


def mad_mlp_adam_step(mlp, grad, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None):
    _check(lib().mad_mlp_adam_step(mlp, _ptr(grad), lr, beta1, beta2, eps, _stream(stream)), "mad_mlp_adam_step")


def mad_mlp_train_epoch(mlp, z, W, dW, perm, n: int, batch: int, c_e: float, c_g, lam_g: float, lr: float,
                        beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, loss_hist=None, stream=None):
    cg = _c_g(c_g)
    _check(lib().mad_mlp_train_epoch(mlp, _ptr(z), _ptr(W), _ptr(dW), _ptr(perm), n, batch, c_e, cg.ctypes.data,
                                     lam_g, lr, beta1, beta2, eps, _ptr(loss_hist), _stream(stream)),
           "mad_mlp_train_epoch")


def mad_problem_add_mlp_term(prob, mlp, rest_pos: np.ndarray):
    r = np.ascontiguousarray(rest_pos, dtype=np.float64)
    _check(lib().mad_problem_add_mlp_term(prob, mlp, r.ctypes.data), "mad_problem_add_mlp_term")


# ---- convenience objects (still marshalling only) -----------------------------------------------
# parameters of the shell density trained on oracle samples (written by tests/train_density.py)
TRAINED_DENSITY = os.path.join(HERE, "data", "shell_density_net.npz")


class Network:
    """The learned density's network (FP32 master parameters, BF16 evaluation copy)."""

    def __init__(self, params: np.ndarray, s_in, s_out: float):
        self.handle = mad_mlp_create(params, s_in, s_out)
        self.s_in = np.asarray(s_in, np.float32)
        self.s_out = float(s_out)

    @classmethod
    def from_file(cls, path: str = TRAINED_DENSITY) -> "Network":
        """A network from saved parameters (theta, s_in, s_out arrays of an .npz file)."""
        with np.load(path, allow_pickle=False) as f:
            return cls(f["theta"], f["s_in"], float(f["s_out"][0]))

    def set_params(self, params):
        mad_mlp_set_params(self.handle, params)

    def params(self, which: int = 0) -> np.ndarray:
        return mad_mlp_get_params(self.handle, which)

    def loss_grad(self, z, W, dW, c_e, c_g, lam_g, idx=None, base=0, count=None, out=None, stream=None):
        import torch
        grad, loss = out if out is not None else (torch.empty(MLP_PARAMS, dtype=torch.float32, device=z.device),
                                                   torch.empty(1, dtype=torch.float32, device=z.device))
        n = z.shape[0] if count is None else count
        mad_mlp_loss_grad(self.handle, z, W, dW, idx, base, n, c_e, c_g, lam_g, grad, loss, stream)
        return grad, loss

    def adam_step(self, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        mad_mlp_adam_step(self.handle, grad, lr, beta1, beta2, eps, stream)

    def train_epoch(self, z, W, dW, perm, batch, c_e, c_g, lam_g, lr, beta1=0.9, beta2=0.999, eps=1e-8,
                    loss_hist=None, stream=None):
        mad_mlp_train_epoch(self.handle, z, W, dW, perm, int(perm.shape[0]), batch, c_e, c_g, lam_g, lr, beta1, beta2,
                            eps, loss_hist, stream)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.mad_mlp_destroy(h)
            self.handle = None

class Mesh:
    def __init__(self, tris: np.ndarray, n_verts: int, comp_offsets: np.ndarray | None = None):
        self.handle = mad_mesh_create(n_verts, tris, comp_offsets)
        self.n_verts, self.n_tris, self.n_edges, self.n_diamonds = mad_mesh_info(self.handle)

    def diamonds(self) -> np.ndarray:
        return mad_mesh_copy_diamonds(self.handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.mad_mesh_destroy(h)
            self.handle = None


class Problem:
    """mesh + var_dim + precision -> terms -> finalize -> eval (Sec. 4.2 programming model)."""

    def __init__(self, mesh: Mesh, var_dim: int, precision: int = F64, patch_faces: int = 0,
                 spd_eps: float = 0.0, degenerate_q: float = 0.0, scatter: int = SCATTER_AUTO,
                 lock_spins: int = 0, wg_waves: int = 0):
        o = mad_options_default()
        o.scatter = scatter
        o.lock_spins = lock_spins
        o.wg_waves = wg_waves
        o.patch_faces = patch_faces
        o.spd_eps = spd_eps
        o.degenerate_q = degenerate_q
        self.mesh = mesh
        self.var_dim = var_dim
        self.precision = precision
        self.handle = mad_problem_create(mesh.handle, var_dim, precision, o)

    def add_term(self, kind: int, params=(), rest_pos: np.ndarray | None = None):
        mad_problem_add_term(self.handle, kind, params, rest_pos)

    def reserve_pairs(self, max_pairs: int):
        mad_problem_reserve_pairs(self.handle, max_pairs)

    def insert_pairs(self, pairs, stream=None) -> int:
        """Add the blocks of interaction pairs (device int32 [n, 2]); refreshes nnzb."""
        added = mad_problem_insert_pairs(self.handle, pairs, int(pairs.shape[0]), stream)
        self.n_rows, self.nnzb, self.block_dim = mad_problem_pattern_info(self.handle)
        return added

    def jacobian_pattern(self, device="cuda"):
        import torch
        m, nnz = mad_problem_jacobian_info(self.handle)
        rowptr = torch.empty(m + 1, dtype=torch.int32, device=device)
        colidx = torch.empty(max(nnz, 1), dtype=torch.int32, device=device)
        mad_problem_copy_jacobian_pattern(self.handle, rowptr, colidx)
        return rowptr, colidx[:nnz]

    def jacobian(self, x, stream=None):
        """(r [m] FP64, vals [nnz]) of the residual terms at x (Eq. 3)."""
        import torch
        m, nnz = mad_problem_jacobian_info(self.handle)
        dt = torch.float32 if self.precision == F32 else torch.float64
        r = torch.empty(m, dtype=torch.float64, device=x.device)
        vals = torch.empty(max(nnz, 1), dtype=dt, device=x.device)
        mad_problem_jacobian(self.handle, x, r, vals, stream)
        return r, vals[:nnz]

    def add_vertex_term(self, kind: int, params, vdata):
        mad_problem_add_vertex_term(self.handle, kind, params, vdata)
        self._vdata = getattr(self, "_vdata", []) + [vdata]   # read at every evaluation

    def add_mlp_term(self, net: "Network", rest_pos: np.ndarray):
        mad_problem_add_mlp_term(self.handle, net.handle, rest_pos)
        self._nets = getattr(self, "_nets", []) + [net]    # the network must outlive the problem

    def finalize(self, stream=None):
        mad_problem_finalize(self.handle, stream)
        self.n_rows, self.nnzb, self.block_dim = mad_problem_pattern_info(self.handle)
        self.energy_count = mad_problem_energy_count(self.handle)

    def pattern(self, device="cuda"):
        import torch
        rowptr = torch.empty(self.n_rows + 1, dtype=torch.int32, device=device)
        colidx = torch.empty(max(self.nnzb, 1), dtype=torch.int32, device=device)
        mad_problem_copy_pattern(self.handle, rowptr, colidx)
        return rowptr, colidx[:self.nnzb]

    def outputs(self, device="cuda"):
        """Allocate (energy, grad, hess) device buffers of the right dtype and size."""
        import torch
        dt = torch.float32 if self.precision == F32 else torch.float64
        d = self.var_dim
        energy = torch.empty(self.energy_count, dtype=torch.float64, device=device)
        grad = torch.empty(self.n_rows * d, dtype=dt, device=device)
        hess = torch.empty((self.nnzb, d, d), dtype=dt, device=device)
        return energy, grad, hess

    def eval(self, x, mode: int = ENERGY | GRAD | HESS, out=None, stream=None):
        energy, grad, hess = out if out is not None else self.outputs(x.device)
        mad_problem_eval(self.handle, x, mode, energy if mode & ENERGY else None,
                         grad if mode & GRAD else None, hess if mode & HESS else None, stream)
        return energy, grad, hess

    def eval_static(self, x, mode: int = ENERGY | GRAD | HESS, out=None, stream=None):
        """mad_problem_eval_static: the same evaluation with the library's static scratch (no allocation
        inside the call; `out` must then be given by callers that cannot allocate)."""
        energy, grad, hess = out if out is not None else self.outputs(x.device)
        mad_problem_eval_static(self.handle, x, mode, energy if mode & ENERGY else None,
                                grad if mode & GRAD else None, hess if mode & HESS else None, stream)
        return energy, grad, hess

    def status(self, stream=None):
        return mad_problem_status(self.handle, stream)

    def hvp(self, x, v, mode: int = 0, out=None, stream=None):
        """y = H(x) v without assembling H (mode: MAD_SPD for the clamped Hessian; ENERGY/GRAD extra)."""
        import torch
        energy, grad, _ = out if out is not None else self.outputs(x.device)
        y = torch.empty_like(grad)
        mad_problem_hvp(self.handle, x, v, mode, energy if mode & ENERGY else None, grad if mode & GRAD else None, y,
                        stream)
        return y, energy, grad

    def layout(self) -> dict:
        return mad_problem_layout(self.handle)

    def set_layout(self, scatter: int, patch_faces: int, persistent: int = 0, wg_waves: int = 0, stream=None):
        mad_problem_set_layout(self.handle, scatter, patch_faces, persistent, wg_waves, stream)

    def autotune(self, x, mode: int = ENERGY | GRAD | HESS, out=None, reps: int = 5, force: bool = False,
                 stream=None) -> dict:
        """Time the candidate layouts on x and keep the fastest; returns the timing report."""
        import json
        energy, grad, hess = out if out is not None else self.outputs(x.device)
        mad_problem_autotune(self.handle, x, mode, energy if mode & ENERGY else None, grad if mode & GRAD else None,
                             hess if mode & HESS else None, reps, TUNE_FORCE if force else 0, stream)
        return json.loads(mad_problem_tune_report(self.handle))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.mad_problem_destroy(h)
            self.handle = None
