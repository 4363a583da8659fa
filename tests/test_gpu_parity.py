"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs, element by element. Sizes span several patches with
ragged tails; edge cases cover empty terms, isolated vertices, non-manifold
edges, closed meshes and batched components."""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_00406_amd import meshgen
from tests import parity as PR

pytestmark = pytest.mark.gpu

ALL = 1 | 2 | 4


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_00406_amd import mad
    mad.lib()
    return torch


def run_case(torch, tris, rest, x, var_dim, terms, precision, mode, patch_faces=0, comp_offsets=None,
             spd_eps=0.0, check_energy=True, scatter=0):
    nv = rest.shape[0]
    mesh, prob = PR.build_gpu(tris, rest, nv, var_dim, terms, precision, comp_offsets, patch_faces, spd_eps,
                              scatter)
    P = PR.build_oracle(tris, rest, nv, var_dim, terms)
    rowptr, colidx = prob.pattern()
    assert np.array_equal(rowptr.cpu().numpy(), P.rowptr), "pattern rowptr differs"
    assert np.array_equal(colidx.cpu().numpy(), P.colidx), "pattern colidx differs"
    xt = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64).ravel()).cuda()
    energy, grad, hess = prob.eval(xt, mode | 1)
    torch.cuda.synchronize()
    nonfinite, fallbacks = prob.status()
    ref = P.eval(x, (mode | 1) & 15, spd_eps=spd_eps)
    rtol = PR.RTOL[precision]
    out = {"fallbacks": fallbacks, "nonfinite": nonfinite}
    if check_energy:
        e = energy.cpu().numpy()
        assert abs(e[0] - ref.energy) <= rtol * ref.esum_abs + 1e-300, (e[0], ref.energy, ref.esum_abs)
    # per entry against the contributing elements' scale; for the Hessian also the headline norm-wise error
    # max |H - H_ref| / max |H_ref| under the same bar (the gradient's is reported only: near a stationary
    # point max |g_ref| is itself a sum that cancels, and no bar relative to it is meaningful)
    if mode & 2:
        out["grad"] = PR.assert_close("grad", grad.cpu().numpy(), ref.grad, ref.gscale, rtol)
        out["grad_norm"] = PR.normwise(grad.cpu().numpy(), ref.grad)
    if mode & 4:
        out["hess"] = PR.assert_close("hess", hess.cpu().numpy(), ref.hess, ref.hscale, rtol)
        out["hess_norm"] = PR.normwise(hess.cpu().numpy(), ref.hess)
        assert out["hess_norm"] <= rtol, out
    return out, prob, (energy, grad, hess)


SHELL = [(4, (0.9, 1.3)), (5, (1.1, 1.0))]     # StVK (mu, lambda) + bending (k_b, h)


# ---------------------------------------------------------------- Dirichlet energy, 64 x 64 jittered grid
def test_dirichlet_64_fp64_vs_oracle_and_cot_laplacian(torch_cuda):
    say("dirichlet 64x64 fp64")
    inp = meshgen.dirichlet_grid(64)
    out, prob, (energy, grad, hess) = run_case(torch_cuda, inp.tris, inp.rest, inp.x, 1, [(3, ())], 0, ALL)
    # the assembled Hessian is the cotangent Laplacian, gradient L u, energy u^T L u / 2
    tris, pos, u = inp.tris, inp.rest, inp.x.ravel()
    rows, cols, vals = [], [], []
    for c in range(3):
        a, b, k = tris[:, (c + 1) % 3], tris[:, (c + 2) % 3], tris[:, c]
        e1, e2 = pos[a] - pos[k], pos[b] - pos[k]
        w = 0.5 * np.einsum("ij,ij->i", e1, e2) / np.linalg.norm(np.cross(e1, e2), axis=1)
        rows += [a, b, a, b]; cols += [b, a, a, b]; vals += [-w, -w, w, w]
    rows, cols, vals = map(np.concatenate, (rows, cols, vals))
    from scipy.sparse import coo_matrix
    L = coo_matrix((vals, (rows, cols)), shape=(4096, 4096)).tocsr()
    rp, ci = [t.cpu().numpy() for t in prob.pattern()]
    H = hess.cpu().numpy().ravel()
    ri = np.repeat(np.arange(4096, dtype=np.int64), np.diff(rp).astype(np.int64))
    Lv = np.asarray(L[ri, ci.astype(np.int64)]).ravel()
    assert np.max(np.abs(H - Lv)) <= 1e-12 * np.max(np.abs(Lv))
    Lu = L @ u
    assert np.max(np.abs(grad.cpu().numpy() - Lu)) <= 1e-12 * np.max(np.abs(Lu))
    assert energy.cpu().numpy()[0] == pytest.approx(0.5 * u @ Lu, rel=1e-12)


# ---------------------------------------------------------------- elastic shell: StVK + bending
@pytest.mark.parametrize("scatter", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("spd", [False, True])
def test_shell_cylinder_small(torch_cuda, precision, spd, scatter):
    say("shell cylinder n=40", "fp32" if precision else "fp64", "spd" if spd else "raw", "scatter", scatter)
    inp = meshgen.shell_cylinder(n=40, seed=2001)
    mode = ALL | (8 if spd else 0)
    out, _, _ = run_case(torch_cuda, inp.tris, inp.rest, inp.x, 3, SHELL, precision, mode, patch_faces=96,
                         scatter=scatter)
    assert not out["nonfinite"]
    say("worst err/scale", out)


@pytest.mark.parametrize("precision", [0, 1])
def test_shell_stress_noise_near_degenerate(torch_cuda, precision):
    say("shell cylinder n=48 absolute noise", precision)
    inp = meshgen.shell_cylinder(n=48, seed=2002, noise="absolute")
    out, _, _ = run_case(torch_cuda, inp.tris, inp.rest, inp.x, 3, SHELL, precision, ALL | 8, patch_faces=200)
    say("stress", out)


def test_shell_spd_eps_positive(torch_cuda):
    say("shell spd eps 1e-3")
    inp = meshgen.shell_cylinder(n=20, seed=7)
    run_case(torch_cuda, inp.tris, inp.rest, inp.x, 3, SHELL, 0, ALL | 8, patch_faces=64, spd_eps=1e-3)


# ---------------------------------------------------------------- symmetric Dirichlet
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("spd", [False, True])
def test_symdir_warped_grid(torch_cuda, precision, spd):
    say("symdir warped n=33", precision, spd)
    inp = meshgen.warped_grid(n=33, seed=3001)
    run_case(torch_cuda, inp.tris, inp.rest, inp.x, 2, [(6, ())], precision, ALL | (8 if spd else 0),
             patch_faces=100)


# ---------------------------------------------------------------- catalogue terms of the paper's listings
@pytest.mark.parametrize("precision", [0, 1])
def test_area_and_edge_terms(torch_cuda, precision):
    say("area + edge sqlen", precision)
    tris, pos = meshgen.icosphere(6)
    x = pos + 0.05 * np.random.default_rng(3).normal(size=pos.shape)
    run_case(torch_cuda, tris, pos, x, 3, [(2, ()), (1, ())], precision, ALL, patch_faces=50)
    run_case(torch_cuda, tris, pos, x, 3, [(2, ())], precision, ALL | 8, patch_faces=50)


# ---------------------------------------------------------------- modes
@pytest.mark.parametrize("precision", [0, 1])
def test_modes_are_consistent(torch_cuda, precision):
    say("modes", precision)
    torch = torch_cuda
    inp = meshgen.shell_cylinder(n=24, seed=11)
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, SHELL, precision, patch_faces=64)
    xt = torch.from_numpy(inp.x.ravel().copy()).cuda()
    e_all, g_all, h_all = [t.clone() for t in prob.eval(xt, ALL | 8)]
    e_pas, _, _ = prob.eval(xt, 1)
    e_g, g_g, _ = prob.eval(xt, 1 | 2)
    _, _, h_only = prob.eval(xt, 4 | 8)
    rtol = PR.RTOL[precision]
    assert abs(float(e_pas[0]) - float(e_all[0])) <= 1e-13 * abs(float(e_all[0])) + 1e-300
    assert abs(float(e_g[0]) - float(e_all[0])) <= 1e-13 * abs(float(e_all[0])) + 1e-300
    gd = (g_g - g_all).abs().max().item()
    assert gd <= rtol * g_all.abs().max().item()
    hd = (h_only - h_all).abs().max().item()
    assert hd <= rtol * h_all.abs().max().item()


def test_energy_is_deterministic(torch_cuda):
    say("energy determinism")
    torch = torch_cuda
    inp = meshgen.shell_cylinder(n=64, seed=5)
    for precision in (0, 1):
        mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, SHELL, precision)
        xt = torch.from_numpy(inp.x.ravel().copy()).cuda()
        es = [prob.eval(xt, ALL | 8)[0].cpu().numpy().copy() for _ in range(3)]
        assert all(np.array_equal(es[0], e) for e in es[1:])


# ---------------------------------------------------------------- edge cases
@pytest.mark.parametrize("name", ["two_tris", "octahedron", "nonmanifold", "grid2", "grid3", "dup_face"])
def test_tiny_meshes(torch_cuda, name):
    say("tiny", name)
    if name == "dup_face":
        # a face repeated with the opposite orientation: the shared edge's diamond has v2 == v3
        tris, pos = meshgen.grid(4)
        tris = np.concatenate([tris, [[0, 1, 5], [1, 0, 5]]]).astype(np.int32)
    else:
        tris, pos = meshgen.tiny_meshes()[name]
    x = pos + 0.1 * np.random.default_rng(1).normal(size=pos.shape)
    for precision in (0, 1):
        for scatter in (1, 2):
            out, _, _ = run_case(torch_cuda, tris, pos, x, 3, SHELL, precision, ALL | 8, scatter=scatter)


def test_isolated_vertex_gets_zero_diagonal(torch_cuda):
    say("isolated vertex")
    tris, pos = meshgen.tiny_meshes()["nonmanifold"]
    mesh, prob = PR.build_gpu(tris, pos, pos.shape[0], 3, SHELL, 0)
    rp, ci = [t.cpu().numpy() for t in prob.pattern()]
    assert rp[6] - rp[5] == 1 and ci[rp[5]] == 5
    import torch
    _, g, h = prob.eval(torch.from_numpy(pos.ravel().copy()).cuda(), ALL)
    assert np.all(h.cpu().numpy()[rp[5]] == 0) and np.all(g.cpu().numpy()[15:18] == 0)


def test_single_patch_and_many_patches_agree(torch_cuda):
    say("patch sizes")
    torch = torch_cuda
    inp = meshgen.shell_cylinder(n=30, seed=9)
    res = []
    for pf, sc in ((8, 2), (64, 2), (100000, 2), (64, 1)):
        mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, SHELL, 0, patch_faces=pf, scatter=sc)
        e, g, h = prob.eval(torch.from_numpy(inp.x.ravel().copy()).cuda(), ALL | 8)
        res.append((e.cpu().numpy()[0], g.cpu().numpy(), h.cpu().numpy()))
    for e, g, h in res[1:]:
        assert abs(e - res[0][0]) <= 1e-13 * abs(res[0][0])
        assert np.max(np.abs(g - res[0][1])) <= 1e-13 * np.max(np.abs(res[0][1]))
        assert np.max(np.abs(h - res[0][2])) <= 1e-13 * np.max(np.abs(res[0][2]))


def test_batched_components_energy(torch_cuda):
    say("batched icospheres 12")
    torch = torch_cuda
    inp = meshgen.icosphere_batch(n_meshes=12, mean_verts=900, vmin=500, vmax=3000)
    co = inp.comp_offsets
    out, prob, (energy, grad, hess) = run_case(torch, inp.tris, inp.rest, inp.x, 3, SHELL, 1, ALL | 8,
                                               patch_faces=256, comp_offsets=co)
    e = energy.cpu().numpy()
    assert e.size == 13
    # per-component energies against the oracle on each component alone
    for c in range(12):
        lo, hi = co[c], co[c + 1]
        sel = np.all((inp.tris >= lo) & (inp.tris < hi), axis=1)
        t = inp.tris[sel] - lo
        P = PR.build_oracle(t, inp.rest[lo:hi], hi - lo, 3, SHELL)
        r = P.eval(inp.x[lo:hi], 1)
        assert abs(e[1 + c] - r.energy) <= 1e-5 * r.esum_abs
    assert e[0] == pytest.approx(e[1:].sum(), rel=1e-14)


def test_invalid_eval_arguments(torch_cuda):
    say("invalid eval args")
    torch = torch_cuda
    from paper_2509_00406_amd import mad
    inp = meshgen.shell_cylinder(n=8, seed=1)
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, SHELL, 1)
    xt = torch.from_numpy(inp.x.ravel().copy()).cuda()
    e, g, h = prob.outputs()
    with pytest.raises(mad.MadError):
        mad.mad_problem_eval(prob.handle, xt, 2, e, None, h)        # gradient requested, no buffer
    with pytest.raises(mad.MadError):
        mad.mad_problem_eval(prob.handle, xt, 8 | 1, e, g, h)       # SPD without HESS
    with pytest.raises(mad.MadError):
        mad.mad_problem_eval(prob.handle, None, 1, e, g, h)
    with pytest.raises(mad.MadError):
        mad.mad_problem_finalize(prob.handle)                       # twice


def test_nonfinite_input_is_flagged(torch_cuda):
    say("nonfinite flag")
    torch = torch_cuda
    inp = meshgen.shell_cylinder(n=8, seed=1)
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, SHELL, 1)
    x = inp.x.ravel().copy()
    x[5] = float("nan")
    prob.eval(torch.from_numpy(x).cuda(), ALL | 8)
    nf, _ = prob.status()
    assert nf
    prob.eval(torch.from_numpy(inp.x.ravel().copy()).cuda(), ALL | 8)
    nf, _ = prob.status()
    assert not nf
