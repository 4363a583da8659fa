"""Full-size parity of the parameterisation, batched and learned-density workloads, each in the launch
configuration the benchmark times (whole pattern bit-exact, sampled block rows and gradient rows against the
oracle element by element, energies against an independent vectorised FP64 evaluation):

* symmetric Dirichlet on the 1001 x 1001 warped grid (2,000,000 triangles, 2x2 blocks, clamped), FP32 and
  FP64: the two-DOF persistent multi-patch path at size, and its matrix-free Hessian-vector product (clamped
  and plain) on the same sampled rows;
* 700 geodesic icospheres of lognormal size in one autotuned launch: sampled rows over all meshes and every
  per-component energy, also in FP64 and through the clamped matrix-free product;
* the learned density on the 708 x 708 cylinder (999,698 triangles), FP32 and FP64, and its clamped
  matrix-free product: the network pass loops over many tiles per wave at this size.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_00406_amd import meshgen
from tests import npref
from tests import parity as PR

pytestmark = pytest.mark.gpu
SPD_ALL = 1 | 2 | 4 | 8


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


def sample_rows(nv, k, seed, extra=()):
    rng = np.random.default_rng(seed)
    rows = set(rng.choice(nv, k, replace=False).tolist()) | set(int(r) for r in extra if 0 <= r < nv)
    mask = np.zeros(nv, bool)
    mask[sorted(rows)] = True
    return mask


def sampled_compare(P, mask, x, grad, hess, d, rtol):
    ref = P.eval(x, O.GRAD | O.HESS | O.SPD, row_mask=mask)
    rows = np.nonzero(mask)[0]
    gi = np.concatenate([np.arange(d * r, d * r + d) for r in rows])
    g = PR.assert_close("grad(sampled)", grad[gi], ref.grad[gi], ref.gscale[gi], rtol)
    bi = np.concatenate([np.arange(P.rowptr[r], P.rowptr[r + 1]) for r in rows])
    h = PR.assert_close("hess(sampled)", hess[bi], ref.hess[bi], ref.hscale[bi], rtol)
    return g, h, bi.size


# ------------------------------------------------------------------ symmetric Dirichlet, 1001^2
@pytest.fixture(scope="module")
def symdir_full():
    say("symdir 1001 oracle setup")
    inp = meshgen.warped_grid(n=1001, seed=3001)
    P = PR.build_oracle(inp.tris, inp.rest, inp.n_verts, 2, [(6, ())])
    n = 1001
    mask = sample_rows(inp.n_verts, 240, 321, extra=(0, n - 1, n, n * n - 1, n * n - n, n * (n // 2) + n // 2))
    e_ref, e_abs = npref.symdir_energy(inp.tris, inp.rest, inp.x)
    return inp, P, mask, e_ref, e_abs


@pytest.mark.parametrize("precision", [1, 0])
def test_symdir_1001_sampled(torch_cuda, symdir_full, precision):
    from paper_2509_00406_amd import mad
    torch = torch_cuda
    inp, P, mask, e_ref, e_abs = symdir_full
    say("symdir 1001", "fp32" if precision else "fp64")
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 2, [(6, ())], precision)
    lay = prob.layout()
    assert lay["scatter"] == mad.SCATTER_PATCH and lay["persistent"] == 1 and lay["n_patches"] > 1000
    rp, ci = [t.cpu().numpy() for t in prob.pattern()]
    assert np.array_equal(rp, P.rowptr) and np.array_equal(ci, P.colidx)
    assert rp[-1] == 7006001
    x = torch.from_numpy(inp.x.ravel().copy()).cuda()
    energy, grad, hess = prob.eval(x, SPD_ALL)
    torch.cuda.synchronize()
    nonfinite, fallbacks = prob.status()
    assert not nonfinite
    rtol = PR.RTOL[precision]
    g, h, nb = sampled_compare(P, mask, inp.x, grad.cpu().numpy(), hess.cpu().numpy(), 2, rtol)
    e = float(energy.cpu()[0])
    assert abs(e - e_ref) <= rtol * e_abs, (e, e_ref, e_abs)
    say(f"layout {lay}; worst grad {g:.2e} hess {h:.2e} over {nb} blocks; energy {e:.12e} vs {e_ref:.12e}; "
        f"fp64 fallbacks {fallbacks}")


@pytest.mark.parametrize("precision,spd", [(1, True), (1, False), (0, True), (0, False)])
def test_symdir_1001_hvp(torch_cuda, symdir_full, precision, spd):
    """The matrix-free product (Sec. 5.5 matrix-free mode) at the benchmark size: y = H v on the sampled rows
    against the oracle's sampled block rows applied to the same v (per entry within rtol of
    sum_b scale_b |v|), clamped and plain, with the same pass's energy."""
    from paper_2509_00406_amd import mad
    torch = torch_cuda
    inp, P, mask, e_ref, e_abs = symdir_full
    say("symdir 1001 hvp", "fp32" if precision else "fp64", "clamped" if spd else "plain")
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 2, [(6, ())], precision)
    x = np.ascontiguousarray(inp.x, dtype=np.float64).ravel()
    v = np.random.default_rng(78).normal(size=x.size)
    y, energy, _ = prob.hvp(torch.from_numpy(x).cuda(), torch.from_numpy(v).cuda(),
                            mad.ENERGY | (mad.SPD if spd else 0))
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    ref = P.eval(inp.x, O.HESS | (O.SPD if spd else 0), row_mask=mask)
    rows = np.nonzero(mask)[0]
    yref = np.zeros((rows.size, 2))
    yscale = np.zeros((rows.size, 2))
    V = v.reshape(-1, 2)
    for n, r in enumerate(rows):
        for b in range(P.rowptr[r], P.rowptr[r + 1]):
            c = P.colidx[b]
            yref[n] += ref.hess[b].reshape(2, 2) @ V[c]
            yscale[n] += ref.hscale[b].reshape(2, 2) @ np.abs(V[c])
    gi = np.concatenate([np.arange(2 * r, 2 * r + 2) for r in rows])
    rtol = PR.RTOL[precision]
    w = PR.assert_close("hvp(sampled)", y[gi], yref.ravel(), yscale.ravel(), rtol)
    e = float(energy.cpu()[0])
    assert abs(e - e_ref) <= rtol * e_abs, (e, e_ref, e_abs)
    say(f"hvp: worst {w:.2e} over {rows.size} rows")


# ------------------------------------------------------------------ 700 icospheres, autotuned
ICO_TERMS = [(4, (1.0, 1.0)), (5, (1.0, 1.0))]


@pytest.fixture(scope="module")
def ico_full():
    say("700 icospheres oracle setup")
    inp = meshgen.icosphere_batch(n_meshes=700)
    P = PR.build_oracle(inp.tris, inp.rest, inp.n_verts, 3, ICO_TERMS)
    co = inp.comp_offsets
    # rows of the first, last and a spread of meshes, plus random ones
    extra = [int(co[c]) for c in (0, 1, 350, 698, 699)] + [int(co[c + 1]) - 1 for c in (0, 350, 699)]
    mask = sample_rows(inp.n_verts, 240, 654, extra=extra)
    e_ref, e_abs = npref.shell_energy_by_component(inp.tris, inp.rest, inp.x, P.topo.diamonds,
                                                   P.topo.diamond_faces, (1.0, 1.0), (1.0, 1.0), co)
    return inp, P, mask, e_ref, e_abs


def check_component_energies(e, e_ref, e_abs, rtol):
    assert e.shape[0] == 701
    bad = np.nonzero(np.abs(e[1:] - e_ref) > rtol * e_abs)[0]
    assert bad.size == 0, (bad[:5], e[1 + bad[:5]], e_ref[bad[:5]])
    assert abs(e[0] - e_ref.sum()) <= rtol * e_abs.sum()


def test_icospheres_700_autotuned(torch_cuda, ico_full):
    torch = torch_cuda
    inp, P, mask, e_ref, e_abs = ico_full
    co = inp.comp_offsets
    say("700 icospheres GPU, autotune")
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, ICO_TERMS, 1, comp_offsets=co)
    x = torch.from_numpy(inp.x.ravel().copy()).cuda()
    out = prob.outputs()
    tune = prob.autotune(x, SPD_ALL, out=out, reps=3, force=True)
    lay = prob.layout()
    rp, ci = [t.cpu().numpy() for t in prob.pattern()]
    assert np.array_equal(rp, P.rowptr) and np.array_equal(ci, P.colidx)
    energy, grad, hess = prob.eval(x, SPD_ALL, out=out)
    torch.cuda.synchronize()
    nonfinite, fallbacks = prob.status()
    assert not nonfinite
    rtol = PR.RTOL[1]
    g, h, nb = sampled_compare(P, mask, inp.x, grad.cpu().numpy(), hess.cpu().numpy(), 3, rtol)
    check_component_energies(energy.cpu().numpy(), e_ref, e_abs, rtol)
    say(f"chosen {tune.get('chosen')} layout {lay}; worst grad {g:.2e} hess {h:.2e} over {nb} blocks; "
        f"700 component energies in bounds; fp64 fallbacks {fallbacks}")


def test_icospheres_700_fp64(torch_cuda, ico_full):
    """The batched persistent launch in FP64 at the default layout: sampled rows and every component energy
    at the FP64 tolerance."""
    torch = torch_cuda
    inp, P, mask, e_ref, e_abs = ico_full
    say("700 icospheres GPU, fp64")
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, ICO_TERMS, 0, comp_offsets=inp.comp_offsets)
    lay = prob.layout()
    assert lay["persistent"] == 1
    x = torch.from_numpy(inp.x.ravel().copy()).cuda()
    energy, grad, hess = prob.eval(x, SPD_ALL)
    torch.cuda.synchronize()
    assert not prob.status()[0]
    rtol = PR.RTOL[0]
    g, h, nb = sampled_compare(P, mask, inp.x, grad.cpu().numpy(), hess.cpu().numpy(), 3, rtol)
    check_component_energies(energy.cpu().numpy(), e_ref, e_abs, rtol)
    say(f"layout {lay}; worst grad {g:.2e} hess {h:.2e} over {nb} blocks; 700 component energies in bounds")


def test_icospheres_700_hvp_fp32(torch_cuda, ico_full):
    """The clamped matrix-free product over the 700 meshes in one launch: y = H v on the sampled rows against the
    oracle's sampled block rows applied to the same v, and the per-component energies of the same pass."""
    from paper_2509_00406_amd import mad
    torch = torch_cuda
    inp, P, mask, e_ref, e_abs = ico_full
    say("700 icospheres GPU, clamped hvp fp32")
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, ICO_TERMS, 1, comp_offsets=inp.comp_offsets)
    x = np.ascontiguousarray(inp.x, dtype=np.float64).ravel()
    v = np.random.default_rng(79).normal(size=x.size)
    y, energy, _ = prob.hvp(torch.from_numpy(x).cuda(), torch.from_numpy(v).cuda(), mad.ENERGY | mad.SPD)
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    ref = P.eval(inp.x, O.HESS | O.SPD, row_mask=mask)
    rows = np.nonzero(mask)[0]
    yref = np.zeros((rows.size, 3))
    yscale = np.zeros((rows.size, 3))
    V = v.reshape(-1, 3)
    for n, r in enumerate(rows):
        for b in range(P.rowptr[r], P.rowptr[r + 1]):
            c = P.colidx[b]
            yref[n] += ref.hess[b].reshape(3, 3) @ V[c]
            yscale[n] += ref.hscale[b].reshape(3, 3) @ np.abs(V[c])
    gi = np.concatenate([np.arange(3 * r, 3 * r + 3) for r in rows])
    rtol = PR.RTOL[1]
    w = PR.assert_close("hvp(sampled)", y[gi], yref.ravel(), yscale.ravel(), rtol)
    check_component_energies(energy.cpu().numpy(), e_ref, e_abs, rtol)
    say(f"hvp: worst {w:.2e} over {rows.size} rows; 700 component energies in bounds")


# ------------------------------------------------------------------ learned density, 708^2
@pytest.fixture(scope="module")
def mlp_full():
    from tests.test_gpu_mlp import bf16_round, oracle_params, seeded_network
    say("mlp 708 oracle setup")
    inp = meshgen.shell_cylinder(n=708, seed=5001)
    theta, s_in, s_out = seeded_network(seed=17, scale=0.6)
    tb = bf16_round(theta)
    P = O.Problem(inp.tris, inp.rest, inp.n_verts, 3)
    P.add_term(O.MLP, oracle_params(tb, s_in, s_out))
    P.build_pattern()
    n = 708
    mask = sample_rows(inp.n_verts, 200, 987, extra=(0, n - 1, n * n - 1, n * (n // 2) + n // 2))
    e_ref, e_abs = npref.mlp_energy(inp.tris, inp.rest, inp.x, tb, s_in.astype(np.float64), float(s_out))
    return inp, P, mask, (theta, s_in, s_out), e_ref, e_abs


@pytest.mark.parametrize("precision", [1, 0])
def test_mlp_708_sampled(torch_cuda, mlp_full, precision):
    from paper_2509_00406_amd import mad
    from tests.test_gpu_mlp import RTOL_MLP
    torch = torch_cuda
    inp, P, mask, (theta, s_in, s_out), e_ref, e_abs = mlp_full
    say("mlp 708", "fp32" if precision else "fp64")
    mesh = mad.Mesh(inp.tris, inp.n_verts)
    prob = mad.Problem(mesh, 3, precision)
    net = mad.Network(theta, s_in, s_out)
    prob.add_mlp_term(net, inp.rest)
    prob.finalize()
    rp, ci = [t.cpu().numpy() for t in prob.pattern()]
    assert np.array_equal(rp, P.rowptr) and np.array_equal(ci, P.colidx)
    assert rp[-1] == 3503186
    x = torch.from_numpy(inp.x.ravel().copy()).cuda()
    energy, grad, hess = prob.eval(x, SPD_ALL)
    torch.cuda.synchronize()
    nonfinite, fallbacks = prob.status()
    assert not nonfinite
    rtol = max(PR.RTOL[precision], RTOL_MLP)
    g, h, nb = sampled_compare(P, mask, inp.x, grad.cpu().numpy(), hess.cpu().numpy(), 3, rtol)
    e = float(energy.cpu()[0])
    assert abs(e - e_ref) <= rtol * e_abs, (e, e_ref, e_abs)
    say(f"worst grad {g:.2e} hess {h:.2e} over {nb} blocks; energy {e:.12e} vs {e_ref:.12e}")


def test_mlp_708_hvp_fp32(torch_cuda, mlp_full):
    """The clamped matrix-free product through the network pass at 708^2 (many network tiles per wave): y = H v
    on the sampled rows against the oracle's sampled block rows applied to the same v, and the pass's energy."""
    from paper_2509_00406_amd import mad
    from tests.test_gpu_mlp import RTOL_MLP
    torch = torch_cuda
    inp, P, mask, (theta, s_in, s_out), e_ref, e_abs = mlp_full
    say("mlp 708 clamped hvp fp32")
    mesh = mad.Mesh(inp.tris, inp.n_verts)
    prob = mad.Problem(mesh, 3, 1)
    prob.add_mlp_term(mad.Network(theta, s_in, s_out), inp.rest)
    prob.finalize()
    x = np.ascontiguousarray(inp.x, dtype=np.float64).ravel()
    v = np.random.default_rng(80).normal(size=x.size)
    y, energy, _ = prob.hvp(torch.from_numpy(x).cuda(), torch.from_numpy(v).cuda(), mad.ENERGY | mad.SPD)
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    ref = P.eval(inp.x, O.HESS | O.SPD, row_mask=mask)
    rows = np.nonzero(mask)[0]
    yref = np.zeros((rows.size, 3))
    yscale = np.zeros((rows.size, 3))
    V = v.reshape(-1, 3)
    for n, r in enumerate(rows):
        for b in range(P.rowptr[r], P.rowptr[r + 1]):
            c = P.colidx[b]
            yref[n] += ref.hess[b].reshape(3, 3) @ V[c]
            yscale[n] += ref.hscale[b].reshape(3, 3) @ np.abs(V[c])
    gi = np.concatenate([np.arange(3 * r, 3 * r + 3) for r in rows])
    rtol = max(PR.RTOL[1], RTOL_MLP)
    w = PR.assert_close("hvp(sampled)", y[gi], yref.ravel(), yscale.ravel(), rtol)
    e = float(energy.cpu()[0])
    assert abs(e - e_ref) <= rtol * e_abs, (e, e_ref, e_abs)
    say(f"hvp: worst {w:.2e} over {rows.size} rows")
