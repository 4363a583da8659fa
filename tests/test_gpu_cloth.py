"""GPU parity of the mass-spring cloth step (Sec. 7.1: edge springs plus per-vertex inertia and
gravity, raw and filtered Hessians) through the C ABI against the oracle: the block pattern
bit-exact, energy, gradient and Hessian entries within the parity bar (rtol 1e-12 FP64 / 1e-5 FP32
of the contributing elements' magnitudes), matrix-free products, the per-vertex data read from the
caller's device array at every evaluation, and the full 1000 x 1000 step on sampled rows."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_00406_amd import meshgen
from tests import npref
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


def build_gpu(torch, inp, precision, scatter=0, patch_faces=0, spd_eps=0.0):
    from paper_2509_00406_amd import mad
    mesh = mad.Mesh(inp.tris, inp.n_verts)
    prob = mad.Problem(mesh, 3, precision, patch_faces=patch_faces, spd_eps=spd_eps, scatter=scatter)
    prob.add_term(mad.SPRING, inp.meta["spring_params"], inp.rest)
    vd = torch.from_numpy(np.ascontiguousarray(inp.meta["vdata"])).cuda()
    prob.add_vertex_term(mad.INERTIA, inp.meta["inertia_params"], vd)
    prob.finalize()
    return mesh, prob, vd


def build_oracle(inp, vdata=None):
    P = O.Problem(inp.tris, inp.rest, inp.n_verts, 3)
    P.add_term(O.SPRING, inp.meta["spring_params"])
    P.add_term(O.INERTIA, inp.meta["inertia_params"],
               vertex_data=inp.meta["vdata"] if vdata is None else vdata)
    P.build_pattern()
    return P


def compare(torch, prob, P, x, mode, precision, spd_eps=0.0):
    xt = torch.from_numpy(np.ascontiguousarray(x).ravel().copy()).cuda()
    energy, grad, hess = prob.eval(xt, mode)
    torch.cuda.synchronize()
    ref = P.eval(x, mode, spd_eps=spd_eps)
    rtol = PR.RTOL[precision]
    e = float(energy.cpu()[0])
    assert abs(e - ref.energy) <= rtol * ref.esum_abs, (e, ref.energy)
    out = {}
    if mode & 2:
        out["grad"] = PR.assert_close("grad", grad.cpu().numpy(), ref.grad, ref.gscale, rtol)
    if mode & 4:
        out["hess"] = PR.assert_close("hess", hess.cpu().numpy(), ref.hess, ref.hscale, rtol)
    nonfinite, fallbacks = prob.status()
    assert not nonfinite
    out["fallbacks"] = fallbacks
    return out


@pytest.mark.parametrize("scatter", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("spd", [False, True])
def test_cloth_step_small(torch_cuda, precision, spd, scatter):
    say("cloth n=33", "fp32" if precision else "fp64", "filtered" if spd else "raw", "scatter", scatter)
    inp = meshgen.cloth(n=33, seed=6011)
    _, prob, _ = build_gpu(torch_cuda, inp, precision, scatter=scatter, patch_faces=96)
    P = build_oracle(inp)
    rp, ci = [t.cpu().numpy() for t in prob.pattern()]
    assert np.array_equal(rp, P.rowptr) and np.array_equal(ci, P.colidx)
    out = compare(torch_cuda, prob, P, inp.x, ALL | (8 if spd else 0), precision)
    say("worst err/scale", out)


@pytest.mark.parametrize("precision", [0, 1])
def test_cloth_filtering_floor(torch_cuda, precision):
    # a positive floor lifts the springs' translations and compressed directions, and the
    # inertia blocks of vertices whose mass is below it
    say("cloth filtered eps", precision)
    inp = meshgen.cloth(n=20, seed=6012)
    eps = 2.0 * inp.meta["vdata"][0, 0]
    _, prob, _ = build_gpu(torch_cuda, inp, precision, patch_faces=64, spd_eps=eps)
    P = build_oracle(inp)
    compare(torch_cuda, prob, P, inp.x, ALL | 8, precision, spd_eps=eps)


@pytest.mark.parametrize("precision", [0, 1])
def test_cloth_vertex_data_read_every_evaluation(torch_cuda, precision):
    # a new time step rewrites xhat (and here the masses) in the caller's array: the next
    # evaluation sees it without any call
    torch = torch_cuda
    say("cloth vdata update", precision)
    inp = meshgen.cloth(n=24, seed=6013)
    _, prob, vd = build_gpu(torch, inp, precision, patch_faces=80)
    P = build_oracle(inp)
    compare(torch, prob, P, inp.x, ALL | 8, precision)
    rng = np.random.default_rng(5)
    new = inp.meta["vdata"].copy()
    new[:, 0] *= rng.uniform(0.5, 2.0, size=new.shape[0])
    new[:, 1:] += 0.01 * rng.normal(size=(new.shape[0], 3))
    vd.copy_(torch.from_numpy(new))
    P2 = build_oracle(inp, vdata=new)
    compare(torch, prob, P2, inp.x, ALL | 8, precision)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("spd", [False, True])
def test_cloth_hvp(torch_cuda, precision, spd):
    torch = torch_cuda
    from paper_2509_00406_amd import mad
    say("cloth hvp", precision, spd)
    inp = meshgen.cloth(n=30, seed=6014)
    _, prob, _ = build_gpu(torch, inp, precision, patch_faces=90)
    P = build_oracle(inp)
    x = inp.x.ravel().copy()
    v = np.random.default_rng(9).normal(size=x.size)
    y, _, _ = prob.hvp(torch.from_numpy(x).cuda(), torch.from_numpy(v).cuda(), mad.SPD if spd else 0)
    torch.cuda.synchronize()
    yref, yscale = P.hvp(x, v, spd=spd)
    PR.assert_close("hvp", y.cpu().numpy(), yref, yscale, PR.RTOL[precision])


def test_cloth_vertex_term_errors(torch_cuda):
    from paper_2509_00406_amd import mad
    inp = meshgen.cloth(n=8, seed=6015)
    mesh = mad.Mesh(inp.tris, inp.n_verts)
    prob = mad.Problem(mesh, 3, 0)
    with pytest.raises(mad.MadError):
        prob.add_term(mad.INERTIA, inp.meta["inertia_params"], None)       # needs the vertex entry point
    host = np.ascontiguousarray(inp.meta["vdata"])
    with pytest.raises(mad.MadError):
        mad.mad_problem_add_vertex_term(prob.handle, mad.INERTIA, inp.meta["inertia_params"], host)  # host memory
    vd = torch_cuda.from_numpy(host).cuda()
    with pytest.raises(mad.MadError):
        mad.mad_problem_add_vertex_term(prob.handle, mad.SPRING, inp.meta["spring_params"], vd)  # not a vertex kind


@pytest.mark.parametrize("precision", [1, 0])
def test_cloth_full_size_sampled(torch_cuda, precision):
    # the benchmark's configuration: 1000 x 1000 vertices, 2,996,001 springs + 1,000,000 vertices,
    # filtered Hessian; the pattern bit-exact, sampled rows element by element, total energy against
    # an independent vectorised evaluation; then the filtered matrix-free product on the same rows
    torch = torch_cuda
    from paper_2509_00406_amd import mad
    n = 1000
    say("cloth full 1000", precision)
    inp = meshgen.cloth(n=n, seed=6001)
    _, prob, _ = build_gpu(torch, inp, precision)
    P = build_oracle(inp)
    rp, ci = [t.cpu().numpy() for t in prob.pattern()]
    assert np.array_equal(rp, P.rowptr) and np.array_equal(ci, P.colidx)
    assert rp[-1] == n * n + 2 * 2996001
    x = torch.from_numpy(inp.x.ravel().copy()).cuda()
    energy, grad, hess = prob.eval(x, mad.ENERGY | mad.GRAD | mad.HESS | mad.SPD)
    torch.cuda.synchronize()
    nonfinite, _ = prob.status()
    assert not nonfinite
    rng = np.random.default_rng(321)
    rows = set(rng.choice(n * n, 200, replace=False).tolist()) | {0, n - 1, n * n - 1, n * (n // 2) + n // 2}
    mask = np.zeros(n * n, bool)
    mask[sorted(rows)] = True
    ref = P.eval(inp.x, O.GRAD | O.HESS | O.SPD, row_mask=mask)
    rtol = PR.RTOL[precision]
    r = np.nonzero(mask)[0]
    gi = np.concatenate([np.arange(3 * i, 3 * i + 3) for i in r])
    g = grad.cpu().numpy()
    PR.assert_close("grad(sampled)", g[gi], ref.grad[gi], ref.gscale[gi], rtol)
    bi = np.concatenate([np.arange(P.rowptr[i], P.rowptr[i + 1]) for i in r])
    h = hess.cpu().numpy()
    PR.assert_close("hess(sampled)", h[bi], ref.hess[bi], ref.hscale[bi], rtol)
    e_ref, e_abs = npref.cloth_energy(inp.tris, inp.rest, inp.x, inp.meta["vdata"], inp.meta["spring_params"],
                                      inp.meta["inertia_params"])
    assert abs(float(energy.cpu()[0]) - e_ref) <= rtol * e_abs
    # the filtered matrix-free product of the same step on the same rows
    v = np.random.default_rng(82).normal(size=x.numel())
    y, ey, _ = prob.hvp(x, torch.from_numpy(v).cuda(), mad.ENERGY | mad.SPD)
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    V = v.reshape(-1, 3)
    yref = np.zeros((r.size, 3))
    yscale = np.zeros((r.size, 3))
    for k, i in enumerate(r):
        for b in range(P.rowptr[i], P.rowptr[i + 1]):
            c = P.colidx[b]
            yref[k] += ref.hess[b].reshape(3, 3) @ V[c]
            yscale[k] += ref.hscale[b].reshape(3, 3) @ np.abs(V[c])
    PR.assert_close("hvp(sampled)", y[gi], yref.ravel(), yscale.ravel(), rtol)
    assert abs(float(ey.cpu()[0]) - e_ref) <= rtol * e_abs
