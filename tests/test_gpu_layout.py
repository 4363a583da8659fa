"""GPU parity of the layout choices: the persistent launch (workgroups taking
patches largest-first from a queue) against one workgroup per patch, layout
rebuilds on a finalized problem, and the timing autotuner with its cache. Every
layout is also checked against the FP64 oracle."""
import sys

import numpy as np
import pytest

from paper_2509_00406_amd import meshgen
from tests import parity as PR

pytestmark = pytest.mark.gpu

ALL = 1 | 2 | 4
SHELL = [(4, (0.9, 1.3)), (5, (1.1, 1.0))]


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


def check_vs_oracle(P, x, out, precision, mode):
    ref = P.eval(x, mode & 15)
    rtol = PR.RTOL[precision]
    e, g, h = (t.cpu().numpy() for t in out)
    assert abs(e[0] - ref.energy) <= rtol * ref.esum_abs
    PR.assert_close("grad", g, ref.grad, ref.gscale, rtol)
    PR.assert_close("hess", h, ref.hess, ref.hscale, rtol)


@pytest.mark.parametrize("precision", [0, 1])
def test_persistent_matches_one_workgroup_per_patch(torch_cuda, precision):
    say("persistent vs grid", precision)
    torch = torch_cuda
    from paper_2509_00406_amd import mad
    inp = meshgen.shell_cylinder(n=40, seed=21)
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, SHELL, precision, patch_faces=64)
    P = PR.build_oracle(inp.tris, inp.rest, inp.n_verts, 3, SHELL)
    xt = torch.from_numpy(inp.x.ravel().copy()).cuda()
    res = []
    for persistent in (0, 1, 0):
        prob.set_layout(mad.SCATTER_PATCH, 64, persistent)
        lay = prob.layout()
        assert lay["persistent"] == persistent and lay["scatter"] == mad.SCATTER_PATCH and lay["n_patches"] > 8
        out = prob.eval(xt, ALL | 8)
        torch.cuda.synchronize()
        check_vs_oracle(P, inp.x, out, precision, ALL | 8)
        res.append([t.cpu().numpy().copy() for t in out])
    # same patches, same per-patch partial sums: the energy is bit-identical
    assert res[0][0][0] == res[1][0][0] == res[2][0][0]
    # a second persistent evaluation reuses the queue counter (it is cleared per evaluation)
    prob.set_layout(mad.SCATTER_PATCH, 64, 1)
    for _ in range(2):
        out = prob.eval(xt, ALL | 8)
        torch.cuda.synchronize()
        check_vs_oracle(P, inp.x, out, precision, ALL | 8)


def test_relayout_between_strategies(torch_cuda):
    say("relayout atomic <-> patch")
    torch = torch_cuda
    from paper_2509_00406_amd import mad
    inp = meshgen.shell_cylinder(n=30, seed=22)
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, SHELL, 0)
    P = PR.build_oracle(inp.tris, inp.rest, inp.n_verts, 3, SHELL)
    xt = torch.from_numpy(inp.x.ravel().copy()).cuda()
    rp0, ci0 = (t.cpu().numpy() for t in prob.pattern())
    for sc, pf, pe in ((1, 512, 0), (2, 16, 1), (2, 100000, 0), (1, 32, 0), (2, 512, 0)):
        prob.set_layout(sc, pf, pe)
        rp, ci = (t.cpu().numpy() for t in prob.pattern())
        assert np.array_equal(rp, rp0) and np.array_equal(ci, ci0)
        out = prob.eval(xt, ALL | 8)
        torch.cuda.synchronize()
        check_vs_oracle(P, inp.x, out, 0, ALL | 8)
    with pytest.raises(mad.MadError):
        prob.set_layout(mad.SCATTER_ATOMIC, 512, 1)   # persistent needs the patch scatter
    with pytest.raises(mad.MadError):
        prob.set_layout(mad.SCATTER_PATCH, 0, 0)
    with pytest.raises(mad.MadError):
        prob.set_layout(7, 512, 0)


def test_autotune_batched_and_cache(torch_cuda):
    say("autotune batched icospheres")
    torch = torch_cuda
    inp = meshgen.icosphere_batch(n_meshes=10, mean_verts=900, vmin=500, vmax=3000)
    co = inp.comp_offsets
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, SHELL, 1, comp_offsets=co)
    P = PR.build_oracle(inp.tris, inp.rest, inp.n_verts, 3, SHELL)
    xt = torch.from_numpy(inp.x.ravel().copy()).cuda()
    out = prob.outputs()
    rep = prob.autotune(xt, ALL | 8, out=out, reps=2, force=True)
    assert rep["cached"] is False and len(rep["candidates"]) == 9
    assert all(c["ms"] > 0 for c in rep["candidates"])
    best = min(rep["candidates"], key=lambda c: c["ms"])
    lay = prob.layout()
    assert lay["patch_faces"] == rep["chosen"]["patch_faces"] == best["effective_faces"]
    assert lay["persistent"] == rep["chosen"]["persistent"] == best["persistent"]
    out = prob.eval(xt, ALL | 8)
    torch.cuda.synchronize()
    check_vs_oracle(P, inp.x, out, 1, ALL | 8)
    e = out[0].cpu().numpy()
    assert e.size == 11 and e[0] == pytest.approx(e[1:].sum(), rel=1e-14)
    # an identical problem takes the cached choice without timing
    mesh2, prob2 = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, SHELL, 1, comp_offsets=co)
    rep2 = prob2.autotune(xt, ALL | 8, reps=2)
    assert rep2["cached"] is True
    assert prob2.layout() == lay
    out2 = prob2.eval(xt, ALL | 8)
    torch.cuda.synchronize()
    check_vs_oracle(P, inp.x, out2, 1, ALL | 8)
