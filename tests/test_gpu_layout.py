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
    # patch targets 128..1024 x persistent or not x tiles of 4 and 8 waves, plus the atomic and colored scatters
    assert rep["cached"] is False and len(rep["candidates"]) == 18
    assert {c["scatter"] for c in rep["candidates"]} == {"patch", "atomic", "color"}
    assert {c["wg_waves"] for c in rep["candidates"]} == {4, 8}
    assert all(c["ms"] > 0 for c in rep["candidates"])
    best = min(rep["candidates"], key=lambda c: c["ms"])
    lay = prob.layout()
    assert lay["patch_faces"] == rep["chosen"]["patch_faces"] == best["effective_faces"]
    assert lay["persistent"] == rep["chosen"]["persistent"] == best["persistent"]
    assert lay["wg_waves"] == rep["chosen"]["wg_waves"] == best["wg_waves"]
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


@pytest.mark.parametrize("persistent", [0, 1])
def test_eight_wave_tile(torch_cuda, persistent):
    """The 8-wave tile (FP32): a workgroup with the CU's LDS to itself (larger patches) for the shell terms, two
    8-wave workgroups per CU for light terms; parity with the oracle, and FP64 keeps the 4-wave tile."""
    torch = torch_cuda
    from paper_2509_00406_amd import mad
    say("eight-wave tile, persistent", persistent)
    inp = meshgen.shell_cylinder(n=60, seed=23)
    P = PR.build_oracle(inp.tris, inp.rest, inp.n_verts, 3, SHELL)
    xt = torch.from_numpy(inp.x.ravel().copy()).cuda()
    mesh = mad.Mesh(inp.tris, inp.n_verts)
    faces = {}
    for waves in (4, 8):
        prob = mad.Problem(mesh, 3, mad.F32, wg_waves=waves, patch_faces=4096)
        for k, prm in SHELL:
            prob.add_term(k, prm, inp.rest)
        prob.finalize()
        prob.set_layout(mad.SCATTER_PATCH, 4096, persistent)
        lay = prob.layout()
        assert lay["wg_waves"] == waves
        faces[waves] = lay["patch_faces"]
        for mode in (1, 1 | 2, ALL, ALL | 8):
            out = prob.eval(xt, mode)
            torch.cuda.synchronize()
            ref = P.eval(inp.x, mode)
            e = out[0].cpu().numpy()
            assert abs(e[0] - ref.energy) <= PR.RTOL[1] * ref.esum_abs
            if mode & 2:
                PR.assert_close("grad", out[1].cpu().numpy(), ref.grad, ref.gscale, PR.RTOL[1])
            if mode & 4:
                PR.assert_close("hess", out[2].cpu().numpy(), ref.hess, ref.hscale, PR.RTOL[1])
        assert prob.status() == (False, 0)
    # the 148 KB budget of the 8-wave tile fits larger patches than the 76 KB one
    assert faces[8] > faces[4], faces
    say("patch targets after the LDS fit:", faces)
    # light terms (springs + inertia) with the 8-wave tile, and FP64, which keeps four waves
    cl = meshgen.cloth(n=40, seed=6001)
    vdata = torch.from_numpy(cl.meta["vdata"]).cuda()
    from oracle import oracle as O
    Pc = O.Problem(cl.tris, cl.rest, cl.n_verts, 3)
    Pc.add_term(O.SPRING, cl.meta["spring_params"])
    Pc.add_term(O.INERTIA, cl.meta["inertia_params"], vertex_data=cl.meta["vdata"])
    Pc.build_pattern()
    ref = Pc.eval(cl.x, ALL | 8)
    for prec in (mad.F32, mad.F64):
        m2 = mad.Mesh(cl.tris, cl.n_verts)
        pc = mad.Problem(m2, 3, prec, wg_waves=8)
        pc.add_term(mad.SPRING, cl.meta["spring_params"], cl.rest)
        pc.add_vertex_term(mad.INERTIA, cl.meta["inertia_params"], vdata)
        pc.finalize()
        pc.set_layout(mad.SCATTER_PATCH, 256, persistent)
        assert pc.layout()["wg_waves"] == (8 if prec == mad.F32 else 4)
        out = pc.eval(torch.from_numpy(cl.x.ravel().copy()).cuda(), ALL | 8)
        torch.cuda.synchronize()
        rtol = PR.RTOL[prec]
        assert abs(out[0].cpu().numpy()[0] - ref.energy) <= rtol * ref.esum_abs
        PR.assert_close("grad", out[1].cpu().numpy(), ref.grad, ref.gscale, rtol)
        PR.assert_close("hess", out[2].cpu().numpy(), ref.hess, ref.hscale, rtol)
