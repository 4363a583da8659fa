"""GPU parity of the colored scatter (the coloring alternative of Sec. 5.5: each term's elements colored so that
no two of a color share a vertex, one launch per color, plain read-add-writes into zeroed outputs) against the
FP64 oracle: shell terms in FP64 and FP32 (with the FP64 redo of near-degenerate elements), 2x2 and 1x1 blocks,
springs with per-vertex inertia, per-component energies of a batch, the matrix-free product, residual terms
and their Jacobian, and a pattern grown by interaction pairs. The colored result is bitwise reproducible."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_00406_amd import meshgen
from tests import parity as PR

pytestmark = pytest.mark.gpu
ALL = 1 | 2 | 4
SHELL = [(4, (0.9, 1.3)), (5, (1.1, 1.0))]
COLOR = 3


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


def check(P, x, out, precision, mode, comp=False):
    ref = P.eval(x, mode & 15)
    rtol = PR.RTOL[precision]
    e, g, h = (t.cpu().numpy() for t in out)
    assert abs(e[0] - ref.energy) <= rtol * ref.esum_abs
    if mode & 2:
        PR.assert_close("grad", g, ref.grad, ref.gscale, rtol)
    if mode & 4:
        PR.assert_close("hess", h, ref.hess, ref.hscale, rtol)
        assert PR.normwise(h, ref.hess) <= rtol


@pytest.mark.parametrize("precision", [0, 1])
def test_color_shell(torch_cuda, precision):
    torch = torch_cuda
    say("colored shell", precision)
    inp = meshgen.shell_cylinder(n=40, seed=41)
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, SHELL, precision, scatter=COLOR)
    assert prob.layout()["scatter"] == COLOR
    P = PR.build_oracle(inp.tris, inp.rest, inp.n_verts, 3, SHELL)
    x = torch.from_numpy(inp.x.ravel().copy()).cuda()
    for mode in (1, 1 | 2, ALL, ALL | 8):
        out = prob.eval(x, mode)
        torch.cuda.synchronize()
        check(P, inp.x, out, precision, mode)
    a = [t.cpu().numpy().copy() for t in prob.eval(x, ALL | 8)]
    b = [t.cpu().numpy().copy() for t in prob.eval(x, ALL | 8)]
    for u, v in zip(a, b):
        assert np.array_equal(u, v), "the colored scatter is bitwise reproducible"
    assert prob.status() == (False, 0)


def test_color_stress_fp32_redo(torch_cuda):
    torch = torch_cuda
    say("colored shell, absolute noise, fp32")
    inp = meshgen.shell_cylinder(n=48, seed=2002, noise="absolute")
    from paper_2509_00406_amd import mad
    mesh = mad.Mesh(inp.tris, inp.n_verts)
    prob = mad.Problem(mesh, 3, mad.F32, scatter=COLOR, degenerate_q=1.0)   # every element redone in FP64
    for k, prm in SHELL:
        prob.add_term(k, prm, inp.rest)
    prob.finalize()
    P = PR.build_oracle(inp.tris, inp.rest, inp.n_verts, 3, SHELL)
    out = prob.eval(torch.from_numpy(inp.x.ravel().copy()).cuda(), ALL | 8)
    torch.cuda.synchronize()
    nonfinite, fallbacks = prob.status()
    assert not nonfinite and fallbacks == mesh.n_tris + mesh.n_diamonds
    check(P, inp.x, out, 1, ALL | 8)


@pytest.mark.parametrize("precision", [0, 1])
def test_color_symdir_and_dirichlet(torch_cuda, precision):
    torch = torch_cuda
    say("colored symdir + dirichlet", precision)
    inp = meshgen.warped_grid(n=33, seed=3001)
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 2, [(6, ())], precision, scatter=COLOR)
    P = PR.build_oracle(inp.tris, inp.rest, inp.n_verts, 2, [(6, ())])
    out = prob.eval(torch.from_numpy(inp.x.ravel().copy()).cuda(), ALL | 8)
    torch.cuda.synchronize()
    check(P, inp.x, out, precision, ALL | 8)
    dg = meshgen.dirichlet_grid(32)
    mesh, prob = PR.build_gpu(dg.tris, dg.rest, dg.rest.shape[0], 1, [(3, ())], precision, scatter=COLOR)
    P = PR.build_oracle(dg.tris, dg.rest, dg.rest.shape[0], 1, [(3, ())])
    out = prob.eval(torch.from_numpy(dg.x.ravel().copy()).cuda(), ALL)
    torch.cuda.synchronize()
    check(P, dg.x, out, precision, ALL)


def test_color_batched_components(torch_cuda):
    torch = torch_cuda
    say("colored icosphere batch")
    inp = meshgen.icosphere_batch(n_meshes=8, mean_verts=900, vmin=500, vmax=2000)
    co = inp.comp_offsets
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, SHELL, 1, comp_offsets=co, scatter=COLOR)
    P = PR.build_oracle(inp.tris, inp.rest, inp.n_verts, 3, SHELL)
    out = prob.eval(torch.from_numpy(inp.x.ravel().copy()).cuda(), ALL | 8)
    torch.cuda.synchronize()
    check(P, inp.x, out, 1, ALL | 8)
    e = out[0].cpu().numpy()
    for c in range(len(co) - 1):
        lo, hi = int(co[c]), int(co[c + 1])
        sel = np.all((inp.tris >= lo) & (inp.tris < hi), axis=1)
        Pc = PR.build_oracle(inp.tris[sel] - lo, inp.rest[lo:hi], hi - lo, 3, SHELL)
        rc = Pc.eval(inp.x[lo:hi], 1)
        assert abs(e[1 + c] - rc.energy) <= PR.RTOL[1] * rc.esum_abs


def test_color_cloth_hvp_and_residuals(torch_cuda):
    torch = torch_cuda
    from paper_2509_00406_amd import mad
    say("colored cloth, hvp, residual terms")
    cl = meshgen.cloth(n=30, seed=6001)
    vdata = torch.from_numpy(cl.meta["vdata"]).cuda()
    mesh = mad.Mesh(cl.tris, cl.n_verts)
    prob = mad.Problem(mesh, 3, mad.F64, scatter=COLOR)
    prob.add_term(mad.SPRING, cl.meta["spring_params"], cl.rest)
    prob.add_vertex_term(mad.INERTIA, cl.meta["inertia_params"], vdata)
    prob.finalize()
    P = O.Problem(cl.tris, cl.rest, cl.n_verts, 3)
    P.add_term(O.SPRING, cl.meta["spring_params"])
    P.add_term(O.INERTIA, cl.meta["inertia_params"], vertex_data=cl.meta["vdata"])
    P.build_pattern()
    x = torch.from_numpy(cl.x.ravel().copy()).cuda()
    out = prob.eval(x, ALL | 8)
    torch.cuda.synchronize()
    check(P, cl.x, out, 0, ALL | 8)
    v = np.random.default_rng(3).normal(size=cl.x.size)
    y, _, _ = prob.hvp(x, torch.from_numpy(v).cuda(), mad.SPD)
    torch.cuda.synchronize()
    yref, yscale = P.hvp(cl.x, v, spd=True)
    PR.assert_close("hvp", y.cpu().numpy(), yref, yscale, PR.RTOL[0])
    # residual terms: the Jacobian's rows stay owned by their elements whatever the element order
    wt = np.zeros((cl.n_verts, 4))
    wt[::5, 0] = 2.0
    wt[:, 1:] = cl.rest
    wd = torch.from_numpy(wt).cuda()
    mesh2 = mad.Mesh(cl.tris, cl.n_verts)
    pr = mad.Problem(mesh2, 3, mad.F64, scatter=COLOR)
    pr.add_term(mad.RES_EDGE, (3.0,), cl.rest)
    pr.add_vertex_term(mad.RES_POSITION, (), wd)
    pr.finalize()
    Pr = O.Problem(cl.tris, cl.rest, cl.n_verts, 3)
    Pr.add_term(O.RES_EDGE, (3.0,))
    Pr.add_term(O.RES_POSITION, (), vertex_data=wt)
    Pr.build_pattern()
    r, vals = pr.jacobian(x)
    rp, ci = pr.jacobian_pattern()
    jr, jrp, jci, jv = Pr.jacobian(cl.x)
    assert np.array_equal(rp.cpu().numpy(), jrp) and np.array_equal(ci.cpu().numpy(), jci)
    assert np.max(np.abs(r.cpu().numpy() - jr)) <= 1e-12 * max(1.0, np.max(np.abs(jr)))
    assert np.max(np.abs(vals.cpu().numpy() - jv)) <= 1e-12 * np.max(np.abs(jv))
    out = pr.eval(x, ALL)
    torch.cuda.synchronize()
    check(Pr, cl.x, out, 0, ALL)


def test_color_after_pair_insertion(torch_cuda):
    torch = torch_cuda
    from paper_2509_00406_amd import mad
    say("colored scatter after pair insertion")
    inp = meshgen.shell_cylinder(n=24, seed=43)
    mesh = mad.Mesh(inp.tris, inp.n_verts)
    prob = mad.Problem(mesh, 3, mad.F32, scatter=COLOR)
    for k, prm in SHELL:
        prob.add_term(k, prm, inp.rest)
    prob.reserve_pairs(500)
    prob.finalize()
    pairs = np.random.default_rng(5).integers(0, inp.n_verts, size=(300, 2)).astype(np.int32)
    prob.insert_pairs(torch.from_numpy(pairs).cuda())
    P = PR.build_oracle(inp.tris, inp.rest, inp.n_verts, 3, SHELL)
    rp0, ci0 = O.insert_pairs(P.rowptr, P.colidx, pairs, inp.n_verts)[:2]
    rp, ci = (t.cpu().numpy() for t in prob.pattern())
    assert np.array_equal(rp, rp0) and np.array_equal(ci, ci0)
    out = prob.eval(torch.from_numpy(inp.x.ravel().copy()).cuda(), ALL | 8)
    torch.cuda.synchronize()
    P.rowptr, P.colidx = rp0, ci0
    check(P, inp.x, out, 1, ALL | 8)
