"""mad_problem_eval_static, the evaluation for callers that cannot allocate, against mad_problem_eval
through the C ABI: the same energy (bitwise: a fixed-order sum), the same pattern, gradients and Hessian
blocks within the parity tolerance of the oracle's per-entry scale, on two calls in a row whose second
problem is smaller (so stale contents of the static scratch from the first call must not leak into the
second), for the persistent and the one-workgroup-per-patch launch, FP32 (with the FP64 redo queue)
and FP64, 2x2 blocks, and the learned density (network outputs in the static scratch). A problem too
large for the scratch is refused before any launch, and the calls leave the device's free memory
unchanged."""
import sys

import numpy as np
import pytest

from paper_2509_00406_amd import meshgen
from tests import parity as PR

pytestmark = pytest.mark.gpu
SPD_ALL = 1 | 2 | 4 | 8
SHELL = [(4, (1.0, 1.0)), (5, (1.0, 1.0))]


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


def compare(torch, prob, P, x_np, precision, mode=SPD_ALL):
    """static vs plain evaluation vs oracle, on one problem; returns the worst ratios"""
    x = torch.from_numpy(np.ascontiguousarray(x_np, dtype=np.float64).ravel()).cuda()
    ref_e, ref_g, ref_h = prob.eval(x, mode)
    out = prob.outputs()
    for t in out:          # poison the outputs: every requested entry must be written
        t.fill_(float("nan"))
    e, g, h = prob.eval_static(x, mode, out=out)
    torch.cuda.synchronize()
    nonfinite, _ = prob.status()
    assert not nonfinite
    assert np.array_equal(e.cpu().numpy(), ref_e.cpu().numpy()), "energy differs from mad_problem_eval"
    oref = P.eval(x_np, mode)
    rtol = PR.RTOL[precision]
    assert abs(float(e.cpu()[0]) - oref.energy) <= rtol * oref.esum_abs
    w = {}
    for name, a, b, sc in (("grad", g, ref_g, oref.gscale), ("hess", h, ref_h, oref.hscale)):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        w[name] = PR.assert_close(name + " static vs eval", a, b, sc, rtol)
        PR.assert_close(name + " static vs oracle", a, oref.grad if name == "grad" else oref.hess, sc, rtol)
    return w


@pytest.mark.parametrize("precision,persistent", [(1, 1), (1, 0), (0, 1)])
def test_static_eval_two_calls_second_smaller(torch_cuda, precision, persistent):
    torch = torch_cuda
    for n in (40, 14):    # the second problem is smaller
        say(f"static eval shell {n}x{n} precision {precision} persistent {persistent}")
        inp = meshgen.shell_cylinder(n=n, seed=2001)
        mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, SHELL, precision, patch_faces=96)
        lay = prob.layout()
        prob.set_layout(lay["scatter"], lay["patch_faces"], persistent)
        P = PR.build_oracle(inp.tris, inp.rest, inp.n_verts, 3, SHELL)
        w = compare(torch, prob, P, inp.x, precision)
        say(f"  {prob.layout()}; worst vs eval: grad {w['grad']:.2e} hess {w['hess']:.2e}")


def test_static_eval_batched_components(torch_cuda):
    """Disjoint meshes in one problem: the per-component energies come from the static array's reduction
    slots; two calls in a row, the second on fewer, smaller meshes."""
    torch = torch_cuda
    for nm, mean_v in ((6, 900), (3, 700)):
        say(f"static eval {nm} icospheres")
        inp = meshgen.icosphere_batch(n_meshes=nm, mean_verts=mean_v, vmin=mean_v - 300, vmax=mean_v + 400)
        mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, SHELL, 1, comp_offsets=inp.comp_offsets)
        P = PR.build_oracle(inp.tris, inp.rest, inp.n_verts, 3, SHELL)
        w = compare(torch, prob, P, inp.x, 1)
        say(f"  {prob.layout()}; worst vs eval: grad {w['grad']:.2e} hess {w['hess']:.2e}")


def test_static_eval_fp64_redo_queue(torch_cuda):
    """FP32 with the quality threshold at 1 (the equilateral triangle's quality; these faces are near
    right isosceles, quality about 0.87): every element goes through the FP64 redo queue, which lives in
    the static scratch"""
    from paper_2509_00406_amd import mad
    torch = torch_cuda
    inp = meshgen.shell_cylinder(n=24, seed=2002, noise="absolute")
    mesh = mad.Mesh(inp.tris, inp.n_verts)
    prob = mad.Problem(mesh, 3, mad.F32, patch_faces=96, degenerate_q=1.0)
    for kind, prm in SHELL:
        prob.add_term(kind, prm, inp.rest)
    prob.finalize()
    P = PR.build_oracle(inp.tris, inp.rest, inp.n_verts, 3, SHELL)
    x = torch.from_numpy(inp.x.ravel().copy()).cuda()
    prob.eval(x, SPD_ALL)
    torch.cuda.synchronize()
    _, fb_plain = prob.status()
    assert fb_plain == mesh.n_tris + mesh.n_diamonds
    w = compare(torch, prob, P, inp.x, 1)
    say(f"redo queue: {fb_plain} elements redone in FP64; worst vs eval: grad {w['grad']:.2e} hess {w['hess']:.2e}")


def test_static_eval_symdir_and_modes(torch_cuda):
    torch = torch_cuda
    inp = meshgen.warped_grid(n=33, seed=3001)
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 2, [(6, ())], 1, patch_faces=128)
    P = PR.build_oracle(inp.tris, inp.rest, inp.n_verts, 2, [(6, ())])
    for mode in (1, 1 | 2, 1 | 2 | 4, SPD_ALL):
        x = torch.from_numpy(inp.x.ravel().copy()).cuda()
        ref = prob.eval(x, mode)
        out = prob.outputs()
        got = prob.eval_static(x, mode, out=out)
        torch.cuda.synchronize()
        assert np.array_equal(got[0].cpu().numpy(), ref[0].cpu().numpy())
        oref = P.eval(inp.x, mode)
        if mode & 2:
            PR.assert_close("grad", got[1].cpu().numpy(), ref[1].cpu().numpy(), oref.gscale, PR.RTOL[1])
        if mode & 4:
            PR.assert_close("hess", got[2].cpu().numpy(), ref[2].cpu().numpy(), oref.hscale, PR.RTOL[1])


def test_static_eval_learned_density(torch_cuda):
    from oracle import oracle as O
    from paper_2509_00406_amd import mad
    from tests.test_gpu_mlp import RTOL_MLP, bf16_round, oracle_params, seeded_network
    torch = torch_cuda
    inp = meshgen.shell_cylinder(n=20, seed=5001)
    theta, s_in, s_out = seeded_network(seed=17, scale=0.6)
    mesh = mad.Mesh(inp.tris, inp.n_verts)
    prob = mad.Problem(mesh, 3, mad.F32, patch_faces=96)
    prob.add_mlp_term(mad.Network(theta, s_in, s_out), inp.rest)
    prob.finalize()
    P = O.Problem(inp.tris, inp.rest, inp.n_verts, 3)
    P.add_term(O.MLP, oracle_params(bf16_round(theta), s_in, s_out))
    P.build_pattern()
    x = torch.from_numpy(inp.x.ravel().copy()).cuda()
    ref = prob.eval(x, SPD_ALL)
    got = prob.eval_static(x, SPD_ALL, out=prob.outputs())
    torch.cuda.synchronize()
    assert np.array_equal(got[0].cpu().numpy(), ref[0].cpu().numpy())
    oref = P.eval(inp.x, SPD_ALL)
    rtol = max(PR.RTOL[1], RTOL_MLP)
    PR.assert_close("grad", got[1].cpu().numpy(), ref[1].cpu().numpy(), oref.gscale, rtol)
    PR.assert_close("hess", got[2].cpu().numpy(), ref[2].cpu().numpy(), oref.hscale, rtol)


def test_static_eval_refuses_oversized_problem(torch_cuda):
    """a problem whose scratch exceeds the static array (the learned density's network outputs alone take
    136 bytes per triangle, 97.6 MB on a 600 x 600 grid): MAD_E_CAPACITY before any launch"""
    from paper_2509_00406_amd import mad
    from tests.test_gpu_mlp import seeded_network
    torch = torch_cuda
    inp = meshgen.shell_cylinder(n=600, seed=5001)
    mesh = mad.Mesh(inp.tris, inp.n_verts)
    prob = mad.Problem(mesh, 3, mad.F32)
    prob.add_mlp_term(mad.Network(*seeded_network(seed=17, scale=0.6)), inp.rest)
    prob.finalize()
    x = torch.from_numpy(inp.x.ravel().copy()).cuda()
    out = prob.outputs()
    with pytest.raises(mad.MadError) as e:
        prob.eval_static(x, SPD_ALL, out=out)
    assert e.value.code == -9 and "static scratch" in str(e.value)
    say(str(e.value))
    prob.eval(x, SPD_ALL, out=out)      # the plain evaluation still works
    torch.cuda.synchronize()
    assert prob.status() == (False, 0)


def test_static_eval_allocates_nothing(torch_cuda):
    torch = torch_cuda
    inp = meshgen.shell_cylinder(n=48, seed=2001)
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, SHELL, 1, patch_faces=128)
    x = torch.from_numpy(inp.x.ravel().copy()).cuda()
    out = prob.outputs()
    prob.eval_static(x, SPD_ALL, out=out)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(5):
        prob.eval_static(x, SPD_ALL, out=out)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    assert prob.status() == (False, 0)
