"""GPU parity of the matrix-free Hessian-vector product (through the C ABI)
against the oracle's definition (assembled Hessian times v), for raw and
clamped Hessians, both scatter strategies, FP64 and FP32. Tolerance: each
product entry within rtol of sum over its row's blocks of the oracle's
per-entry Hessian scale times |v| (the product analogue of the assembly bar)."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_00406_amd import meshgen
from tests import parity as PR

pytestmark = pytest.mark.gpu

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


def run_hvp(torch, inp, var_dim, terms, precision, spd, scatter=0, patch_faces=0, seed=3):
    from paper_2509_00406_amd import mad
    nv = inp.n_verts
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, nv, var_dim, terms, precision, inp.comp_offsets, patch_faces, 0.0,
                              scatter)
    P = PR.build_oracle(inp.tris, inp.rest, nv, var_dim, terms)
    x = np.ascontiguousarray(inp.x, dtype=np.float64).ravel()
    v = np.random.default_rng(seed).normal(size=x.size)
    xt = torch.from_numpy(x).cuda()
    vt = torch.from_numpy(v).cuda()
    mode = mad.ENERGY | mad.GRAD | (mad.SPD if spd else 0)
    y, energy, grad = prob.hvp(xt, vt, mode)
    torch.cuda.synchronize()
    yref, yscale = P.hvp(x, v, spd=spd)
    rtol = PR.RTOL[precision]
    worst = PR.assert_close("hvp", y.cpu().numpy(), yref, yscale, rtol)
    # the same pass's energy and gradient equal a plain evaluation's
    ref = P.eval(x, 1 | 2)
    assert abs(energy.cpu().numpy()[0] - ref.energy) <= rtol * ref.esum_abs
    PR.assert_close("grad", grad.cpu().numpy(), ref.grad, ref.gscale, rtol)
    nonfinite, _ = prob.status()
    assert not nonfinite
    say("worst |err|/scale", worst)
    return prob, xt, vt, y


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("spd", [False, True])
@pytest.mark.parametrize("scatter", [1, 2])
def test_hvp_shell(torch_cuda, precision, spd, scatter):
    say("hvp shell", precision, spd, scatter)
    inp = meshgen.shell_cylinder(n=40, seed=41)
    run_hvp(torch_cuda, inp, 3, SHELL, precision, spd, scatter=scatter, patch_faces=96)


def test_hvp_dirichlet_is_laplacian_times_v(torch_cuda):
    say("hvp dirichlet")
    inp = meshgen.dirichlet_grid(64)
    run_hvp(torch_cuda, inp, 1, [(3, ())], 0, False)


def test_hvp_symdir_and_stress_fallback(torch_cuda):
    say("hvp symdir + stress shell fp32 (FP64 redo of degenerate elements)")
    inp = meshgen.warped_grid(n=41, seed=42)
    run_hvp(torch_cuda, inp, 2, [(6, ())], 1, True)
    inp = meshgen.shell_cylinder(n=48, seed=2002, noise="absolute")
    prob, _, _, _ = run_hvp(torch_cuda, inp, 3, SHELL, 1, True)


def test_hvp_matches_assembled_product_on_gpu(torch_cuda):
    # the matrix-free product equals the assembled (block-CSR) Hessian times v, both from the GPU
    torch = torch_cuda
    say("hvp vs assembled")
    inp = meshgen.icosphere_batch(n_meshes=4, mean_verts=900, vmin=600, vmax=1500)
    prob, xt, vt, y = run_hvp(torch, inp, 3, SHELL, 0, True)
    e, g, h = prob.eval(xt, 1 | 2 | 4 | 8)
    rowptr, colidx = prob.pattern()
    rp, ci = rowptr.cpu().numpy(), colidx.cpu().numpy()
    H = h.cpu().numpy()
    v = vt.cpu().numpy().reshape(-1, 3)
    ya = np.zeros_like(v)
    for i in range(len(rp) - 1):
        for b in range(rp[i], rp[i + 1]):
            ya[i] += H[b] @ v[ci[b]]
    assert np.max(np.abs(ya.ravel() - y.cpu().numpy())) <= 1e-11 * np.max(np.abs(ya))
