"""Full-size parity on the benchmark workload (1024 x 1024 shell cylinder,
2,093,058 triangles + 3,137,541 bending diamonds, 13,606,924 blocks), in the
launch configuration the benchmark times: the whole pattern bit-exact,
gradient rows and Hessian block rows of sampled vertices against the oracle
element by element, and the total energy against an independent vectorised
FP64 evaluation."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_00406_amd import meshgen
from tests import npref
from tests import parity as PR

pytestmark = pytest.mark.gpu

N = 1024
STVK_PRM, BEND_PRM = (1.0, 1.0), (1.0, 1.0)
TERMS = [(4, STVK_PRM), (5, BEND_PRM)]


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def full():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("full-size oracle setup")
    inp = meshgen.shell_cylinder(n=N, seed=2001)
    P = PR.build_oracle(inp.tris, inp.rest, inp.n_verts, 3, TERMS)
    rng = np.random.default_rng(123)
    rows = set(rng.choice(inp.n_verts, 240, replace=False).tolist())
    rows |= {0, 1, N - 1, N, N * N - 1, N * N - N, N * (N // 2) + N // 2}   # corners, boundary, middle
    mask = np.zeros(inp.n_verts, bool)
    mask[sorted(rows)] = True
    return inp, P, mask


def sampled_compare(P, mask, x, grad, hess, rtol):
    ref = P.eval(x, O.GRAD | O.HESS | O.SPD, row_mask=mask)
    rows = np.nonzero(mask)[0]
    gi = np.concatenate([np.arange(3 * r, 3 * r + 3) for r in rows])
    g = PR.assert_close("grad(sampled)", grad[gi], ref.grad[gi], ref.gscale[gi], rtol)
    bi = np.concatenate([np.arange(P.rowptr[r], P.rowptr[r + 1]) for r in rows])
    h = PR.assert_close("hess(sampled)", hess[bi], ref.hess[bi], ref.hscale[bi], rtol)
    assert PR.normwise(hess[bi], ref.hess[bi]) <= rtol   # the headline norm-wise error over the sampled rows
    return g, h, bi.size


@pytest.mark.parametrize("precision", [1, 0])
def test_full_shell_sampled(full, precision):
    import torch
    from paper_2509_00406_amd import mad
    inp, P, mask = full
    say("full shell 1024", "fp32" if precision else "fp64")
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, TERMS, precision)
    rp, ci = [t.cpu().numpy() for t in prob.pattern()]
    assert np.array_equal(rp, P.rowptr) and np.array_equal(ci, P.colidx)
    assert rp[-1] == 13606924
    x = torch.from_numpy(inp.x.ravel().copy()).cuda()
    energy, grad, hess = prob.eval(x, mad.ENERGY | mad.GRAD | mad.HESS | mad.SPD)
    torch.cuda.synchronize()
    nonfinite, fallbacks = prob.status()
    assert not nonfinite
    rtol = PR.RTOL[precision]
    g, h, nb = sampled_compare(P, mask, inp.x, grad.cpu().numpy(), hess.cpu().numpy(), rtol)
    e_ref, e_abs = npref.shell_energy(inp.tris, inp.rest, inp.x, P.topo.diamonds, P.topo.diamond_faces,
                                      STVK_PRM, BEND_PRM)
    e = float(energy.cpu()[0])
    assert abs(e - e_ref) <= rtol * e_abs, (e, e_ref, e_abs)
    say(f"worst grad {g:.2e} hess {h:.2e} over {nb} blocks; energy {e:.12e} vs {e_ref:.12e}; "
        f"fp64 fallbacks {fallbacks}")


def test_full_shell_stress_noise_fp32(full):
    import torch
    from paper_2509_00406_amd import mad
    inp, P, mask = full
    say("full shell 1024 absolute noise fp32")
    st = meshgen.shell_cylinder(n=N, seed=2002, noise="absolute")
    mesh, prob = PR.build_gpu(st.tris, st.rest, st.n_verts, 3, TERMS, 1)
    x = torch.from_numpy(st.x.ravel().copy()).cuda()
    energy, grad, hess = prob.eval(x, mad.ENERGY | mad.GRAD | mad.HESS | mad.SPD)
    torch.cuda.synchronize()
    nonfinite, fallbacks = prob.status()
    g, h, nb = sampled_compare(P, mask, st.x, grad.cpu().numpy(), hess.cpu().numpy(), PR.RTOL[1])
    e_ref, e_abs = npref.shell_energy(st.tris, st.rest, st.x, P.topo.diamonds, P.topo.diamond_faces,
                                      STVK_PRM, BEND_PRM)
    assert abs(float(energy.cpu()[0]) - e_ref) <= 1e-5 * e_abs
    say(f"stress: worst grad {g:.2e} hess {h:.2e}; fp64 fallbacks {fallbacks}; nonfinite {nonfinite}")


@pytest.mark.parametrize("scatter", ["atomic", "color"])
def test_full_shell_other_scatters_fp32(full, scatter):
    """The paper's device-wide atomic scatter and its coloring alternative at the benchmark size: sampled rows
    against the oracle and the energy against the independent FP64 evaluation, FP32."""
    import torch
    from paper_2509_00406_amd import mad
    inp, P, mask = full
    say("full shell 1024 fp32, scatter", scatter)
    sc = {"atomic": mad.SCATTER_ATOMIC, "color": mad.SCATTER_COLOR}[scatter]
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, TERMS, 1, scatter=sc)
    assert prob.layout()["scatter"] == sc
    x = torch.from_numpy(inp.x.ravel().copy()).cuda()
    energy, grad, hess = prob.eval(x, mad.ENERGY | mad.GRAD | mad.HESS | mad.SPD)
    torch.cuda.synchronize()
    nonfinite, fallbacks = prob.status()
    assert not nonfinite
    g, h, nb = sampled_compare(P, mask, inp.x, grad.cpu().numpy(), hess.cpu().numpy(), PR.RTOL[1])
    e_ref, e_abs = npref.shell_energy(inp.tris, inp.rest, inp.x, P.topo.diamonds, P.topo.diamond_faces,
                                      STVK_PRM, BEND_PRM)
    e = float(energy.cpu()[0])
    assert abs(e - e_ref) <= PR.RTOL[1] * e_abs, (e, e_ref, e_abs)
    say(f"{scatter}: worst grad {g:.2e} hess {h:.2e} over {nb} blocks; fp64 fallbacks {fallbacks}")


@pytest.mark.parametrize("precision", [1, 0])
def test_full_shell_hvp(full, precision):
    """The matrix-free clamped Hessian-vector product at the benchmark size: y = H v on the sampled rows against
    the oracle's sampled Hessian rows applied to the same v (per entry within rtol of sum_b scale_b |v|), and the
    same pass's gradient on those rows."""
    import torch
    from paper_2509_00406_amd import mad
    inp, P, mask = full
    say("full shell 1024", "fp32" if precision else "fp64", "clamped Hessian-vector product")
    mesh, prob = PR.build_gpu(inp.tris, inp.rest, inp.n_verts, 3, TERMS, precision)
    x = np.ascontiguousarray(inp.x, dtype=np.float64).ravel()
    v = np.random.default_rng(77).normal(size=x.size)
    y, energy, grad = prob.hvp(torch.from_numpy(x).cuda(), torch.from_numpy(v).cuda(),
                               mad.ENERGY | mad.GRAD | mad.SPD)
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    ref = P.eval(inp.x, O.GRAD | O.HESS | O.SPD, row_mask=mask)
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
    w = PR.assert_close("hvp(sampled)", y[gi], yref.ravel(), yscale.ravel(), PR.RTOL[precision])
    g = PR.assert_close("grad(sampled)", grad.cpu().numpy()[gi], ref.grad[gi], ref.gscale[gi], PR.RTOL[precision])
    e_ref, e_abs = npref.shell_energy(inp.tris, inp.rest, inp.x, P.topo.diamonds, P.topo.diamond_faces,
                                      STVK_PRM, BEND_PRM)
    assert abs(float(energy.cpu()[0]) - e_ref) <= PR.RTOL[precision] * e_abs
    say(f"hvp: worst {w:.2e} over {rows.size} rows, grad {g:.2e}")
