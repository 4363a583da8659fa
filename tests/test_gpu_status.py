"""Internal errors surface at the boundary: a patch kernel whose LDS-lock wait gives up adds no block
without the lock, flags the evaluation, and mad_problem_status reports MAD_E_INTERNAL (the condition is
forced from the host with a zero spin bound, so every kernel still runs to completion)."""
import numpy as np
import pytest
import torch

from paper_2509_00406_amd import mad, meshgen

pytestmark = pytest.mark.gpu
MODE = mad.ENERGY | mad.GRAD | mad.HESS | mad.SPD


def shell_problem(prec, **kw):
    inp = meshgen.shell_cylinder(n=24, seed=2001)
    mesh = mad.Mesh(inp.tris, inp.n_verts)
    prob = mad.Problem(mesh, 3, prec, patch_faces=128, **kw)
    prob.add_term(mad.STVK, (1.0, 1.0), inp.rest)
    prob.add_term(mad.BENDING, (1.0, 1.0), inp.rest)
    prob.finalize()
    return mesh, prob, torch.from_numpy(inp.x.ravel().copy()).cuda()


@pytest.mark.parametrize("prec", [mad.F32, mad.F64])
def test_lock_timeout_is_reported(prec):
    print(f"lock time-out, precision {prec}", flush=True)
    mesh, prob, x = shell_problem(prec, lock_spins=mad.LOCK_NO_WAIT)
    prob.eval(x, MODE)
    with pytest.raises(mad.MadError) as e:
        prob.status()
    assert e.value.code == -10 and "LDS lock" in str(e.value)
    # the flags were reset by the failing call; an evaluation that adds no blocks takes no lock
    prob.eval(x, mad.ENERGY | mad.GRAD)
    assert prob.status() == (False, 0)
    prob.eval(x, MODE)
    with pytest.raises(mad.MadError):
        prob.status()


def test_default_lock_reports_ok():
    mesh, prob, x = shell_problem(mad.F32)
    ref = prob.eval(x, MODE)
    torch.cuda.synchronize()
    nonfinite, _ = prob.status()
    assert not nonfinite
    # an explicit, generous bound gives the same result as the default
    mesh2, prob2, _ = shell_problem(mad.F32, lock_spins=1 << 20)
    out = prob2.eval(x, MODE)
    prob2.status()
    for a, b in ((out[1], ref[1]), (out[2], ref[2])):   # same sums up to the LDS summation order
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.abs(a - b).max() <= 1e-5 * np.abs(b).max()
