"""Vertices of any valence (Sec. 6.1 builds the pattern for general triangle meshes): closed double fans whose
two poles each lie on k triangles and 2k bending diamonds. The pattern builder sorts each row's candidates in
LDS up to 2,048 of them (k = 60: 721 candidates at a pole) and in a global scratch range beyond (k = 300:
3,601; k = 1,000: 12,001). The rim is pleated (rim vertices alternately above and below the plane) so the
k triangles around a pole keep a usable shape (quality >= 0.2 at k = 300, against 0.08 for a flat fan),
and the parity bar applies as everywhere else; at k = 1,000 the pattern is checked bit-exact."""
import math
import sys

import numpy as np
import pytest

from tests import parity as PR

pytestmark = pytest.mark.gpu
SHELL = [(4, (1.0, 1.0)), (5, (1.0, 1.0))]


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def double_fan(k, seed=9, pleat=0.1, sigma=2e-4):
    """poles 0 (z = 1) and k+1 (z = -1), rim 1..k on the unit circle at z = +-pleat alternately (k even);
    faces (0, a, b) and (k+1, b, a)"""
    rim = np.arange(k)
    a, b = 1 + rim, 1 + (rim + 1) % k
    tris = np.concatenate([np.stack([np.zeros(k, int), a, b], 1), np.stack([np.full(k, k + 1), b, a], 1)])
    ang = 2 * math.pi * rim / k
    rest = np.zeros((k + 2, 3))
    rest[1:k + 1, 0], rest[1:k + 1, 1] = np.cos(ang), np.sin(ang)
    rest[1:k + 1, 2] = np.where(rim % 2 == 0, pleat, -pleat)
    rest[0, 2], rest[k + 1, 2] = 1.0, -1.0
    x = rest * np.array([1.05, 0.97, 1.1]) + np.random.default_rng(seed).normal(0, sigma, rest.shape)
    return tris.astype(np.int32), rest, x


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("k", [60, 300])
@pytest.mark.parametrize("precision", [0, 1])
def test_high_valence_fan(torch_cuda, k, precision):
    torch = torch_cuda
    say(f"double fan k={k} precision {precision}")
    tris, rest, x = double_fan(k)
    nv = k + 2
    P = PR.build_oracle(tris, rest, nv, 3, SHELL)
    mesh, prob = PR.build_gpu(tris, rest, nv, 3, SHELL, precision)
    rp, ci = [t.cpu().numpy() for t in prob.pattern()]
    assert np.array_equal(rp, P.rowptr) and np.array_equal(ci, P.colidx)
    assert rp[1] - rp[0] == k + 2          # the pole couples to every vertex (bending reaches the other pole)
    xt = torch.from_numpy(x.ravel().copy()).cuda()
    mode = 1 | 2 | 4 | 8
    energy, grad, hess = prob.eval(xt, mode)
    torch.cuda.synchronize()
    nonfinite, fallbacks = prob.status()
    assert not nonfinite
    ref = P.eval(x, mode)
    rtol = PR.RTOL[precision]
    assert abs(float(energy.cpu()[0]) - ref.energy) <= rtol * ref.esum_abs
    g = PR.assert_close("grad", grad.cpu().numpy(), ref.grad, ref.gscale, rtol)
    h = PR.assert_close("hess", hess.cpu().numpy(), ref.hess, ref.hscale, rtol)
    say(f"  {prob.layout()}: worst grad {g:.2e} hess {h:.2e}, fp64 redo {fallbacks}")


def test_valence_1000_pattern(torch_cuda):
    torch = torch_cuda
    k = 1000
    say(f"double fan k={k} pattern")
    tris, rest, x = double_fan(k)
    P = PR.build_oracle(tris, rest, k + 2, 3, SHELL)
    mesh, prob = PR.build_gpu(tris, rest, k + 2, 3, SHELL, 1)
    rp, ci = [t.cpu().numpy() for t in prob.pattern()]
    assert np.array_equal(rp, P.rowptr) and np.array_equal(ci, P.colidx)
    energy, grad, hess = prob.eval(torch.from_numpy(x.ravel().copy()).cuda(), 1 | 2 | 4 | 8)
    torch.cuda.synchronize()
    assert prob.status()[0] is False and np.isfinite(hess.cpu().numpy()).all()
