"""GPU parity of residual terms and the sparse Jacobian (Sec. 4.1 Eq. 3, Sec. 6.1) through the C ABI:
the row-owned CSR pattern bit-exact against the oracle's, residuals and Jacobian values within the
parity bar (rtol 1e-12 FP64 / 1e-5 FP32 of each row's largest entry), the Gauss-Newton scalar form
(1/2 |r|^2, J^T r, J^T J) through the ordinary evaluation and the matrix-free product, for the
positional residual of the paper's vector-term example and an edge-length residual, mixed with a
scalar term, in both scatter strategies, and a Gauss-Newton solve built on them."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_00406_amd import meshgen
from tests import parity as PR

pytestmark = pytest.mark.gpu


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


def workload(n, seed):
    """A grid sheet pulled toward targets on a random subset of vertices: edge-length residuals keep
    the rest lengths, positional residuals pull the constrained vertices (w = 0 elsewhere)."""
    tris, rest = meshgen.grid(n)
    rng = np.random.default_rng(seed)
    x = rest + 0.05 * rng.normal(size=rest.shape)
    vd = np.zeros((n * n, 4))
    vd[:, 0] = rng.uniform(0.5, 2.0, n * n) * (rng.random(n * n) < 0.25)
    vd[:, 1:] = rest + np.array([0.0, 0.0, 0.2]) + 0.05 * rng.normal(size=rest.shape)
    return tris, rest, x, vd


def build(torch, tris, rest, vd, precision, scatter=0, patch_faces=0, with_scalar=False):
    from paper_2509_00406_amd import mad
    nv = rest.shape[0]
    mesh = mad.Mesh(tris, nv)
    prob = mad.Problem(mesh, 3, precision, patch_faces=patch_faces, scatter=scatter)
    prob.add_term(mad.RES_EDGE, (3.0,), rest)
    vdt = torch.from_numpy(np.ascontiguousarray(vd)).cuda()
    prob.add_vertex_term(mad.RES_POSITION, (), vdt)
    if with_scalar:
        prob.add_term(mad.STVK, (1.0, 1.0), rest)
    prob.finalize()
    P = O.Problem(tris, rest, nv, 3)
    P.add_term(O.RES_EDGE, (3.0,))
    P.add_term(O.RES_POSITION, (), vertex_data=vd)
    if with_scalar:
        P.add_term(O.STVK, (1.0, 1.0))
    P.build_pattern()
    return mesh, prob, P, vdt


def check_jacobian(torch, prob, P, x, precision):
    xt = torch.from_numpy(x.ravel().copy()).cuda()
    rp, ci = [t.cpu().numpy() for t in prob.jacobian_pattern()]
    r, vals = prob.jacobian(xt)
    torch.cuda.synchronize()
    rr, rpr, cir, vr = P.jacobian(x)
    assert np.array_equal(rp, rpr) and np.array_equal(ci, cir)
    rtol = PR.RTOL[precision]
    # each row against its largest entry (an element's local Jacobian row)
    rowmax = np.maximum.reduceat(np.abs(vr), rpr[:-1]) if len(vr) else np.zeros(0)
    scale = np.repeat(rowmax, np.diff(rpr))
    PR.assert_close("J", vals.cpu().numpy(), vr, scale, rtol)
    # residuals: FP64 primal on both paths
    assert np.max(np.abs(r.cpu().numpy() - rr)) <= 1e-12 * max(1.0, np.max(np.abs(rr)))
    nonfinite, _ = prob.status()
    assert not nonfinite
    return rr, rpr, cir, vr


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scatter", [1, 2])
def test_jacobian_and_gauss_newton(torch_cuda, precision, scatter):
    torch = torch_cuda
    say("jacobian + gauss-newton", precision, scatter)
    tris, rest, x, vd = workload(20, 31)
    _, prob, P, _ = build(torch, tris, rest, vd, precision, scatter=scatter, patch_faces=60)
    check_jacobian(torch, prob, P, x, precision)
    # the scalar form: 1/2 |r|^2, J^T r and J^T J in the block pattern
    for spd in (False, True):
        mode = 1 | 2 | 4 | (8 if spd else 0)
        e, g, h = prob.eval(torch.from_numpy(x.ravel().copy()).cuda(), mode)
        torch.cuda.synchronize()
        ref = P.eval(x, mode)
        rtol = PR.RTOL[precision]
        assert abs(float(e.cpu()[0]) - ref.energy) <= rtol * ref.esum_abs
        PR.assert_close("J^T r", g.cpu().numpy(), ref.grad, ref.gscale, rtol)
        PR.assert_close("J^T J", h.cpu().numpy(), ref.hess, ref.hscale, rtol)


def test_gauss_newton_matrix_equals_jt_j_of_the_gpu_jacobian(torch_cuda):
    # both from the GPU: the assembled block matrix equals J^T J of the CSR Jacobian
    torch = torch_cuda
    say("JtJ from GPU J")
    tris, rest, x, vd = workload(16, 32)
    _, prob, P, _ = build(torch, tris, rest, vd, 0)
    xt = torch.from_numpy(x.ravel().copy()).cuda()
    rp, ci = [t.cpu().numpy() for t in prob.jacobian_pattern()]
    r, vals = prob.jacobian(xt)
    _, g, h = prob.eval(xt, 1 | 2 | 4)
    torch.cuda.synchronize()
    nv = rest.shape[0]
    J = np.zeros((len(rp) - 1, 3 * nv))
    J[np.repeat(np.arange(len(rp) - 1), np.diff(rp)), ci] = vals.cpu().numpy()
    JtJ = J.T @ J
    brp, bci = [t.cpu().numpy() for t in prob.pattern()]
    H = h.cpu().numpy()
    D = np.zeros_like(JtJ)
    for i in range(nv):
        for b in range(brp[i], brp[i + 1]):
            D[3 * i:3 * i + 3, 3 * bci[b]:3 * bci[b] + 3] = H[b]
    assert np.max(np.abs(D - JtJ)) <= 1e-12 * np.max(np.abs(JtJ))
    assert np.max(np.abs(g.cpu().numpy() - J.T @ r.cpu().numpy())) <= 1e-12 * np.max(np.abs(J.T @ r.cpu().numpy()))


@pytest.mark.parametrize("precision", [0, 1])
def test_mixed_with_scalar_term_and_hvp(torch_cuda, precision):
    torch = torch_cuda
    from paper_2509_00406_amd import mad
    say("residual + StVK, hvp", precision)
    tris, rest, x, vd = workload(18, 33)
    _, prob, P, _ = build(torch, tris, rest, vd, precision, patch_faces=50, with_scalar=True)
    check_jacobian(torch, prob, P, x, precision)          # the scalar term owns no rows
    xt = torch.from_numpy(x.ravel().copy()).cuda()
    v = np.random.default_rng(4).normal(size=x.size)
    y, _, _ = prob.hvp(xt, torch.from_numpy(v).cuda(), mad.SPD)
    torch.cuda.synchronize()
    yref, ys = P.hvp(x.ravel(), v, spd=True)
    PR.assert_close("hvp", y.cpu().numpy(), yref, ys, PR.RTOL[precision])


def test_vertex_targets_read_every_evaluation(torch_cuda):
    torch = torch_cuda
    tris, rest, x, vd = workload(12, 34)
    _, prob, P, vdt = build(torch, tris, rest, vd, 0)
    check_jacobian(torch, prob, P, x, 0)
    vd2 = vd.copy()
    vd2[:, 0] = 1.0                                        # constrain every vertex
    vd2[:, 1:] += 0.3
    vdt.copy_(torch.from_numpy(vd2))
    P2 = O.Problem(tris, rest, rest.shape[0], 3)
    P2.add_term(O.RES_EDGE, (3.0,))
    P2.add_term(O.RES_POSITION, (), vertex_data=vd2)
    check_jacobian(torch, prob, P2, x, 0)


def test_gauss_newton_iterations_reduce_the_residual(torch_cuda):
    # Levenberg-Marquardt (damped Gauss-Newton) on the GPU's J^T J, J^T r and 1/2 |r|^2, dense solves on
    # the host at this size: the least-squares objective falls at every accepted step, by far overall,
    # and the gradient drops by orders of magnitude (a flat sheet under edge-length residuals has
    # nearly free out-of-plane directions, hence the damping)
    torch = torch_cuda
    say("gauss-newton solve")
    tris, rest, x, vd = workload(10, 35)
    vd[0, 0] = vd[9, 0] = 5.0                              # pin two corners at least
    _, prob, P, _ = build(torch, tris, rest, vd, 0)
    nv = rest.shape[0]
    brp, bci = [t.cpu().numpy() for t in prob.pattern()]

    def energy(y):
        e, _, _ = prob.eval(torch.from_numpy(y.ravel().copy()).cuda(), 1)
        return float(e.cpu()[0])

    xk = x.copy()
    f0 = f = energy(xk)
    mu, g0 = 1e-3, None
    for it in range(25):
        e, g, h = prob.eval(torch.from_numpy(xk.ravel().copy()).cuda(), 1 | 2 | 4)
        torch.cuda.synchronize()
        H = np.zeros((3 * nv, 3 * nv))
        Hb = h.cpu().numpy()
        for i in range(nv):
            for b in range(brp[i], brp[i + 1]):
                H[3 * i:3 * i + 3, 3 * bci[b]:3 * bci[b] + 3] = Hb[b]
        gg = g.cpu().numpy()
        g0 = np.linalg.norm(gg) if g0 is None else g0
        for _ in range(40):
            step = np.linalg.solve(H + mu * np.eye(3 * nv), -gg).reshape(nv, 3)
            fn = energy(xk + step)
            if fn < f:
                xk, f, mu = xk + step, fn, max(mu * 0.3, 1e-12)
                break
            mu *= 10
    _, g, _ = prob.eval(torch.from_numpy(xk.ravel().copy()).cuda(), 1 | 2)
    assert f < 0.05 * f0
    assert np.linalg.norm(g.cpu().numpy()) < 1e-2 * g0


@pytest.mark.parametrize("precision", [1, 0])
def test_jacobian_full_size_1000(torch_cuda, precision):
    """The benchmark's residual workload at its size (1000 x 1000 grid: 2,996,001 edge-length residuals and
    3,000,000 positional residual rows): the whole CSR pattern of J bit-exact, every value and residual against
    the oracle, and the Gauss-Newton form (J^T r, J^T J) on sampled block rows."""
    torch = torch_cuda
    from paper_2509_00406_amd import mad
    say("jacobian full size 1000", precision)
    n = 1000
    tris, rest = meshgen.grid(n)
    rng = np.random.default_rng(7001)
    x = rest + 0.05 * rng.normal(size=rest.shape)
    vd = np.zeros((n * n, 4))
    vd[:, 0] = rng.uniform(0.5, 2.0, n * n) * (rng.random(n * n) < 0.25)
    vd[:, 1:] = rest + np.array([0.0, 0.0, 0.2]) + 0.05 * rng.normal(size=rest.shape)
    _, prob, P, _ = build(torch, tris, rest, vd, precision)
    rr, rpr, _, _ = check_jacobian(torch, prob, P, x, precision)
    e, g, h = prob.eval(torch.from_numpy(x.ravel().copy()).cuda(), mad.ENERGY | mad.GRAD | mad.HESS)
    torch.cuda.synchronize()
    mask = np.zeros(n * n, bool)
    mask[np.random.default_rng(8).choice(n * n, 200, replace=False)] = True
    mask[[0, n - 1, n * n - 1, n * (n // 2) + n // 2]] = True
    ref = P.eval(x, O.GRAD | O.HESS, row_mask=mask)
    rows = np.nonzero(mask)[0]
    gi = np.concatenate([np.arange(3 * r, 3 * r + 3) for r in rows])
    rtol = PR.RTOL[precision]
    PR.assert_close("J^T r(sampled)", g.cpu().numpy()[gi], ref.grad[gi], ref.gscale[gi], rtol)
    bi = np.concatenate([np.arange(P.rowptr[r], P.rowptr[r + 1]) for r in rows])
    PR.assert_close("J^T J(sampled)", h.cpu().numpy()[bi], ref.hess[bi], ref.hscale[bi], rtol)
    # the energy is half the squared residual norm, summed in FP64
    e_ref = 0.5 * float(np.sum(rr * rr))
    assert abs(float(e.cpu()[0]) - e_ref) <= 1e-12 * e_ref
