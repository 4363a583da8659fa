"""GPU parity of dynamic sparsity (Sec. 6.3 and the CSR update of the appendix) through the C ABI:
the pattern after inserting interaction pairs bit-exact against the oracle's definition (sorted
union), evaluations afterwards against the oracle assembled into the new pattern (inserted blocks
that no term touches are zero), repeated insertions (the two pattern buffers swap each time), a
relayout after insertion, the atomic scatter, the errors, and the full-size shell."""
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


def build(inp, precision, reserve, scatter=0, patch_faces=0):
    from paper_2509_00406_amd import mad
    mesh = mad.Mesh(inp.tris, inp.n_verts)
    prob = mad.Problem(mesh, 3, precision, patch_faces=patch_faces, scatter=scatter)
    for kind, prm in SHELL:
        prob.add_term(kind, prm, inp.rest)
    prob.reserve_pairs(reserve)
    prob.finalize()
    return mesh, prob


def random_pairs(nv, n, rng, P=None):
    """Random vertex pairs plus some self pairs, repeats and pairs already in the pattern."""
    pr = rng.integers(0, nv, size=(n, 2))
    pr[: n // 20, 1] = pr[: n // 20, 0]                  # self pairs
    pr[n // 20: n // 10] = pr[n // 10: n // 10 + (n // 10 - n // 20)]   # repeats
    if P is not None:                                    # pairs already present (mesh edges)
        e = P.topo.edges[rng.choice(len(P.topo.edges), n // 10, replace=False)]
        pr[-(n // 10):] = e
    return np.ascontiguousarray(pr, dtype=np.int32)


def check_eval(torch, prob, P, inp, precision, spd=True):
    mode = 1 | 2 | 4 | (8 if spd else 0)
    x = torch.from_numpy(inp.x.ravel().copy()).cuda()
    e, g, h = prob.eval(x, mode)
    torch.cuda.synchronize()
    ref = P.eval(inp.x, mode)
    rtol = PR.RTOL[precision]
    assert abs(float(e.cpu()[0]) - ref.energy) <= rtol * ref.esum_abs
    PR.assert_close("grad", g.cpu().numpy(), ref.grad, ref.gscale, rtol)
    hh = h.cpu().numpy()
    PR.assert_close("hess", hh, ref.hess, ref.hscale, rtol)
    return hh, ref


def insert_and_check(torch, prob, P, pairs, nv):
    rp0, ci0 = [t.cpu().numpy() for t in prob.pattern()]
    added = prob.insert_pairs(torch.from_numpy(pairs).cuda())
    rp, ci = [t.cpu().numpy() for t in prob.pattern()]
    rref, cref, _ = O.insert_pairs(rp0, ci0, pairs, nv)
    assert np.array_equal(rp, rref) and np.array_equal(ci, cref)
    assert added == len(cref) - len(ci0) and prob.nnzb == len(cref)
    P.rowptr, P.colidx = rref, cref
    return added


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("seed", [0, 1])
def test_insert_then_evaluate(torch_cuda, precision, seed):
    torch = torch_cuda
    say("insert pairs shell n=24", precision, seed)
    inp = meshgen.shell_cylinder(n=24, seed=40 + seed)
    nv = inp.n_verts
    _, prob = build(inp, precision, reserve=800, patch_faces=64)
    P = PR.build_oracle(inp.tris, inp.rest, nv, 3, SHELL)
    rng = np.random.default_rng(seed)
    added = insert_and_check(torch, prob, P, random_pairs(nv, 400, rng, P), nv)
    assert added > 0
    hh, ref = check_eval(torch, prob, P, inp, precision)
    # the inserted blocks no term touches are exactly zero
    untouched = np.all(ref.hscale.reshape(len(hh), -1) == 0, axis=1)
    assert untouched.sum() >= added and np.all(hh[untouched] == 0)


@pytest.mark.parametrize("scatter", [1, 2])
def test_repeated_insertions_and_relayout(torch_cuda, scatter):
    torch = torch_cuda
    from paper_2509_00406_amd import mad
    say("insert twice + relayout, scatter", scatter)
    inp = meshgen.shell_cylinder(n=30, seed=44)
    nv = inp.n_verts
    _, prob = build(inp, 1, reserve=1300, scatter=scatter, patch_faces=80)   # room for four insertions
    P = PR.build_oracle(inp.tris, inp.rest, nv, 3, SHELL)
    rng = np.random.default_rng(7)
    for _ in range(3):
        insert_and_check(torch, prob, P, random_pairs(nv, 300, rng), nv)
        check_eval(torch, prob, P, inp, 1)
    # a relayout after the insertions keeps the pattern and the results
    lay = prob.layout()
    prob.set_layout(lay["scatter"], 40, 1 if scatter == 2 else 0)
    rp, ci = [t.cpu().numpy() for t in prob.pattern()]
    assert np.array_equal(rp, P.rowptr) and np.array_equal(ci, P.colidx)
    check_eval(torch, prob, P, inp, 1)
    insert_and_check(torch, prob, P, random_pairs(nv, 300, rng), nv)
    check_eval(torch, prob, P, inp, 1, spd=False)
    # the matrix-free product does not depend on the pattern
    x = torch.from_numpy(inp.x.ravel().copy()).cuda()
    v = torch.randn_like(x)
    y, _, _ = prob.hvp(x, v, mad.SPD)
    torch.cuda.synchronize()
    yref, ys = P.hvp(inp.x.ravel(), v.cpu().numpy(), spd=True)
    PR.assert_close("hvp", y.cpu().numpy(), yref, ys, PR.RTOL[1])


def test_insert_errors_leave_the_pattern_unchanged(torch_cuda):
    torch = torch_cuda
    from paper_2509_00406_amd import mad
    inp = meshgen.shell_cylinder(n=12, seed=45)
    nv = inp.n_verts
    mesh = mad.Mesh(inp.tris, nv)
    p0 = mad.Problem(mesh, 3, 1)
    for kind, prm in SHELL:
        p0.add_term(kind, prm, inp.rest)
    pairs = torch.from_numpy(np.array([[0, nv - 1]], np.int32)).cuda()
    with pytest.raises(mad.MadError) as ex:
        p0.insert_pairs(pairs)                       # before finalize
    assert ex.value.code == -7
    p0.finalize()
    with pytest.raises(mad.MadError) as ex:
        p0.insert_pairs(pairs)                       # no reserve
    assert ex.value.code == -7
    with pytest.raises(mad.MadError) as ex:
        p0.reserve_pairs(10)                         # after finalize
    assert ex.value.code == -7
    _, prob = build(inp, 1, reserve=10)
    rp0, ci0 = [t.cpu().numpy() for t in prob.pattern()]
    big = torch.from_numpy(np.zeros((11, 2), np.int32)).cuda()
    with pytest.raises(mad.MadError) as ex:
        prob.insert_pairs(big)                       # more pairs than reserved
    assert ex.value.code == -1
    bad = torch.from_numpy(np.array([[0, 1], [2, nv]], np.int32)).cuda()
    with pytest.raises(mad.MadError) as ex:
        prob.insert_pairs(bad)                       # vertex out of range
    assert ex.value.code == -1
    rp, ci = [t.cpu().numpy() for t in prob.pattern()]
    assert np.array_equal(rp, rp0) and np.array_equal(ci, ci0)
    far = np.array([[i, nv - 1 - i] for i in range(10)], np.int32)   # 20 new blocks: fills the reserve
    assert prob.insert_pairs(torch.from_numpy(far).cuda()) == 20
    rp1, ci1 = [t.cpu().numpy() for t in prob.pattern()]
    more = torch.from_numpy(np.array([[0, nv // 2 + 3]], np.int32)).cuda()
    with pytest.raises(mad.MadError) as ex:
        prob.insert_pairs(more)                      # beyond the reserved room
    assert ex.value.code == -9
    rp, ci = [t.cpu().numpy() for t in prob.pattern()]
    assert np.array_equal(rp, rp1) and np.array_equal(ci, ci1)
    assert prob.insert_pairs(torch.from_numpy(far).cuda()) == 0   # present pairs add nothing


def test_insert_full_size_shell(torch_cuda):
    # 1024 x 1024 shell (13,606,924 blocks) and 200,000 random pairs: bit-exact pattern, and the
    # evaluation afterwards keeps every old block's value
    torch = torch_cuda
    from paper_2509_00406_amd import mad
    say("insert full size")
    n = 1024
    inp = meshgen.shell_cylinder(n=n, seed=2001)
    nv = inp.n_verts
    mesh, prob = build(inp, 1, reserve=200000)
    x = torch.from_numpy(inp.x.ravel().copy()).cuda()
    mode = mad.ENERGY | mad.GRAD | mad.HESS | mad.SPD
    _, g0, h0 = prob.eval(x, mode)
    h0 = h0.cpu().numpy()
    rp0, ci0 = [t.cpu().numpy() for t in prob.pattern()]
    pairs = np.ascontiguousarray(np.random.default_rng(11).integers(0, nv, size=(200000, 2)), dtype=np.int32)
    added = prob.insert_pairs(torch.from_numpy(pairs).cuda())
    rp, ci = [t.cpu().numpy() for t in prob.pattern()]
    rref, cref, mp = O.insert_pairs(rp0, ci0, pairs, nv)
    assert np.array_equal(rp, rref) and np.array_equal(ci, cref)
    assert added == len(cref) - len(ci0)
    _, g1, h1 = prob.eval(x, mode)
    torch.cuda.synchronize()
    h1 = h1.cpu().numpy()
    new = np.ones(len(cref), bool)
    new[mp] = False
    assert np.all(h1[new] == 0)
    # same values in the old blocks up to the order of the FP32 sums (atomics in the redo queue)
    assert np.max(np.abs(h1[mp] - h0)) <= 1e-6 * np.max(np.abs(h0))
    assert torch.allclose(g0, g1, rtol=0, atol=1e-6 * float(g0.abs().max()))
