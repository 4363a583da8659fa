"""The threaded oracle evaluation (used to time the oracle on all host cores) is bit-identical to the
serial oracle: each output entry is the same sequence of additions. Checked in the parity build and in the
-O3 -march=native timing build (each against its own serial evaluation)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_00406_amd import meshgen

MODES = [O.ENERGY | O.GRAD | O.HESS | O.SPD, O.ENERGY | O.GRAD | O.HESS, O.ENERGY | O.GRAD, O.ENERGY]


def problems():
    sh = meshgen.shell_cylinder(n=18, seed=2002, noise="absolute")
    P = O.Problem(sh.tris, sh.rest, sh.n_verts, 3)
    P.add_term(O.STVK, (1.0, 0.7))
    P.add_term(O.BENDING, (1.0, 1.0))
    yield "shell", P, sh.x
    sd = meshgen.warped_grid(n=15, seed=3002)
    P = O.Problem(sd.tris, sd.rest, sd.n_verts, 2)
    P.add_term(O.SYMDIR, ())
    yield "symdir", P, sd.x
    cl = meshgen.cloth(n=12, seed=6002)
    P = O.Problem(cl.tris, cl.rest, cl.n_verts, 3)
    P.add_term(O.SPRING, cl.meta["spring_params"])
    P.add_term(O.INERTIA, cl.meta["inertia_params"], vertex_data=cl.meta["vdata"])
    yield "cloth", P, cl.x
    P = O.Problem(sh.tris, sh.rest, sh.n_verts, 3)
    P.add_term(O.SHELL_TRI, (1.0, 0.8, 0.5))
    P.add_term(O.TRI_AREA, ())
    yield "shell_tri", P, sh.x
    dg = meshgen.dirichlet_grid(n=12)
    P = O.Problem(dg.tris, dg.rest, dg.n_verts, 1)
    P.add_term(O.DIRICHLET, ())
    yield "dirichlet", P, dg.x


def same(a, b):
    if a is None or b is None:
        return a is None and b is None
    return np.array_equal(np.asarray(a).view(np.uint64), np.asarray(b).view(np.uint64))


@pytest.mark.parametrize("build", ["parity", "fast"])
def test_parallel_eval_is_bit_identical(build):
    handle = O.lib() if build == "parity" else O.load(O.build_fast())
    with O.using(handle):
        for name, P, x in problems():
            for mode in MODES:
                ref = P.eval(x, mode, scales=False)
                for threads in (1, 3, 8):
                    r = P.eval_par(x, mode, threads=threads)
                    assert np.float64(r.energy).view(np.uint64) == np.float64(ref.energy).view(np.uint64), name
                    assert np.float64(r.esum_abs).view(np.uint64) == np.float64(ref.esum_abs).view(np.uint64)
                    assert same(r.grad, ref.grad), (name, mode, threads)
                    assert same(r.hess, ref.hess), (name, mode, threads)


def test_fast_build_agrees_with_parity_build_to_rounding():
    name, P, x = next(problems())
    ref = P.eval(x, O.ENERGY | O.GRAD | O.HESS | O.SPD)
    with O.using(O.load(O.build_fast())):
        r = P.eval_par(x, O.ENERGY | O.GRAD | O.HESS | O.SPD, threads=4)
    assert abs(r.energy - ref.energy) <= 1e-12 * ref.esum_abs
    assert np.all(np.abs(r.grad - ref.grad) <= 1e-11 * ref.gscale + 1e-300)
    assert np.all(np.abs(r.hess - ref.hess).ravel() <= 1e-11 * ref.hscale.ravel() + 1e-300)
