"""The vectorised numpy energies agree with the oracle on small meshes."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_00406_amd import meshgen
from tests import npref


@pytest.mark.parametrize("noise", ["relative", "absolute"])
def test_npref_shell_energy_matches_oracle(noise):
    inp = meshgen.shell_cylinder(n=20, seed=4, noise=noise)
    P = O.Problem(inp.tris, inp.rest, inp.n_verts, 3)
    P.add_term(O.STVK, (0.9, 1.3))
    P.add_term(O.BENDING, (1.1, 1.0))
    r = P.eval(inp.x, O.ENERGY)
    e, s = npref.shell_energy(inp.tris, inp.rest, inp.x, P.topo.diamonds, P.topo.diamond_faces, (0.9, 1.3), (1.1, 1.0))
    assert e == pytest.approx(r.energy, rel=1e-12)
    assert s == pytest.approx(r.esum_abs, rel=1e-12)


def test_npref_cloth_energy_matches_oracle():
    from oracle import oracle as O
    inp = meshgen.cloth(n=30, seed=6003)
    P = O.Problem(inp.tris, inp.rest, inp.n_verts, 3)
    P.add_term(O.SPRING, inp.meta["spring_params"])
    P.add_term(O.INERTIA, inp.meta["inertia_params"], vertex_data=inp.meta["vdata"])
    r = P.eval(inp.x, O.ENERGY)
    e, s = npref.cloth_energy(inp.tris, inp.rest, inp.x, inp.meta["vdata"], inp.meta["spring_params"],
                              inp.meta["inertia_params"])
    assert abs(e - r.energy) <= 1e-13 * s
    assert s == pytest.approx(r.esum_abs, rel=1e-12)
