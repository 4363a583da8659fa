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


def test_npref_symdir_energy_matches_oracle():
    inp = meshgen.warped_grid(n=25, seed=3007)
    P = O.Problem(inp.tris, inp.rest, inp.n_verts, 2)
    P.add_term(O.SYMDIR, ())
    r = P.eval(inp.x, O.ENERGY)
    e, s = npref.symdir_energy(inp.tris, inp.rest, inp.x)
    assert abs(e - r.energy) <= 1e-13 * s
    assert s == pytest.approx(r.esum_abs, rel=1e-12)


def test_npref_per_component_energy_matches_oracle():
    inp = meshgen.icosphere_batch(n_meshes=4, mean_verts=700, vmin=600, vmax=900)
    co = inp.comp_offsets
    P = O.Problem(inp.tris, inp.rest, inp.n_verts, 3)
    P.add_term(O.STVK, (1.0, 1.0))
    P.add_term(O.BENDING, (1.0, 1.0))
    e, s = npref.shell_energy_by_component(inp.tris, inp.rest, inp.x, P.topo.diamonds, P.topo.diamond_faces,
                                           (1.0, 1.0), (1.0, 1.0), co)
    for c in range(len(co) - 1):
        lo, hi = int(co[c]), int(co[c + 1])
        sel = np.all((inp.tris >= lo) & (inp.tris < hi), axis=1)
        Q = O.Problem(inp.tris[sel] - lo, inp.rest[lo:hi], hi - lo, 3)
        Q.add_term(O.STVK, (1.0, 1.0))
        Q.add_term(O.BENDING, (1.0, 1.0))
        r = Q.eval(inp.x[lo:hi], O.ENERGY)
        assert abs(e[c] - r.energy) <= 1e-13 * s[c]
        assert s[c] == pytest.approx(r.esum_abs, rel=1e-12)


def test_npref_mlp_energy_matches_oracle():
    inp = meshgen.shell_cylinder(n=14, seed=5011)
    r = np.random.default_rng(3)
    H = 64
    theta = np.concatenate([r.normal(scale=0.5, size=6 * H), r.normal(scale=0.5, size=H),
                            r.normal(scale=0.12, size=H * H), r.normal(scale=0.5, size=H),
                            r.normal(scale=0.3, size=H), [0.1]])
    s_in, s_out = r.uniform(0.5, 2.0, 6), 0.8
    t = theta
    P = O.Problem(inp.tris, inp.rest, inp.n_verts, 3)
    P.add_term(O.MLP, O.mlp_pack(s_out, s_in, t[:6 * H].reshape(H, 6), t[6 * H:7 * H],
                                 t[7 * H:7 * H + H * H].reshape(H, H), t[7 * H + H * H:8 * H + H * H],
                                 t[8 * H + H * H:9 * H + H * H], t[9 * H + H * H]))
    ref = P.eval(inp.x, O.ENERGY)
    e, s = npref.mlp_energy(inp.tris, inp.rest, inp.x, theta, s_in, s_out)
    assert abs(e - ref.energy) <= 1e-12 * s
    assert s == pytest.approx(ref.esum_abs, rel=1e-12)
