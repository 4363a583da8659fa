"""CPU-side tests of the product library: it loads, exports every entry point
that include/mad.h declares, validates arguments before any device work, and
its host topology (edges, diamonds) is bit-exact against the oracle's."""
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_00406_amd import mad, meshgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "mad.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mad_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(mad.LIB_PATH), "libmad.so is not built"
    declared = header_functions()
    assert len(declared) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", mad.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (mad_[a-z_]+)\b", out))
    missing = [f for f in declared if f not in exported]
    assert not missing, f"declared but not exported: {missing}"
    assert declared == mad.exported_symbols(), "binding does not mirror the header"
    lib = mad.lib()
    for f in declared:
        assert hasattr(lib, f)


def test_library_is_gfx950_code_object():
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", mad.LIB_PATH], capture_output=True, text=True)
    if out.returncode != 0:
        pytest.skip("roc-obj-ls unavailable")
    assert "gfx950" in out.stdout


def test_version_and_defaults():
    assert mad.mad_version() == 100
    o = mad.mad_options_default()
    assert o.patch_faces == 0 and o.spd_eps == 0.0 and o.scatter == mad.SCATTER_PATCH


@pytest.mark.parametrize("name", ["two_tris", "octahedron", "nonmanifold", "grid5"])
def test_host_topology_matches_oracle(name):
    tris, pos = meshgen.tiny_meshes()[name]
    m = mad.Mesh(tris, pos.shape[0])
    topo = O.topology(tris, pos.shape[0])
    assert m.n_edges == topo.edges.shape[0]
    assert np.array_equal(m.diamonds(), topo.diamonds)


def test_host_topology_matches_oracle_larger():
    for tris, nv in [(meshgen.grid(64)[0], 64 * 64), (meshgen.icosphere(9)[0], 10 * 81 + 2)]:
        m = mad.Mesh(tris, nv)
        topo = O.topology(tris, nv)
        assert m.n_edges == topo.edges.shape[0]
        assert np.array_equal(m.diamonds(), topo.diamonds)


def test_mesh_validation_errors():
    with pytest.raises(mad.MadError) as e:
        mad.Mesh(np.array([[0, 1, 4]], np.int32), 4)
    assert e.value.code == -2
    with pytest.raises(mad.MadError) as e:
        mad.Mesh(np.array([[0, 1, 1]], np.int32), 4)
    assert e.value.code == -2
    with pytest.raises(mad.MadError) as e:
        mad.Mesh(np.array([[0, 1, 2]], np.int32), 0)
    assert e.value.code == -1
    # component offsets must partition the vertices, and faces may not straddle components
    with pytest.raises(mad.MadError) as e:
        mad.Mesh(np.array([[0, 1, 2]], np.int32), 6, np.array([0, 2, 6]))
    assert e.value.code == -2
    with pytest.raises(mad.MadError) as e:
        mad.Mesh(np.array([[0, 1, 2]], np.int32), 6, np.array([0, 3, 5]))
    assert e.value.code == -1


def test_problem_validation_errors():
    tris, pos = meshgen.grid(3)
    m = mad.Mesh(tris, 9)
    with pytest.raises(mad.MadError) as e:
        mad.Problem(m, 4)
    assert e.value.code == -1
    p = mad.Problem(m, 3, mad.F32)
    with pytest.raises(mad.MadError) as e:
        p.add_term(mad.SYMDIR, (), pos)            # VarDim 2 term on a VarDim 3 problem
    assert e.value.code == -8
    with pytest.raises(mad.MadError) as e:
        p.add_term(mad.STVK, (1.0, 1.0), None)     # needs rest positions
    assert e.value.code == -1
    bad = pos.copy()
    bad[4] = bad[0]                                # collapses rest triangles
    with pytest.raises(mad.MadError) as e:
        p.add_term(mad.STVK, (1.0, 1.0), bad)
    assert e.value.code == -3
    with pytest.raises(mad.MadError) as e:
        p.add_term(mad.BENDING, (1.0, float("nan")), pos)
    assert e.value.code == -1
    with pytest.raises(mad.MadError) as e:
        mad.mad_problem_eval(p.handle, np.zeros(27), mad.ENERGY, np.zeros(1), stream=0)
    assert e.value.code == -7                      # eval before finalize
    with pytest.raises(mad.MadError) as e:
        p.reserve_pairs(-1)
    assert e.value.code == -1
    with pytest.raises(mad.MadError) as e:
        mad.mad_problem_insert_pairs(p.handle, np.zeros((1, 2), np.int32), 1, stream=0)
    assert e.value.code == -7                      # insertion before finalize
    with pytest.raises(mad.MadError) as e:
        p.add_term(mad.INERTIA, (0.1, 0.0, 0.0, -9.8), None)
    assert e.value.code == -1                      # vertex terms have their own entry point
    o = mad.mad_options_default()
    o.spd_eps = -1.0
    with pytest.raises(mad.MadError) as e:
        mad.mad_problem_create(m.handle, 3, mad.F64, o)
    assert e.value.code == -1
    o = mad.mad_options_default()
    o.reserved[3] = 7
    with pytest.raises(mad.MadError) as e:
        mad.mad_problem_create(m.handle, 3, mad.F64, o)
    assert e.value.code == -1
    o = mad.mad_options_default()
    o.lock_spins = -2                              # below MAD_LOCK_NO_WAIT
    with pytest.raises(mad.MadError) as e:
        mad.mad_problem_create(m.handle, 3, mad.F64, o)
    assert e.value.code == -1
    o.lock_spins = mad.LOCK_NO_WAIT
    mad.mad_problem_destroy(mad.mad_problem_create(m.handle, 3, mad.F64, o))


def test_status_codes_mirror_header():
    txt = open(os.path.join(ROOT, "include", "mad.h")).read()
    codes = {int(v): k for k, v in re.findall(r"\b(MAD_(?:OK|E_[A-Z_]+))\s*=\s*(-?\d+)", txt)}
    assert codes == mad.STATUS
    assert re.search(r"MAD_LOCK_NO_WAIT\s*=\s*-1\b", txt) and mad.LOCK_NO_WAIT == -1
