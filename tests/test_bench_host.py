"""Host-side checks of the benchmark's measurement code (no GPU): the algorithmic byte counts that the
HBM rooflines divide by, recounted from the arrays the oracle builds for the same meshes; the per-dispatch
counter summary and its FP-operation count on a hand-written counter file; the refusal of more than one GPU."""
import os
import subprocess
import sys

import numpy as np

from oracle import oracle as O
from paper_2509_00406_amd import meshgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_shell_alg_bytes_recounted_from_arrays():
    inp = meshgen.shell_cylinder(n=16, seed=2001)
    topo = O.topology(inp.tris, inp.n_verts)
    rt = O.rest_tri(inp.tris, inp.rest)
    rd = O.rest_diamond(topo, inp.tris, inp.rest)
    P = O.Problem(inp.tris, inp.rest, inp.n_verts, 3)
    P.add_term(O.STVK, (1.0, 1.0))
    P.add_term(O.BENDING, (1.0, 1.0))
    rowptr, colidx = P.build_pattern()
    x = np.ascontiguousarray(inp.x, dtype=np.float64)
    reads = (x.nbytes + inp.tris.astype(np.int32).nbytes + topo.diamonds.astype(np.int32).nbytes + rt.nbytes + rd.nbytes
             + rowptr.astype(np.int32).nbytes + colidx.astype(np.int32).nbytes)
    nnzb = colidx.size
    for eb in (4, 8):
        writes = inp.n_verts * 3 * eb + nnzb * 9 * eb + 8   # gradient, every 3x3 block, the FP64 energy
        got = bench.alg_bytes(inp.n_verts, inp.tris.shape[0], topo.diamonds.shape[0], nnzb, eb)
        assert got == reads + writes, (got, reads + writes)


def test_symdir_alg_bytes_recounted_from_arrays():
    inp = meshgen.warped_grid(n=12, seed=3001)
    rt = O.rest_tri(inp.tris, inp.rest)
    P = O.Problem(inp.tris, inp.rest, inp.n_verts, 2)
    P.add_term(O.SYMDIR, ())
    rowptr, colidx = P.build_pattern()
    x = np.ascontiguousarray(inp.x, dtype=np.float64)
    assert x.shape[-1] == 2 or x.size == 2 * inp.n_verts
    reads = x.nbytes + inp.tris.astype(np.int32).nbytes + rt.nbytes + rowptr.nbytes + colidx.nbytes
    nnzb = colidx.size
    for eb in (4, 8):
        writes = inp.n_verts * 2 * eb + nnzb * 4 * eb + 8
        got = bench.symdir_alg_bytes(inp.n_verts, inp.tris.shape[0], nnzb, eb)
        assert got == reads + writes, (got, reads + writes)


def test_summarize_counters_per_dispatch_and_fp_ops(tmp_path):
    d = tmp_path / "pass" / "host"
    d.mkdir(parents=True)
    rows = ["Kernel_Name,Counter_Name,Counter_Value,Dispatch_Id"]
    # two dispatches of one kernel, counters split over two agents' rows each; one dispatch of another
    vals = {"SQ_INSTS_VALU_FMA_F32": (30, 50), "SQ_INSTS_VALU_MUL_F32": (10, 10), "SQ_INSTS_VALU_ADD_F32": (4, 6),
            "SQ_INSTS_VALU_TRANS_F32": (1, 3), "SQ_INSTS_VALU_FMA_F64": (2, 2)}
    for disp in (1, 2):
        for c, (a, b) in vals.items():
            v = a if disp == 1 else b
            rows.append(f"kern_a,{c},{v / 2},{disp}")
            rows.append(f"kern_a,{c},{v / 2},{disp}")
    rows.append("kern_b,FETCH_SIZE,100,3")
    (d / "run_counter_collection.csv").write_text("\n".join(rows) + "\n")
    out = bench.summarize_counters(str(tmp_path / "pass"), n_elements=16)
    a = out["kern_a"]
    assert a["dispatches"] == 2
    assert a["SQ_INSTS_VALU_FMA_F32"] == 40 and a["SQ_INSTS_VALU_TRANS_F32"] == 2
    # 64 lanes x (2 FMA + MUL + ADD + TRANS), F32 and F64, per dispatch: 64 x (80 + 10 + 5 + 2 + 4)
    assert a["fp_ops_per_dispatch"] == 64 * 101
    assert a["fp_ops_per_element"] == 64 * 101 / 16
    assert out["kern_b"] == {"dispatches": 1, "FETCH_SIZE": 100.0}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stdout
