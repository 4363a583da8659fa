"""Pins of the oracle's pattern update for new interaction pairs (Sec. 6.3, the CSR update of the
appendix): brute force with Python sets, and the properties the update must have (old blocks kept,
symmetric patterns stay symmetric, the result independent of pair order and of batching, present
pairs and self pairs adding nothing, old blocks' new indices pointing at the same (row, column))."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_00406_amd import meshgen


def brute(rowptr, colidx, pairs, nv):
    rows = [set(colidx[rowptr[r]:rowptr[r + 1]].tolist()) for r in range(nv)]
    for a, b in np.asarray(pairs).reshape(-1, 2).tolist():
        if a != b:
            rows[a].add(b)
            rows[b].add(a)
    rp = [0]
    ci = []
    for r in range(nv):
        ci += sorted(rows[r])
        rp.append(len(ci))
    return np.array(rp), np.array(ci)


def random_pattern(nv, density, rng, symmetric=True):
    m = rng.random((nv, nv)) < density
    if symmetric:
        m = m | m.T
    np.fill_diagonal(m, True)
    rp = np.concatenate([[0], np.cumsum(m.sum(1))]).astype(np.int32)
    ci = np.concatenate([np.nonzero(m[r])[0] for r in range(nv)]).astype(np.int32)
    return rp, ci


@pytest.mark.parametrize("seed", range(6))
def test_insert_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    nv = int(rng.integers(1, 40))
    rp, ci = random_pattern(nv, rng.uniform(0.0, 0.3), rng, symmetric=bool(seed % 2))
    pairs = rng.integers(0, nv, size=(int(rng.integers(0, 60)), 2))
    rp2, ci2, mp = O.insert_pairs(rp, ci, pairs, nv)
    brp, bci = brute(rp, ci, pairs, nv)
    assert np.array_equal(rp2, brp) and np.array_equal(ci2, bci)
    rows_old = np.repeat(np.arange(nv), np.diff(rp))
    rows_new = np.repeat(np.arange(nv), np.diff(rp2))
    assert np.array_equal(rows_new[mp], rows_old) and np.array_equal(ci2[mp], ci)


def test_insert_properties_on_a_mesh_pattern():
    tris, pos = meshgen.grid(12)
    P = O.Problem(tris, pos, 144, 3)
    P.add_term(O.STVK, (1.0, 1.0))
    rp, ci = P.build_pattern()
    rng = np.random.default_rng(3)
    pairs = rng.integers(0, 144, size=(300, 2))
    rp2, ci2, mp = O.insert_pairs(rp, ci, pairs, 144)
    # symmetric in, symmetric out
    A = np.zeros((144, 144), bool)
    A[np.repeat(np.arange(144), np.diff(rp2)), ci2] = True
    assert np.array_equal(A, A.T)
    # rows sorted and unique
    for r in range(144):
        row = ci2[rp2[r]:rp2[r + 1]]
        assert np.all(np.diff(row) > 0)
    # order of the pairs, swapping a pair's ends, batching: all the same result
    perm = rng.permutation(len(pairs))
    for q in (pairs[perm], pairs[:, ::-1]):
        r3, c3, _ = O.insert_pairs(rp, ci, q, 144)
        assert np.array_equal(r3, rp2) and np.array_equal(c3, ci2)
    ra, ca, _ = O.insert_pairs(rp, ci, pairs[:120], 144)
    rb, cb, _ = O.insert_pairs(ra, ca, pairs[120:], 144)
    assert np.array_equal(rb, rp2) and np.array_equal(cb, ci2)
    # pairs already present, and self pairs, change nothing
    rows = np.repeat(np.arange(144), np.diff(rp))
    present = np.stack([rows, ci], 1)
    r4, c4, m4 = O.insert_pairs(rp, ci, np.concatenate([present, np.stack([rows, rows], 1)]), 144)
    assert np.array_equal(r4, rp) and np.array_equal(c4, ci) and np.array_equal(m4, np.arange(len(ci)))
    # the count: old blocks plus the distinct new off-diagonal blocks
    keys = set(zip(rows.tolist(), ci.tolist()))
    new = {(a, b) for a, b in pairs.tolist() if a != b} | {(b, a) for a, b in pairs.tolist() if a != b}
    assert rp2[-1] == len(keys | new)


def test_insert_rejects_out_of_range():
    rp, ci = random_pattern(5, 0.2, np.random.default_rng(1))
    with pytest.raises(ValueError):
        O.insert_pairs(rp, ci, np.array([[0, 5]]), 5)
