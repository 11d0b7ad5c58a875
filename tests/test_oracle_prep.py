"""Pins for the oracle's ligand preparation (moving sets, fragments, pair list).

The paper (Sec. 2.1) only states that torsion genes turn rotatable bonds and
that the intramolecular energy sums over atom pairs; the exclusion reading is
pinned here by hand-worked fixtures (tests/golden/prep_*.json), by a
brute-force Floyd-Warshall distance matrix and by a parent-pointer definition
of the moving sets, none of which share code with the oracle's BFS.
"""
import itertools

import numpy as np
import pytest

from oracle import dock_ref as R
from paper_2410_10447_amd import synth
from tests.helpers import ligand_from_bonds, load_golden

FF = synth.force_field()


@pytest.mark.parametrize("name", ["prep_chain7.json", "prep_branched9.json", "prep_rigid6.json"])
def test_golden_topologies(name):
    g = load_golden(name)
    lig = ligand_from_bonds(g["bonds"], g["rot_bonds"])
    p = R.prepare(lig, FF)
    assert [list(map(int, a)) for a in p.axis] == g["axis"]
    for k, mv in enumerate(g["moving"]):
        assert sorted(np.nonzero(p.moving[k])[0].tolist()) == mv
    frags = {}
    for i, f in enumerate(p.frag):
        frags.setdefault(int(f), []).append(i)
    assert sorted(frags.values()) == sorted(g["fragments"])
    assert p.pairs.tolist() == g["pairs"]
    if "depth" in g:
        assert p.depth.tolist() == g["depth"]


def floyd_warshall(n, bonds):
    INF = 10 ** 9
    d = np.full((n, n), INF, dtype=np.int64)
    np.fill_diagonal(d, 0)
    for u, v in bonds:
        d[u, v] = d[v, u] = 1
    for k in range(n):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    return d


def parent_pointers(n, bonds, root=0):
    par = [-1] * n
    seen = {root}
    frontier = [root]
    while frontier:
        nxt = []
        for u in frontier:
            for a, b in bonds:
                for x, y in ((a, b), (b, a)):
                    if x == u and y not in seen:
                        par[y] = u
                        seen.add(y)
                        nxt.append(y)
        frontier = nxt
    return par


@pytest.mark.parametrize("seed,n,t", [(11, 12, 4), (12, 24, 6), (13, 48, 10), (14, 70, 20), (15, 5, 3)])
def test_random_ligands_against_bruteforce(seed, n, t):
    lig = synth.ligand(n, t, seed)
    p = R.prepare(lig, FF)
    bonds = [tuple(map(int, b)) for b in lig.bonds]
    D = floyd_warshall(n, bonds)
    assert np.array_equal(D, p.graph_dist)
    par = parent_pointers(n, bonds)

    def ancestors(i):
        out = []
        while i != -1:
            out.append(i)
            i = par[i]
        return out

    # moving set of torsion k = atoms whose root path passes through b_k
    for k in range(p.n_torsions):
        a, b = p.axis[k]
        assert par[b] == a
        want = [i for i in range(n) if b in ancestors(i)]
        assert np.nonzero(p.moving[k])[0].tolist() == want
        assert len(want) >= 2  # b_k has degree >= 2 for an internal bond
    # T + 1 fragments, sets nested or disjoint
    assert p.n_frag == p.n_torsions + 1
    for k1, k2 in itertools.combinations(range(p.n_torsions), 2):
        m1, m2 = p.moving[k1], p.moving[k2]
        inter = (m1 & m2).sum()
        assert inter in (0, min(m1.sum(), m2.sum()))
    # fragment = same set of enclosing torsions
    sig = [tuple(p.moving[:, i]) for i in range(n)]
    for i, j in itertools.combinations(range(n), 2):
        assert (p.frag[i] == p.frag[j]) == (sig[i] == sig[j])
    # pair list = brute-force definition
    want = [(i, j) for i, j in itertools.combinations(range(n), 2)
            if D[i, j] >= 4 and sig[i] != sig[j]]
    assert [tuple(x) for x in p.pairs.tolist()] == want


def test_pair_parameters_closed_forms():
    lig = synth.ligand(30, 8, 21)
    p = R.prepare(lig, FF)
    for k, (i, j) in enumerate(p.pairs):
        ci, cj = int(lig.cls[i]), int(lig.cls[j])
        hb = (ci in FF.donors and cj in FF.acceptors) or (cj in FF.donors and ci in FF.acceptors)
        assert hb == bool(p.pair_hb[k])
        if hb:
            d, a = (ci, cj) if ci in FF.donors else (cj, ci)
            assert p.r0[k] == FF.hb_r0[FF.donors.index(d), FF.acceptors.index(a)]
            assert p.eps[k] == FF.hb_eps[FF.donors.index(d), FF.acceptors.index(a)]
        else:
            assert p.r0[k] == FF.radius[ci] + FF.radius[cj]
            assert np.isclose(p.eps[k], np.sqrt(FF.eps[ci] * FF.eps[cj]), rtol=1e-15)
        assert np.isclose(p.qq[k], 332.06363 * lig.charge[i] * lig.charge[j], rtol=1e-15)


def test_single_atom_and_empty_torsions():
    lig = ligand_from_bonds(np.zeros((0, 2), np.int32), [])
    p = R.prepare(lig, FF)
    assert p.n_atoms == 1 and p.n_torsions == 0 and p.pairs.shape == (0, 2) and p.n_frag == 1
