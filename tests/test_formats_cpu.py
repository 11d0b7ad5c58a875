"""AutoDock .map reading and writing (host IO). The fixture tests/golden/tiny.map
is a hand-written 2 x 2 x 2-cell map whose value at node (x, y, z) is
x + 10 y + 100 z, which pins the node order (x fastest) and the origin rule
(CENTER - NELEMENTS / 2 * SPACING)."""
import os

import numpy as np
import pytest

from paper_2410_10447_amd import formats, synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny.map")


def test_golden_map_node_order_and_origin():
    m = formats.read_map(GOLDEN)
    assert m.values.shape == (3, 3, 3)
    z, y, x = np.meshgrid(np.arange(3), np.arange(3), np.arange(3), indexing="ij")
    assert np.array_equal(m.values, (x + 10 * y + 100 * z).astype(np.float32))
    assert m.spacing == 0.5 and m.origin == (0.5, 1.5, 2.5)


def test_round_trip_is_exact(tmp_path):
    rng = np.random.default_rng(1)
    v = (rng.normal(size=(5, 7, 3)) * 10.0 ** rng.integers(-8, 6, size=(5, 7, 3))).astype(np.float32)
    p = tmp_path / "a.map"
    formats.write_map(p, v, 0.375, (-1.5, 2.25, 0.0))
    m = formats.read_map(p)
    assert np.array_equal(m.values.view(np.uint32), v.view(np.uint32))
    assert m.spacing == 0.375 and np.allclose(m.origin, (-1.5, 2.25, 0.0), atol=1e-12)


def test_bad_files_are_rejected(tmp_path):
    text = open(GOLDEN).read()
    with pytest.raises(ValueError):
        formats.read_map(text.replace("SPACING", "SPACE"), from_text=True)
    with pytest.raises(ValueError):
        formats.read_map("\n".join(text.splitlines()[:-1]) + "\n", from_text=True)   # one value short
    with pytest.raises(ValueError):
        formats.write_map(tmp_path / "b.map", np.zeros((4, 3, 3), np.float32), 0.5, (0, 0, 0))


def test_load_maps_stacks_in_library_order(tmp_path):
    g = synth.grids(9, 5, 3)                 # 9 nodes per axis: 8 cells, writable as .map
    paths = []
    for k in range(5):
        p = tmp_path / f"m{k}.map"
        formats.write_map(p, g.maps[k], g.spacing, g.origin)
        paths.append(p)
    st = formats.load_maps(paths[:3], paths[3], paths[4])
    assert np.array_equal(st.maps, np.asarray(g.maps, np.float32))
    assert st.spacing == g.spacing and np.allclose(st.origin, g.origin, atol=1e-6)
    formats.write_map(tmp_path / "odd.map", g.maps[0], g.spacing * 2, g.origin)
    with pytest.raises(ValueError):
        formats.load_maps(paths[:3], paths[3], tmp_path / "odd.map")


# ---------------------------------------------------------------------------
# PDBQT ligands. Two hand-written fixtures with hand-derived topologies:
# * pyridine_ethanol.pdbqt: a pyridine ring (N1 an acceptor, NA; C2..C6
#   aromatic) with a 2-hydroxyethyl chain C7-C8-O9-H10 at C4 (para to N1);
#   three torsions (C4-C7, C7-C8, C8-O9), four rigid fragments (the ring,
#   C7, C8, O9+H10). Pairs >= 4 bonds apart in different fragments: H10 with
#   C4 (4 bonds), C3, C5 (5), C2, C6 (6), N1 (7); O9 with C3, C5, C2, C6, N1;
#   C8 with C2, C6, N1; C7 with N1: 15 pairs, one of them donor-acceptor
#   (H10, HD, with N1, NA).
# * biphenyl.pdbqt: two aromatic rings joined by C1-C7, one torsion, two
#   fragments; the pair (a, b), a on ring 1 and b on ring 2, is d_1(a, C1) +
#   1 + d_2(C7, b) bonds apart, so it is kept when d_1 + d_2 >= 3: 36 pairs
#   minus the 13 with d_1 + d_2 <= 2 (1 + 2 + 2 + 2 + 2 + 4) = 23 pairs.
# ---------------------------------------------------------------------------

PDBQT1 = os.path.join(os.path.dirname(__file__), "golden", "pyridine_ethanol.pdbqt")
PDBQT2 = os.path.join(os.path.dirname(__file__), "golden", "biphenyl.pdbqt")


def _named_pairs(lig, pairs):
    return sorted(tuple(sorted((lig.names[int(i)], lig.names[int(j)]))) for i, j in pairs)


def test_pdbqt_pyridine_ethanol_topology():
    from oracle import dock_ref as R
    from paper_2410_10447_amd import dock
    lig = formats.read_pdbqt(PDBQT1)
    assert lig.names == ["N1", "C2", "C3", "C4", "C5", "C6", "C7", "C8", "O9", "H10"]
    assert lig.types == ["NA", "A", "A", "A", "A", "A", "C", "C", "OA", "HD"]
    assert lig.cls.tolist() == [3, 1, 1, 1, 1, 1, 0, 0, 4, 6]
    assert lig.charge.tolist() == [-0.26, 0.1, 0.02, 0.01, 0.02, 0.1, 0.05, 0.2, -0.39, 0.21]
    assert lig.root == 0
    names = lig.names
    bonds = sorted(tuple(sorted((names[u], names[v]))) for u, v in lig.bonds)
    assert bonds == sorted([("C2", "N1"), ("C2", "C3"), ("C3", "C4"), ("C4", "C5"), ("C5", "C6"),
                            ("C6", "N1"), ("C4", "C7"), ("C7", "C8"), ("C8", "O9"), ("H10", "O9")])
    rot = [tuple(sorted((names[u], names[v]))) for u, v in lig.bonds[lig.rot_bonds]]
    assert rot == [("C4", "C7"), ("C7", "C8"), ("C8", "O9")]
    ff = synth.force_field()
    p = R.prepare(lig, ff)
    want = sorted(tuple(sorted(x)) for x in
                  [("H10", a) for a in ("C4", "C3", "C5", "C2", "C6", "N1")]
                  + [("O9", a) for a in ("C3", "C5", "C2", "C6", "N1")]
                  + [("C8", a) for a in ("C2", "C6", "N1")] + [("C7", "N1")])
    assert p.n_frag == 4 and _named_pairs(lig, p.pairs) == want
    assert _named_pairs(lig, p.pairs[p.pair_hb]) == [("H10", "N1")]
    L = dock.Ligand(lig, ff, upload=False)
    ex = L.export()
    assert (L.n_torsions, L.n_fragments, L.n_pairs) == (3, 4, 15)
    assert _named_pairs(lig, ex["pairs"]) == want
    assert _named_pairs(lig, ex["pairs"][ex["pair_hb"]]) == [("H10", "N1")]


def test_pdbqt_biphenyl_rings_stay_rigid():
    from oracle import dock_ref as R
    from paper_2410_10447_amd import dock
    lig = formats.read_pdbqt(PDBQT2)
    assert lig.n_atoms == 12 and lig.bonds.shape == (13, 2) and lig.n_torsions == 1
    ff = synth.force_field()
    p = R.prepare(lig, ff)
    ring1 = {f"C{k}" for k in range(1, 7)}
    named = _named_pairs(lig, p.pairs)
    assert len(named) == 23 and p.n_frag == 2 and not p.pair_hb.any()
    assert all((a in ring1) != (b in ring1) for a, b in named)
    L = dock.Ligand(lig, ff, upload=False)
    assert (L.n_fragments, L.n_pairs) == (2, 23)
    assert _named_pairs(lig, L.export()["pairs"]) == named
    # the moving side of the torsion is the whole second ring
    assert set(np.nonzero(p.moving[0])[0].tolist()) == set(range(6, 12))


def test_pdbqt_round_trip_of_ring_ligands(tmp_path):
    """write_pdbqt then read_pdbqt: the same atoms (coordinates to the
    file's 3 decimals, charges to its 3 decimals), bonds and torsions, up to
    the file's atom order. Bonds come from the CONECT records here (the
    synthetic ligands put arbitrary types on 1.5 A bonds, which covalent
    radii would not all perceive; the fixtures above test perception)."""
    from oracle import dock_ref as R
    inv = {0: "C", 1: "A", 2: "N", 3: "NA", 4: "OA", 5: "SA", 6: "HD", 7: "HS"}
    ff = synth.force_field()
    for seed, (nr, nc, t) in enumerate([(1, 3, 2), (2, 6, 4), (3, 9, 6)]):
        lig = synth.ring_ligand(nr, nc, t, 900 + seed)
        lig.charge = np.round(lig.charge, 3)
        types = [inv[int(c)] for c in lig.cls]
        path = tmp_path / f"l{seed}.pdbqt"
        formats.write_pdbqt(path, lig, types)
        back = formats.read_pdbqt(path)
        # file order -> original index, by coordinates
        perm = [int(np.argmin(np.linalg.norm(lig.xyz - x, axis=1))) for x in back.xyz]
        assert sorted(perm) == list(range(lig.n_atoms))
        assert np.abs(back.xyz - lig.xyz[perm]).max() <= 5e-4
        assert np.array_equal(back.charge, lig.charge[perm]) and np.array_equal(back.cls, lig.cls[perm])
        orig = {tuple(sorted(b)) for b in lig.bonds.tolist()}
        got = {tuple(sorted((perm[u], perm[v]))) for u, v in back.bonds.tolist()}
        assert got == orig
        rot_o = {tuple(sorted(lig.bonds[k].tolist())) for k in lig.rot_bonds}
        rot_b = {tuple(sorted((perm[u], perm[v]))) for u, v in back.bonds[back.rot_bonds].tolist()}
        assert rot_b == rot_o and perm[back.root] == lig.root
        assert R.prepare(back, ff).pairs.shape == R.prepare(lig, ff).pairs.shape


def test_pdbqt_rejects_bad_files():
    text = open(PDBQT1).read()
    with pytest.raises(ValueError):
        formats.read_pdbqt(text.replace("BRANCH   8   9", "BRANCH   8  10"), from_text=True)   # not a bond
    with pytest.raises(ValueError):
        formats.read_pdbqt(text.replace(" HD", " XX"), from_text=True)                      # unknown type
    with pytest.raises(ValueError):
        formats.read_pdbqt("REMARK nothing\n", from_text=True)
