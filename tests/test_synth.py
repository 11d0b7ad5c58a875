"""The seeded generators are deterministic and produce the stated shapes."""
import numpy as np

from paper_2410_10447_amd import synth


def test_deterministic_and_shapes():
    a = synth.score_workload(16)
    b = synth.score_workload(16)
    la, lb = a.ligands[0], b.ligands[0]
    assert synth.digest(la.xyz, la.charge, la.cls, la.bonds, la.rot_bonds, a.grids.maps,
                        a.genotypes[0]) == \
        synth.digest(lb.xyz, lb.charge, lb.cls, lb.bonds, lb.rot_bonds, b.grids.maps,
                     b.genotypes[0])
    assert la.n_atoms == 24 and la.n_torsions == 6
    assert a.grids.maps.shape == (10, 40, 40, 40) and a.grids.maps.dtype == np.float32
    assert a.genotypes[0].shape == (16, 13)


def test_ligand_geometry():
    lig = synth.ligand(48, 10, 1000)
    b = lig.bonds
    d = np.linalg.norm(lig.xyz[b[:, 0]] - lig.xyz[b[:, 1]], axis=1)
    assert np.allclose(d, 1.5, atol=1e-12)
    assert np.abs(lig.xyz.mean(axis=0)).max() < 1e-12
    deg = np.bincount(b.ravel(), minlength=48)
    assert deg.max() <= 4
    for k in lig.rot_bonds:
        u, v = b[k]
        assert deg[u] >= 2 and deg[v] >= 2


def test_uneven_sizes_in_range():
    w = synth.uneven_workload(n_ligands=8, per_ligand=4, grid_n=16)
    for lig, g in zip(w.ligands, w.genotypes):
        assert 12 <= lig.n_atoms <= 128 and 0 <= lig.n_torsions <= 32
        assert g.shape == (4, 7 + lig.n_torsions)
