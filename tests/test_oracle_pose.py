"""Pins for the oracle's genotype -> pose (Sec. 2.1: position, orientation, torsions).

Checked against: the identity genotype, rigid-body facts (bond lengths and
intra-fragment distances do not depend on the genotype), quaternion sign/scale
invariance, 2*pi periodicity, SciPy's rotation matrix (a library routine,
scalar-last order), and the textbook dihedral of a 4-atom chain.
"""
import itertools

import numpy as np
from scipy.spatial.transform import Rotation

from oracle import dock_ref as R
from paper_2410_10447_amd import synth
from tests.helpers import ligand_from_bonds

FF = synth.force_field()


def _rand_genotypes(rng, n, T):
    t = rng.uniform(-5, 5, (n, 3))
    q = rng.normal(size=(n, 4))
    psi = rng.uniform(-np.pi, np.pi, (n, T))
    return np.concatenate([t, q, psi], axis=1)


def test_identity_genotype_gives_reference():
    lig = synth.ligand(24, 6, 0)
    p = R.prepare(lig, FF)
    g = np.zeros((1, 7 + p.n_torsions))
    g[0, 3] = 1.0
    x = R.pose(p, g)[0]
    # psi = 0 rotations are the identity up to the (y - p) + p round trip
    assert np.abs(x - p.y0).max() < 1e-14


def test_rigid_invariants():
    lig = synth.ligand(48, 10, 1000)
    p = R.prepare(lig, FF)
    rng = np.random.default_rng(1)
    g = _rand_genotypes(rng, 16, p.n_torsions)
    x = R.pose(p, g)
    b = np.asarray(lig.bonds)
    bl = np.linalg.norm(x[:, b[:, 0]] - x[:, b[:, 1]], axis=-1)
    assert np.abs(bl - 1.5).max() < 1e-12
    for f in range(p.n_frag):
        idx = np.nonzero(p.frag == f)[0]
        for i, j in itertools.combinations(idx, 2):
            d = np.linalg.norm(x[:, i] - x[:, j], axis=-1)
            d0 = np.linalg.norm(p.y0[i] - p.y0[j])
            assert np.abs(d - d0).max() < 1e-12
    # bonded angles across a rotatable bond are kept too: distance a_k's
    # neighbours to b_k is invariant; torsion changes only dihedrals
    for k in range(p.n_torsions):
        a, bb = p.axis[k]
        d = np.linalg.norm(x[:, a] - x[:, bb], axis=-1)
        assert np.abs(d - 1.5).max() < 1e-12


def test_quaternion_sign_scale_and_torsion_period():
    lig = synth.ligand(30, 8, 5)
    p = R.prepare(lig, FF)
    rng = np.random.default_rng(2)
    g = _rand_genotypes(rng, 8, p.n_torsions)
    x = R.pose(p, g)
    g2 = g.copy(); g2[:, 3:7] *= -1.0
    g3 = g.copy(); g3[:, 3:7] *= 2.5
    g4 = g.copy(); g4[:, 7:] += 2 * np.pi
    for gg in (g2, g3, g4):
        assert np.abs(R.pose(p, gg) - x).max() < 1e-12


def test_quat_matrix_matches_scipy():
    rng = np.random.default_rng(3)
    q = rng.normal(size=(50, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    ours = R.quat_matrix(q)
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    assert np.abs(ours - ref).max() < 1e-14


def _dihedral(a, b, c, d):
    b1, b2, b3 = b - a, c - b, d - c
    n1, n2 = np.cross(b1, b2), np.cross(b2, b3)
    return np.arctan2(np.linalg.norm(b2) * np.dot(b1, n2), np.dot(n1, n2))


def test_four_atom_chain_dihedral_moves_by_psi():
    lig = ligand_from_bonds([[0, 1], [1, 2], [2, 3]], [1], seed=4)
    p = R.prepare(lig, FF)
    assert p.axis.tolist() == [[1, 2]]
    for psi in (0.3, -1.2, 2.9):
        g = np.array([[0, 0, 0, 1, 0, 0, 0, psi]], dtype=float)
        x = R.pose(p, g)[0]
        d0 = _dihedral(*p.y0)
        d1 = _dihedral(*x)
        diff = (d1 - d0 + np.pi) % (2 * np.pi) - np.pi
        assert abs(diff - psi) < 1e-12
        # the fixed side stays put, the moving atom stays on its circle
        assert np.abs(x[:3] - p.y0[:3]).max() < 1e-12


def test_leaf_first_equals_composed_fragment_transforms():
    """The pose equals each atom mapped by the product of its enclosing torsions.

    Independent construction: for atom i, apply rotations of the torsions that
    contain it, root-most last, each about the *reference* axis of its bond.
    """
    lig = synth.ligand(40, 12, 8)
    p = R.prepare(lig, FF)
    rng = np.random.default_rng(9)
    psi = rng.uniform(-np.pi, np.pi, p.n_torsions)
    y = R.internal_coords(p, psi[None, :])[0]
    for i in range(p.n_atoms):
        ks = [k for k in range(p.n_torsions) if p.moving[k, i]]
        ks.sort(key=lambda k: -p.moving[k].sum())     # root-most (largest) first
        v = p.y0[i].copy()
        for k in reversed(ks):                        # deepest first
            a, b = p.axis[k]
            u = (p.y0[b] - p.y0[a]) / np.linalg.norm(p.y0[b] - p.y0[a])
            c, s = np.cos(psi[k]), np.sin(psi[k])
            K = np.array([[0, -u[2], u[1]], [u[2], 0, -u[0]], [-u[1], u[0], 0]])
            Rk = np.eye(3) + s * K + (1 - c) * K @ K
            v = Rk @ (v - p.y0[a]) + p.y0[a]
        assert np.abs(v - y[i]).max() < 1e-12
