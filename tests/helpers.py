"""Shared helpers for tests: build ligands from golden fixtures."""
import json
import os

import numpy as np

from paper_2410_10447_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def ligand_from_bonds(bonds, rot_bonds, seed=0, cls=None, charge=None):
    """A ligand with the given topology and coordinates from a seeded embedding.

    Coordinates are placed so bonded atoms are 1.5 A apart (each child at a
    random direction from its parent); only the topology matters to the
    preparation tests.
    """
    bonds = np.asarray(bonds, dtype=np.int32).reshape(-1, 2)
    n = int(bonds.max()) + 1 if len(bonds) else 1
    rng = np.random.default_rng(seed)
    xyz = np.zeros((n, 3))
    placed = {0}
    pending = list(map(tuple, bonds))
    while pending:
        for e in list(pending):
            u, v = int(e[0]), int(e[1])
            if u in placed and v in placed:          # a ring closure: topology only
                pending.remove(e)
            elif u in placed and v not in placed:
                d = rng.normal(size=3)
                xyz[v] = xyz[u] + 1.5 * d / np.linalg.norm(d)
                placed.add(v)
                pending.remove(e)
            elif v in placed and u not in placed:
                d = rng.normal(size=3)
                xyz[u] = xyz[v] + 1.5 * d / np.linalg.norm(d)
                placed.add(u)
                pending.remove(e)
    if cls is None:
        cls = rng.integers(0, 8, n)
    if charge is None:
        charge = rng.normal(0, 0.2, n)
    return synth.Ligand(xyz=xyz, charge=np.asarray(charge, float), cls=np.asarray(cls, np.int32),
                        bonds=bonds, rot_bonds=np.asarray(rot_bonds, np.int32))
