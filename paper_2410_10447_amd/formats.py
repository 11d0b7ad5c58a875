"""AutoDock grid-map files (`.map`): read them into the map stack the library
takes, and write them (host IO; the kernels never see files).

The format (AutoDock 4): six header lines

    GRID_PARAMETER_FILE <name>
    GRID_DATA_FILE <name>
    MACROMOLECULE <name>
    SPACING <h>
    NELEMENTS <nx> <ny> <nz>      (even counts of cells; nodes per axis = count + 1)
    CENTER <cx> <cy> <cz>

then one value per node, x fastest, then y, then z. The grid's lowest node is
CENTER - (NELEMENTS / 2) * SPACING on each axis.
"""
from __future__ import annotations

import io
from dataclasses import dataclass

import numpy as np

_KEYS = ("GRID_PARAMETER_FILE", "GRID_DATA_FILE", "MACROMOLECULE", "SPACING", "NELEMENTS", "CENTER")


@dataclass
class GridMap:
    values: np.ndarray     # [nz][ny][nx] float32
    spacing: float
    origin: tuple          # lowest node (x, y, z)


def read_map(path_or_text, from_text: bool = False) -> GridMap:
    """Parses one .map file (or its text with from_text=True)."""
    f = io.StringIO(path_or_text) if from_text else open(path_or_text, "r")
    with f:
        head = {}
        for _ in range(6):
            parts = f.readline().split()
            if not parts or parts[0] not in _KEYS:
                raise ValueError(f"bad .map header line: {' '.join(parts)!r}")
            head[parts[0]] = parts[1:]
        h = float(head["SPACING"][0])
        n = [int(v) for v in head["NELEMENTS"]]
        if len(n) != 3 or any(v < 1 for v in n) or not h > 0:
            raise ValueError("bad NELEMENTS or SPACING")
        c = [float(v) for v in head["CENTER"]]
        nodes = [v + 1 for v in n]
        vals = np.loadtxt(f, dtype=np.float64, ndmin=1)
    if vals.size != nodes[0] * nodes[1] * nodes[2]:
        raise ValueError(f".map holds {vals.size} values, expected {nodes[0] * nodes[1] * nodes[2]}")
    origin = tuple(c[k] - (n[k] / 2.0) * h for k in range(3))
    return GridMap(vals.astype(np.float32).reshape(nodes[2], nodes[1], nodes[0]), h, origin)


def write_map(path, values, spacing: float, origin, macromolecule="receptor",
              grid_parameter_file="grid.gpf", grid_data_file="grid.maps.fld"):
    """Writes values [nz][ny][nx] (odd node counts) with 9 significant digits,
    which round-trip float32 exactly."""
    v = np.asarray(values, np.float32)
    nz, ny, nx = v.shape
    n = (nx - 1, ny - 1, nz - 1)
    if any(k % 2 for k in n):
        raise ValueError(".map grids have an even number of cells per axis")
    center = [origin[k] + (n[k] / 2.0) * spacing for k in range(3)]
    with open(path, "w") as f:
        f.write(f"GRID_PARAMETER_FILE {grid_parameter_file}\n")
        f.write(f"GRID_DATA_FILE {grid_data_file}\n")
        f.write(f"MACROMOLECULE {macromolecule}\n")
        f.write(f"SPACING {spacing:.9g}\n")
        f.write(f"NELEMENTS {n[0]} {n[1]} {n[2]}\n")
        f.write(f"CENTER {center[0]:.9g} {center[1]:.9g} {center[2]:.9g}\n")
        np.savetxt(f, v.reshape(-1), fmt="%.9g")


@dataclass
class MapStack:
    """Maps in the order the library takes them (type maps by atom class,
    then the electrostatic and the desolvation map), the shape of what
    `dock.Grids.from_synth` uploads."""
    maps: np.ndarray       # [M][nz][ny][nx] float32
    spacing: float
    origin: tuple


def load_maps(type_map_paths, elec_path, desolv_path) -> MapStack:
    """Reads the type maps (index = atom class) and the electrostatic and
    desolvation maps; all must share spacing, node counts and origin."""
    ms = [read_map(p) for p in list(type_map_paths) + [elec_path, desolv_path]]
    first = ms[0]
    for m in ms[1:]:
        if m.values.shape != first.values.shape or m.spacing != first.spacing or \
                not np.allclose(m.origin, first.origin, rtol=0, atol=1e-6):
            raise ValueError("maps of one set must share spacing, size and origin")
    return MapStack(np.stack([m.values for m in ms]), first.spacing, first.origin)


# ---------------------------------------------------------------------------
# PDBQT ligands (AutoDock 4): the ligand's atoms with their partial charges
# and AutoDock atom types, and its torsion tree (ROOT ... ENDROOT, nested
# BRANCH a b ... ENDBRANCH a b blocks, each BRANCH naming the rotatable bond
# from atom a, on the root side, to atom b). Columns follow the PDB ATOM
# record: serial 7-11, name 13-16, x/y/z 31-38/39-46/47-54, partial charge
# 71-76, atom type 78-79.
# ---------------------------------------------------------------------------

# AutoDock atom type -> atom class of the force-field table the library
# takes. The table the library uses here is synthetic (8 classes: donors 6
# and 7, acceptors 3 and 4), so this mapping is a reading: carbon 0,
# aromatic carbon 1, nitrogen 2, acceptor nitrogen 3, acceptor oxygen 4,
# sulphur and halogens 5, polar hydrogen on N/O 6, polar hydrogen on S 7.
AD_TYPE_CLASS = {"C": 0, "A": 1, "N": 2, "NA": 3, "NS": 3, "OA": 4, "OS": 4, "O": 4,
                 "S": 5, "SA": 5, "F": 5, "Cl": 5, "CL": 5, "Br": 5, "BR": 5, "I": 5, "P": 2,
                 "HD": 6, "HS": 7, "H": 0}

# covalent radii (A) by element, for bond perception from coordinates
_COVALENT = {"C": 0.76, "N": 0.71, "O": 0.66, "S": 1.05, "P": 1.07, "H": 0.31, "F": 0.57,
             "Cl": 1.02, "Br": 1.20, "I": 1.39}
_TYPE_ELEMENT = {"C": "C", "A": "C", "N": "N", "NA": "N", "NS": "N", "OA": "O", "OS": "O", "O": "O",
                 "S": "S", "SA": "S", "P": "P", "H": "H", "HD": "H", "HS": "H", "F": "F",
                 "Cl": "Cl", "CL": "Cl", "Br": "Br", "BR": "Br", "I": "I"}
BOND_TOLERANCE = 0.45      # A beyond the sum of covalent radii


@dataclass
class PdbqtLigand:
    """A ligand read from PDBQT, with the fields the library's ligand
    description takes (xyz, charge, cls, bonds, rot_bonds, root) plus the
    file's atom names, types and serial numbers."""
    xyz: np.ndarray        # float64 [N, 3]
    charge: np.ndarray     # float64 [N]
    cls: np.ndarray        # int32 [N]
    bonds: np.ndarray      # int32 [n_bonds, 2]
    rot_bonds: np.ndarray  # int32 [T], indices into bonds, in BRANCH order
    root: int
    names: list
    types: list
    serials: list

    @property
    def n_atoms(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_torsions(self) -> int:
        return int(self.rot_bonds.shape[0])


def perceive_bonds(xyz, types, tolerance: float = BOND_TOLERANCE):
    """Bonds from coordinates: atoms i < j are bonded when their distance is
    at most the sum of their covalent radii plus `tolerance` (and above
    0.4 A). Returns int32 [n_bonds, 2], sorted."""
    xyz = np.asarray(xyz, np.float64)
    rad = np.array([_COVALENT[_TYPE_ELEMENT[t]] for t in types])
    d = np.linalg.norm(xyz[:, None, :] - xyz[None, :, :], axis=2)
    lim = rad[:, None] + rad[None, :] + tolerance
    i, j = np.nonzero(np.triu((d <= lim) & (d > 0.4), k=1))
    return np.stack([i, j], axis=1).astype(np.int32).reshape(-1, 2)


def read_pdbqt(path_or_text, from_text: bool = False, tolerance: float = BOND_TOLERANCE) -> PdbqtLigand:
    """Parses a PDBQT ligand (the first MODEL if there are several). Bonds
    come from CONECT records when the file has any, else from coordinates
    (perceive_bonds); every BRANCH must name a bond. The root atom is the
    first atom of the ROOT block."""
    text = path_or_text if from_text else open(path_or_text).read()
    serials, names, types, xyz, charge = [], [], [], [], []
    branches, conect = [], []
    root_serial = None
    in_root = False
    for line in text.splitlines():
        rec = line[:6].strip()
        if rec == "ENDMDL":
            break
        if rec in ("ATOM", "HETATM"):
            serial = int(line[6:11])
            t = line[77:79].strip() if len(line) > 77 else ""
            if not t:
                raise ValueError(f"atom {serial}: no AutoDock type (columns 78-79)")
            if t not in AD_TYPE_CLASS:
                raise ValueError(f"atom {serial}: AutoDock type {t!r} has no class in AD_TYPE_CLASS")
            serials.append(serial)
            names.append(line[12:16].strip())
            types.append(t)
            xyz.append([float(line[30:38]), float(line[38:46]), float(line[46:54])])
            charge.append(float(line[70:76]))
            if in_root and root_serial is None:
                root_serial = serial
        elif rec == "ROOT":
            in_root = True
        elif rec == "ENDROOT":
            in_root = False
        elif rec == "BRANCH":
            a, b = (int(v) for v in line.split()[1:3])
            branches.append((a, b))
        elif rec == "CONECT":
            f = [int(v) for v in line.split()[1:]]
            conect += [(f[0], g) for g in f[1:]]
    if not serials:
        raise ValueError("no ATOM/HETATM records")
    index = {s: k for k, s in enumerate(serials)}
    if len(index) != len(serials):
        raise ValueError("repeated atom serial number")
    xyz = np.asarray(xyz, np.float64)
    if conect:
        pairs = {tuple(sorted((index[a], index[b]))) for a, b in conect}
        bonds = np.array(sorted(pairs), dtype=np.int32).reshape(-1, 2)
    else:
        bonds = perceive_bonds(xyz, types, tolerance)
    where = {tuple(b): k for k, b in enumerate(bonds.tolist())}
    rot = []
    for a, b in branches:
        if a not in index or b not in index:
            raise ValueError(f"BRANCH {a} {b} names an unknown atom")
        key = tuple(sorted((index[a], index[b])))
        if key not in where:
            raise ValueError(f"BRANCH {a} {b} is not a bond")
        rot.append(where[key])
    cls = np.array([AD_TYPE_CLASS[t] for t in types], dtype=np.int32)
    return PdbqtLigand(xyz, np.asarray(charge, np.float64), cls, bonds, np.asarray(rot, np.int32).reshape(-1),
                       index[root_serial] if root_serial is not None else 0, names, types, serials)


def write_pdbqt(path, lig, types, names=None, conect: bool = True):
    """Writes a ligand (xyz, charge, bonds, rot_bonds, root) as PDBQT: ROOT
    holds the root atom's rigid fragment, each rotatable bond opens a BRANCH
    holding the fragment on its far side, nested as the torsion tree is.
    With `conect` the bonds are also written as CONECT records (so a reader
    need not perceive them from coordinates). Serial numbers follow the
    file order."""
    xyz = np.asarray(lig.xyz, np.float64)
    n = xyz.shape[0]
    bonds = np.asarray(lig.bonds, np.int64).reshape(-1, 2)
    rot = set(int(k) for k in np.asarray(lig.rot_bonds).reshape(-1))
    adj = [[] for _ in range(n)]
    for k, (u, v) in enumerate(bonds.tolist()):
        adj[u].append((v, k))
        adj[v].append((u, k))
    names = names or [f"{_TYPE_ELEMENT[t]}{k + 1}" for k, t in enumerate(types)]
    serial = {}
    out = []

    def atom_line(i):
        serial[i] = len(serial) + 1
        return (f"ATOM  {serial[i]:5d} {names[i]:<4s} LIG A   1    "
                f"{xyz[i, 0]:8.3f}{xyz[i, 1]:8.3f}{xyz[i, 2]:8.3f}  1.00  0.00    "
                f"{float(lig.charge[i]):+6.3f} {types[i]:<2s}")

    def fragment(start, seen):
        """Atoms reachable from start without crossing a rotatable bond:
        start first, then the rest in index order."""
        comp, stack = [], [start]
        seen.add(start)
        while stack:
            u = stack.pop()
            comp.append(u)
            for v, k in adj[u]:
                if k not in rot and v not in seen:
                    seen.add(v)
                    stack.append(v)
        return [start] + sorted(c for c in comp if c != start)

    seen = set()

    def branches(comp):
        for i in comp:
            for v, k in sorted(adj[i]):
                if k in rot and v not in seen:
                    a_serial, b_serial = serial[i], len(serial) + 1
                    out.append(f"BRANCH {a_serial:3d} {b_serial:3d}")
                    sub = fragment(v, seen)
                    out.extend(atom_line(j) for j in sub)
                    branches(sub)
                    out.append(f"ENDBRANCH {a_serial:3d} {b_serial:3d}")

    root = int(getattr(lig, "root", 0))
    out.append("ROOT")
    root_comp = fragment(root, seen)
    out.extend(atom_line(i) for i in root_comp)
    out.append("ENDROOT")
    branches(root_comp)
    out.append(f"TORSDOF {len(rot)}")
    if conect:
        for u, v in bonds.tolist():
            out.append(f"CONECT{serial[u]:5d}{serial[v]:5d}")
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
