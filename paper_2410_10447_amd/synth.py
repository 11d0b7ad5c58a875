"""Seeded synthetic inputs for the docking hot path.

This module only draws random numbers and lays them out; it contains none of
the scoring function's arithmetic (no pose construction, interpolation, pair
terms or optimiser). Both the HIP path and the FP64 oracle consume the arrays it
returns, so the two sides see bit-identical inputs.

The paper's complexes (Sec. 5) and their AutoDock grid maps are not available,
so every workload is a synthetic stand-in with the shapes of the paper's
problem (Sec. 2.1: a ligand with N_rot rotatable bonds against fixed receptor
grids):

* ligand: a random tree of atoms with 1.5 A bonds, 8 atom classes, Gaussian
  partial charges, rotatable bonds picked among internal bonds; or a ligand
  with planar rings (ring_ligand) joined by single bonds;
* force-field table: per-class radius, well depth, solvation and volume, and
  a donor x acceptor hydrogen-bond table (synthetic ranges, seed 7);
* grids: one map per atom type plus an electrostatic and a desolvation map,
  each a clipped sum of 32 Gaussians on a cubic lattice of spacing 0.375 A;
* genotypes: translation in the box, uniform random unit quaternion,
  torsions uniform in [-pi, pi].
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

N_CLASSES = 8
DONOR_CLASSES = (6, 7)
ACCEPTOR_CLASSES = (3, 4)
BOND_LENGTH = 1.5
MIN_NONBONDED = 2.0
GRID_SPACING = 0.375
GRID_CLIP = (-2.0, 1.0e5)
FF_SEED = 7


@dataclass
class Ligand:
    """Raw ligand description, as a caller would hand it over."""
    xyz: np.ndarray        # float64 [N, 3], reference conformation (A)
    charge: np.ndarray     # float64 [N], partial charges (e)
    cls: np.ndarray        # int32 [N], atom class in [0, 8)
    bonds: np.ndarray      # int32 [n_bonds, 2]: tree edges (parent, child), plus ring bonds
    rot_bonds: np.ndarray  # int32 [T], indices into `bonds`
    root: int = 0
    seed: int = 0
    n_torsions_requested: int = 0

    @property
    def n_atoms(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_torsions(self) -> int:
        return int(self.rot_bonds.shape[0])

    @property
    def n_genes(self) -> int:
        return 7 + self.n_torsions


@dataclass
class ForceField:
    """Per-class parameters (synthetic, seeded) and the H-bond table."""
    radius: np.ndarray     # float64 [C], vdW radius R (A)
    eps: np.ndarray        # float64 [C], well depth (kcal/mol)
    solv: np.ndarray       # float64 [C], atomic solvation parameter s
    vol: np.ndarray        # float64 [C], atomic volume V (A^3)
    hb_r0: np.ndarray      # float64 [2, 2], [donor 6/7][acceptor 3/4] (A)
    hb_eps: np.ndarray     # float64 [2, 2] (kcal/mol)
    donors: tuple = DONOR_CLASSES
    acceptors: tuple = ACCEPTOR_CLASSES


@dataclass
class Grids:
    """Receptor grid maps, planar layout [n_maps][nz][ny][nx], x fastest."""
    maps: np.ndarray       # float32 [M, nz, ny, nx]
    spacing: float
    origin: np.ndarray     # float64 [3], coordinate of node (0,0,0), (x,y,z)
    seed: int = 0

    @property
    def n_maps(self) -> int:
        return int(self.maps.shape[0])

    @property
    def dims(self) -> tuple:
        """(nx, ny, nz)"""
        return (int(self.maps.shape[3]), int(self.maps.shape[2]), int(self.maps.shape[1]))


def force_field(seed: int = FF_SEED, n_classes: int = N_CLASSES) -> ForceField:
    rng = np.random.default_rng(seed)
    radius = rng.uniform(1.0, 2.1, n_classes)
    eps = rng.uniform(0.02, 0.25, n_classes)
    solv = rng.uniform(-0.003, 0.001, n_classes)
    vol = rng.uniform(0.0, 35.0, n_classes)
    hb_r0 = rng.uniform(1.8, 2.0, (2, 2))
    hb_eps = rng.uniform(1.0, 5.0, (2, 2))
    return ForceField(radius, eps, solv, vol, hb_r0, hb_eps)


def _unit_vectors(rng, k):
    v = rng.normal(size=(k, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def ligand(n_atoms: int, n_torsions: int, seed: int) -> Ligand:
    """Random connected tree with 1.5 A bonds.

    Each new atom picks a parent uniformly among atoms of degree < 4 and a
    direction uniformly on the sphere; the draw is repeated (up to 100 times
    per atom) until the new atom is at least 2.0 A from every atom other than
    its parent. The structure is then centred on its centroid. Rotatable bonds
    are drawn without replacement among internal bonds (both ends of degree
    >= 2); when fewer exist than requested, all internal bonds are used.
    """
    if n_atoms < 1:
        raise ValueError("n_atoms must be >= 1")
    rng = np.random.default_rng(seed)
    xyz = np.zeros((n_atoms, 3))
    degree = np.zeros(n_atoms, dtype=np.int64)
    bonds = []
    for i in range(1, n_atoms):
        placed = False
        for _ in range(100):
            cand = np.nonzero(degree[:i] < 4)[0]
            parent = int(cand[rng.integers(len(cand))])
            pos = xyz[parent] + BOND_LENGTH * _unit_vectors(rng, 1)[0]
            d = np.linalg.norm(xyz[:i] - pos, axis=1)
            d[parent] = np.inf
            if i == 1 or d.min() >= MIN_NONBONDED:
                placed = True
                break
        if not placed:
            raise RuntimeError(f"could not place atom {i} (seed {seed})")
        xyz[i] = pos
        degree[parent] += 1
        degree[i] += 1
        bonds.append((parent, i))
    xyz -= xyz.mean(axis=0)
    bonds = np.array(bonds, dtype=np.int32).reshape(-1, 2)
    internal = [b for b, (u, v) in enumerate(bonds) if degree[u] >= 2 and degree[v] >= 2]
    t_eff = min(n_torsions, len(internal))
    if t_eff > 0:
        rot = np.sort(rng.choice(np.array(internal), size=t_eff, replace=False)).astype(np.int32)
    else:
        rot = np.zeros(0, dtype=np.int32)
    cls = rng.integers(0, N_CLASSES, n_atoms).astype(np.int32)
    charge = rng.normal(0.0, 0.2, n_atoms)
    return Ligand(xyz=xyz, charge=charge, cls=cls, bonds=bonds, rot_bonds=rot,
                  root=0, seed=seed, n_torsions_requested=n_torsions)


RING_BOND = 1.4


def ring_ligand(n_rings: int, n_chain: int, n_torsions: int, seed: int, ring_size: int = 6) -> Ligand:
    """Ligand of planar rings (regular polygons with 1.4 A edges) and chain
    atoms, joined by 1.5 A single bonds into a connected graph whose rings
    stay inside rigid fragments.

    Units (a ring or one chain atom, in a seeded random order) are attached
    one at a time by a single bond to an atom with a free valence (ring atoms
    take one substituent, chain atoms up to four bonds): from a ring atom the
    bond points away from its ring's centre in the ring plane, from a chain
    atom in a uniform direction; a new ring lies in a random plane containing
    the bond, its attaching atom on the bond. A placement is redrawn (up to
    200 times) until every new atom is at least 2.0 A from every existing
    atom except the one it bonds to. Rotatable bonds are drawn among the
    single bonds between units with both ends bonded elsewhere (never a ring
    bond). The structure is centred on its centroid; classes and charges as
    in `ligand`.
    """
    if n_rings < 0 or n_chain < 0 or n_rings + n_chain < 1 or ring_size < 3:
        raise ValueError("need at least one unit and rings of >= 3 atoms")
    rng = np.random.default_rng(seed)
    units = np.array([1] * n_rings + [0] * n_chain)
    units = units[rng.permutation(len(units))]
    R = RING_BOND / (2.0 * np.sin(np.pi / ring_size))        # circumradius
    xyz, bonds, degree, ring_of, centre = [], [], [], [], []
    single = []                                              # inter-unit bonds

    def ring_atoms(p0, direction, normal):
        w = np.cross(normal, direction)
        c = p0 + R * direction
        th = 2.0 * np.pi * np.arange(ring_size) / ring_size
        return c, c[None, :] + R * (np.cos(th)[:, None] * (-direction)[None, :] + np.sin(th)[:, None] * w[None, :])

    for k, is_ring in enumerate(units):
        if k == 0:
            if is_ring:
                d0 = _unit_vectors(rng, 1)[0]
                n0 = np.cross(d0, _unit_vectors(rng, 1)[0])
                c, pts = ring_atoms(np.zeros(3), d0, n0 / np.linalg.norm(n0))
            else:
                c, pts = None, np.zeros((1, 3))
            base = 0
        else:
            placed = False
            for _ in range(200):
                cand = [i for i in range(len(xyz)) if degree[i] < (3 if ring_of[i] >= 0 else 4)]
                a = int(cand[rng.integers(len(cand))])
                if ring_of[a] >= 0:
                    d = xyz[a] - centre[ring_of[a]]
                    d /= np.linalg.norm(d)
                else:
                    d = _unit_vectors(rng, 1)[0]
                p0 = xyz[a] + BOND_LENGTH * d
                if is_ring:
                    nrm = np.cross(d, _unit_vectors(rng, 1)[0])
                    c, pts = ring_atoms(p0, d, nrm / np.linalg.norm(nrm))
                else:
                    c, pts = None, p0[None, :]
                old = np.asarray(xyz)
                dist = np.linalg.norm(old[None, :, :] - pts[:, None, :], axis=2)
                dist[0, a] = np.inf                         # the new bond
                if dist.min() >= MIN_NONBONDED:
                    placed = True
                    break
            if not placed:
                raise RuntimeError(f"could not place unit {k} (seed {seed})")
            base = len(xyz)
            single.append(len(bonds))
            bonds.append((a, base))
            degree[a] += 1
        r_id = len(centre) if is_ring else -1
        if is_ring:
            centre.append(c)
        for i, pt in enumerate(pts):
            xyz.append(pt)
            degree.append(1 if k > 0 and i == 0 else 0)
            ring_of.append(r_id)
        if is_ring:
            for i in range(ring_size):
                bonds.append((base + i, base + (i + 1) % ring_size))
                degree[base + i] += 1
                degree[base + (i + 1) % ring_size] += 1
    xyz = np.asarray(xyz, dtype=np.float64)
    xyz -= xyz.mean(axis=0)
    n_atoms = xyz.shape[0]
    bonds = np.array(bonds, dtype=np.int32).reshape(-1, 2)
    internal = [b for b in single if degree[bonds[b, 0]] >= 2 and degree[bonds[b, 1]] >= 2]
    t_eff = min(n_torsions, len(internal))
    if t_eff > 0:
        rot = np.sort(rng.choice(np.array(internal), size=t_eff, replace=False)).astype(np.int32)
    else:
        rot = np.zeros(0, dtype=np.int32)
    cls = rng.integers(0, N_CLASSES, n_atoms).astype(np.int32)
    charge = rng.normal(0.0, 0.2, n_atoms)
    return Ligand(xyz=xyz, charge=charge, cls=cls, bonds=bonds, rot_bonds=rot,
                  root=0, seed=seed, n_torsions_requested=n_torsions)


def grids(n: int, n_maps: int, seed: int, spacing: float = GRID_SPACING,
          n_gauss: int = 32, n_walls: int = 4) -> Grids:
    """Cubic grid of n^3 nodes, box centred on the origin.

    Each map is a sum of 32 Gaussians with centres uniform in the box. The
    atom-type maps (all but the last two) mix 28 smooth ones (amplitude
    U[-4, 4], width U[1, 3] A) with 4 steep repulsive "walls" (amplitude
    10^U[3, 5.5], width U[0.5, 1] A) that reach the 1e5 clip; the
    electrostatic and desolvation maps (the last two) are scaled by the atom
    charge and its magnitude, so they hold only smooth Gaussians (a wall there
    would become a bottomless well for one sign of charge). Node values are
    clipped to [-2, 1e5] and stored as float32.
    """
    rng = np.random.default_rng(seed)
    half = (n - 1) * spacing / 2.0
    origin = np.array([-half, -half, -half])
    ax = origin[0] + spacing * np.arange(n)
    maps = np.zeros((n_maps, n, n, n), dtype=np.float64)
    for m in range(n_maps):
        walls = n_walls if m < n_maps - 2 else 0
        smooth = n_gauss - walls
        centres = rng.uniform(-half, half, (n_gauss, 3))
        amp = np.concatenate([rng.uniform(-4.0, 4.0, smooth),
                              10.0 ** rng.uniform(3.0, 5.5, walls)])
        sig = np.concatenate([rng.uniform(1.0, 3.0, smooth),
                              rng.uniform(0.5, 1.0, walls)])
        acc = np.zeros((n, n, n))
        for g in range(n_gauss):
            s2 = 2.0 * sig[g] ** 2
            ex = np.exp(-(ax - centres[g, 0]) ** 2 / s2)
            ey = np.exp(-(ax - centres[g, 1]) ** 2 / s2)
            ez = np.exp(-(ax - centres[g, 2]) ** 2 / s2)
            acc += amp[g] * ez[:, None, None] * ey[None, :, None] * ex[None, None, :]
        maps[m] = acc
    maps = np.clip(maps, GRID_CLIP[0], GRID_CLIP[1]).astype(np.float32)
    return Grids(maps=maps, spacing=spacing, origin=origin, seed=seed)


def ligand_radius(lig: Ligand) -> float:
    """Largest distance of a reference atom from the reference centroid."""
    c = lig.xyz - lig.xyz.mean(axis=0)
    return float(np.linalg.norm(c, axis=1).max()) if lig.n_atoms else 0.0


def genotypes(lig: Ligand, grd: Grids, n: int, seed: int) -> np.ndarray:
    """Random starting genotypes, float32 [n, 7 + T].

    Layout (tx, ty, tz, qw, qx, qy, qz, psi_1..psi_T). The translation is
    uniform in the cube of half-width max(0, L/2 - R_lig), with L the box edge
    and R_lig the ligand radius, so the reference conformation starts inside
    the box; q is a normalised 4-D Gaussian (uniform on SO(3)); torsions are
    uniform in [-pi, pi].
    """
    rng = np.random.default_rng(seed)
    nx, ny, nz = grd.dims
    L = (min(nx, ny, nz) - 1) * grd.spacing
    hw = max(0.0, L / 2.0 - ligand_radius(lig))
    t = rng.uniform(-hw, hw, (n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    psi = rng.uniform(-np.pi, np.pi, (n, lig.n_torsions))
    g = np.concatenate([t, q, psi], axis=1)
    return g.astype(np.float32)


# ---------------------------------------------------------------------------
# Named workloads (seeds: ligand 1000c, grids 1000c+1, genotypes 1000c+2).
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    ligands: list
    grids: Grids
    ff: ForceField
    genotypes: list            # one float32 [n_i, G_i] array per ligand
    iterations: int = 0
    rho: float = 0.8
    eps: float = 1e-2
    meta: dict = field(default_factory=dict)


def score_workload(n_genotypes: int = 256) -> Workload:
    """Single 24-atom, 6-torsion ligand on 40^3 x 10 maps; random genotypes."""
    c = 0
    lig = ligand(24, 6, 1000 * c)
    grd = grids(40, 10, 1000 * c + 1)
    g = genotypes(lig, grd, n_genotypes, 1000 * c + 2)
    return Workload("score_n24_t6_g40", [lig], grd, force_field(), [g])


def ls_workload(n_individuals: int = 3000, iterations: int = 300) -> Workload:
    """One 48-atom, 10-torsion ligand on 64^3 x 10 maps, 3000 individuals."""
    c = 1
    lig = ligand(48, 10, 1000 * c)
    grd = grids(64, 10, 1000 * c + 1)
    g = genotypes(lig, grd, n_individuals, 1000 * c + 2)
    return Workload("ls_n48_t10_g64_i3000", [lig], grd, force_field(), [g],
                    iterations=iterations)


def uneven_workload(n_ligands: int = 64, per_ligand: int = 100, iterations: int = 300,
                    grid_n: int = 96) -> Workload:
    """64 ligands, atoms U{12..128}, torsions U{0..32}, on one 96^3 x 12 set."""
    c = 3
    rng = np.random.default_rng(1000 * c)
    sizes = rng.integers(12, 129, n_ligands)
    tors = rng.integers(0, 33, n_ligands)
    seeds = rng.integers(0, 2**31 - 1, n_ligands)
    grd = grids(grid_n, 12, 1000 * c + 1)
    ligs, gens = [], []
    for k in range(n_ligands):
        lig = ligand(int(sizes[k]), int(tors[k]), int(seeds[k]))
        ligs.append(lig)
        gens.append(genotypes(lig, grd, per_ligand, int(seeds[k]) + 2))
    return Workload(f"uneven_l{n_ligands}_i{per_ligand}_g{grid_n}", ligs, grd,
                    force_field(), gens, iterations=iterations)


def digest(*arrays) -> str:
    """SHA-256 over the raw bytes of the given arrays (shape and dtype included)."""
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()
