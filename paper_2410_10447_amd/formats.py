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
