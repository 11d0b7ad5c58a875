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
