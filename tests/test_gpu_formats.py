"""Grid maps read from AutoDock .map files score exactly as the same maps
uploaded from memory (the file path only changes where the values come from)."""
import numpy as np
import pytest

from paper_2410_10447_amd import formats, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_maps_from_files_score_bit_identically(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_10447_amd import dock
    grd = synth.grids(41, 10, 501)            # 40 cells per axis: a valid .map size
    lig = synth.ligand(24, 6, 502)
    gen = torch.from_numpy(synth.genotypes(lig, grd, 128, 503)).cuda()
    paths = []
    for k in range(grd.maps.shape[0]):
        p = tmp_path / f"map{k}.map"
        formats.write_map(p, grd.maps[k], grd.spacing, grd.origin)
        paths.append(p)
    stack = formats.load_maps(paths[:-2], paths[-2], paths[-1])
    ff = synth.force_field()
    L = dock.Ligand(lig, ff)
    e_mem, g_mem = dock.score_batch(dock.Grids.from_synth(grd), L, gen)
    e_file, g_file = dock.score_batch(dock.Grids.from_synth(stack), L, gen)
    torch.cuda.synchronize()
    assert torch.equal(e_mem, e_file) and torch.equal(g_mem, g_file)
