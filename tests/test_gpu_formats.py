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


@pytest.mark.parametrize("name", ["pyridine_ethanol.pdbqt", "biphenyl.pdbqt", "ring_synth"])
def test_ring_ligands_score_and_search_parity(name):
    """Ligands with rings (read from PDBQT, or generated with planar rings):
    scoring parity with the FP64 oracle at the kernel's own positions, and a
    20-step search whose best points meet the oracle."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import os
    from oracle import dock_ref as R
    from paper_2410_10447_amd import dock
    from tests.gpu_common import check, check_reported, gpu_points
    if name == "ring_synth":
        lig = synth.ring_ligand(4, 24, 12, 931)
    else:
        lig = formats.read_pdbqt(os.path.join(os.path.dirname(__file__), "golden", name))
    grd = synth.grids(48, 10, 932)
    ff = synth.force_field()
    gen = synth.genotypes(lig, grd, 256, 933)
    G = dock.Grids.from_synth(grd)
    L = dock.Ligand(lig, ff)
    prep = R.prepare(lig, ff)
    for v in (0, 1):
        E, g, ao = gpu_points(dock, G, L, gen, v)
        check(f"{name} score v{v}", prep, grd, gen, E, g, ao, variant=v)
    st = dock.LSState.start(torch.from_numpy(gen).cuda())
    dock.local_search([(G, L, st)], 20)
    torch.cuda.synchronize()
    s = st.to_numpy()
    check_reported(f"{name} search best points", dock, G, L, prep, grd, s["best_genotype"], s["best_energy"])
