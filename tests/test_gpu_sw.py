"""GPU parity of the Solis-Wets search (dock_solis_wets_batch) against the
reference (oracle/sw_ref.py).

The accept decisions compare energies, so both sides take them in the
kernel's precision: the reference replays the search with the kernel's logged
float32 trial energies as its decisions, and
* every logged energy must match the FP64 score of its trial point at the
  kernel's positions of it (the scoring tolerances of the FP32 path),
* the trial pattern (second trial made or not) must be identical,
* the final state (genotypes, bias, rho, run counters) must be bit-exact,
  since every state update is float32 arithmetic in a fixed order.
"""
import numpy as np
import pytest

from oracle import dock_ref as R
from oracle import sw_ref as SW
from paper_2410_10447_amd import synth
from tests.gpu_common import check_reported

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_10447_amd import dock
    dock.lib()
    return dock


def _setup(dk, lig, grid, ff, gen0):
    G = dk.Grids.from_synth(grid)
    L = dk.Ligand(lig, ff)
    g = torch.from_numpy(np.ascontiguousarray(gen0, np.float32)).cuda()
    E0, _ = dk.score_batch(G, L, g)
    return G, L, g, E0


def _replay_check(dk, lig, grid, ff, gen0, iters, variant, seed):
    G, L, g, E0 = _setup(dk, lig, grid, ff, gen0)
    n, Gn = g.shape
    rng = np.random.default_rng(seed)
    normals = rng.normal(size=(iters, n, Gn)).astype(np.float32)
    scale = SW.gene_scale(Gn)
    st = dk.SWState.start(g, E0)
    log = dk.solis_wets(G, L, st, torch.from_numpy(normals).cuda(),
                        torch.from_numpy(scale).cuda(), variant=variant, log=True)
    torch.cuda.synchronize()
    log = log.cpu().numpy()                                 # [n, iters, 2]
    prep = R.prepare(lig, ff)
    results = []

    def energy_fn(c):
        r = R.score(prep, grid, np.asarray(c, np.float64))
        results.append((np.asarray(c, np.float32).copy(), r))
        return r.energy

    ref = SW.sw_start(np.asarray(gen0, np.float32), E0.cpu().numpy().astype(np.float64))
    tried = SW.sw_run(energy_fn, ref, normals, scale, decide_energies=log.transpose(1, 0, 2))
    glog = log.transpose(1, 0, 2)                           # [iters, n, 2]
    assert np.array_equal(np.isnan(glog), np.isnan(tried)), "trial patterns differ"
    # logged energies against the FP64 score of the same trial points, at the
    # kernel's positions of them (from a scoring evaluation: the pose code is
    # shared; the energy-only evaluation sums the pair energies per lane)
    pts, es = [], []
    for it in range(iters):
        for t in range(2):
            c, r = results[2 * it + t]
            m = ~np.isnan(glog[it, :, t])
            pts.append(c[m])
            es.append(glog[it, m, t])
    check_reported(f"sw trials N={lig.n_atoms} v{variant}", dk, G, L, prep, grid, np.concatenate(pts),
                   np.concatenate(es), variant=variant, exact_rescore=False)
    st_np = {k: getattr(st, k).cpu().numpy() for k in ("genotype", "energy", "bias", "rho", "counts")}
    assert np.array_equal(st_np["genotype"].view(np.uint32), ref.x.view(np.uint32))
    assert np.array_equal(st_np["bias"].view(np.uint32), ref.bias.view(np.uint32))
    assert np.array_equal(st_np["rho"], ref.rho)
    assert np.array_equal(st_np["counts"][:, 0], ref.succ) and np.array_equal(st_np["counts"][:, 1], ref.fail)
    assert np.array_equal(st_np["energy"], ref.energy.astype(np.float32))
    assert np.all(st_np["energy"] <= E0.cpu().numpy())
    return st_np


@pytest.mark.parametrize("variant", [0, 1])
def test_sw_replay_parity_benchmark_ligand(dk, variant):
    w = synth.ls_workload(48)
    print(f"sw replay 48 atoms variant={variant}", flush=True)
    _replay_check(dk, w.ligands[0], w.grids, w.ff, w.genotypes[0], iters=12, variant=variant, seed=5)


def test_sw_replay_parity_two_slot_ligand(dk):
    ff = synth.force_field()
    lig = synth.ligand(90, 12, 77)
    grd = synth.grids(40, 10, 78)
    gen = synth.genotypes(lig, grd, 16, 79)
    print("sw replay 90 atoms", flush=True)
    _replay_check(dk, lig, grd, ff, gen, iters=6, variant=0, seed=6)


def test_sw_chunked_equals_single(dk):
    w = synth.ls_workload(64)
    G, L, g, E0 = _setup(dk, w.ligands[0], w.grids, w.ff, w.genotypes[0])
    n, Gn = g.shape
    normals = torch.from_numpy(np.random.default_rng(8).normal(size=(20, n, Gn)).astype(np.float32)).cuda()
    scale = torch.from_numpy(SW.gene_scale(Gn)).cuda()
    a = dk.SWState.start(g, E0)
    dk.solis_wets(G, L, a, normals, scale)
    b = dk.SWState.start(g, E0)
    dk.solis_wets(G, L, b, normals[:7], scale)
    dk.solis_wets(G, L, b, normals[7:], scale)
    torch.cuda.synchronize()
    for k in ("genotype", "energy", "bias", "rho", "counts"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    assert torch.all(a.energy <= E0)
