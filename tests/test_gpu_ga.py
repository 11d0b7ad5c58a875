"""GPU parity of the GA generation step (dock_ga_step) against the reference
step: bit-exact, since every random number is an input and the step's only
arithmetic is one float32 addition per mutated gene. Shapes span several
256-thread blocks with a ragged tail, one member per run, the longest
genotype, and the docking job the benchmark runs (20 runs x 150 members, 17
genes)."""
import numpy as np
import pytest

from oracle import ga_ref as GA

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_10447_amd import dock
    dock.lib()
    return dock


def _inputs(R, P, G, seed, energy_kind="normal"):
    rng = np.random.default_rng(seed)
    gen = rng.normal(size=(R, P, G)).astype(np.float32)
    if energy_kind == "normal":
        E = rng.normal(size=(R, P)).astype(np.float32)
    elif energy_kind == "ties":
        E = rng.integers(-2, 3, size=(R, P)).astype(np.float32)   # many equal energies
    else:                                                          # NaN and inf sprinkled in
        E = rng.normal(size=(R, P)).astype(np.float32)
        E[rng.random((R, P)) < 0.2] = np.nan
        E[rng.random((R, P)) < 0.1] = np.inf
    cand = rng.integers(0, P, size=(R, P, 4), dtype=np.int32)
    coins = rng.random((R, P, 3), dtype=np.float32)
    cuts = rng.integers(0, G + 1, size=(R, P, 2), dtype=np.int32)
    mut_coin = rng.random((R, P, G), dtype=np.float32)
    mut_delta = ((rng.random((R, P, G), dtype=np.float32) - 0.5) * 3.0).astype(np.float32)
    return gen, E, cand, coins, cuts, mut_coin, mut_delta


def _run(dk, arrays, p_t, p_c, p_m, elitism):
    dev = [torch.from_numpy(a).cuda() for a in arrays]
    children, best = dk.ga_step(*dev, p_t, p_c, p_m, elitism)
    torch.cuda.synchronize()
    return children.cpu().numpy(), best.cpu().numpy()


@pytest.mark.parametrize("shape", [(3, 7, 7), (2, 33, 17), (1, 1, 39), (5, 61, 13), (20, 150, 17)])
@pytest.mark.parametrize("elitism", [0, 1])
def test_ga_step_bit_exact(dk, shape, elitism):
    R, P, G = shape
    arrays = _inputs(R, P, G, seed=R * 1000 + P * 10 + G)
    print(f"ga_step shape={shape} elitism={elitism}", flush=True)
    got, best = _run(dk, arrays, 0.6, 0.8, 0.02, elitism)
    want, want_best = GA.ga_step(*arrays, 0.6, 0.8, 0.02, elitism)
    assert np.array_equal(best, want_best)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("kind", ["ties", "nonfinite"])
@pytest.mark.parametrize("probs", [(0.6, 0.8, 0.02), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0)])
def test_ga_step_ties_nonfinite_and_extreme_rates(dk, kind, probs):
    R, P, G = 4, 50, 17
    arrays = _inputs(R, P, G, seed=7 if kind == "ties" else 8, energy_kind=kind)
    print(f"ga_step kind={kind} probs={probs}", flush=True)
    got, best = _run(dk, arrays, *probs, 1)
    want, want_best = GA.ga_step(*arrays, *probs, 1)
    assert np.array_equal(best, want_best)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_ga_step_clamps_out_of_range_draws(dk):
    R, P, G = 2, 9, 11
    gen, E, cand, coins, cuts, mc, md = _inputs(R, P, G, seed=9)
    cand[0, :, 0] = -5
    cand[1, :, 1] = P + 3
    cuts[0, :, 0] = -2
    cuts[1, :, 1] = G + 9
    arrays = (gen, E, cand, coins, cuts, mc, md)
    got, best = _run(dk, arrays, 0.6, 0.9, 0.1, 0)
    want, want_best = GA.ga_step(*arrays, 0.6, 0.9, 0.1, 0)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_ga_step_twice_then_smaller(dk):
    """Two calls in a row reuse nothing from each other: the second, smaller
    call matches the reference on its own inputs."""
    for shape, seed in (((6, 100, 17), 11), ((2, 5, 9), 12)):
        arrays = _inputs(*shape, seed=seed)
        got, best = _run(dk, arrays, 0.6, 0.8, 0.05, 1)
        want, want_best = GA.ga_step(*arrays, 0.6, 0.8, 0.05, 1)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
        assert np.array_equal(best, want_best)


def test_ga_step_rejects_bad_arguments(dk):
    R, P, G = 2, 4, 7
    dev = [torch.from_numpy(a).cuda() for a in _inputs(R, P, G, seed=13)]
    with pytest.raises(dk.DockError):
        dk.ga_step(*dev, float("nan"), 0.8, 0.02, 1)
    with pytest.raises(dk.DockError):        # children overlapping the parents
        dk.ga_step(*dev, 0.6, 0.8, 0.02, 1, children=dev[0])


def test_lga_generation_keeps_the_elite(dk):
    """One generation of the LGA on the device (GA step, scoring, local
    search): with elitism, child 0 of each run is the run's best genotype, so
    its score equals the parent's, and after the local search (which keeps
    each individual's best point) no run's best energy has risen."""
    from paper_2410_10447_amd import synth
    wl = synth.ls_workload(600)
    grids = dk.Grids.from_synth(wl.grids)
    lig = dk.Ligand(wl.ligands[0], wl.ff)
    R, P = 4, 150
    G = lig.n_genes
    gen0 = torch.from_numpy(np.asarray(wl.genotypes[0], np.float32)[: R * P]).cuda()
    E0, _ = dk.score_batch(grids, lig, gen0)
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    draws = dk.ga_draws(R, P, G, g, "cuda")
    children, best = dk.ga_step(gen0.view(R, P, G), E0.view(R, P), *draws, 0.6, 0.8, 0.02, True)
    E1, _ = dk.score_batch(grids, lig, children.view(R * P, G))
    torch.cuda.synchronize()
    b = best.cpu().numpy()
    e0 = E0.view(R, P).cpu().numpy()
    e1 = E1.view(R, P).cpu().numpy()
    assert np.array_equal(e1[:, 0], e0[np.arange(R), b])
    assert np.array_equal(children[:, 0].cpu().numpy(),
                          gen0.view(R, P, G)[torch.arange(R, device="cuda"), best.long()].cpu().numpy())
    st = dk.LSState.start(children.view(R * P, G))
    dk.local_search([(grids, lig, st)], iterations=30)
    torch.cuda.synchronize()
    e2 = st.best_energy.view(R, P).cpu().numpy()
    m0 = e0.min(axis=1)
    # the search's first point is the elite itself, evaluated by the same
    # FP32 code; the bound allows only rounding
    assert np.all(e2.min(axis=1) <= m0 + 1e-5 * np.maximum(np.abs(m0), 1.0))


def test_lga_job_budget_monotone_and_oracle_checked(dk):
    """A small docking job (3 runs x 40 members, 20 search iterations): the
    per-run best energy never rises from generation to generation (elitism
    plus a search that keeps its start point), the evaluation budget stops
    the job before a generation that would exceed it, and the reported best
    genotypes score, under the FP64 reference, to the reported energies."""
    from oracle import dock_ref as R
    from paper_2410_10447_amd import lga, synth
    from tests.gpu_common import check_reported
    wl = synth.ls_workload(120)
    grids = dk.Grids.from_synth(wl.grids)
    lig = dk.Ligand(wl.ligands[0], wl.ff)
    gen0 = torch.from_numpy(np.asarray(wl.genotypes[0], np.float32)).cuda()
    n, its = gen0.shape[0], 20
    budget = 3 * n * (its + 1) + n            # initial search + 2 generations fit, a third does not
    res = lga.run_lga(grids, lig, gen0, n_runs=3, generations=5, ls_iterations=its,
                      eval_budget=budget, seed=3)
    assert res.generations == 2 and res.evaluations == 3 * n * (its + 1)
    h = np.stack(res.history)
    assert h.shape == (3, 3)
    assert np.all(np.diff(h, axis=0) <= 0), h
    prep = R.prepare(wl.ligands[0], wl.ff)
    check_reported("lga job best points", dk, grids, lig, prep, wl.grids, res.best_genotype,
                   res.best_energy)


def test_lga_job_early_stop(dk):
    """The convergence rule ends the job: with a tolerance no improvement can
    exceed, the job stops after `patience` generations."""
    from paper_2410_10447_amd import lga, synth
    wl = synth.ls_workload(60)
    grids = dk.Grids.from_synth(wl.grids)
    lig = dk.Ligand(wl.ligands[0], wl.ff)
    gen0 = torch.from_numpy(np.asarray(wl.genotypes[0], np.float32)).cuda()
    res = lga.run_lga(grids, lig, gen0, n_runs=2, generations=6, ls_iterations=10,
                      stop_patience=2, stop_tol=1e9, seed=4)
    assert res.stopped_early and res.generations == 2 and len(res.history) == 3
    res = lga.run_lga(grids, lig, gen0, n_runs=2, generations=3, ls_iterations=10,
                      stop_patience=2, stop_tol=-1.0, seed=4)     # never converged
    assert not res.stopped_early and res.generations == 3


@pytest.mark.parametrize("n,rate", [(0, 0.5), (1, 0.5), (7, 0.0), (1000, 1.0), (1023, 0.3), (1025, 0.3),
                                    (7500, 0.06), (20000, 0.5)])
def test_select_gather_scatter_bit_exact(dk, n, rate):
    """Rows selected for the local search (draw < rate, increasing order)
    against the reference selection, then a gather of those rows and a
    scatter of modified rows back: both exact copies."""
    from oracle import ga_ref as GR
    rng = np.random.default_rng(n + int(rate * 100))
    draws = rng.random(n).astype(np.float32)
    if n > 10:
        draws[5] = np.float32(rate)            # equal to the rate: not selected
    want = GR.select_rows(draws, rate)
    idx, cnt = dk.select_rows(torch.from_numpy(draws).cuda(), rate)
    torch.cuda.synchronize()
    m = int(cnt.item())
    assert m == len(want)
    assert np.array_equal(idx.cpu().numpy()[:m], want)
    G = 17
    pop = rng.normal(size=(n, G)).astype(np.float32)
    sub = dk.gather_rows(torch.from_numpy(pop).cuda(), idx, m)
    torch.cuda.synchronize()
    assert np.array_equal(sub.cpu().numpy(), pop[want])
    new = (sub * 2.0 + 1.0).contiguous()
    dst = torch.from_numpy(pop).cuda()
    dk.scatter_rows(new, idx, dst)
    e = torch.from_numpy(rng.normal(size=n).astype(np.float32)).cuda()
    e_new = torch.arange(m, dtype=torch.float32, device="cuda")
    e_ref = e.cpu().numpy().copy()
    dk.scatter_rows(e_new, idx, e)
    torch.cuda.synchronize()
    ref = pop.copy()
    ref[want] = pop[want] * np.float32(2.0) + np.float32(1.0)
    e_ref[want] = np.arange(m, dtype=np.float32)
    assert np.array_equal(dst.cpu().numpy(), ref)
    assert np.array_equal(e.cpu().numpy(), e_ref)


def test_lga_job_partial_local_search_rate(dk):
    """A docking job that searches only the children whose draw is below the
    local-search rate (0.3): every phase searches the selected share, the
    evaluation count is the scoring of every member plus the searches, the
    unsearched members keep their scores, per-run best energies never rise,
    and the reported best points meet the oracle."""
    from oracle import dock_ref as R
    from paper_2410_10447_amd import lga, synth
    from tests.gpu_common import check_reported
    wl = synth.ls_workload(200)
    grids = dk.Grids.from_synth(wl.grids)
    lig = dk.Ligand(wl.ligands[0], wl.ff)
    gen0 = torch.from_numpy(np.asarray(wl.genotypes[0], np.float32)).cuda()
    n, its = gen0.shape[0], 20
    res = lga.run_lga(grids, lig, gen0, n_runs=4, generations=3, ls_iterations=its, seed=11, ls_rate=0.3)
    assert res.generations == 3 and len(res.searched) == 4
    assert all(0 < m < n for m in res.searched)
    assert abs(np.mean(res.searched) - 0.3 * n) < 0.1 * n
    assert res.evaluations == sum(n + m * (its + 1) for m in res.searched)
    h = np.stack(res.history)
    assert np.all(np.diff(h, axis=0) <= 0), h
    prep = R.prepare(wl.ligands[0], wl.ff)
    check_reported("lga job at rate 0.3, best points", dk, grids, lig, prep, wl.grids, res.best_genotype,
                   res.best_energy)
    # the same seed gives the same job, bit for bit
    res2 = lga.run_lga(grids, lig, gen0, n_runs=4, generations=3, ls_iterations=its, seed=11, ls_rate=0.3)
    assert res2.searched == res.searched
    assert np.array_equal(res2.best_energy, res.best_energy)
    assert np.array_equal(res2.best_genotype, res.best_genotype)
