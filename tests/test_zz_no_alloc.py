"""dock_local_search_batch_static (the library-resident workspace) against
dock_local_search_batch (caller workspace): same items, same kernels, so the
results must agree bit for bit. Two calls in a row, the second with fewer
items and individuals, so a stale table or work counter left in the
library's workspace by the first call would show."""
import numpy as np
import pytest

from paper_2410_10447_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_10447_amd import dock
    dock.lib()
    return dock


def _jobs(dk, spec, grids, ff):
    """spec: (atoms, torsions, seed, individuals, threads_per_ind, variant[, two per wave])."""
    jobs = []
    for n_atoms, n_tors, seed, n, tpi, var, *two in spec:
        lig = synth.ligand(n_atoms, n_tors, seed)
        L = dk.Ligand(lig, ff)
        gen = synth.genotypes(lig, grids[1], n, seed + 1)
        st = dk.LSState.start(torch.from_numpy(gen).cuda())
        jobs.append(dk.LsJob(grids[0], L, st, var, threads_per_ind=tpi, two_per_wave=bool(two and two[0])))
    return jobs


def _twin(dk, jobs):
    return [dk.LsJob(j.grids, j.ligand, j.state.clone(), j.variant, threads_per_ind=j.threads_per_ind,
                     two_per_wave=j.two_per_wave)
            for j in jobs]


def _assert_same(a_jobs, b_jobs):
    for k, (a, b) in enumerate(zip(a_jobs, b_jobs)):
        an, bn = a.state.to_numpy(), b.state.to_numpy()
        for f in an:
            assert np.array_equal(an[f], bn[f], equal_nan=True), (k, f)


def test_static_workspace_equals_caller_workspace(dk):
    grd = synth.grids(48, 10, 9001)
    G = dk.Grids.from_synth(grd)
    ff = synth.force_field()
    # first call: all five kernel families (one-slot, two-slot one-wave,
    # two-wave, four-wave, two individuals per wave) and two variants, so the
    # call has five parts
    spec1 = [(48, 10, 9100, 96, 64, 0), (100, 14, 9200, 40, 64, 1), (90, 12, 9300, 33, 128, 0),
             (20, 3, 9400, 70, 64, 1), (70, 9, 9600, 21, 256, 1), (24, 5, 9700, 31, 64, 0, True)]
    jobs_s = _jobs(dk, spec1, (G, grd), ff)
    jobs_r = _twin(dk, jobs_s)
    print(f"\n[no-alloc] call 1: {len(spec1)} items, {sum(s[3] for s in spec1)} individuals, 25 iterations",
          flush=True)
    dk.local_search_static(jobs_s, 25, final_eval=False)
    dk.local_search(jobs_r, 25, final_eval=False)
    torch.cuda.synchronize()
    _assert_same(jobs_s, jobs_r)
    # second call: fewer items and individuals, continuing the first two
    # items' states, plus a fresh small item; final evaluation on
    spec2 = [(30, 5, 9500, 17, 64, 0)]
    new_s = _jobs(dk, spec2, (G, grd), ff)
    new_r = _twin(dk, new_s)
    sub_s = [jobs_s[1], new_s[0]]
    sub_r = [jobs_r[1], new_r[0]]
    print("[no-alloc] call 2: 2 items, 57 individuals, 10 iterations + final evaluation", flush=True)
    dk.local_search_static(sub_s, 10, final_eval=True)
    dk.local_search(sub_r, 10, final_eval=True)
    torch.cuda.synchronize()
    _assert_same(sub_s, sub_r)
    _assert_same(jobs_s, jobs_r)          # untouched items stay equal too
    s = sub_s[0].state.to_numpy()
    assert np.all(s["iters_done"] == 35) and np.all(np.isfinite(s["best_energy"]))
    s = sub_s[1].state.to_numpy()
    assert np.all(s["iters_done"] == 10) and np.all(np.isfinite(s["energy"]))


def test_static_workspace_rejects_too_many_items(dk):
    grd = synth.grids(40, 10, 9011)
    G = dk.Grids.from_synth(grd)
    jobs = _jobs(dk, [(24, 6, 9600, 2, 64, 0)], (G, grd), synth.force_field())
    many = jobs * (dk.STATIC_MAX_ITEMS + 1)
    before = jobs[0].state.clone()
    with pytest.raises(dk.DockError):
        dk.local_search_static(many, 5)
    torch.cuda.synchronize()
    after = jobs[0].state.to_numpy()
    for f, v in before.to_numpy().items():
        assert np.array_equal(v, after[f], equal_nan=True), f
