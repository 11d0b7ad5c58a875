"""Serving loop on the GPU: continuous batching across jobs, and each job's
result is the same alone and in the mix (bit for bit: the kernel computes
every individual independently, in a fixed order, and chunked searches equal
unchunked ones)."""
import numpy as np
import pytest

from paper_2410_10447_amd import serve, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    grids = [synth.grids(48, 10, 501), synth.grids(56, 12, 502)]
    ff = synth.force_field()
    ex = serve.GpuExecutor(grids, ff)
    rng = np.random.default_rng(9)
    specs = []
    for k in range(6):
        lig = synth.ligand(int(rng.integers(12, 70)), int(rng.integers(0, 12)), 900 + k)
        gid = k % 2
        gen = synth.genotypes(lig, grids[gid], 300, 950 + k)
        specs.append(serve.JobSpec(job_id=k, ligand=lig, grid_id=gid, genotypes=gen,
                                   arrival=0.002 * k, iterations=60))
    return ex, specs


def test_alone_equals_mixed(setup):
    ex, specs = setup
    srv = serve.Server(ex, max_individuals=100_000, device_budget=1 << 30, chunk_iters=16)
    st = srv.run(specs)
    assert len(st.completed) == len(specs) and not st.failed
    mixed = {r.spec.job_id: r.result for r in st.completed}
    # some launch carried more than one job
    assert st.chunks < sum(-(-s.iterations // 16) for s in specs)
    for s in specs[:3]:
        srv1 = serve.Server(ex, max_individuals=100_000, device_budget=1 << 30, chunk_iters=25)
        one = srv1.run([serve.JobSpec(s.job_id, s.ligand, s.grid_id, s.genotypes, 0.0, s.iterations)])
        r = one.completed[0].result
        assert np.array_equal(r["best_energy"], mixed[s.job_id]["best_energy"])
        assert np.array_equal(r["best_genotype"], mixed[s.job_id]["best_genotype"])
    summ = st.summary()
    print(f"\n[serve] {summ}", flush=True)
    assert summ["p99_s"] >= summ["p50_s"] > 0


def test_cancelled_job_leaves_the_others_unchanged(setup):
    """A long job withdrawn while its chunks run gets no final evaluation and
    no result, its state is released, and every other job's result is bit for
    bit that of a run without it."""
    ex, specs = setup
    base = specs[:3]
    srv0 = serve.Server(ex, max_individuals=100_000, device_budget=1 << 30, chunk_iters=16)
    ref = {r.spec.job_id: r.result for r in srv0.run(base).completed}
    s = specs[3]
    long = serve.JobSpec(s.job_id, s.ligand, s.grid_id, s.genotypes, 0.0, iterations=100_000,
                         cancel_at=0.05)
    srv = serve.Server(ex, max_individuals=100_000, device_budget=1 << 30, chunk_iters=16)
    st = srv.run(list(base) + [long])
    assert [r.spec.job_id for r in st.cancelled] == [s.job_id]
    assert st.cancelled[0].result is None and st.cancelled[0].iters_done < long.iterations
    assert len(st.completed) == 3 and not st.failed
    for r in st.completed:
        assert np.array_equal(r.result["best_energy"], ref[r.spec.job_id]["best_energy"])
        assert np.array_equal(r.result["best_genotype"], ref[r.spec.job_id]["best_genotype"])
    assert srv.used_bytes == 0 and srv.used_individuals == 0
    print(f"\n[serve cancel] job {s.job_id} withdrawn after {st.cancelled[0].iters_done} steps", flush=True)
