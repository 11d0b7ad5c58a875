"""Serving loop logic on a simulated device (no GPU): continuous batching,
admission by footprint, FIFO, per-job step accounting, failure handling,
cancellation."""
import numpy as np
import pytest

from paper_2410_10447_amd import serve


def _spec(i, n, arrival, iters=300, genes=17):
    g = np.full((n, genes), float(i), np.float32)
    return serve.JobSpec(job_id=i, ligand=None, grid_id=0, genotypes=g, arrival=arrival,
                         iterations=iters)


def _run(specs, **kw):
    ex = serve.FakeExecutor(sec_per_eval=kw.pop("spe", 1e-8), fail_on=kw.pop("fail_on", None))
    srv = serve.Server(ex, clock=ex.clock, **kw)
    st = srv.run(specs, poll=1e-3)
    return ex, srv, st


def test_every_job_gets_its_steps_and_one_final_eval():
    specs = [_spec(i, 100 + 10 * i, arrival=0.01 * i) for i in range(12)]
    ex, srv, st = _run(specs, max_individuals=10_000, device_budget=1 << 30, chunk_iters=50)
    assert len(st.completed) == 12 and not st.failed
    per_job = {}
    for chunk in ex.launched:
        for jid, k, fin in chunk:
            assert 1 <= k <= 50
            d = per_job.setdefault(jid, [0, 0])
            assert d[1] == 0, "steps after the final evaluation"
            d[0] += k
            d[1] += int(fin)
    assert all(v == [300, 1] for v in per_job.values())
    assert st.evals == sum(s.genotypes.shape[0] * 301 for s in specs)
    for r in st.completed:
        assert r.result["iters"] == 300 and r.result["final"]
        assert r.done >= r.admitted >= r.spec.arrival


def test_continuous_batching_mixes_jobs_at_different_progress():
    specs = [_spec(0, 500, 0.0), _spec(1, 500, 0.0005), _spec(2, 500, 0.002)]
    ex, srv, st = _run(specs, max_individuals=10_000, device_budget=1 << 30, chunk_iters=20,
                       spe=1e-7)
    # some launch carries job 0 and a job that joined later, with different remaining work
    progress = {0: 0, 1: 0, 2: 0}
    mixed = False
    for chunk in ex.launched:
        ids = [j for j, _, _ in chunk]
        if len(ids) > 1 and len({progress[j] for j in ids}) > 1:
            mixed = True
        for j, k, _ in chunk:
            progress[j] += k
    assert mixed
    assert len(st.completed) == 3


def test_admission_by_footprint_and_fifo():
    specs = [_spec(i, 1000, 0.0) for i in range(6)]
    fp = serve.state_bytes(1000, 17)
    ex, srv, st = _run(specs, max_individuals=10_000, device_budget=2 * fp, chunk_iters=100)
    assert st.peak_device_bytes <= 2 * fp
    # never more than two jobs in one launch
    assert max(len(c) for c in ex.launched) <= 2
    admitted = [r.spec.job_id for r in sorted(st.completed, key=lambda r: r.admitted)]
    assert admitted == sorted(admitted)
    assert [r.spec.job_id for r in st.completed] == list(range(6))


def test_individual_cap_blocks_queue_head():
    specs = [_spec(0, 900, 0.0), _spec(1, 900, 0.0), _spec(2, 50, 0.0)]
    ex, srv, st = _run(specs, max_individuals=1000, device_budget=1 << 30, chunk_iters=300)
    first = ex.launched[0]
    assert [j for j, _, _ in first] == [0]           # FIFO: job 2 waits behind job 1
    assert len(st.completed) == 3


def test_job_that_can_never_fit_is_rejected():
    ex = serve.FakeExecutor()
    srv = serve.Server(ex, max_individuals=100, device_budget=1 << 30, clock=ex.clock)
    with pytest.raises(ValueError):
        srv.submit(_spec(0, 1000, 0.0))


def test_injected_launch_failure_fails_only_its_jobs():
    specs = [_spec(0, 100, 0.0), _spec(1, 100, 0.5), _spec(2, 100, 1.0)]
    ex, srv, st = _run(specs, max_individuals=10_000, device_budget=1 << 30, chunk_iters=50,
                       fail_on={1})
    assert [r.spec.job_id for r in st.failed] == [1]
    assert sorted(r.spec.job_id for r in st.completed) == [0, 2]
    assert srv.used_bytes == 0 and srv.used_individuals == 0


def test_stalled_chunk_times_out():
    class Stall(serve.FakeExecutor):
        def launch(self, plan, max_iters):
            tok = super().launch(plan, max_iters)
            if any(h["spec"].job_id == 7 for h, _, _ in plan):
                return float("inf")
            return tok

        def wait(self, token, poll):
            self.t += 0.05 if token == float("inf") else max(0.0, token - self.t)

    ex = Stall()
    srv = serve.Server(ex, max_individuals=10_000, device_budget=1 << 30, chunk_iters=300,
                       clock=ex.clock, chunk_timeout=1.0, depth=1)
    st = srv.run([_spec(7, 10, 0.0)], poll=1e-3)
    assert [r.spec.job_id for r in st.failed] == [7]
    assert "timed out" in st.failed[0].error


def test_poisson_arrivals_rate():
    t = serve.poisson_arrivals(20.0, 100.0, seed=4)
    assert abs(len(t) / 100.0 - 20.0) < 2.0
    assert all(0 <= a < 100 for a in t) and t == sorted(t)


def test_latency_percentiles_under_load():
    arr = serve.poisson_arrivals(20.0, 5.0, seed=1)
    specs = [_spec(i, 750, a) for i, a in enumerate(arr)]
    ex, srv, st = _run(specs, max_individuals=30_000, device_budget=1 << 30, chunk_iters=50,
                       spe=2e-9)
    s = st.summary()
    assert s["jobs"] == len(specs)
    assert 0 < s["p50_s"] <= s["p99_s"]
    assert s["evals_per_s"] > 0


def test_lazy_starting_points_and_progress_reports():
    """A job may carry a function that draws its starting points when it is
    admitted; the result equals the job with the array given up front, and
    the progress callback fires on the server clock."""
    drawn = []

    def lazy(i, n):
        def draw():
            drawn.append(i)
            return np.full((n, 17), float(i), np.float32)
        return draw

    eager = [_spec(i, 50 + 5 * i, arrival=0.02 * i) for i in range(6)]
    lazy_specs = [serve.JobSpec(job_id=s.job_id, ligand=None, grid_id=0,
                                genotypes=lazy(s.job_id, s.count), arrival=s.arrival,
                                iterations=s.iterations, n=s.count) for s in eager]
    assert all(l.count == e.count for l, e in zip(lazy_specs, eager))
    _, _, st_e = _run(eager, max_individuals=10_000, device_budget=1 << 30, chunk_iters=50)
    ex = serve.FakeExecutor(sec_per_eval=1e-6)
    srv = serve.Server(ex, clock=ex.clock, max_individuals=10_000, device_budget=1 << 30,
                       chunk_iters=50)
    reports = []
    st_l = srv.run(lazy_specs, poll=1e-3, progress=lambda now, s: reports.append(now),
                   progress_every=0.05)
    assert sorted(drawn) == list(range(6)) or set(drawn) == set(range(6))
    res_e = {r.spec.job_id: r.result["value"] for r in st_e.completed}
    res_l = {r.spec.job_id: r.result["value"] for r in st_l.completed}
    assert res_e == res_l
    assert st_l.evals == st_e.evals
    assert reports and all(b > a for a, b in zip(reports, reports[1:]))


def test_cancel_queued_job_never_runs():
    """A job withdrawn while it waits for admission leaves the queue; the job
    behind it moves up."""
    fp = serve.state_bytes(1000, 17)
    specs = [_spec(0, 1000, 0.0), _spec(1, 1000, 0.0), _spec(2, 1000, 0.0)]
    specs[1].cancel_at = 1e-6
    ex, srv, st = _run(specs, max_individuals=10_000, device_budget=fp, chunk_iters=100)
    assert [r.spec.job_id for r in st.cancelled] == [1]
    assert st.cancelled[0].result is None and st.cancelled[0].error == "cancelled"
    assert all(j != 1 for c in ex.launched for j, _, _ in c)
    assert sorted(r.spec.job_id for r in st.completed) == [0, 2]
    assert srv.used_bytes == 0 and srv.used_individuals == 0
    assert st.summary()["cancelled"] == 1


def test_cancel_admitted_job_stops_at_a_chunk_boundary():
    """A job withdrawn in flight gets no further chunk and no final
    evaluation; its state is released once no enqueued chunk carries it, and
    the other jobs' results are those of a run without it."""
    kw = dict(max_individuals=10_000, device_budget=1 << 30, chunk_iters=50, spe=1e-7)
    _, _, ref = _run([_spec(0, 500, 0.0), _spec(2, 500, 0.0)], **kw)
    specs = [_spec(0, 500, 0.0), _spec(1, 500, 0.0), _spec(2, 500, 0.0)]
    specs[1].cancel_at = 0.01          # chunks of the three jobs take 7.5 ms each
    ex, srv, st = _run(specs, **kw)
    steps = sum(k for c in ex.launched for j, k, _ in c if j == 1)
    assert 0 < steps < 300
    assert not any(fin for c in ex.launched for j, _, fin in c if j == 1)
    assert [r.spec.job_id for r in st.cancelled] == [1] and st.cancelled[0].result is None
    assert 1 not in ex.live and srv.used_bytes == 0 and srv.used_individuals == 0
    assert sorted(r.spec.job_id for r in st.completed) == [0, 2]
    want = {r.spec.job_id: r.result for r in ref.completed}
    assert {r.spec.job_id: r.result for r in st.completed} == want


def test_cancel_of_unknown_or_finished_job_is_refused():
    ex = serve.FakeExecutor()
    srv = serve.Server(ex, max_individuals=10_000, device_budget=1 << 30, clock=ex.clock)
    assert not srv.cancel(5)
    st = srv.run([_spec(0, 10, 0.0, iters=20)], poll=1e-3)
    assert len(st.completed) == 1
    assert not srv.cancel(0) and not st.cancelled
