"""Host-side pieces of the benchmark: the work model against the oracle's,
the roofline object, the traffic figure's source check, and the one-GPU
guard (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from oracle import dock_ref as R  # noqa: E402
from oracle import work as W  # noqa: E402
from paper_2410_10447_amd import synth  # noqa: E402


@pytest.mark.parametrize("n_atoms,n_tors,seed", [(48, 10, None), (24, 6, None), (100, 14, 4100), (7, 0, 11)])
def test_work_model_matches_the_oracles_sizes(n_atoms, n_tors, seed):
    """The benchmark prices an evaluation with the same model as the oracle,
    at the pair, atom and torsion counts of the oracle's preparation."""
    if seed is None:
        w = synth.ls_workload(2) if n_atoms == 48 else synth.score_workload(2)
        lig, ff = w.ligands[0], w.ff
    else:
        lig, ff = synth.ligand(n_atoms, n_tors, seed), synth.force_field()
    prep = R.prepare(lig, ff)
    P, N, T = len(prep.pairs), prep.n_atoms, prep.n_torsions
    assert bench.work_per_eval(P, N, T) == W.model_slots(P, N, T)
    if n_atoms == 48:
        assert bench.work_per_eval(P, N, T) == 74875


def test_roofline_object():
    r = bench.roofline(903000, 2.5e-3, 74875, traffic=3.0e9, kernel="k")
    assert r["bound"] == "alu" and r["unit"] == "Tops/s" and r["kernel"] == "k"
    assert r["achieved"] == pytest.approx(903000 * 74875 / 2.5e-3 / 1e12)
    assert r["peak"] == pytest.approx(78.65) and r["peak_nonpacked"] == pytest.approx(39.325)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.65)
    assert r["frac_nonpacked"] == pytest.approx(2 * r["frac"])
    assert r["traffic"] == 3.0e9


def test_traffic_only_for_the_counted_kernel_sources(monkeypatch):
    """The committed HBM counters apply to the kernel sources they were taken
    on: a different source hash gives no traffic figure."""
    t = dict(bench.TRAFFIC)
    monkeypatch.setattr(bench, "TRAFFIC", dict(t, kernel_sha256=bench.kernel_sha256()))
    got = bench.traffic_bytes()
    assert got == pytest.approx(1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]))
    monkeypatch.setattr(bench, "TRAFFIC", dict(t, kernel_sha256="0" * 64))
    assert bench.traffic_bytes() is None


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stdout
