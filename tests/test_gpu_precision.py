"""Per-variant precision report of the block sum (the paper's Sec. 4.2 and
its error table, Sec. 5.1): for every reduction variant, the per-individual
error of E and of the genotype gradient against the FP64 oracle (evaluated at
the kernel's own atom positions), at random starting poses and at the best
points of 300-step searches, for the 48-atom, 10-torsion benchmark ligand.
The table is printed; the bounds are those of tests/gpu_common.check (FP32
tolerances; the 2-term BF16 split also by its own 2^-16 bound)."""
import numpy as np
import pytest

from oracle import dock_ref as R
from paper_2410_10447_amd import synth
from tests.gpu_common import check, gpu_points

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

VARIANTS = [0, 1, 2, 3, 4]
N_POINTS = 2000


@pytest.fixture(scope="module")
def dk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_10447_amd import dock
    dock.lib()
    return dock


def _q(a, p):
    return float(np.quantile(a, p)) if len(a) else 0.0


def test_precision_report_all_variants(dk):
    w = synth.ls_workload(3000)
    lig = w.ligands[0]
    G = dk.Grids.from_synth(w.grids)
    L = dk.Ligand(lig, w.ff)
    prep = R.prepare(lig, w.ff)
    starts = w.genotypes[0][:N_POINTS]
    st = dk.LSState.start(torch.from_numpy(w.genotypes[0]).cuda())
    dk.local_search([(G, L, st)], 300, variant=0, final_eval=True)
    torch.cuda.synchronize()
    ends = st.best_genotype.cpu().numpy()[:N_POINTS]
    names = {0: "shuffle FP32", 1: "MFMA FP32", 2: "MFMA BF16 2-term", 3: "MFMA FP16 2-term",
             4: "MFMA BF16 3-term"}
    rows = []
    for v in VARIANTS:
        for where, gens in (("random starts", starts), ("300-step best points", ends)):
            E, g, ao = gpu_points(dk, G, L, gens, v)
            # the 2-term BF16 split is held to its own 2^-16 bound (counted,
            # not capped): its error, not the conditioning, exceeds 1e-5 there
            rep = check(f"precision v{v} {where}", prep, w.grids, gens, E, g, ao, variant=v,
                        cond_cap=1.0 if v == 2 else 0.01)
            rows.append((names[v], where, rep))
    print("\n| variant | points | n | E err p50 | E err p99 | E err max | E > 1e-5 (conditioning) | "
          "g err p50 | g err p99 | g err max | g > 1e-4 (at a kink) |")
    print("|---|---|---|---|---|---|---|---|---|---|---|")
    for name, where, r in rows:
        print(f"| {name} | {where} | {r.n} | {_q(r.e_err, 0.5):.2e} | {_q(r.e_err, 0.99):.2e} | "
              f"{r.e_err.max():.2e} | {int((r.e_err > 1e-5).sum())} ({int(r.cond.sum())}) | {_q(r.g_err, 0.5):.2e} | "
              f"{_q(r.g_err, 0.99):.2e} | {r.g_err.max():.2e} | {int((r.g_err > 1e-4).sum())} "
              f"({int(((r.g_err > 1e-4) & r.kink).sum())}) |", flush=True)
    # the FP32 variants and the 3-term split meet the E bound at every point
    # but the conditioning exceptions (capped inside check)
    for name, where, r in rows:
        if name in (names[0], names[1], names[4]):
            assert np.all((r.e_err <= 1e-5) | r.cond), (name, where)
