"""Pins of the oracle's operation tally (oracle/work.py): the counting
scalars count textbook expressions exactly, the tally runs the same
computation as the float64 oracle (same energy), and its per-stage counts
scale with the sizes that fix them (pairs by kind, atoms)."""
import numpy as np
import pytest

from oracle import dock_ref as R
from oracle import work as W
from paper_2410_10447_amd import synth


def _count(fn):
    st, out = W._measure(fn)
    return st["ops"], st, out


def test_textbook_expressions():
    x = W._counting(np.array([1.5, -2.0, 0.25]))
    # Horner form of a cubic: 3 multiplies, 3 additions per element
    ops, st, _ = _count(lambda: ((2.0 * x + 3.0) * x - 1.0) * x + 0.5)
    assert ops == {"mul": 9, "add": 6, "sub": 3}
    assert st["slots"] == 18 and st["transcendental"] == 0
    # Euclidean norm of a 3-vector: 3 squares, 2 additions, 1 square root
    v = W._counting(np.array([[3.0, 4.0, 12.0]]))
    ops, st, out = _count(lambda: R._norm(v))
    assert ops == {"mul": 3, "add": 2, "sqrt": 1} and st["slots"] == 5 + 4
    assert out[0, 0].v == 13.0
    # a division by a computed value is a transcendental, by a constant not
    ops, st, _ = _count(lambda: 1.0 / x[0] + x[1] / 4.0)
    assert ops == {"div": 1, "divc": 1, "add": 1} and st["slots"] == 4 + 1 + 1
    # constants alone are not counted
    c = W._counting(np.array([2.0, 3.0]), counting=False)
    ops, st, _ = _count(lambda: np.sqrt(c[0] * c[1] + 1.0))
    assert ops == {} and st["slots"] == 0


def test_tally_runs_the_oracles_computation():
    w = synth.ls_workload(3)
    prep = R.prepare(w.ligands[0], w.ff)
    for k in range(3):
        t = W.tally(prep, w.grids, w.genotypes[0][k])
        ref = R.score(prep, w.grids, w.genotypes[0][k:k + 1]).energy[0]
        assert t["energy"] == pytest.approx(ref, rel=1e-12, abs=1e-9)
        assert t["total"]["slots"] == sum(t[s]["slots"] for s in
                                          ("pose", "grid", "pairs", "sums", "gradient", "adadelta"))


def _pair_stage(lig, ff, grd, gen):
    prep = R.prepare(lig, ff)
    return prep, W.tally(prep, grd, gen)["pairs"]["slots"]


def test_pair_and_grid_stages_scale_with_their_sizes():
    """The pair stage costs a fixed amount per van der Waals pair and per
    hydrogen-bond pair (plus the energy sum), the grid stage a fixed amount
    per atom inside the box: a model fitted on two ligands predicts a third."""
    ff = synth.force_field()
    grd = synth.grids(64, 10, 31)
    rows, costs, grid = [], [], []
    for n, t, seed in ((30, 5, 501), (48, 10, 502), (70, 12, 503), (90, 14, 504)):
        lig = synth.ligand(n, t, seed)
        gen = synth.genotypes(lig, grd, 1, seed + 1)[0]
        gen[0:3] = 0.0                      # centred: every atom inside the box
        prep = R.prepare(lig, ff)
        tl = W.tally(prep, grd, gen)
        P, H = prep.pairs.shape[0], int(prep.pair_hb.sum())
        rows.append([P - H, H, 1.0])
        costs.append(tl["pairs"]["slots"])
        grid.append((prep.n_atoms, tl["grid"]["slots"]))
    A = np.array(rows, dtype=np.float64)
    coef, *_ = np.linalg.lstsq(A[:3], np.array(costs[:3], np.float64), rcond=None)
    assert np.allclose(A[3] @ coef, costs[3], rtol=0, atol=1e-6)
    per_atom = {c // n for n, c in grid}
    assert len(per_atom) == 1 and all(c % n == 0 for n, c in grid)
    # an HB pair costs more than a vdW pair (two more powers of s)
    assert coef[1] > coef[0] > 0


def test_model_for_the_benchmark_ligand():
    w = synth.ls_workload(1)
    prep = R.prepare(w.ligands[0], w.ff)
    P, N, T = prep.pairs.shape[0], prep.n_atoms, prep.n_torsions
    assert (P, N, T) == (886, 48, 10)
    assert W.model_slots(P, N, T) == 75 * 886 + 150 * 48 + 80 * 10 + 25 * 17 == 74875
    # the oracle's own formulation takes more work than the model
    assert W.tally(prep, w.grids, w.genotypes[0][0])["total"]["slots"] > W.model_slots(P, N, T)
