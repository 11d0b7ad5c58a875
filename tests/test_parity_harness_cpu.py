"""The GPU parity harness (tests/gpu_common.check) on the CPU: it accepts the
oracle's own energies at FP32 positions, and it rejects energies computed by
an oracle with a planted mistake, so that its conditioning bound cannot pass
a wrong term. The mistakes are planted in the oracle, on the CPU."""
import numpy as np
import pytest

from oracle import dock_ref as R
from paper_2410_10447_amd import synth
from tests.gpu_common import check, oracle_at


@pytest.fixture(scope="module")
def case():
    w = synth.score_workload(256)
    lig = w.ligands[0]
    prep = R.prepare(lig, w.ff)
    gen = np.asarray(w.genotypes[0], np.float32)
    x = R.pose(prep, gen.astype(np.float64))
    # the kernel's per-atom output: positions relative to t, in FP32
    rel = (x - gen[:, None, 0:3].astype(np.float64)).astype(np.float32)
    atom_out = np.zeros((gen.shape[0], prep.n_atoms, 8), np.float32)
    atom_out[:, :, 0:3] = rel
    return w, prep, gen, atom_out


def _energies(prep, grd, gen, atom_out):
    from tests.gpu_common import world_positions
    return oracle_at(prep, grd, gen, world_positions(gen, atom_out)).energy


def test_accepts_the_oracle_itself(case):
    w, prep, gen, ao = case
    E = _energies(prep, w.grids, gen, ao)
    rep = check("harness self", prep, w.grids, gen, E, None, ao)
    assert rep.e_err.max() == 0.0 and not rep.cond.any()


@pytest.mark.parametrize("name,factor", [("DESOLV_SIGMA", 1.01), ("DIEL_K", 1.01), ("K_OUT", 1.5),
                                         ("ELEC_SCALE", 1.01), ("E_CAP", 0.999)])
def test_rejects_a_planted_constant(case, monkeypatch, name, factor):
    """A constant of one term off by 0.1-50 %: every individual whose energy
    it moves by more than ten times the FP32 tolerance falls outside the
    bounds, but for the share the conditioning bound may cover (1 %)."""
    w, prep, gen, ao = case
    if name == "K_OUT":
        # half of the poses moved 8 A along x (the box is 15 A wide): some
        # atoms outside, where the penalty applies
        gen = gen.copy()
        gen[::2, 0] += 8.0
    monkeypatch.setattr(R, name, getattr(R, name) * factor)
    if name == "DIEL_K":
        monkeypatch.setattr(R, "DIEL_B", R.DIEL_EPS0 - R.DIEL_A)
    prep_bad = R.prepare(w.ligands[0], w.ff) if name == "ELEC_SCALE" else prep
    E_bad = _energies(prep_bad, w.grids, gen, ao)
    monkeypatch.undo()
    E_ok = _energies(prep, w.grids, gen, ao)
    rep = check("harness planted " + name, prep, w.grids, gen, E_bad, None, ao, assert_ok=False)
    bad = ~((rep.e_err <= 1e-5) | rep.cond | rep.split)
    moved = np.abs(E_bad - E_ok) > 1e-4 * np.maximum(np.abs(E_ok), 1.0)
    print(f"[harness planted {name}] moved {int(moved.sum())} of {len(moved)}, flagged {int(bad[moved].sum())}")
    assert moved.sum() >= 8, (name, int(moved.sum()))
    assert bad[moved].mean() >= 0.99 - 1.0 / moved.sum(), (name, bad[moved].mean())
    with pytest.raises(AssertionError):
        check("harness planted " + name, prep, w.grids, gen, E_bad, None, ao)
