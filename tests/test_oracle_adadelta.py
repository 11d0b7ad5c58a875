"""Pins for the oracle's ADADELTA local search (Sec. 2.1; Zeiler 2012, Alg. 1).

The update is pinned against a library routine, torch.optim.Adadelta with
lr = 1 (the same algorithm, in float64), both on random gradient sequences and
end-to-end: a one-atom ligand without torsions on grid maps holding linear
fields has a constant translation gradient and zero torque, so the oracle's
trajectory must equal the library optimiser run on that constant gradient.
"""
import numpy as np
import torch

from oracle import dock_ref as R
from paper_2410_10447_amd import synth
from tests.helpers import ligand_from_bonds


def _torch_adadelta(x0, grads, rho, eps):
    p = torch.tensor(x0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adadelta([p], lr=1.0, rho=rho, eps=eps)
    out = []
    for g in grads:
        opt.zero_grad()
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        out.append(p.detach().numpy().copy())
    return out


def test_step_matches_library_on_random_gradients():
    rng = np.random.default_rng(0)
    n, G = 5, 12
    x = rng.normal(size=(n, G))
    x[:, 3:7] /= np.linalg.norm(x[:, 3:7], axis=1, keepdims=True)
    grads = [rng.normal(scale=10.0, size=(n, G)) for _ in range(15)]
    ref = _torch_adadelta(x, grads, 0.8, 1e-2)
    a2 = np.zeros_like(x); d2 = np.zeros_like(x)
    for k, g in enumerate(grads):
        x, a2, d2 = R.adadelta_step(x, g, a2, d2, 0.8, 1e-2)
        # all genes but the quaternion follow the library exactly
        keep = [c for c in range(G) if c not in (3, 4, 5, 6)]
        assert np.abs(x[:, keep] - ref[k][:, keep]).max() < 1e-12
        assert np.abs(np.linalg.norm(x[:, 3:7], axis=1) - 1).max() < 1e-14


def test_one_atom_linear_field_trajectory():
    n = 32
    h = 0.375
    half = (n - 1) * h / 2
    ax = -half + h * np.arange(n)
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    coef = {0: (2.0, -1.0, 3.0), 8: (1.0, 1.0, -2.0), 9: (-1.0, 0.0, 0.5)}
    maps = np.zeros((10, n, n, n), dtype=np.float32)
    for m, (a, b, c) in coef.items():
        maps[m] = (a * X + b * Y + c * Z).astype(np.float32)
        assert np.array_equal(maps[m].astype(np.float64), a * X + b * Y + c * Z)
    grd = synth.Grids(maps=maps, spacing=h, origin=np.array([-half] * 3))
    q = -0.3
    lig = ligand_from_bonds(np.zeros((0, 2), np.int32), [], cls=[0], charge=[q])
    prep = R.prepare(lig, synth.force_field())
    g_const = np.array(coef[0]) + q * np.array(coef[8]) + abs(q) * np.array(coef[9])
    x0 = np.array([[0.3, -0.2, 0.1, 0.6, 0.0, 0.8, 0.0]])
    st = R.ls_init(x0)
    trace = []
    R.local_search(prep, grd, st, 20, rho=0.8, eps=1e-2, trace=trace)
    ref = _torch_adadelta(x0[0, :3], [g_const] * 20, 0.8, 1e-2)
    for k in range(20):
        xt, Et, gt = trace[k]
        assert np.abs(gt[0, :3] - g_const).max() < 1e-12
        assert np.abs(gt[0, 3:7]).max() == 0.0          # zero torque
        assert np.abs(trace[k + 1][0][0, :3] - ref[k]).max() < 1e-12
        assert np.array_equal(trace[k + 1][0][0, 3:7], x0[0, 3:7])
    # energy decreases monotonically along a constant descent direction
    E = [tr[1][0] for tr in trace]
    assert all(E[k + 1] < E[k] for k in range(20))
    assert st.best_energy[0] == min(E)


def test_best_tracking_first_minimum_wins():
    w = synth.ls_workload(8)
    prep = R.prepare(w.ligands[0], w.ff)
    st = R.ls_init(w.genotypes[0])
    trace = []
    R.local_search(prep, w.grids, st, 30, trace=trace)
    Es = np.stack([t[1] for t in trace])           # [31, n]
    xs = np.stack([t[0] for t in trace])
    k = np.argmin(Es, axis=0)                      # argmin returns the first minimum
    assert np.array_equal(st.best_energy, Es[k, np.arange(8)])
    assert np.array_equal(st.best_genotype, xs[k, np.arange(8)])
    assert len(trace) == 31 and np.all(st.iters_done == 30)


def test_chunked_equals_single():
    w = synth.ls_workload(6)
    prep = R.prepare(w.ligands[0], w.ff)
    a = R.ls_init(w.genotypes[0])
    R.local_search(prep, w.grids, a, 30)
    b = R.ls_init(w.genotypes[0])
    for _ in range(2):
        R.local_search(prep, w.grids, b, 10, final_eval=False)
    R.local_search(prep, w.grids, b, 10, final_eval=True)
    for f in ("genotype", "acc_g2", "acc_dx2", "best_genotype", "best_energy", "energy"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
