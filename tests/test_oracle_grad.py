"""Pins for the oracle's analytic gradient with respect to the genotype.

Sec. 2.1: the local search needs the gradient of the score with respect to
the genotype (translation, orientation and torsion genes), built from the
per-atom gradients and the torque. Pinned by central finite differences of the
oracle's own energy on every genotype coordinate (all four quaternion
components and every torsion), and the torque by finite differences along
world-frame rotations of the quaternion. Points where the stencil crosses a
grid-cell face, the box boundary, the 1e5 cap or the r^2 clamp are skipped,
since the score is only piecewise smooth there.
"""
import numpy as np
import pytest

from oracle import dock_ref as R
from paper_2410_10447_amd import synth

FF = synth.force_field()


def _regime(prep, grd, gen):
    """Discrete state that must not change inside an FD stencil."""
    x = R.pose(prep, gen)
    nx, ny, nz = grd.dims
    dims = np.array([nx, ny, nz])
    lo = grd.origin
    hi = lo + (dims - 1) * grd.spacing
    xc = np.clip(x, lo, hi)
    u = (xc - lo) / grd.spacing
    cell = np.clip(np.floor(u), 0, dims - 2)
    out = x != xc
    i, j = prep.pairs[:, 0], prep.pairs[:, 1]
    d = x[:, j] - x[:, i]
    r2 = np.sum(d * d, axis=-1)
    _, _, elj, _, _ = R.pair_energy(r2, prep.r0, prep.eps, prep.pair_hb, prep.qq, prep.dsolv)
    return np.concatenate([cell.reshape(len(gen), -1), out.reshape(len(gen), -1),
                           (elj >= 1e5), (r2 < 1e-4)], axis=1)


def _fd_check(prep, grd, gen, h=1e-6, rel=1e-6):
    res = R.score(prep, grd, gen)
    base = _regime(prep, grd, gen)
    G = gen.shape[1]
    checked = 0
    for c in range(G):
        gp = gen.copy(); gp[:, c] += h
        gm = gen.copy(); gm[:, c] -= h
        ok = np.all(_regime(prep, grd, gp) == base, axis=1) & np.all(_regime(prep, grd, gm) == base, axis=1)
        Ep = R.score(prep, grd, gp).energy
        Em = R.score(prep, grd, gm).energy
        fd = (Ep - Em) / (2 * h)
        scale = np.maximum(np.linalg.norm(res.grad, axis=1), 1.0)
        # FD round-off is about eps_mach |E| / h; allow it on top of `rel`
        tol = rel + 4 * np.finfo(float).eps * np.abs(res.energy) / h / scale
        err = np.abs(fd - res.grad[:, c]) / scale
        assert np.all(err[ok] <= tol[ok]), (c, err[ok].max())
        checked += ok.sum()
    assert checked >= 0.8 * gen.shape[0] * G
    return res


@pytest.mark.parametrize("wl", ["score", "ls"])
def test_genotype_gradient_fd_random_starts(wl):
    w = synth.score_workload(64) if wl == "score" else synth.ls_workload(64)
    prep = R.prepare(w.ligands[0], w.ff)
    gen = w.genotypes[0].astype(np.float64)
    _fd_check(prep, w.grids, gen)


def test_genotype_gradient_fd_relaxed_points():
    """After a few ADADELTA steps: moderate energies, small gradients."""
    w = synth.ls_workload(24)
    prep = R.prepare(w.ligands[0], w.ff)
    st = R.ls_init(w.genotypes[0])
    R.local_search(prep, w.grids, st, 40, final_eval=False)
    _fd_check(prep, w.grids, st.genotype)


def test_genotype_gradient_fd_unnormalised_quaternion():
    w = synth.score_workload(32)
    prep = R.prepare(w.ligands[0], w.ff)
    gen = w.genotypes[0].astype(np.float64)
    gen[:, 3:7] *= np.linspace(0.3, 3.0, 32)[:, None]
    res = _fd_check(prep, w.grids, gen)
    # the quaternion gradient is tangent to the 3-sphere
    dots = np.sum(res.grad[:, 3:7] * gen[:, 3:7], axis=1)
    assert np.abs(dots).max() <= 1e-9 * np.abs(res.grad[:, 3:7]).max()


def test_torque_is_rotation_derivative():
    w = synth.score_workload(16)
    prep = R.prepare(w.ligands[0], w.ff)
    gen = w.genotypes[0].astype(np.float64)
    res = R.score(prep, w.grids, gen)
    h = 1e-6
    base = _regime(prep, w.grids, gen)
    for k in range(3):
        e = np.zeros(4); e[0] = np.cos(h / 2); e[1 + k] = np.sin(h / 2)
        em = e.copy(); em[1 + k] = -em[1 + k]
        gp = gen.copy(); gp[:, 3:7] = R.quat_mul(e[None], gen[:, 3:7])
        gm = gen.copy(); gm[:, 3:7] = R.quat_mul(em[None], gen[:, 3:7])
        ok = np.all(_regime(prep, w.grids, gp) == base, axis=1) & \
            np.all(_regime(prep, w.grids, gm) == base, axis=1)
        fd = (R.score(prep, w.grids, gp).energy - R.score(prep, w.grids, gm).energy) / (2 * h)
        scale = np.maximum(np.linalg.norm(res.torque, axis=1), 1.0)
        tol = 1e-6 + 4 * np.finfo(float).eps * np.abs(res.energy) / h / scale
        assert np.all((np.abs(fd - res.torque[:, k]) / scale)[ok] <= tol[ok])
