"""Pins for the oracle's intramolecular pair terms.

Checked against: rigid-body invariance of the internal energy (it cannot
depend on translation or orientation), vanishing net force and net torque of
central pair forces, closed-form minima of the 12-6 and 12-10 terms, the
limits of the Mehler-Solmajer dielectric, a finite difference of each pair
term in r, and an O(N^2) double loop.
"""
import numpy as np

from oracle import dock_ref as R
from paper_2410_10447_amd import synth

FF = synth.force_field()


def _genos(rng, n, T, psi=None):
    t = rng.uniform(-5, 5, (n, 3))
    q = rng.normal(size=(n, 4))
    if psi is None:
        psi = rng.uniform(-np.pi, np.pi, (n, T))
    return np.concatenate([t, q, psi], axis=1)


def test_rigid_body_invariance_and_zero_net_force_torque():
    lig = synth.ligand(48, 10, 1000)
    p = R.prepare(lig, FF)
    rng = np.random.default_rng(0)
    psi = np.repeat(rng.uniform(-np.pi, np.pi, (1, p.n_torsions)), 12, axis=0)
    g = _genos(rng, 12, p.n_torsions, psi)
    x = R.pose(p, g)
    E, gi = R.intra_terms(p, x)
    assert np.abs(E - E[0]).max() <= 1e-9 * max(1.0, abs(E[0]))
    scale = np.abs(gi).max()
    assert np.abs(gi.sum(axis=1)).max() <= 1e-12 * max(1.0, scale) * p.n_atoms
    tau = np.cross(x - g[:, None, 0:3], gi).sum(axis=1)
    assert np.abs(tau).max() <= 1e-11 * max(1.0, scale) * p.n_atoms


def test_closed_form_minima():
    for hb in (False, True):
        r0 = np.array([3.1])
        eps = np.array([0.7])
        e, w, elj, eel, eds = R.pair_energy(r0 ** 2, r0, eps, np.array([hb]),
                                            np.array([0.0]), np.array([0.0]))
        assert np.isclose(elj[0], -0.7, rtol=1e-15)
        assert abs(w[0]) < 1e-14
        # minimum: energy rises on both sides
        for rr in (3.0, 3.2):
            e2, *_ = R.pair_energy(np.array([rr * rr]), r0, eps, np.array([hb]),
                                   np.array([0.0]), np.array([0.0]))
            assert e2[0] > e[0]


def test_dielectric_limits():
    e0, _ = R.dielectric(np.array([0.0]))
    einf, _ = R.dielectric(np.array([1e4]))
    assert abs(e0[0] - 1.3466) < 1e-4       # A + B/(1+k)
    assert abs(einf[0] - 78.4) < 1e-9


def test_pair_energy_derivative_fd():
    rng = np.random.default_rng(3)
    r = rng.uniform(1.5, 9.0, 400)
    r0 = rng.uniform(2.0, 4.2, 400)
    eps = rng.uniform(0.02, 5.0, 400)
    hb = rng.uniform(size=400) < 0.3
    qq = rng.normal(0, 20, 400)
    ds = rng.normal(0, 0.1, 400)
    e, w, *_ = R.pair_energy(r * r, r0, eps, hb, qq, ds)
    ok = e < 1e4                                    # away from the cap
    h = 1e-6
    ep, *_ = R.pair_energy((r + h) ** 2, r0, eps, hb, qq, ds)
    em, *_ = R.pair_energy((r - h) ** 2, r0, eps, hb, qq, ds)
    fd = (ep - em) / (2 * h)
    dedr = w * r
    assert np.all(np.abs(fd - dedr)[ok] <= 1e-6 * np.maximum(1.0, np.abs(dedr[ok])))


def test_cap_and_clamp():
    e, w, elj, *_ = R.pair_energy(np.array([0.5 ** 2, 1e-6]), np.array([4.0, 4.0]),
                                  np.array([0.2, 0.2]), np.array([False, True]),
                                  np.array([1.0, 1.0]), np.array([0.1, 0.1]))
    assert elj[0] == 1e5 and elj[1] == 1e5
    assert w[1] == 0.0                  # r^2 below the clamp: no force
    # capped: only elec + desolvation contribute to w
    _, w_ref, *_ = R.pair_energy(np.array([0.25]), np.array([4.0]), np.array([0.0]),
                                 np.array([False]), np.array([1.0]), np.array([0.1]))
    assert np.isclose(w[0], w_ref[0], rtol=1e-14)


def test_vectorised_matches_double_loop():
    lig = synth.ligand(24, 6, 0)
    p = R.prepare(lig, FF)
    rng = np.random.default_rng(5)
    x = R.pose(p, _genos(rng, 6, p.n_torsions))
    E1, g1 = R.intra_terms(p, x)
    E2, g2 = R.intra_terms_bruteforce(p, x)
    assert np.allclose(E1, E2, rtol=1e-13, atol=1e-9)
    assert np.allclose(g1, g2, rtol=1e-12, atol=1e-9)
