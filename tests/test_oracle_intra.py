"""Pins for the oracle's intramolecular pair terms.

Checked against: rigid-body invariance of the internal energy (it cannot
depend on translation or orientation), vanishing net force and net torque of
central pair forces, closed-form minima of the 12-6 and 12-10 terms, the
limits of the Mehler-Solmajer dielectric, a finite difference of each pair
term in r, an O(N^2) double loop, and closed-form values of the
electrostatic and desolvation terms (Gaussian half-width, Coulomb asymptotes
of r * E_el, a hand-set ligand whose desolvation weight and energy are
computed by hand).
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


# ---------------------------------------------------------------------------
# Closed-form value pins of the electrostatic and desolvation terms. Each
# fails if the corresponding formula of the oracle is perturbed (a sigma^2
# in place of 2 sigma^2, another sigma, r^2 in the Coulomb denominator,
# another dielectric plateau, the charge term of the solvation parameter
# dropped or on the wrong atom).
# ---------------------------------------------------------------------------

def _terms(r, qq=0.0, dsolv=0.0):
    """Pair terms at distances r with the 12-6/12-10 term switched off."""
    r = np.asarray(r, dtype=np.float64)
    n = r.shape[0]
    return R.pair_energy(r * r, np.full(n, 2.0), np.zeros(n), np.zeros(n, bool),
                         np.full(n, qq), np.full(n, dsolv))


def test_desolvation_gaussian_closed_forms():
    # Gaussian exp(-r^2 / (2 sigma^2)) with sigma = 3.5 A at unit weight:
    # 1 at the origin, 1/2 at the half-width r = sigma sqrt(2 ln 2),
    # exp(-1/2) at r = sigma, exp(-2) at r = 2 sigma
    sigma = 3.5
    r = np.array([0.01, sigma * np.sqrt(2.0 * np.log(2.0)), sigma, 2.0 * sigma])
    e, w, elj, eel, eds = _terms(r, dsolv=1.0)
    assert np.all(elj == 0.0) and np.all(eel == 0.0)
    assert abs(eds[0] - 1.0) < 1e-5                 # r^2 = 1e-4: 1 - 4.1e-6
    assert abs(eds[1] - 0.5) < 1e-15
    assert abs(eds[2] - np.exp(-0.5)) < 1e-15
    assert abs(eds[3] - np.exp(-2.0)) < 1e-15
    # slope of the Gaussian: d/dr = -r / sigma^2 * value, so w = -value / sigma^2
    assert np.allclose(w, -eds / sigma ** 2, rtol=1e-14, atol=0)
    # the weight scales the term linearly
    _, _, _, _, eds3 = _terms(r, dsolv=-3.0)
    assert np.allclose(eds3, -3.0 * eds, rtol=1e-15)


def test_coulomb_dielectric_asymptotes():
    # E_el = qq / (r eps(r)): r E_el -> qq / 78.4 far away (eps0 = 78.4) and
    # -> qq / 1.3466 near contact (eps(0) = A + B / (1 + k)); the slope of
    # eps at 0 is about 2.77 per A, so at r = 0.01 A r E_el lies within 2.1 %
    # below qq / 1.3466
    qq = 41.5
    e, w, elj, eel, eds = _terms(np.array([1.0e4, 0.01]), qq=qq)
    assert np.all(eds == 0.0)
    assert abs(eel[0] * 1.0e4 - qq / 78.4) < 1e-12 * qq
    near = eel[1] * 0.01
    assert qq / 1.3466 * 0.979 < near <= qq / 1.3466 * (1 + 1e-4)
    # far away the force is that of a plain Coulomb law in a medium of 78.4:
    # dE/dr = -qq / (78.4 r^2), so w = dE/dr / r = -qq / (78.4 r^3)
    assert abs(w[0] - (-qq / (78.4 * 1.0e12))) < 1e-9 * qq / (78.4 * 1.0e12)
    # the energy is odd in the charge product
    _, _, _, eel_neg, _ = _terms(np.array([1.0e4, 0.01]), qq=-qq)
    assert np.array_equal(eel_neg, -eel)


def _chain5(cls, charge):
    """Five atoms on a straight line, 1.5 A apart (0-1-2-3-4), bonds 1-2 and
    2-3 rotatable: the only listed pair is (0, 4), 6 A apart."""
    from paper_2410_10447_amd import synth
    xyz = np.array([[1.5 * k, 0.0, 0.0] for k in range(5)])
    bonds = np.array([[0, 1], [1, 2], [2, 3], [3, 4]], np.int32)
    return synth.Ligand(xyz=xyz, charge=np.asarray(charge, float), cls=np.asarray(cls, np.int32),
                        bonds=bonds, rot_bonds=np.array([1, 2], np.int32))


def _ff_hand():
    """Hand-set parameters: every well depth zero (no 12-6 / 12-10 term)."""
    from paper_2410_10447_amd import synth
    ff = synth.force_field()
    solv = np.array([-0.002, 0.001, 0.0005, -0.001, 0.0, 0.0, 0.0, 0.0])
    vol = np.array([10.0, 20.0, 15.0, 5.0, 0.0, 0.0, 0.0, 0.0])
    return synth.ForceField(radius=ff.radius, eps=np.zeros(8), solv=solv, vol=vol,
                            hb_r0=ff.hb_r0, hb_eps=np.zeros((2, 2)))


def test_desolvation_weight_hand_set_ligand():
    # atom 0: class 0 (s = -0.002, V = 10), q = +0.5;
    # atom 4: class 1 (s = 0.001, V = 20), q = -0.25.
    # S_0 = -0.002 + 0.01097 * 0.5 = 0.003485, S_4 = 0.001 + 0.01097 * 0.25
    # = 0.0037425; weight S_0 V_4 + S_4 V_0 = 0.0697 + 0.037425 = 0.107125
    lig = _chain5([0, 2, 2, 2, 1], [0.5, 0.0, 0.0, 0.0, -0.25])
    p = R.prepare(lig, _ff_hand())
    assert p.pairs.tolist() == [[0, 4]]
    assert abs(p.dsolv[0] - 0.107125) < 1e-15
    assert abs(p.qq[0] - 332.06363 * -0.125) < 1e-12
    # swapping the two atoms' charges changes the weight (the charge term
    # belongs to the atom's own S, multiplied by the partner's volume):
    # S_0 = -0.002 + 0.0027425 = 0.0007425, S_4 = 0.001 + 0.005485 = 0.006485;
    # 0.0007425 * 20 + 0.006485 * 10 = 0.01485 + 0.06485 = 0.0797
    p2 = R.prepare(_chain5([0, 2, 2, 2, 1], [-0.25, 0.0, 0.0, 0.0, 0.5]), _ff_hand())
    assert abs(p2.dsolv[0] - 0.0797) < 1e-15


def test_desolvation_energy_of_hand_set_ligand():
    # neutral atoms 6 A apart at weight 0.107125 - 0.01097 * 0.5 * 20
    # - 0.01097 * 0.25 * 10 = -0.002 * 20 + 0.001 * 10 = -0.03: the internal
    # energy is -0.03 exp(-36 / 24.5) and does not depend on the pose
    lig = _chain5([0, 2, 2, 2, 1], [0.0] * 5)
    p = R.prepare(lig, _ff_hand())
    assert abs(p.dsolv[0] - (-0.03)) < 1e-17
    x = R.pose(p, np.array([[0.3, -0.2, 0.1, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0],
                            [1.0, 2.0, 3.0, 0.5, 0.5, -0.5, 0.5, 0.0, 0.0]]))
    E, g = R.intra_terms(p, x)
    assert np.allclose(E, -0.03 * np.exp(-36.0 / 24.5), rtol=1e-13, atol=0)
    # for a negative weight dE/dr = -|c| (-r / s^2) exp(...) > 0: the gradient
    # on atom 4 points away from atom 0 (the force, its negative, attracts)
    d = x[:, 4] - x[:, 0]
    assert np.all(np.sum(g[:, 4] * d, axis=-1) > 0)
