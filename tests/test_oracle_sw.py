"""Pins of the Solis-Wets reference (oracle/sw_ref.py) on energy functions
whose outcome is known in advance: a constant (every trial fails), a
quadratic bowl seen from a point where the forward or only the reverse trial
improves, and convergence on a bowl."""
import numpy as np

from oracle import sw_ref as SW

F = np.float32


def bowl(c):
    c = np.asarray(c, np.float64)
    return lambda g: np.sum((np.asarray(g, np.float64) - c) ** 2, axis=1)


def test_constant_energy_fails_every_trial_and_contracts():
    n, G = 3, 5
    st = SW.sw_start(np.ones((n, G), F), np.zeros(n))
    st.bias[:] = F(1.0)
    z = np.random.default_rng(0).normal(size=(9, n, G)).astype(F)
    tried = SW.sw_run(lambda g: np.zeros(len(g)), st, z, np.ones(G, F))
    assert np.all(st.x == 1.0)                               # never moved (strictly lower needed)
    assert np.all(st.bias == F(0.5) ** 9)                    # halved at every failure
    assert np.all(st.rho == F(0.25))                         # halved after failures 4 and 8
    assert np.all(st.fail == 1) and np.all(st.succ == 0)
    assert np.all(np.isfinite(tried))                        # both trials made every time


def test_forward_success_moves_and_updates_bias():
    # from 0 towards a minimum at +1 along gene 0, with a positive deviation
    st = SW.sw_start(np.zeros((1, 3), F), bowl([1.0, 0.0, 0.0])(np.zeros((1, 3), F)))
    st.bias[:] = np.array([[0.25, 0.0, 0.0]], F)
    z = np.array([[[0.5, 0.0, 0.0]]], F)
    tried = SW.sw_run(bowl([1.0, 0.0, 0.0]), st, z, np.ones(3, F))
    dev = F(1.0) * (F(1.0) * F(0.5))
    assert st.x[0, 0] == F(F(0.0 + 0.25) + dev)              # x + bias + dev = 0.75
    assert st.bias[0, 0] == F(F(0.2) * F(0.25) + F(0.4) * dev)
    assert st.succ[0] == 1 and st.fail[0] == 0
    assert np.isnan(tried[0, 0, 1])                          # the reverse trial was not needed
    assert st.energy[0] == (0.75 - 1.0) ** 2


def test_reverse_success_when_forward_overshoots():
    # minimum at -1: the forward trial (+0.5) worsens, the reverse one (-0.5) improves
    st = SW.sw_start(np.zeros((1, 2), F), np.array([1.0]))
    z = np.array([[[0.5, 0.0]]], F)
    tried = SW.sw_run(bowl([-1.0, 0.0]), st, z, np.ones(2, F))
    assert tried[0, 0, 0] == (0.5 + 1.0) ** 2 and tried[0, 0, 1] == (-0.5 + 1.0) ** 2
    assert st.x[0, 0] == F(-0.5)
    assert st.bias[0, 0] == F(0.0 - F(0.4) * F(0.5))
    assert st.succ[0] == 1


def test_success_runs_expand_rho():
    # a linear slope: every forward step goes downhill
    st = SW.sw_start(np.zeros((1, 1), F), np.array([0.0]))
    z = np.full((8, 1, 1), 0.1, F)
    SW.sw_run(lambda g: -np.asarray(g, np.float64)[:, 0], st, z, np.ones(1, F))
    assert st.rho[0] == F(4.0) and st.succ[0] == 0          # doubled after successes 4 and 8


def test_converges_on_a_bowl_and_never_rises():
    rng = np.random.default_rng(3)
    n, G = 8, 6
    c = rng.normal(size=G)
    f = bowl(c)
    x0 = rng.normal(size=(n, G)).astype(F) * 3
    st = SW.sw_start(x0, f(x0))
    e_prev = st.energy.copy()
    for _ in range(40):
        SW.sw_run(f, st, rng.normal(size=(10, n, G)).astype(F), np.full(G, 0.3, F))
        assert np.all(st.energy <= e_prev)
        e_prev = st.energy.copy()
    assert np.all(np.abs(st.energy - f(st.x)) <= 1e-12 * np.maximum(1.0, st.energy))
    assert np.all(st.energy < 1e-2), st.energy


def test_decisions_can_follow_supplied_energies():
    # supplied energies that accept every forward trial override a constant energy function
    st = SW.sw_start(np.zeros((2, 3), F), np.array([0.0, 0.0]))
    z = np.ones((3, 2, 3), F)
    dec = np.full((3, 2, 2), np.nan)
    dec[:, :, 0] = -np.arange(1, 4)[:, None]
    SW.sw_run(lambda g: np.zeros(len(g)), st, z, np.ones(3, F), decide_energies=dec)
    assert np.all(st.succ == 3) and np.all(st.energy == -3.0)
