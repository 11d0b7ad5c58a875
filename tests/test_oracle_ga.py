"""Pins of the GA generation step reference (oracle/ga_ref.py): special cases
that reduce to a minimum, a maximum or a plain copy, and the defining
properties of two-point crossover and additive mutation, on members whose
gene values name the member and the gene."""
import numpy as np

from oracle import ga_ref as GA


def _population(R, P, G):
    # gene g of member m of run r holds 1000 r + 10 m + g / 64: every value
    # names its run, member and gene, and all are exact in float32
    r, m, g = np.meshgrid(np.arange(R), np.arange(P), np.arange(G), indexing="ij")
    return (1000 * r + 10 * m + g / 64.0).astype(np.float32)


def _member(v, r):
    return int(round((float(v) - 1000 * r) // 10))


def _draws(R, P, G, seed):
    rng = np.random.default_rng(seed)
    cand = rng.integers(0, P, size=(R, P, 4), dtype=np.int32)
    coins = rng.random((R, P, 3), dtype=np.float32)
    cuts = rng.integers(0, G + 1, size=(R, P, 2), dtype=np.int32)
    mut_coin = rng.random((R, P, G), dtype=np.float32)
    mut_delta = (rng.random((R, P, G), dtype=np.float32) - 0.5).astype(np.float32)
    return cand, coins, cuts, mut_coin, mut_delta


def test_tournament_extremes_pick_min_and_max():
    R, P, G = 3, 9, 7
    gen = _population(R, P, G)
    rng = np.random.default_rng(1)
    E = rng.permutation(R * P).reshape(R, P).astype(np.float32)  # distinct energies
    cand, coins, cuts, mc, md = _draws(R, P, G, 2)
    for p_t, pick in ((1.0, min), (0.0, max)):
        out, _ = GA.ga_step(gen, E, cand, coins, cuts, mc, md, p_t, 0.0, 0.0, 0)
        for r in range(R):
            for k in range(P):
                a, b = cand[r, k, 0], cand[r, k, 1]
                want = pick((E[r, a], a), (E[r, b], b))[1]
                assert np.array_equal(out[r, k], gen[r, want])


def test_tournament_tie_takes_first_candidate_and_nan_ranks_last():
    gen = _population(1, 4, 7)
    E = np.array([[np.nan, 2.0, 2.0, 5.0]], dtype=np.float32)
    cand = np.array([[[2, 1, 0, 3]] * 4], dtype=np.int32)
    coins = np.zeros((1, 4, 3), dtype=np.float32)          # tournament draws 0 < p: the fitter wins
    z = np.zeros((1, 4, 7), dtype=np.float32)
    one = np.ones((1, 4, 7), dtype=np.float32)
    out, best = GA.ga_step(gen, E, cand, coins, np.zeros((1, 4, 2), np.int32), one, z, 0.5, 0.0, 0.0, 0)
    assert all(np.array_equal(out[0, k], gen[0, 2]) for k in range(4))   # tie 2.0 vs 2.0: first
    # elitism: the NaN at index 0 is not best; of the equal minima the lower index is
    assert best[0] == 1
    out, _ = GA.ga_step(gen, E, cand, coins, np.zeros((1, 4, 2), np.int32), one, z, 0.5, 0.0, 0.0, 1)
    assert np.array_equal(out[0, 0], gen[0, 1])
    # second tournament: NaN (member 0) against 5.0 (member 3): 5.0 is fitter
    assert GA.tournament(GA.fitness_key(E[0]), 0, 3, 0.0, 0.5) == 3


def test_elitism_copies_the_run_minimum_unchanged():
    R, P, G = 4, 6, 9
    gen = _population(R, P, G)
    rng = np.random.default_rng(3)
    E = rng.normal(size=(R, P)).astype(np.float32)
    cand, coins, cuts, mc, md = _draws(R, P, G, 4)
    out, best = GA.ga_step(gen, E, cand, coins, cuts, np.zeros_like(mc), md, 0.6, 1.0, 1.0, 1)
    for r in range(R):
        assert best[r] == min(range(P), key=lambda m: (E[r, m], m))
        assert np.array_equal(out[r, 0], gen[r, best[r]])        # no crossover, no mutation


def test_two_point_crossover_segment_comes_from_second_parent():
    R, P, G = 2, 12, 13
    gen = _population(R, P, G)
    E = np.zeros((R, P), dtype=np.float32)
    cand, coins, cuts, mc, md = _draws(R, P, G, 5)
    cuts[0, 1] = (4, 4)           # empty segment
    cuts[0, 2] = (9, 2)           # reversed cut points
    cuts[1, 3] = (0, G)           # whole genotype
    out, _ = GA.ga_step(gen, E, cand, coins, cuts, mc, md, 1.0, 1.0, 0.0, 0)
    for r in range(R):
        for k in range(P):
            # equal energies: each tournament returns its first candidate
            p1, p2 = cand[r, k, 0], cand[r, k, 2]
            lo, hi = min(cuts[r, k]), max(cuts[r, k])
            for g in range(G):
                src = p2 if lo <= g < hi else p1
                assert _member(out[r, k, g], r) == src
                assert out[r, k, g] == gen[r, src, g]


def test_mutation_adds_the_displacement_exactly_where_drawn():
    R, P, G = 2, 7, 11
    gen = _population(R, P, G)
    E = np.zeros((R, P), dtype=np.float32)
    cand, coins, cuts, mc, md = _draws(R, P, G, 6)
    out, _ = GA.ga_step(gen, E, cand, coins, cuts, mc, md, 1.0, 0.0, 0.3, 0)
    for r in range(R):
        for k in range(P):
            parent = gen[r, cand[r, k, 0]]
            for g in range(G):
                if mc[r, k, g] < np.float32(0.3):
                    # one float32 rounding of the exact sum
                    exact = float(parent[g]) + float(md[r, k, g])
                    assert out[r, k, g] == np.float32(exact)
                else:
                    assert out[r, k, g] == parent[g]
    # p = 0 changes nothing, p = 1 every gene
    out0, _ = GA.ga_step(gen, E, cand, coins, cuts, mc, md, 1.0, 0.0, 0.0, 0)
    assert np.array_equal(out0, gen[np.arange(R)[:, None], cand[:, :, 0]])
    out1, _ = GA.ga_step(gen, E, cand, coins, cuts, mc, np.ones_like(md), 1.0, 0.0, 1.0, 0)
    assert np.all(out1 == gen[np.arange(R)[:, None], cand[:, :, 0]] + np.float32(1.0))


def test_out_of_range_draws_are_clamped():
    gen = _population(1, 5, 7)
    E = np.arange(5, dtype=np.float32)[None]
    cand = np.array([[[-3, 99, 7, -1]] * 5], dtype=np.int32)
    cuts = np.array([[[-5, 50]] * 5], dtype=np.int32)
    coins = np.zeros((1, 5, 3), dtype=np.float32)
    z = np.zeros((1, 5, 7), dtype=np.float32)
    out, _ = GA.ga_step(gen, E, cand, coins, cuts, np.ones_like(z), z, 1.0, 1.0, 0.0, 0)
    # candidates clamp to (0, 4) and (4, 0): parents 0 and 0; cuts to (0, 7)
    assert all(np.array_equal(out[0, k], gen[0, 0]) for k in range(5))


def test_select_rows_special_cases():
    """Rate 0 selects nothing, rate above every draw selects every row, a
    rate equal to a draw excludes that row (strict comparison), and the
    selection is the set {r : draw_r < rate} in increasing order."""
    from oracle import ga_ref as GR
    d = np.array([0.5, 0.1, 0.9, 0.3, 0.3, 0.0], np.float32)
    assert GR.select_rows(d, 0.0).tolist() == []
    assert GR.select_rows(d, 1.0).tolist() == [0, 1, 2, 3, 4, 5]
    assert GR.select_rows(d, 0.3).tolist() == [1, 5]
    assert GR.select_rows(d, np.nextafter(np.float32(0.3), np.float32(1))).tolist() == [1, 3, 4, 5]
    rng = np.random.default_rng(3)
    x = rng.random(1000).astype(np.float32)
    sel = GR.select_rows(x, 0.25)
    assert np.array_equal(sel, np.flatnonzero(x < np.float32(0.25)))
    assert abs(len(sel) - 250) < 60
    assert GR.select_rows(np.zeros(0, np.float32), 0.5).shape == (0,)
