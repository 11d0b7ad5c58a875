"""Reference of one generation step of the genetic algorithm of the LGA.

TEST INFRASTRUCTURE ONLY: only tests, the smoke check and the benchmark's
CPU-baseline leg may use this module. Nothing here is shared with the HIP
path.

What the paper fixes and what is read into it
---------------------------------------------
Sec. 2.1 fixes only the structure: the Lamarckian GA alternates a genetic
global search, which produces new genotypes, with a local search that improves
each of them; a docking job holds many independent LGA runs. The paper names
no operator. The operators below are the standard ones of the AutoDock LGA
(Morris et al. 1998), stated as readings:

* elitism: with `elitism` set, child 0 of every run is an unchanged copy of
  the run's best genotype (lowest energy; among equal energies the lowest
  index; a NaN energy ranks as +inf);
* selection: every other child takes two parents, each chosen by a binary
  tournament between two candidate members: the fitter one (lower energy,
  the first candidate on a tie, NaN as +inf) wins when the tournament draw is
  below `p_tournament`, else the other one;
* crossover: when the crossover draw is below `p_crossover`, two-point
  crossover: genes [lo, hi) come from the second parent, with lo and hi the
  smaller and larger of the two cut draws; otherwise the child copies the
  first parent;
* mutation: gene g of a child changes when its mutation draw is below
  `p_mutation`, by adding its displacement draw (one float32 addition).

Every random number is an input (drawn by the caller): candidate indices
(clamped to [0, pop - 1]), three uniform draws per child (two tournaments, the
crossover), two cut points (clamped to [0, n_genes]), and per gene a uniform
draw and a displacement. Decisions compare float32 values with float32
thresholds and the only arithmetic is the float32 addition of the mutation,
so the result is exact: a correct implementation reproduces it bit for bit.
"""
from __future__ import annotations

import numpy as np


def fitness_key(energies):
    """Energies as the selection compares them: NaN ranks as +inf."""
    e = np.asarray(energies, dtype=np.float32)
    return np.where(np.isnan(e), np.float32(np.inf), e)


def run_best(energies):
    """Index of each run's best member: the first index of the minimal key
    (energies (R, P))."""
    return np.argmin(fitness_key(energies), axis=1).astype(np.int32)


def tournament(key, a, b, u, p_tournament):
    """Binary tournament between members a and b of one run."""
    better, worse = (a, b) if key[a] <= key[b] else (b, a)
    return better if np.float32(u) < np.float32(p_tournament) else worse


def ga_step(genotypes, energies, cand, coins, cuts, mut_coin, mut_delta,
            p_tournament, p_crossover, p_mutation, elitism):
    """One generation of children from one population per run.

    genotypes (R, P, G) float32, energies (R, P) float32, cand (R, P, 4) int32
    (tournament candidates of the two parents), coins (R, P, 3) float32
    (tournament 1, tournament 2, crossover), cuts (R, P, 2) int32, mut_coin and
    mut_delta (R, P, G) float32. Returns (children (R, P, G) float32, best (R,)
    int32). Pure Python loops over children: meant for small populations.
    """
    gen = np.asarray(genotypes, dtype=np.float32)
    R, P, G = gen.shape
    key = fitness_key(energies)
    best = run_best(energies)
    cand = np.clip(np.asarray(cand, dtype=np.int64), 0, P - 1)
    cuts = np.clip(np.asarray(cuts, dtype=np.int64), 0, G)
    coins = np.asarray(coins, dtype=np.float32)
    mut_coin = np.asarray(mut_coin, dtype=np.float32)
    mut_delta = np.asarray(mut_delta, dtype=np.float32)
    out = np.empty_like(gen)
    for r in range(R):
        for k in range(P):
            if elitism and k == 0:
                out[r, k] = gen[r, best[r]]
                continue
            p1 = tournament(key[r], cand[r, k, 0], cand[r, k, 1], coins[r, k, 0], p_tournament)
            p2 = tournament(key[r], cand[r, k, 2], cand[r, k, 3], coins[r, k, 1], p_tournament)
            child = gen[r, p1].copy()
            if coins[r, k, 2] < np.float32(p_crossover):
                lo, hi = sorted((int(cuts[r, k, 0]), int(cuts[r, k, 1])))
                child[lo:hi] = gen[r, p2, lo:hi]
            for g in range(G):
                if mut_coin[r, k, g] < np.float32(p_mutation):
                    child[g] = np.float32(child[g] + mut_delta[r, k, g])
            out[r, k] = child
    return out, best


def select_rows(draws, rate):
    """Rows that take the local search at `rate` (reading: AutoDock searches
    each child with probability equal to the local-search rate, Sec. 2.1 for
    the structure): row r is selected when its uniform draw is below the rate
    (float32 comparison). Returns the selected rows in increasing order."""
    d = np.asarray(draws, dtype=np.float32)
    return np.array([r for r in range(d.shape[0]) if d[r] < np.float32(rate)], dtype=np.int32)
