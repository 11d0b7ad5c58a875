"""A Lamarckian GA docking job on the device: independent runs, each a
population that alternates the genetic step (dock_ga_step) with the ADADELTA
local search (dock_local_search_batch) on its children (Sec. 2.1: the GA makes
new genotypes, the local search improves them; a docking job holds many LGA
runs, and each run ends at a generation cap or an evaluation budget). With a
local-search rate below one, every child is scored (dock_score_batch) and
only the children whose uniform draw falls below the rate are searched: they
are selected (dock_select_rows), gathered into a compact state
(dock_gather_rows), searched, and their best points and energies written back
(dock_scatter_rows).

Host sequencing only: every step runs in the library's kernels; random inputs
of the GA step are drawn on the device with a seeded torch generator. The
search's best points and energies (Lamarckian write-back) form the next
population.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import dock


def converged(history, patience: int, tol: float) -> bool:
    """Early stopping: True when no run's best energy improved by more than
    `tol` over the last `patience` generations (history: per generation, the
    [n_runs] best energies, oldest first). patience <= 0 never stops."""
    if patience <= 0 or len(history) <= patience:
        return False
    then = np.asarray(history[-1 - patience], np.float64)
    now = np.asarray(history[-1], np.float64)
    return bool(np.all(then - now <= tol))


@dataclass
class LgaResult:
    best_energy: np.ndarray      # [n_runs] float32: each run's best energy
    best_genotype: np.ndarray    # [n_runs, G] float32
    evaluations: int             # scoring evaluations spent (all runs)
    generations: int             # generations completed after the initial search
    stopped_early: bool = False  # ended by the convergence rule
    history: list = field(default_factory=list)   # per generation: [n_runs] best energies (host)
    searched: list = field(default_factory=list)  # per search phase: individuals searched


def run_lga(grids, ligand, genotypes, n_runs: int, generations: int, ls_iterations: int = 300,
            eval_budget: int = 0, p_tournament: float = 0.6, p_crossover: float = 0.8,
            p_mutation: float = 0.02, seed: int = 0, variant: int = dock.REDUCE_SHUFFLE,
            threads_per_ind: int = 0, stop_patience: int = 0, stop_tol: float = 1e-3,
            ls_rate: float = 1.0) -> LgaResult:
    """Runs the job from `genotypes` ([n_runs * pop, G] float32 CUDA tensor,
    run-major). The initial population is searched first; then each
    generation makes pop children per run and searches them: all of them at
    ls_rate >= 1, else the children whose draw (seeded, one per child) is
    below ls_rate, after scoring every child (the initial population is
    treated the same way). A generation that would take the job past
    `eval_budget` (if > 0; a rate below one counts its expected cost) is not
    started. With stop_patience > 0 the job also ends once no run's best
    energy has improved by more than stop_tol (kcal/mol) over the last
    stop_patience generations (early stopping; `converged`). Everything runs
    on the current stream."""
    import torch
    n, G = genotypes.shape
    if n_runs < 1 or n % n_runs != 0:
        raise ValueError("genotypes rows must be n_runs * pop")
    if not (ls_rate >= 0.0):
        raise ValueError("ls_rate must be >= 0")
    pop = n // n_runs
    full = ls_rate >= 1.0
    # the search's evaluations incl. the final point; a partial rate scores
    # every child and searches the expected share
    per_gen = n * (ls_iterations + 1) if full else n + int(round(ls_rate * n)) * (ls_iterations + 1)
    dev = genotypes.device
    ws = torch.empty(max(dock.workspace_bytes(1), 64), dtype=torch.uint8, device=dev)
    rng = torch.Generator(device=dev)
    rng.manual_seed(seed)
    searched = []

    def search(gen):
        st = dock.LSState.start(gen)
        dock.local_search([dock.LsJob(grids, ligand, st, threads_per_ind=threads_per_ind)],
                          ls_iterations, variant=variant, workspace=ws)
        return st

    def phase(gen):
        """Population (genotypes, energies) after the search phase; the
        evaluations it spent."""
        if full:
            st = search(gen)
            searched.append(n)
            return st.best_genotype, st.best_energy, n * (ls_iterations + 1)
        pop_g = gen.contiguous().clone()
        pop_e, _ = dock.score_batch(grids, ligand, pop_g, variant=variant, with_grad=False)
        draws = torch.rand(n, generator=rng, device=dev, dtype=torch.float32)
        index, count = dock.select_rows(draws, ls_rate)
        m = int(count.item())                      # host needs the size of the search
        searched.append(m)
        if m > 0:
            st = search(dock.gather_rows(pop_g, index, m))
            dock.scatter_rows(st.best_genotype, index, pop_g)
            dock.scatter_rows(st.best_energy, index, pop_e)
        return pop_g, pop_e, n + m * (ls_iterations + 1)

    def run_best(pop_e, pop_g=None):
        # reporting on the host: each run's best member (first of equal energies)
        torch.cuda.synchronize()
        e = pop_e.cpu().numpy().reshape(n_runs, pop)
        k = np.argmin(e, axis=1)
        rows = np.arange(n_runs)
        g = pop_g.cpu().numpy().reshape(n_runs, pop, G)[rows, k] if pop_g is not None else None
        return e[rows, k], g

    pop_g, pop_e, evals = phase(genotypes)
    history = [run_best(pop_e)[0]]
    done = 0
    stopped = False
    for _ in range(generations):
        if eval_budget > 0 and evals + per_gen > eval_budget:
            break
        if converged(history, stop_patience, stop_tol):
            stopped = True
            break
        draws = dock.ga_draws(n_runs, pop, G, rng, dev)
        children, _ = dock.ga_step(pop_g.view(n_runs, pop, G), pop_e.view(n_runs, pop), *draws,
                                   p_tournament, p_crossover, p_mutation, True)
        pop_g, pop_e, spent = phase(children.view(n, G))
        evals += spent
        done += 1
        history.append(run_best(pop_e)[0])
    e, g = run_best(pop_e, pop_g)
    return LgaResult(e, g, evals, done, stopped, history, searched)
