"""A Lamarckian GA docking job on the device: independent runs, each a
population that alternates the genetic step (dock_ga_step) with the ADADELTA
local search (dock_local_search_batch) on every child (Sec. 2.1: the GA makes
new genotypes, the local search improves each of them; a docking job holds
many LGA runs, and each run ends at a generation cap or an evaluation
budget).

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


def run_lga(grids, ligand, genotypes, n_runs: int, generations: int, ls_iterations: int = 300,
            eval_budget: int = 0, p_tournament: float = 0.6, p_crossover: float = 0.8,
            p_mutation: float = 0.02, seed: int = 0, variant: int = dock.REDUCE_SHUFFLE,
            threads_per_ind: int = 0, stop_patience: int = 0, stop_tol: float = 1e-3) -> LgaResult:
    """Runs the job from `genotypes` ([n_runs * pop, G] float32 CUDA tensor,
    run-major). The initial population is searched first; then each
    generation makes pop children per run and searches all of them. A
    generation that would take the job past `eval_budget` (if > 0) is not
    started. With stop_patience > 0 the job also ends once no run's best
    energy has improved by more than stop_tol (kcal/mol) over the last
    stop_patience generations (early stopping; `converged`). Everything runs
    on the current stream."""
    import torch
    n, G = genotypes.shape
    if n_runs < 1 or n % n_runs != 0:
        raise ValueError("genotypes rows must be n_runs * pop")
    pop = n // n_runs
    per_gen = n * (ls_iterations + 1)          # the search's evaluations incl. the final point
    ws = torch.empty(max(dock.workspace_bytes(1), 64), dtype=torch.uint8, device=genotypes.device)

    def search(gen):
        st = dock.LSState.start(gen)
        dock.local_search([dock.LsJob(grids, ligand, st, threads_per_ind=threads_per_ind)],
                          ls_iterations, variant=variant, workspace=ws)
        return st

    def run_best(st, with_genotype=False):
        # reporting on the host: each run's best member (first of equal energies)
        torch.cuda.synchronize()
        e = st.best_energy.cpu().numpy().reshape(n_runs, pop)
        k = np.argmin(e, axis=1)
        rows = np.arange(n_runs)
        g = st.best_genotype.cpu().numpy().reshape(n_runs, pop, G)[rows, k] if with_genotype else None
        return e[rows, k], g

    st = search(genotypes)
    evals = per_gen
    history = [run_best(st)[0]]
    rng = torch.Generator(device=genotypes.device)
    rng.manual_seed(seed)
    done = 0
    stopped = False
    for _ in range(generations):
        if eval_budget > 0 and evals + per_gen > eval_budget:
            break
        if converged(history, stop_patience, stop_tol):
            stopped = True
            break
        draws = dock.ga_draws(n_runs, pop, G, rng, genotypes.device)
        children, _ = dock.ga_step(st.best_genotype.view(n_runs, pop, G),
                                   st.best_energy.view(n_runs, pop), *draws,
                                   p_tournament, p_crossover, p_mutation, True)
        st = search(children.view(n, G))
        evals += per_gen
        done += 1
        history.append(run_best(st)[0])
    e, g = run_best(st, with_genotype=True)
    return LgaResult(e, g, evals, done, stopped, history)
