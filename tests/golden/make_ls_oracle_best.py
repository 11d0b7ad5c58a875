"""Writes ls_oracle_best_n48_t10_i3000.txt: the FP64 oracle's best energy of
each of the 3000 individuals of the 48-atom, 10-torsion local-search workload
(64^3 x 10 maps) after 300 ADADELTA iterations (rho 0.8, eps 1e-2) plus the
final evaluation, one value per line in individual order.

Calls only the oracle and the seeded input generators:
    python tests/golden/make_ls_oracle_best.py [--workers N]
"""
import argparse
import os
import sys
from multiprocessing import get_context

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "ls_oracle_best_n48_t10_i3000.txt")
N, ITERS = 3000, 300


def _slice(args):
    lo, hi = args
    from oracle import dock_ref as R
    from paper_2410_10447_amd import synth
    w = synth.ls_workload(N, ITERS)
    prep = R.prepare(w.ligands[0], w.ff)
    st = R.ls_init(w.genotypes[0][lo:hi])
    R.local_search(prep, w.grids, st, ITERS, rho=w.rho, eps=w.eps, final_eval=True)
    return lo, st.best_energy


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    a = ap.parse_args()
    os.environ["OMP_NUM_THREADS"] = "1"
    step = 125
    chunks = [(lo, min(lo + step, N)) for lo in range(0, N, step)]
    best = [None] * N
    with get_context("spawn").Pool(a.workers) as pool:
        for lo, be in pool.imap_unordered(_slice, chunks):
            best[lo:lo + len(be)] = list(be)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle best energy (kcal/mol) per individual, 48-atom 10-torsion ligand,\n")
        f.write("# 64^3 x 10 maps, 3000 individuals, 300 ADADELTA iterations + final evaluation\n")
        for v in best:
            f.write(f"{v:.17g}\n")
    print(OUT)


if __name__ == "__main__":
    main()
