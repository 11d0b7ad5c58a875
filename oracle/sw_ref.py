"""Reference of the Solis-Wets local search of the LGA.

TEST INFRASTRUCTURE ONLY: only tests, the smoke check and the benchmark's
CPU-baseline leg may use this module. Nothing here is shared with the HIP
path.

What the paper fixes and what is read into it
---------------------------------------------
Sec. 2.1 names Solis-Wets as the second local search of the LGA beside
ADADELTA; it needs energies only, no gradient. The paper gives no step, so
this is the published random-search method of Solis and Wets (1981) in the
form AutoDock uses, stated as readings:

* per iteration a deviation dev = rho * (scale_g * z_g) per gene, with z a
  standard normal draw (an input) and scale_g a per-gene step scale;
* try x + bias + dev; if its energy is lower than the current one, move there
  and set bias = 0.2 bias + 0.4 dev (a success);
* else try x - bias - dev; if lower, move there and set bias = bias - 0.4 dev
  (a success);
* else bias = 0.5 bias (a failure);
* successes and failures are counted in runs: after n_success successes in a
  row rho doubles, after n_failure failures in a row it halves, and the
  count restarts.

Every state update is float32 arithmetic in the order written (products,
then sums; no fused operations), so an implementation that takes the same
accept decisions reproduces the state bit for bit. The decisions compare
energies: `decide_energies` lets a test take them from the implementation's
own float32 energies (the same precision as its decisions) while the energies
themselves are checked against this module's FP64 evaluation.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

F = np.float32


@dataclass
class SWState:
    x: np.ndarray        # [n, G] float32 genotypes
    energy: np.ndarray   # [n] energies of x (float64 here; the decisions' precision is the caller's)
    bias: np.ndarray     # [n, G] float32
    rho: np.ndarray      # [n] float32
    succ: np.ndarray     # [n] int32, successes in a row
    fail: np.ndarray     # [n] int32, failures in a row


def sw_start(x, energy, rho0=1.0):
    x = np.asarray(x, F)
    n = x.shape[0]
    return SWState(x.copy(), np.asarray(energy, np.float64).copy(), np.zeros_like(x),
                   np.full(n, rho0, F), np.zeros(n, np.int32), np.zeros(n, np.int32))


def deviation(rho, scale, z):
    """dev = rho * (scale * z), float32, per individual (rho [n], z [n, G])."""
    return (np.asarray(rho, F)[:, None] * (np.asarray(scale, F)[None, :] * np.asarray(z, F))).astype(F)


def sw_run(energy_fn, st: SWState, normals, scale, n_success=4, n_failure=4,
           decide_energies=None):
    """Runs len(normals) iterations in place on `st`; returns the energies of
    the tried points, [iters, n, 2] float64 (NaN where the second point was
    not tried).

    energy_fn(genotypes [m, G] float32) -> energies [m] float64.
    decide_energies: optional [iters, n, 2] energies that take the accept
    decisions in place of energy_fn's (the state then follows them; the
    current energy is taken from them too, after the initial one).
    """
    normals = np.asarray(normals, F)
    iters, n, G = normals.shape
    tried = np.full((iters, n, 2), np.nan)
    cur = st.energy.astype(np.float64).copy()
    for it in range(iters):
        dev = deviation(st.rho, scale, normals[it])
        c1 = ((st.x + st.bias).astype(F) + dev).astype(F)
        e1 = np.asarray(energy_fn(c1), np.float64)
        tried[it, :, 0] = e1
        d1 = e1 if decide_energies is None else np.asarray(decide_energies[it, :, 0], np.float64)
        c2 = ((st.x - st.bias).astype(F) - dev).astype(F)
        e2_all = np.asarray(energy_fn(c2), np.float64)
        for k in range(n):
            if d1[k] < cur[k]:
                st.x[k] = c1[k]
                cur[k] = d1[k]
                st.bias[k] = (F(0.2) * st.bias[k] + F(0.4) * dev[k]).astype(F)
                st.succ[k] += 1
                st.fail[k] = 0
            else:
                tried[it, k, 1] = e2_all[k]
                d2 = e2_all[k] if decide_energies is None else float(decide_energies[it, k, 1])
                if d2 < cur[k]:
                    st.x[k] = c2[k]
                    cur[k] = d2
                    st.bias[k] = (st.bias[k] - F(0.4) * dev[k]).astype(F)
                    st.succ[k] += 1
                    st.fail[k] = 0
                else:
                    st.bias[k] = (F(0.5) * st.bias[k]).astype(F)
                    st.fail[k] += 1
                    st.succ[k] = 0
            if st.succ[k] >= n_success:
                st.rho[k] = F(2.0) * st.rho[k]
                st.succ[k] = 0
            elif st.fail[k] >= n_failure:
                st.rho[k] = F(0.5) * st.rho[k]
                st.fail[k] = 0
    st.energy = cur
    return tried


def gene_scale(n_genes, translation=1.0, quaternion=0.1, torsion=0.5):
    """Per-gene step scales of the benchmark: Angstrom for the translation,
    unit-quaternion components, radians for the torsions."""
    s = np.full(n_genes, torsion, F)
    s[:3] = translation
    s[3:7] = quaternion
    return s
