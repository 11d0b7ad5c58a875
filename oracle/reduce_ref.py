"""Reference for the block sum of 4-vectors {E, gx, gy, gz}.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The operation (Sec. 3, the reduce-and-broadcast; Sec. 4.2, the matrix form):
every thread of a block holds one 4-vector; the result is the component-wise
sum over the block, made available to every thread.

* `sum4_exact` is the definition itself: the exactly rounded (math.fsum) sum of
  each component, in float64.
* `sum4_matrix` is the paper's formulation (Sec. 4.2) in float64: 64 vectors at
  a time fill a 16x16 matrix A column-major (row 4m+c, column j holds component
  c of vector 4j+m), V accumulates A P with P the all-ones matrix, and W = Q V
  with Q the 4x4 block matrix of 4x4 identities; the sums are W[0..3, 0].
  (The prose speaks of summing "every 4th column"; with Q multiplying from
  the left it sums rows r = r' mod 4, which is what the matrices printed there
  compute, and what is done here.)
* `round_bf16`, `round_f16` and `split_terms` model the split-operand inputs of
  a half-width matrix-unit reduction (precision refinement, Sec. 6): a float32
  value is written as a sum of s narrow terms, each the round-to-nearest-even
  of the remainder left by the previous terms.
"""
from __future__ import annotations

import math

import numpy as np


def sum4_exact(u):
    """Exactly rounded component sums of u [n, 4] -> float64 [4]."""
    u = np.asarray(u, dtype=np.float64).reshape(-1, 4)
    return np.array([math.fsum(u[:, c]) for c in range(4)])


def paper_matrices():
    """P (all ones) and Q (4x4 blocks of I4), both 16x16, float64."""
    P = np.ones((16, 16))
    Q = np.kron(np.ones((4, 4)), np.eye(4))
    return P, Q


def pack_A(u64):
    """16x16 A from 64 vectors: A[4m + c, j] = u[4j + m, c]."""
    A = np.zeros((16, 16))
    for j in range(16):
        for m in range(4):
            for c in range(4):
                A[4 * m + c, j] = u64[4 * j + m, c]
    return A


def sum4_matrix(u):
    """The paper's V <- A P (+ V per 64 vectors), W <- Q V; returns W[0:4, 0]."""
    u = np.asarray(u, dtype=np.float64).reshape(-1, 4)
    n = u.shape[0]
    pad = (-n) % 64
    if pad:
        u = np.concatenate([u, np.zeros((pad, 4))])
    P, Q = paper_matrices()
    V = np.zeros((16, 16))
    for b in range(0, u.shape[0], 64):
        V = pack_A(u[b:b + 64]) @ P + V
    W = Q @ V
    return W[0:4, 0].copy()


def round_bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even); returns float32."""
    x = np.asarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    return np.where(np.isfinite(x), out, x)


def round_f16(x):
    """Round float32 values to IEEE binary16 (nearest, ties to even); returns float32."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)


def split_terms(x, fmt: str, terms: int):
    """Write float32 x as `terms` narrow values: t_0 = rnd(x), t_k = rnd(x - sum_{<k})."""
    rnd = round_bf16 if fmt == "bf16" else round_f16
    x = np.asarray(x, dtype=np.float32)
    rem = x.astype(np.float32)
    out = []
    for _ in range(terms):
        t = rnd(rem)
        out.append(t)
        rem = (rem - t).astype(np.float32)
    return out


def unit_roundoff(fmt: str) -> float:
    """Half the spacing of the narrow format at 1: 2^-8 (bf16), 2^-11 (fp16)."""
    return 2.0 ** -8 if fmt == "bf16" else 2.0 ** -11
