"""Pins for the reduction reference (Sec. 3 reduce-and-broadcast; Sec. 4.2 matrix form).

* the paper's matrix identity W = Q (A P (+V)) gives the component sums: on
  integer-valued data (exact in any order) it equals the exactly rounded sum
  bit for bit, and on random data it agrees to float64 rounding;
* the exactly rounded sum is checked against Python's integer arithmetic on
  scaled integers and against a sorted pairwise sum;
* bf16/fp16 rounding is checked against PyTorch's dtype conversions (library
  round-to-nearest-even), and the split-operand error against its bound
  |x - sum of s terms| <= u^s |x|.
"""
import math

import numpy as np
import pytest
import torch

from oracle import reduce_ref as RR


@pytest.mark.parametrize("n", [1, 63, 64, 65, 256, 1000])
def test_matrix_identity_integer_exact(n):
    rng = np.random.default_rng(n)
    u = rng.integers(-127, 128, (n, 4)).astype(np.float64)
    want = np.array([sum(int(v) for v in u[:, c]) for c in range(4)], dtype=float)
    assert np.array_equal(RR.sum4_exact(u), want)
    assert np.array_equal(RR.sum4_matrix(u), want)


def test_matrix_identity_random():
    rng = np.random.default_rng(1)
    u = rng.normal(size=(1024, 4)) * 10 ** rng.uniform(-3, 5, (1024, 1))
    ex = RR.sum4_exact(u)
    mx = RR.sum4_matrix(u)
    bound = 64 * np.finfo(float).eps * np.abs(u).sum(axis=0)
    assert np.all(np.abs(mx - ex) <= bound)


def test_paper_matrix_shapes_and_layout():
    P, Q = RR.paper_matrices()
    assert P.shape == Q.shape == (16, 16) and np.all(P == 1)
    for r in range(16):
        for c in range(16):
            assert Q[r, c] == (1.0 if r % 4 == c % 4 else 0.0)
    u = np.arange(256, dtype=float).reshape(64, 4)
    A = RR.pack_A(u)
    assert A[0, 0] == u[0, 0] and A[0, 15] == u[60, 0] and A[3, 0] == u[0, 3] and A[4, 0] == u[1, 0]


def test_fsum_against_scaled_integers():
    rng = np.random.default_rng(2)
    k = rng.integers(-2**40, 2**40, (500, 4))
    u = k.astype(np.float64) * 2.0 ** -30
    want = np.array([float(sum(int(v) for v in k[:, c])) * 2.0 ** -30 for c in range(4)])
    assert np.array_equal(RR.sum4_exact(u), want)


def test_bf16_f16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = (rng.normal(size=20000) * 10 ** rng.uniform(-6, 6, 20000)).astype(np.float32)
    x = np.concatenate([x, np.float32([0.0, -0.0, 1.0, 65504.0, 3.0e-5])])
    tb = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(RR.round_bf16(x), tb)
    small = x[np.abs(x) < 6e4]
    th = torch.from_numpy(small).to(torch.float16).to(torch.float32).numpy()
    assert np.array_equal(RR.round_f16(small), th)


@pytest.mark.parametrize("fmt,terms", [("bf16", 2), ("bf16", 3), ("f16", 2)])
def test_split_bound(fmt, terms):
    rng = np.random.default_rng(4)
    # keep fp16 terms normal: |x| in [2^-3, 2^14]
    lo, hi = (-20, 20) if fmt == "bf16" else (-3, 14)
    x = (rng.choice([-1, 1], 5000) * 2.0 ** rng.uniform(lo, hi, 5000)).astype(np.float32)
    t = RR.split_terms(x, fmt, terms)
    s = sum(v.astype(np.float64) for v in t)
    u = RR.unit_roundoff(fmt)
    assert np.all(np.abs(s - x.astype(np.float64)) <= u ** terms * np.abs(x) * (1 + 1e-12))
