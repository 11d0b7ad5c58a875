"""Operation tally of one scoring evaluation and one ADADELTA step.

TEST INFRASTRUCTURE ONLY (see the package docstring): the benchmark reads
this count to state the algorithmic work behind its roofline fraction.

The count is made by the oracle itself: its own functions (pose, grid term,
pair terms, gradient -> genotype, ADADELTA update; Sec. 2.1) run on one
individual whose coordinates are counting scalars (Tally). Every arithmetic
operation those functions apply to a value that depends on the genotype is
recorded once; operations on constants alone (force-field parameters,
charges, map values, grid geometry) are not, since they are fixed per ligand
and receptor. Classes:

* alu: add, subtract, multiply, negate, absolute value, compare (max, min,
  clip, tests), floor, and division by a constant;
* transcendental: sqrt, exp, sin, cos, division by a computed value, and
  powers other than squares (a square counts as one multiply).

Lane-slot weight: alu 1, transcendental 4 (the quarter-rate issue of the
transcendental unit, the convention of the FP32 VALU roofline this work is
priced against). The tally is of the formulas as the oracle writes them
(e.g. it rotates every moving atom of every torsion and evaluates the
dielectric with its own divisions); a kernel may do the same work with
fewer operations.
"""
from __future__ import annotations

import dataclasses
import math
from collections import Counter

import numpy as np

from . import dock_ref as R

_ALU = ("add", "sub", "mul", "neg", "abs", "cmp", "floor", "divc")
_TRANSC = ("sqrt", "exp", "sin", "cos", "div", "pow")


class Tally:
    """A float whose arithmetic is counted into the active Counter. A
    constant Tally (counting=False) stands for a value fixed per ligand
    (e.g. reference coordinates): operations whose operands are all
    constants are not counted and give constants."""

    __slots__ = ("v", "counting")
    counter: Counter = Counter()

    def __init__(self, v, counting=True):
        self.v = float(v)
        self.counting = counting

    @staticmethod
    def _val(o):
        return o.v if isinstance(o, Tally) else o

    def _op(self, kind, v, o=None):
        counting = self.counting or (isinstance(o, Tally) and o.counting)
        if counting:
            Tally.counter[kind] += 1
        return Tally(v, counting)

    def __add__(self, o):
        return self._op("add", self.v + self._val(o), o)

    __radd__ = __add__

    def __sub__(self, o):
        return self._op("sub", self.v - self._val(o), o)

    def __rsub__(self, o):
        return self._op("sub", self._val(o) - self.v, o)

    def __mul__(self, o):
        return self._op("mul", self.v * self._val(o), o)

    __rmul__ = __mul__

    def __truediv__(self, o):
        computed = isinstance(o, Tally) and o.counting
        return self._op("div" if computed else "divc", self.v / self._val(o), o)

    def __rtruediv__(self, o):
        return self._op("div", self._val(o) / self.v, o)

    def __neg__(self):
        return self._op("neg", -self.v)

    def __abs__(self):
        return self._op("abs", abs(self.v))

    def __pow__(self, e):
        e = self._val(e)
        return self._op("mul" if e == 2 else "pow", self.v ** e)

    def sqrt(self):
        return self._op("sqrt", math.sqrt(self.v))

    def exp(self):
        return self._op("exp", math.exp(self.v))

    def sin(self):
        return self._op("sin", math.sin(self.v))

    def cos(self):
        return self._op("cos", math.cos(self.v))

    def __floor__(self):
        if self.counting:
            Tally.counter["floor"] += 1
        return math.floor(self.v)

    def __int__(self):
        return int(self.v)

    def _cmp(self, o, f):
        if self.counting or (isinstance(o, Tally) and o.counting):
            Tally.counter["cmp"] += 1
        return f(self.v, self._val(o))

    def __lt__(self, o):
        return self._cmp(o, lambda a, b: a < b)

    def __le__(self, o):
        return self._cmp(o, lambda a, b: a <= b)

    def __gt__(self, o):
        return self._cmp(o, lambda a, b: a > b)

    def __ge__(self, o):
        return self._cmp(o, lambda a, b: a >= b)

    def __eq__(self, o):
        return self._cmp(o, lambda a, b: a == b)

    __hash__ = None


def _counting(a, counting=True):
    return np.vectorize(lambda v: Tally(v, counting), otypes=[object])(np.asarray(a, dtype=np.float64))


def _measure(fn):
    Tally.counter = Counter()
    out = fn()
    c = Tally.counter
    Tally.counter = Counter()
    alu = sum(c[k] for k in _ALU)
    tr = sum(c[k] for k in _TRANSC)
    return {"alu": alu, "transcendental": tr, "slots": alu + 4 * tr, "ops": dict(c)}, out


def _float_of(a):
    return np.vectorize(lambda t: t.v if isinstance(t, Tally) else float(t), otypes=[np.float64])(a)


def tally(prep: R.Prepared, grd, genotype) -> dict:
    """Per-stage operation counts of one evaluation (energy and gradient) and
    one ADADELTA step at `genotype` [G], the stages as the oracle computes
    them: pose, grid term (all atoms), pair terms (all pairs), gradient ->
    genotype, ADADELTA update. Returns {stage: {alu, transcendental, slots,
    ops}} plus "total". Sizes: prep's atoms, torsions and pairs."""
    gen = _counting(np.asarray(genotype, np.float64)[None, :])
    prep = dataclasses.replace(prep, y0=_counting(prep.y0, counting=False))
    stages = {}
    stages["pose"], x = _measure(lambda: R.pose(prep, gen))
    stages["grid"], (e_in, g_in) = _measure(lambda: R.inter_terms(prep, grd, x))
    stages["pairs"], (e_ia, g_ia) = _measure(lambda: R.intra_terms(prep, x))

    def _total():
        gat = g_in + g_ia
        E = e_in.sum(axis=1) + e_ia
        return gat, E
    stages["sums"], (gat, E) = _measure(_total)
    stages["gradient"], grad = _measure(lambda: R.genotype_gradient(prep, gen, x, gat))
    acc = _counting(np.zeros_like(np.asarray(genotype, np.float64))[None, :], counting=False)
    stages["adadelta"], _ = _measure(lambda: R.adadelta_step(gen, grad, acc, acc, 0.8, 1e-2))
    tot = {"alu": 0, "transcendental": 0, "slots": 0}
    for st in stages.values():
        for k in tot:
            tot[k] += st[k]
    stages["total"] = tot
    stages["energy"] = float(_float_of(E)[0])
    return stages


def model_slots(n_pairs: int, n_atoms: int, n_torsions: int) -> int:
    """The work model of one evaluation in FP32 lane-slots (transcendentals
    weighted 4): 75 per kept pair, 150 per atom, 80 per torsion, 25 per gene
    (G = 7 + T), with the sizes the oracle's preparation tallies."""
    return 75 * n_pairs + 150 * n_atoms + 80 * n_torsions + 25 * (7 + n_torsions)
