"""FP64 CPU oracle for the docking hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or run
anything under this directory; only the tests, the smoke check and the CPU
baseline leg of the benchmark do. The oracle shares no code with the HIP path:
it takes plain NumPy arrays (as produced by the seeded generators) and
recomputes every step of the method in float64, in the order the method states
it, without blocking, fusion or reordering.

Submodules
----------
dock_ref
    ligand preparation (BFS), genotype -> pose, trilinear grid term,
    intramolecular pair terms, gradient -> genotype, ADADELTA local search.
work
    the operation tally of one evaluation: the oracle's own functions run on
    counting scalars (the algorithmic-work figure beside the work model).
reduce_ref
    the block sum of 4-vectors {E, gx, gy, gz}: the exactly rounded sum and the
    paper's matrix formulation (Sec. 4.2), plus split-operand helpers.
"""
from . import dock_ref, reduce_ref  # noqa: F401
