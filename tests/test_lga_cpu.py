"""Early-stopping rule of the LGA job (host logic)."""
import numpy as np

from paper_2410_10447_amd.lga import converged


def test_converged_needs_patience_generations_without_improvement():
    h = [np.array([-10.0, -5.0]), np.array([-11.0, -5.0]), np.array([-11.0005, -5.0]),
         np.array([-11.0005, -5.0002])]
    assert not converged(h, 0, 1e-3)                 # off
    assert not converged(h[:2], 2, 1e-3)             # not enough history
    assert not converged(h[:3], 2, 1e-3)             # run 0 improved by 1.0005 over 2 generations
    assert converged(h, 2, 1e-3)                     # both runs within 1e-3 over the last 2
    assert not converged(h, 2, 1e-4)                 # run 0 improved by 5e-4 > 1e-4
    assert not converged(h, 3, 1e-3)                 # over 3 generations run 0 improved by 1.0005


def test_converged_on_any_single_improving_run_is_false():
    h = [np.zeros(5)] * 4 + [np.array([0.0, 0.0, -0.5, 0.0, 0.0])]
    assert not converged(h, 3, 0.1)
    assert converged(h[:4], 3, 0.1)
