"""Pins of the oracle's objective gradient (tangent-linear method).

The tangent sweep (forward sensitivities, one complex-step JVP of the step
residual per step) is checked against two derivatives that share none of its
steps: the complex step taken through the whole time loop (every assembly and
LU solve in complex arithmetic) and central finite differences of the real loop.
The FD step is large (1e-2 relative) because J ~ 1e-14 carries the LU round-off of
phi_e; truncation at that step is O(1e-4) relative, the bar below is 1e-2.
"""
import numpy as np
import pytest

from knp_inputs import config_case
from oracle.adjoint import gradient_complex_step, gradient_tangent, objective


@pytest.fixture(scope="module")
def small():
    case = config_case(4, per_pitch=4, n_steps=3)
    J, g = gradient_tangent(case, case.theta)
    return case, J, g


def test_tangent_matches_complex_step(small):
    case, J, g = small
    gc = gradient_complex_step(case, case.theta)
    assert np.all(np.isfinite(g)) and np.abs(g).max() > 0
    assert np.abs(g - gc).max() <= 1e-6 * np.abs(gc).max()


def test_tangent_matches_central_differences(small):
    case, J, g = small
    assert np.isclose(J, objective(case, case.theta), rtol=1e-12)
    for c in (0, int(np.argmax(np.abs(g)))):
        h = 1e-2 * case.theta[c]
        tp = case.theta.copy()
        tm = case.theta.copy()
        tp[c] += h
        tm[c] -= h
        fd = (objective(case, tp) - objective(case, tm)) / (2 * h)
        assert abs(fd - g[c]) <= 1e-2 * np.abs(g).max(), (c, fd, g[c])


def test_gradient_is_zero_before_any_step():
    case = config_case(4, per_pitch=4, n_steps=0)
    J, g = gradient_tangent(case, case.theta)
    assert J == 0.0 and np.all(g == 0.0)
