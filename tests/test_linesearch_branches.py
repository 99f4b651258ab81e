"""Every branch of the modified secant step (Sec. 3.3, Algorithm 2), pinned
by hand-derived traces on functions of one variable.

Each case gives f and f' in closed form, the start tau0 and the sequence of
points the search must evaluate, with the branch that produced each point.
The sequences were derived by hand from the algorithm's steps (derivations in
the comments; all points are exact rationals).  Parameters: delta = 0.05,
sigma = 0.1 (so |f'| <= 0.1 |f'(0)| ends the search), gamma = 0.5,
eps = 1e-12; every f has f(0) = -10, so the energy bound is -10 + 1e-11.

The same traces are checked for the oracle (oracle/linesearch.py) and for the
library's host control of the line search (eahp_linesearch_host), which is the
code the GPU path runs between its trial evaluations.
"""
import os
import sys
from fractions import Fraction as Fr

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import linesearch  # noqa: E402
import workloads as W  # noqa: E402

PRM = dict(W.DEFAULT_PARAMS, delta=0.05, sigma=0.1, gamma=0.5, eps=1e-12, ls_maxit=20)


def poly(c):
    """f(t) = -10 - t + c2 t^2/2 + c3 t^3/3 + c4 t^4/4, f'(t) = -1 + c2 t + c3 t^2 + c4 t^3."""
    c2, c3, c4 = c

    def ev(t):
        return (-10.0 - t + c2 * t * t / 2 + c3 * t ** 3 / 3 + c4 * t ** 4 / 4,
                -1.0 + c2 * t + c3 * t * t + c4 * t ** 3)
    return ev


CASES = {
    # f' = -(t - 1)^2 (an inflection at t = 1, f' < 0 elsewhere).
    # tau0 = 3/2: f' = -1/4, not accepted.  Secant on [0, 3/2] with slopes -1,
    # -1/4: (0 + 3/2)/(3/4) = 2 > b, f(2) - f(0) = -2/3 -> [a, b] = [3/2, 2].
    # Secant on [3/2, 2], slopes -1/4, -1: (-3/2 + 1/2)/(-3/4) = 4/3 < a, energy
    # below the bound -> tau = b / gamma = 4, [0, 4].  f'(4) = -9; secant on
    # [0, 4]: 4/(-8) = -1/2, evaluated: f(-1/2) - f(0) = 19/24 > 0 with
    # f' = -9/4 < 0 -> tau = gamma b = 2, [0, 2].  f'(2) = -1 = f'(0): equal
    # slopes, midpoint 1, where f' = 0: accepted after 7 evaluations.
    "right_left_grow_shrink_midpoint": (
        poly((2.0, -1.0, 0.0)), 1.5,
        [(Fr(3, 2), "init"), (Fr(2), "secant"), (Fr(4, 3), "secant"), (Fr(4), "grow"), (Fr(-1, 2), "secant"),
         (Fr(2), "shrink"), (Fr(1), "secant")]),
    # f' = -1 + 2t + 2t^2 - 2t^3.  tau0 = 3/2: f' = -1/4.  Secant on [0, 3/2]:
    # 2 > b (f'(2) = -5, f(2) - f(0) = -2/3) -> [3/2, 2].  Secant on [3/2, 2]:
    # (3/2 (-5) - 2 (-1/4))/(-5 + 1/4) = 28/19 inside, where f - f(0) = 0.4735 > 0
    # and f' = -0.1101 < 0 -> tau = gamma b = 1, [0, 1].  f'(1) = 1 (f too high
    # but the point is not in a bracket update).  Secant on [0, 1]: 1/2, f' = 1/4
    # >= 0 with f below the bound -> [0, 1/2].  Secant: (1/2)/(5/4) = 2/5,
    # f' = -0.008: accepted after 6 evaluations.
    "right_shrink_inside": (
        poly((2.0, 2.0, -2.0)), 1.5,
        [(Fr(3, 2), "init"), (Fr(2), "secant"), (Fr(28, 19), "secant"), (Fr(1), "shrink"), (Fr(1, 2), "secant"),
         (Fr(2, 5), "secant")]),
    # f' = -1 + 2t - t^2/2.  tau0 = 3: f' = 1/2, f - f(0) = 3/2.  Secant on
    # [0, 3]: 3/(3/2) = 2, f' = 1 >= 0 and f - f(0) = 2/3 above the bound ->
    # [0, 2] and the next trial bisects: 1, f' = 1/2, f - f(0) = -1/6 -> [0, 1].
    # Secant: 1/(3/2) = 2/3, f' = 1/9 > 1/10 -> [0, 2/3].  Secant:
    # (2/3)/(10/9) = 3/5, f' = 1/50: accepted after 5 evaluations.
    "bisect_after_high_right_end": (
        poly((2.0, -0.5, 0.0)), 3.0,
        [(Fr(3), "init"), (Fr(2), "secant"), (Fr(1), "bisect"), (Fr(2, 3), "secant"), (Fr(3, 5), "secant")]),
    # f' = t^2 - 1.  tau0 = 2: f' = 3.  Secant on [0, 2]: 2/4 = 1/2, f' = -3/4
    # < 0 -> [1/2, 2].  Secant: (3/2 + 3/2)/(15/4) = 4/5, f' = -9/25 ->
    # [4/5, 2].  Secant: (12/5 + 18/25)/(84/25) = 13/14, f' = -27/196 ->
    # [13/14, 2].  Secant: (39/14 + 54/196)/(615/196) = 40/41, f' = -81/1681:
    # accepted after 5 evaluations (the left end moves, the right end stays).
    "inside_left_end_moves": (
        poly((0.0, 1.0, 0.0)), 2.0,
        [(Fr(2), "init"), (Fr(1, 2), "secant"), (Fr(4, 5), "secant"), (Fr(13, 14), "secant"),
         (Fr(40, 41), "secant")]),
    # f = -10 - t + t^2/4 (f' = -1 + t/2): tau0 = 1, f' = -1/2.  Secant on
    # [0, 1]: 1/(1/2) = 2 > b, f'(2) = 0: accepted after 2 evaluations.
    "quadratic_exact_secant": (
        poly((0.5, 0.0, 0.0)), 1.0, [(Fr(1), "init"), (Fr(2), "secant")]),
    # the same quadratic from its minimiser: accepted at once
    "accept_tau0": (poly((0.5, 0.0, 0.0)), 2.0, [(Fr(2), "init")]),
}


def _expected_taus(trace):
    return [float(t) for t, _ in trace]


@pytest.mark.parametrize("name", sorted(CASES))
def test_oracle_trace(name):
    ev, tau0, want = CASES[name]
    f0, df0 = ev(0.0)
    assert (f0, df0) == (-10.0, -1.0)
    tr = []
    tau, f, df, _, trials = linesearch.secant_step(lambda t: ev(t) + (None,), f0, df0, tau0, PRM["delta"],
                                                   PRM["sigma"], PRM["gamma"], PRM["eps"], PRM["ls_maxit"], trace=tr)
    assert [w for _, w in tr] == [w for _, w in want]
    assert [t for t, _ in tr] == pytest.approx(_expected_taus(want), rel=1e-14, abs=1e-15)
    assert trials == len(want)
    assert tau == pytest.approx(float(want[-1][0]), rel=1e-14)


def _library():
    from paper_2503_16225_amd import binding
    if not os.path.exists(binding.library_path()):
        pytest.skip("libeahp.so is not built")
    return binding


@pytest.mark.parametrize("name", sorted(CASES))
def test_library_host_control_trace(name):
    binding = _library()
    ev, tau0, want = CASES[name]
    seen = []

    def rec(t):
        seen.append(t)
        return ev(t)
    tau, trials = binding.linesearch_host(rec, -10.0, -1.0, tau0, PRM)
    assert seen == pytest.approx(_expected_taus(want), rel=1e-14, abs=1e-15)
    assert trials == len(want)
    assert tau == pytest.approx(float(want[-1][0]), rel=1e-14)


def test_no_acceptable_step_is_an_error():
    """f = -10 - t (f' = -1 everywhere): equal slopes give midpoints 1/2, 3/4,
    7/8, ... all inside with f' < 0, so the left end creeps towards 1 and no
    point passes the curvature test; the search stops after ls_maxit
    evaluations."""
    def ev(t):
        return -10.0 - t, -1.0
    tr = []
    with pytest.raises(linesearch.LineSearchError):
        linesearch.secant_step(lambda t: ev(t) + (None,), -10.0, -1.0, 1.0, 0.05, 0.1, 0.5, 1e-12, 20, trace=tr)
    assert len(tr) == 20
    assert [t for t, _ in tr[:4]] == [1.0, 0.5, 0.75, 0.875]
    binding = _library()
    seen = []
    with pytest.raises(binding.EahpError) as e:
        binding.linesearch_host(lambda t: (seen.append(t), ev(t))[1], -10.0, -1.0, 1.0, PRM)
    assert e.value.status == -6 and len(seen) == 20 and seen[:4] == [1.0, 0.5, 0.75, 0.875]


def test_library_rejects_non_descent():
    binding = _library()
    with pytest.raises(binding.EahpError) as e:
        binding.linesearch_host(lambda t: (-10.0, 1.0), -10.0, 1.0, 1.0, PRM)
    assert e.value.status == -7
