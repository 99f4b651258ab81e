"""Modified secant step size strategy (Sec. 3.3, Algorithm 2).

Test infrastructure: part of the CPU oracle, never called by the library.

f(t) = E(R_Phi(t eta)),  f'(t) = <r(t), T_{t eta}(eta)>  (eq. (3.6) pairing).

The steps follow the printed algorithm in its order: start from [a, b] =
[0, tau0]; while tau fails the termination test, take the secant point of
f' on [a, b], evaluate f and f' there, then

1. if f(tau) is too high and f'(tau) < 0: tau = gamma b, [a, b] = [0, tau];
2. else if tau < a: tau = b / gamma, [a, b] = [0, tau];
3. else if tau > b: [a, b] = [b, tau];
4. else (a <= tau <= b): keep the half of the bracket where f' changes sign.

Termination test: the approximate Wolfe conditions (eq. (3.8)), read as
Hager-Zhang intend them for negative energies:
    f(t) <= f(0) + eps |f(0)|   and   |f'(t)| <= min(sigma, 1 - 2 delta) |f'(0)|.
The same energy bound decides "too high" in branch 1.

Readings where the printed algorithm is silent or at odds with itself:
* equal slopes in the secant denominator: the midpoint of the bracket;
* "tau = gamma b" / "tau = b / gamma" use the bracket end b before the
  update, and every new tau is evaluated (one H-apply per evaluation), so
  the secant point is evaluated also when it falls left of a, before the
  branches are tested (branch 1 then usually fires: left of 0 along a
  descent direction the energy is above f(0) and still decreasing);
* inside the bracket the printed test keeps [a, tau] when f'(tau) < 0 while
  its comment says the interval where f' changes sign is kept; with f'(a) < 0
  that interval is [a, tau] exactly when f'(tau) >= 0, which is also
  Hager-Zhang's update rule, so [a, tau] is kept when f'(tau) >= 0 and
  [tau, b] otherwise;
* not in the printed algorithm: when that in-bracket point has f'(tau) >= 0
  but an energy above the bound, the next trial is the midpoint of the kept
  bracket [a, tau] instead of a secant point.  The secant recurrence keeps
  one end fixed and, when f' is much larger at b than at a, creeps towards a
  by a tiny step per evaluation (from a random start the first accepted step
  can be ~100, and the next search then needs far more than 20 evaluations);
  the Hager-Zhang search the paper builds on likewise bisects when secant
  steps stop shrinking the bracket;
* at most ``maxit`` evaluations, then an error.
"""
from __future__ import annotations

import math


class LineSearchError(RuntimeError):
    pass


def secant_step(evaluate, f0, df0, tau0, delta, sigma, gamma, eps, maxit=20, trace=None):
    """evaluate(t) -> (f, df, payload).  Returns (tau, f, df, payload, trials).

    trace (a list, optional) receives one (tau, branch) pair per evaluation:
    branch "init" for tau0, "secant" for a secant point (the midpoint when the
    slopes are equal), "bisect" for the midpoint after a too-high in-bracket
    point, "shrink" for gamma b (branch 1), "grow" for b / gamma (branch 2)."""
    c = min(sigma, 1.0 - 2.0 * delta)
    fbound = f0 + eps * abs(f0)

    def ok(f, df):
        return f <= fbound and abs(df) <= c * abs(df0)

    trials = 0

    def ev(t, why):
        nonlocal trials
        if trials >= maxit:
            raise LineSearchError("line search: no acceptable step")
        trials += 1
        if trace is not None:
            trace.append((t, why))
        return evaluate(t)

    a, dfa = 0.0, df0
    b = tau0
    fb, dfb, pb = ev(b, "init")
    tau, ft, dft, pt = b, fb, dfb, pb
    bisect = False
    while not ok(ft, dft):
        den = dfb - dfa
        if bisect:
            tau, why = 0.5 * (a + b), "bisect"
        elif den != 0.0 and math.isfinite(den):
            tau, why = (a * dfb - b * dfa) / den, "secant"
        else:
            tau, why = 0.5 * (a + b), "secant"
        bisect = False
        ft, dft, pt = ev(tau, why)
        if ft > fbound and dft < 0.0:
            tau = gamma * b
            a, dfa = 0.0, df0
            b = tau
            fb, dfb, pb = ev(b, "shrink")
            ft, dft, pt = fb, dfb, pb
        elif tau < a:
            tau = b / gamma
            a, dfa = 0.0, df0
            b = tau
            fb, dfb, pb = ev(b, "grow")
            ft, dft, pt = fb, dfb, pb
        elif tau > b:
            a, dfa = b, dfb
            b, fb, dfb, pb = tau, ft, dft, pt
        elif dft >= 0.0:
            b, fb, dfb, pb = tau, ft, dft, pt
            bisect = ft > fbound
        else:
            a, dfa = tau, dft
    return tau, ft, dft, pt, trials
