"""Modified secant step size strategy (Sec. 3.3, Algorithm 2).

f(t) = E(R_Phi(t eta)),  f'(t) = <r(t), T_{t eta}(eta)>  (eq. (3.6) pairing).

Termination test: the approximate Wolfe conditions (eq. (3.8)), read as
Hager-Zhang intend them for negative energies:
    f(t) <= f(0) + eps |f(0)|   and   |f'(t)| <= min(sigma, 1 - 2 delta) |f'(0)|.

Readings where the printed algorithm is silent or at odds with itself:
* equal slopes in the secant denominator: bisect the bracket;
* "tau = gamma b" / "tau = b / gamma" use the bracket end b before the update,
  and every new tau is evaluated (one H-apply per evaluation);
* inside the bracket the printed test keeps [a, tau] when f'(tau) < 0 while
  its comment says the interval where f' changes sign is kept; with f'(a) < 0
  that interval is [a, tau] exactly when f'(tau) >= 0, which is also
  Hager-Zhang's update rule, so [a, tau] is kept when f'(tau) >= 0 and
  [tau, b] otherwise;
* a secant point left of a (this happens where f is concave, i.e. away
  from the partially converged start the paper uses) is not evaluated: it
  goes straight to the enlargement branch tau = b / gamma;
* when the in-bracket point has f'(tau) >= 0 but an energy above
  f(0) + eps |f(0)|, the kept bracket [a, tau] is bisected on the next trial
  instead of taking a secant step (Hager-Zhang's bisection for a too-high
  energy; without it the secant creeps when f' is small at b);
* at most ``maxit`` evaluations, then an error.
"""
from __future__ import annotations

import math


class LineSearchError(RuntimeError):
    pass


def secant_step(evaluate, f0, df0, tau0, delta, sigma, gamma, eps, maxit=20):
    """evaluate(t) -> (f, df, payload).  Returns (tau, f, df, payload, trials)."""
    c = min(sigma, 1.0 - 2.0 * delta)
    fbound = f0 + eps * abs(f0)

    def ok(f, df):
        return f <= fbound and abs(df) <= c * abs(df0)

    trials = 0

    def ev(t):
        nonlocal trials
        if trials >= maxit:
            raise LineSearchError("line search: no acceptable step")
        trials += 1
        return evaluate(t)

    a, dfa = 0.0, df0
    b = tau0
    fb, dfb, pb = ev(b)
    tau, ft, dft, pt = b, fb, dfb, pb
    bisect = False
    while not ok(ft, dft):
        den = dfb - dfa
        if bisect:
            tn = 0.5 * (a + b)
            bisect = False
        elif den != 0.0 and math.isfinite(den):
            tn = (a * dfb - b * dfa) / den
        else:
            tn = 0.5 * (a + b)
        if tn < a:
            tau = b / gamma
            a, dfa = 0.0, df0
            b = tau
            fb, dfb, pb = ev(b)
            tau, ft, dft, pt = b, fb, dfb, pb
            continue
        fn, dfn, pn = ev(tn)
        if fn > fbound and dfn < 0.0:
            tau = gamma * b
            a, dfa = 0.0, df0
            b = tau
            fb, dfb, pb = ev(b)
            tau, ft, dft, pt = b, fb, dfb, pb
        elif tn > b:
            a, dfa = b, dfb
            b, fb, dfb, pb = tn, fn, dfn, pn
            tau, ft, dft, pt = tn, fn, dfn, pn
        else:
            tau, ft, dft, pt = tn, fn, dfn, pn
            if dfn >= 0.0:
                b, fb, dfb, pb = tn, fn, dfn, pn
                bisect = fn > fbound
            else:
                a, dfa = tn, dfn
    return tau, ft, dft, pt, trials
