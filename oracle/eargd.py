"""Energy-adaptive Riemannian gradient descent (EARGD), the gradient-descent
sibling of EARCG that the paper compares against (Sec. 5.2, list of methods;
Sec. 1 introduces it as the method EARCG builds on).

Test infrastructure only: called by tests/ and never by the product path.

The paper names its ingredients (the energy-adaptive gradient of Sec. 4 as
the search direction, a Barzilai-Borwein step size and non-monotone
backtracking) but does not print the step rule.  Readings (also in the design
notes, A28-A31):

* A28 direction and shift: d = -G with G the energy-adaptive gradient of
  eq. (4.6) from the metric solve of Algorithm 4, with the same shift rule as
  EARCG (warm shift while ||R||_F > warm_rtol, then mu; mu doubled while d is
  not a descent direction);
* A29 Barzilai-Borwein step from ambient differences of consecutive iterates,
  S = Phi_k - Phi_{k-1} and Y = G_k - G_{k-1}, with the unweighted pairing
  <A, B> = sum_k Re tr(A_k^* B_k):  tau = <S,S>/|<S,Y>| on odd iterations and
  |<S,Y>|/<Y,Y> on even ones (alternating long and short steps), clamped to
  [tau_min, tau_max]; the first iteration tries tau = 1 (the natural step of
  an energy-adaptive metric, whose gradient is Newton-like); <S,Y> = 0 keeps
  the previous accepted step;
* A30 non-monotone backtracking in the Zhang-Hager form: a trial tau is
  accepted when E(R_Phi(tau d)) <= C_k + rho tau dE_k (R the polar
  retraction, or the qR one when selected), with dE_k the
  derivative of the energy along d (C11: 2 f sum_k w_k Re tr(R_k^* d_k)),
  otherwise tau <- delta tau; C_0 = E_0, Q_0 = 1, Q_{k+1} = theta Q_k + 1,
  C_{k+1} = (theta Q_k C_k + E_{k+1}) / Q_{k+1};
* A31 constants rho = 1e-4, delta = 0.5, theta = 0.85, tau_min = 1e-10,
  tau_max = 1e10, at most ls_maxit energy evaluations per iteration.

Cost model: a trial costs one energy evaluation (density and energy, no
H-apply); the accepted point then needs H Phi (p H-applies per k) for its
residual, plus the metric solve's H-applies.
"""
from __future__ import annotations

import numpy as np

from . import earcg as _earcg
from . import hamiltonian as ham
from . import manifold as mf

TAU_MIN = 1e-10
TAU_MAX = 1e10


class BacktrackError(RuntimeError):
    pass


def energy_slope(model, R, d):
    """dE/dtau at tau = 0 along the tangent d: 2 f sum_k w_k Re tr(R_k^* d_k) (C11)."""
    s = 0.0
    for w, Rk, dk in zip(model.kw, model.blocks(R), model.blocks(d)):
        s += w * float(np.real(np.vdot(Rk, dk)))
    return 2.0 * model.occ * s


def bb_step(S, Y, k, tau_prev):
    """Alternating Barzilai-Borwein step of iteration k >= 1 (A29)."""
    sy = abs(float(np.real(np.vdot(S, Y))))
    if sy == 0.0:
        return tau_prev
    if k % 2 == 1:
        tau = float(np.real(np.vdot(S, S))) / sy
    else:
        tau = sy / float(np.real(np.vdot(Y, Y)))
    return min(max(tau, TAU_MIN), TAU_MAX)


def eargd(model, Phi0, prm, log=None, maxit=None, callback=None):
    """Returns (Phi, state, stats); stats holds per-iteration energies, ||R||_F,
    accepted steps, trial counts and the reference values C_k."""
    prm = dict(prm)
    maxit = prm["maxit"] if maxit is None else maxit
    rho, delta, theta = prm["nm_rho"], prm["nm_backtrack"], prm["nm_theta"]
    p_tot = sum(b.shape[1] for b in model.blocks(Phi0))
    stats = dict(napply=0, fom=[], trials=[], taus=[], rnorm=[], energy=[], mus=[], C=[], slopes=[])

    def mu_for(rn, st):
        if rn <= prm["warm_rtol"]:
            return prm["mu"]
        lam_max = max(float(np.linalg.eigvalsh(L)[-1]) for L in st["lams"])
        return max(prm["mu_warm"], lam_max - float(st["Veff"].min()) + 1.0)

    def gradient(st, mu):
        X, _ = _earcg.metric_solve(model, st["Phi"], st["HPhi"], st["lams"], st["Veff"], mu, prm, stats)
        return mf.ea_gradient(model, st["Phi"], X)

    Phi = Phi0
    st = mf.state(model, Phi)
    st["Phi"] = Phi
    stats["napply"] += p_tot
    rn = float(np.linalg.norm(st["R"]))
    mu = mu_for(rn, st)
    G = gradient(st, mu)
    C, Q = st["E"], 1.0
    tau_prev = 1.0
    Phi_old = G_old = None
    stats["rnorm"].append(rn)
    stats["energy"].append(st["E"])
    stats["C"].append(C)
    it = 0
    while rn > prm["tol"] and it < maxit:
        d = -G
        dE = energy_slope(model, st["R"], d)
        while not dE < 0.0:
            mu *= 2.0
            G = gradient(st, mu)
            d = -G
            dE = energy_slope(model, st["R"], d)
        tau = 1.0 if it == 0 else bb_step(st["Phi"] - Phi_old, G - G_old, it, tau_prev)
        trials = 0
        while True:
            if trials >= prm["ls_maxit"]:
                raise BacktrackError("no acceptable step")
            trials += 1
            Phin, _ = mf.retraction_ops(prm.get("retraction", 0))[0](model, st["Phi"], d, tau)
            En = ham.energy_terms(model, Phin)[0]["total"]
            if En <= C + rho * tau * dE:
                break
            tau *= delta
        new = mf.state(model, Phin)
        new["Phi"] = Phin
        stats["napply"] += p_tot
        stats["trials"].append(trials)
        stats["taus"].append(tau)
        stats["slopes"].append(dE)
        Qn = theta * Q + 1.0
        C = (theta * Q * C + new["E"]) / Qn
        Q = Qn
        rn = float(np.linalg.norm(new["R"]))
        mu = mu_for(rn, new)
        stats["mus"].append(mu)
        Phi_old, G_old = st["Phi"], G
        G = gradient(new, mu)
        st = new
        tau_prev = tau
        it += 1
        stats["rnorm"].append(rn)
        stats["energy"].append(st["E"])
        stats["C"].append(C)
        if log is not None:
            log(f"it {it:3d} E {st['E']:.12f} |R| {rn:.3e} tau {tau:.3e} trials {trials} C {C:.12f} mu {mu}")
        if callback is not None:
            callback(it, st, stats)
    stats["iters"] = it
    return st["Phi"], st, stats
