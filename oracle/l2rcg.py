"""Unpreconditioned L2-gradient Riemannian CG (L2RCG), the comparison method
of Sec. 5.2 that shows what the energy-adaptive metric buys.

Test infrastructure only: called by tests/ and never by the product path.

The paper names it (RCG with the L2 Riemannian gradient, no preconditioner,
an approximated-Hessian step size from a cited work) without printing the
step rule.  Readings (also in the design notes, A33-A34):

* A33 Algorithm 3 with the energy-adaptive gradient G replaced by the L2
  gradient R = H Phi - Phi Lambda (no metric solve, no preconditioner):
  eta_0 = -R_0, eta+ = -R+ + beta T_{tau eta}(eta) with the hybrid
  beta = max(0, min(FR, PRP)), FR = <R+, R+>/<R, R>, PRP = <R+, R+ - T(R)>/<R, R>
  (unweighted pairing), transports of the retraction in use; eta is reset to
  -R when <R, eta> >= 0;
* A34 step size: the minimiser of the quadratic model of the energy along
  the retraction curve with the Hessian approximated by the frozen-potential
  (band-energy) part, tau_H = -dE / h with
  dE = 2 f sum_k w_k Re tr(R_k^* eta_k) and
  h = 2 f sum_k w_k Re tr(eta_k^* (H eta_k - eta_k Lambda_k)),
  the previous accepted step when h <= 0; safeguarded by the non-monotone
  backtracking of EARGD (A30, A31) with energy-only trials.

Cost model: H eta (p H-applies per k) for h, energy-only trials, H Phi of the
accepted point.
"""
from __future__ import annotations

import numpy as np

from . import eargd as _gd
from . import hamiltonian as ham
from . import manifold as mf


def hessian_curvature(model, Veff, Phi, lams, eta):
    """h = 2 f sum_k w_k Re tr(eta_k^* (H eta_k - eta_k Lambda_k)) with H at V_eff."""
    Heta = ham.apply_H(model, Veff, eta)
    s = 0.0
    for w, Ek, HEk, L in zip(model.kw, model.blocks(eta), model.blocks(Heta), lams):
        s += w * float(np.real(np.vdot(Ek, HEk - Ek @ L)))
    return 2.0 * model.occ * s


def l2rcg(model, Phi0, prm, log=None, maxit=None, callback=None):
    prm = dict(prm)
    maxit = prm["maxit"] if maxit is None else maxit
    rho, delta, theta = prm["nm_rho"], prm["nm_backtrack"], prm["nm_theta"]
    retract, transport_self, transport_general = mf.retraction_ops(prm.get("retraction", 0))
    p_tot = sum(b.shape[1] for b in model.blocks(Phi0))
    stats = dict(napply=0, trials=[], taus=[], rnorm=[], energy=[], C=[], slopes=[], betas=[], curv=[])
    st = mf.state(model, Phi0)
    st["Phi"] = Phi0
    stats["napply"] += p_tot
    rn = float(np.linalg.norm(st["R"]))
    eta = -st["R"]
    C, Q = st["E"], 1.0
    tau_prev = 1.0
    stats["rnorm"].append(rn)
    stats["energy"].append(st["E"])
    stats["C"].append(C)
    it = 0
    while rn > prm["tol"] and it < maxit:
        if not mf.pair(model, st["R"], eta) < 0.0:
            eta = -st["R"]
        dE = _gd.energy_slope(model, st["R"], eta)
        h = hessian_curvature(model, st["Veff"], st["Phi"], st["lams"], eta)
        stats["napply"] += p_tot
        tau = -dE / h if h > 0.0 else tau_prev
        tau = min(max(tau, _gd.TAU_MIN), _gd.TAU_MAX)
        trials = 0
        while True:
            if trials >= prm["ls_maxit"]:
                raise _gd.BacktrackError("no acceptable step")
            trials += 1
            Phin, facs = retract(model, st["Phi"], eta, tau)
            En = ham.energy_terms(model, Phin)[0]["total"]
            if En <= C + rho * tau * dE:
                break
            tau *= delta
        new = mf.state(model, Phin)
        new["Phi"] = Phin
        stats["napply"] += p_tot
        Qn = theta * Q + 1.0
        C = (theta * Q * C + new["E"]) / Qn
        Q = Qn
        Teta = transport_self(model, Phin, eta, tau, facs)
        TR = transport_general(model, Phin, tau * eta, st["R"], facs)
        rr = mf.pair(model, st["R"], st["R"])
        fr = mf.pair(model, new["R"], new["R"]) / rr
        prp = mf.pair(model, new["R"], new["R"] - TR) / rr
        beta = max(0.0, min(fr, prp))
        eta = -new["R"] + beta * Teta
        stats["trials"].append(trials)
        stats["taus"].append(tau)
        stats["slopes"].append(dE)
        stats["curv"].append(h)
        stats["betas"].append(beta)
        st = new
        tau_prev = tau
        rn = float(np.linalg.norm(st["R"]))
        it += 1
        stats["rnorm"].append(rn)
        stats["energy"].append(st["E"])
        stats["C"].append(C)
        if log is not None:
            log(f"it {it:3d} E {st['E']:.12f} |R| {rn:.3e} tau {tau:.3e} beta {beta:.3f} trials {trials}")
        if callback is not None:
            callback(it, st, stats)
    stats["iters"] = it
    return st["Phi"], st, stats
