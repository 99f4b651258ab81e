"""Energy-adaptive Riemannian conjugate gradient (Sec. 4.4, Algorithm 3).

At a point Phi (per k-point where the method is per block):
    Lambda = (Phi^* H Phi) Hermitised,  R = H Phi - Phi Lambda,
    Sigma  = Lambda - mu I  (shift of Prop. 4.4, Sec. 4.3),
    X      = FOM solution of H X - X Sigma = Phi with X0 = Phi / mu (eq. (5.2)),
    G      = Phi - X (Phi^* X)^-1                 (discrete eq. (4.6)).
Iteration: tau from Algorithm 2 started at the previous tau (tau_-1 = 1),
Phi+ = pf(Phi + tau eta), T(eta) by the closed form for xi = tau eta,
T(G) by the Lyapunov form (Prop. 3.1), hybrid FR-PRP beta (Sec. 3.4),
eta+ = -G+ + beta T(eta).

Readings for a seeded random start (the paper starts from a partially
converged SCF state, Sec. 5.2, where Prop. 4.4's coercivity holds):
* while ||R||_F > warm_rtol the shift correction is
  max(mu_warm, lambda_max(Lambda) - min_r V_eff(r) + 1): since
  H >= min V_eff (kinetic and projector terms are non-negative), every
  H - s_l, s_l an eigenvalue of Sigma = Lambda - mu I, is then positive
  definite, the metric is coercive (Remark 4.1 with a uniform bound) and the
  FOM is a Galerkin solve of definite systems; once ||R||_F <= warm_rtol
  the paper's mu is used;
* if f'(0) = <R, eta> >= 0 the direction is reset to -G; if -G is not a
  descent direction either, mu is doubled and G recomputed.
Convergence is measured by ||R||_F (the quantity the paper plots).
"""
from __future__ import annotations

import numpy as np

from . import fom as _fom
from . import hamiltonian as ham
from . import linesearch as _ls
from . import manifold as mf


def metric_solve(model, Phi, HPhi, lams, Veff, mu, prm, stats=None):
    """X of H X - X Sigma = Phi per k with Sigma = Lambda - mu I, X0 = Phi / mu."""
    Xs = []
    alphas = mf.tpa_alpha(model, Phi)
    info_all = []
    for ik, (Pk, Hk) in enumerate(zip(model.blocks(Phi), model.blocks(HPhi))):
        p = Pk.shape[1]
        Sigma = lams[ik] - mu * np.eye(p)
        X0 = Pk / mu
        HX0 = Hk / mu
        kin = model.bases[ik]["kin"]
        al = alphas[ik]
        X, info = _fom.fom(lambda V, ik=ik: ham.apply_H_k(model, ik, Veff, V), Pk, Sigma, X0, HX0,
                           lambda Y: mf.tpa_apply(kin, al, Y), prm["fom_rtol"], prm["fom_maxit"],
                           prm["rank_tol"])
        Xs.append(X)
        info_all.append(info)
    if stats is not None:
        stats["napply"] += sum(i["napply"] for i in info_all)
        stats["fom"].append(info_all)
    return np.concatenate(Xs, axis=0), info_all


def evaluate_point(model, Phi, eta, tau, retraction=0):
    """f(tau), f'(tau) and everything the accepted step reuses."""
    retract, transport_self, _ = mf.retraction_ops(retraction)
    Phin, facs = retract(model, Phi, eta, tau)
    st = mf.state(model, Phin)
    Teta = transport_self(model, Phin, eta, tau, facs)
    df = mf.pair(model, st["R"], Teta)
    st.update(Phi=Phin, facs=facs, Teta=Teta)
    return st["E"], df, st


def earcg(model, Phi0, prm, log=None, maxit=None, callback=None):
    prm = dict(prm)
    maxit = prm["maxit"] if maxit is None else maxit
    p_tot = sum(b.shape[1] for b in model.blocks(Phi0))
    stats = dict(napply=0, fom=[], trials=[], taus=[], rnorm=[], energy=[], betas=[], mus=[])
    Phi = Phi0
    st = mf.state(model, Phi)
    stats["napply"] += p_tot

    def mu_for(rn, st):
        if rn <= prm["warm_rtol"]:
            return prm["mu"]
        lam_max = max(float(np.linalg.eigvalsh(L)[-1]) for L in st["lams"])
        return max(prm["mu_warm"], lam_max - float(st["Veff"].min()) + 1.0)

    def gradient(st, mu):
        X, _ = metric_solve(model, st["Phi"], st["HPhi"], st["lams"], st["Veff"], mu, prm, stats)
        return mf.ea_gradient(model, st["Phi"], X)

    st["Phi"] = Phi
    rn = float(np.linalg.norm(st["R"]))
    mu = mu_for(rn, st)
    G = gradient(st, mu)
    eta = -G
    tau_prev = 1.0
    stats["rnorm"].append(rn)
    stats["energy"].append(st["E"])
    it = 0
    while rn > prm["tol"] and it < maxit:
        df0 = mf.pair(model, st["R"], eta)
        if not df0 < 0.0:
            eta = -G
            df0 = mf.pair(model, st["R"], eta)
            while not df0 < 0.0:
                mu *= 2.0
                G = gradient(st, mu)
                eta = -G
                df0 = mf.pair(model, st["R"], eta)
        tau, f, df, new, trials = _ls.secant_step(
            lambda t: evaluate_point(model, st["Phi"], eta, t, prm.get("retraction", 0)), st["E"], df0, tau_prev,
            prm["delta"], prm["sigma"], prm["gamma"], prm["eps"], prm["ls_maxit"])
        stats["napply"] += trials * p_tot
        stats["trials"].append(trials)
        stats["taus"].append(tau)
        rn = float(np.linalg.norm(new["R"]))
        mu = mu_for(rn, new)
        stats["mus"].append(mu)
        Gn = gradient(new, mu)
        TG = mf.retraction_ops(prm.get("retraction", 0))[2](model, new["Phi"], tau * eta, G, new["facs"])
        rg = mf.pair(model, st["R"], G)
        fr = mf.pair(model, new["R"], Gn) / rg
        prp = mf.pair(model, new["R"], Gn - TG) / rg
        beta = max(0.0, min(fr, prp))
        stats["betas"].append(beta)
        eta = -Gn + beta * new["Teta"]
        G = Gn
        st = new
        tau_prev = tau
        it += 1
        stats["rnorm"].append(rn)
        stats["energy"].append(st["E"])
        if log is not None:
            log(f"it {it:3d} E {st['E']:.12f} |R| {rn:.3e} tau {tau:.3e} beta {beta:.3f} "
                f"trials {trials} fom {[i['iters'] for i in stats['fom'][-1]]} mu {mu}")
        if callback is not None:
            callback(it, st, stats)
    stats["iters"] = it
    return st["Phi"], st, stats
