"""Stiefel-manifold quantities on the k-point product manifold (FP64).

Discrete forms of Sec. 2.2-4 (outer product V^* W, inner product
Re tr(V^* W), Sec. 5.1) applied per k-point block (product manifold,
eq. (5.1)).  All functions take stacked blocks plus the model's offsets.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import hamiltonian as ham


def blocks(model, X):
    return model.blocks(X)


def pair(model, A, B):
    """<A, B> = sum_k Re tr(A_k^* B_k) (unweighted pairing over k)."""
    return float(np.real(np.vdot(A, B)))


def lam_residual(model, Phi, HPhi):
    """Lambda_k = (M + M^*)/2 with M = Phi_k^* (H Phi)_k (eq. (2.6)) and the
    residual R_k = (H Phi)_k - Phi_k Lambda_k (Sec. 2.2)."""
    lams, R = [], []
    for Pk, Hk in zip(model.blocks(Phi), model.blocks(HPhi)):
        M = Pk.conj().T @ Hk
        L = 0.5 * (M + M.conj().T)
        lams.append(L)
        R.append(Hk - Pk @ L)
    return lams, np.concatenate(R, axis=0)


def eig_herm(M):
    w, V = np.linalg.eigh(0.5 * (M + M.conj().T))
    return w, V


def polar(Psi):
    """Polar factor pf(Psi) = Psi V D^-1/2 V^* and sf(Psi) = V D^1/2 V^*,
    from the eigendecomposition Psi^* Psi = V D V^* (eq. (3.1))."""
    d, V = eig_herm(Psi.conj().T @ Psi)
    if np.any(d <= 0):
        raise np.linalg.LinAlgError("Gram matrix not positive definite")
    isq = (V * d ** -0.5) @ V.conj().T
    sq = (V * d ** 0.5) @ V.conj().T
    return Psi @ isq, sq, d, V


def retract(model, Phi, eta, tau):
    """R_Phi(tau eta) = pf(Phi + tau eta) per k (eq. (3.2)).
    Returns (Phi_new, list of (S, d, V) per k)."""
    outs, facs = [], []
    for Pk, Ek in zip(model.blocks(Phi), model.blocks(eta)):
        Q, S, d, V = polar(Pk + tau * Ek)
        outs.append(Q)
        facs.append((S, d, V))
    return np.concatenate(outs, axis=0), facs


def transport_self(model, Phi_new, eta, tau, facs):
    """Closed form for xi = tau eta (Sec. 3.2):
    T(eta) = eta S^-1 - tau R(tau eta) (eta S^-1)^* (eta S^-1)."""
    out = []
    for Qk, Ek, (S, d, V) in zip(model.blocks(Phi_new), model.blocks(eta), facs):
        Sinv = (V * d ** -0.5) @ V.conj().T
        ES = Ek @ Sinv
        out.append(ES - tau * Qk @ (ES.conj().T @ ES))
    return np.concatenate(out, axis=0)


def transport_general(model, Phi_new, xi, v, facs):
    """Differentiated polar retraction (Prop. 3.1, eqs. (3.3)-(3.4)):
    T_xi(v) = (v - R(xi) X) S^-1 with S X + X S = xi^* v + v^* xi,
    solved in the eigenbasis of S = V D^1/2 V^*."""
    out = []
    for Qk, Xk, Vk, (S, d, V) in zip(model.blocks(Phi_new), model.blocks(xi), model.blocks(v), facs):
        B = Xk.conj().T @ Vk
        B = B + B.conj().T
        s = np.sqrt(d)
        Bt = V.conj().T @ B @ V
        Xt = Bt / (s[:, None] + s[None, :])
        X = V @ Xt @ V.conj().T
        Sinv = (V * d ** -0.5) @ V.conj().T
        out.append((Vk - Qk @ X) @ Sinv)
    return np.concatenate(out, axis=0)


# -- qR retraction (Sec. 3.1 names it as the alternative to the polar one) -----
def qf(Psi):
    """Q factor of Psi = qf(Psi) R with R upper triangular and positive on
    the diagonal (Gram-Schmidt orthonormalisation), from the Cholesky factor
    of Psi^* Psi = R^* R.  Returns (Q, R, R^-1)."""
    p = Psi.shape[1]
    R = np.linalg.cholesky(Psi.conj().T @ Psi).conj().T
    Rinv = sla.solve_triangular(R, np.eye(p), lower=False)
    return Psi @ Rinv, R, Rinv


def retract_qr(model, Phi, eta, tau):
    """R^qr_Phi(tau eta) = qf(Phi + tau eta) per k; factors (R, R^-1) per k."""
    outs, facs = [], []
    for Pk, Ek in zip(model.blocks(Phi), model.blocks(eta)):
        Q, R, Rinv = qf(Pk + tau * Ek)
        outs.append(Q)
        facs.append((R, Rinv))
    return np.concatenate(outs, axis=0), facs


def transport_qr(model, Phi_new, v, facs):
    """Differentiated qR retraction: with psi = Q R and M = Q^* v R^-1,
    D qf(psi)[v] = Q Omega + (I - Q Q^*) v R^-1, where Omega is the
    skew-Hermitian matrix with the strictly lower triangle of M, the negated
    conjugate transpose of it above the diagonal and i Im(M_jj) on the
    diagonal (differentiating psi = Q R with Q^* Q = I and R upper triangular
    with a real diagonal).  Depends only on the new point and its factors."""
    out = []
    for Qk, Vk, (R, Rinv) in zip(model.blocks(Phi_new), model.blocks(v), facs):
        M = Qk.conj().T @ Vk @ Rinv
        L = np.tril(M, -1)
        Om = L - L.conj().T + 1j * np.diag(np.imag(np.diag(M)))
        out.append(Qk @ Om + (Vk - Qk @ (Qk.conj().T @ Vk)) @ Rinv)
    return np.concatenate(out, axis=0)


def retraction_ops(kind):
    """(retract, transport_self, transport_general) of the polar (0) or qR (1)
    retraction, with the signatures of the polar functions."""
    if kind == 1:
        return (retract_qr,
                lambda model, Phi_new, eta, tau, facs: transport_qr(model, Phi_new, eta, facs),
                lambda model, Phi_new, xi, v, facs: transport_qr(model, Phi_new, v, facs))
    return retract, transport_self, transport_general


def tpa_alpha(model, Phi):
    """alpha_jk = sum_G |k+G|^2/2 |phi_jk(G)|^2 (orbital-wise mean kinetic energy)."""
    return [np.sum(b["kin"][:, None] * np.abs(Pk) ** 2, axis=0)
            for b, Pk in zip(model.bases, model.blocks(Phi))]


def tpa_apply(kin, alpha, X):
    """TPA preconditioner P^-1 on column j: x_G / (|k+G|^2/2 + alpha_j) (Sec. 5.1)."""
    return X / (kin[:, None] + alpha[None, :])


def ea_gradient(model, Phi, X):
    """Discrete energy-adaptive gradient G = Phi - X (Phi^* X)^-1 (Sec. 5.2,
    from eq. (4.6)), per k-point."""
    out = []
    for Pk, Xk in zip(model.blocks(Phi), model.blocks(X)):
        M = Pk.conj().T @ Xk
        out.append(Pk - np.linalg.solve(M.T, Xk.T).T)
    return np.concatenate(out, axis=0)


# -- exact energy-adaptive objects (test pins only) -----------------------------
def ea_gradient_exact_dense(Hk, Phik, Sigma):
    """Prop. 4.2 with a dense H: grad = Phi - A^-1(Phi X_Phi) where X_Phi in
    Herm(p) solves <A^-1(Phi X), Phi> + <Phi, A^-1(Phi X)> = 2 I (eq. (4.5)),
    A(v) = H v - v Sigma.  Solved by vectorising the linear map X -> lhs over
    a Hermitian basis (brute force, tiny sizes only)."""
    n, p = Phik.shape
    w, Q = np.linalg.eigh(Hk)
    s, U = np.linalg.eigh(Sigma)

    def Ainv(Y):
        return Q @ ((Q.conj().T @ Y @ U) / (w[:, None] - s[None, :])) @ U.conj().T

    basis = []
    for a in range(p):
        for b in range(a, p):
            E = np.zeros((p, p), complex)
            if a == b:
                E[a, a] = 1.0
                basis.append(E)
            else:
                E[a, b] = 1.0
                E[b, a] = 1.0
                basis.append(E.copy())
                E = np.zeros((p, p), complex)
                E[a, b] = 1j
                E[b, a] = -1j
                basis.append(E)
    cols = []
    for E in basis:
        Z = Ainv(Phik @ E)
        L = Z.conj().T @ Phik + Phik.conj().T @ Z
        cols.append(np.concatenate([L.real.ravel(), L.imag.ravel()]))
    Mat = np.array(cols).T
    rhs = np.concatenate([(2.0 * np.eye(p)).ravel(), np.zeros(p * p)])
    coef, *_ = np.linalg.lstsq(Mat, rhs, rcond=None)
    X = sum(c * E for c, E in zip(coef, basis))
    return Phik - Ainv(Phik @ X)


def sylvester_exact(Hk, Sigma, Phik):
    """Exact X of H X - X Sigma = Phi (eq. (5.2)) via eigendecompositions."""
    w, Q = np.linalg.eigh(Hk)
    s, U = np.linalg.eigh(Sigma)
    Ct = Q.conj().T @ Phik @ U
    Yt = Ct / (w[:, None] - s[None, :])
    return Q @ Yt @ U.conj().T


def state(model, Phi):
    """Energy, density, V_eff, H Phi, Lambda per k and residual at Phi."""
    terms, rho, Veff = ham.energy_terms(model, Phi)
    HPhi = ham.apply_H(model, Veff, Phi)
    lams, R = lam_residual(model, Phi, HPhi)
    return dict(E=terms["total"], terms=terms, rho=rho, Veff=Veff, HPhi=HPhi, lams=lams, R=R)
