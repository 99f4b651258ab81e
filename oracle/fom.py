"""Preconditioned block FOM for H X - X Sigma = Phi (Appendix A, Algorithm 4).

Steps in the paper's order, per k-point:

    C   = Phi - (H X0 - X0 Sigma)
    V_1 = unitary factor of a rank-revealing QR of P^-1 C
    W_1 = H V_1,  A_1 = V_1^* W_1,  C_1 = V_1^* C
    loop j = 1, 2, ...
        solve A_j Y - Y Sigma = C_j
        E_j = C - (W_j Y - V_j Y Sigma)        (= -(H X_j - X_j Sigma - Phi))
        stop when ||E_j||_F / ||C||_F <= rtol (Sec. 5.2 stopping rule)
        R_j = (I - V_j V_j^*) P^-1 E_j
        V~ = unitary factor of a rank-revealing QR of R_j
        append V~ to V and H V~ to W, border A with V_j^* H V~ and V~^* H V~,
        C_{j+1} = [C_j ; V~^* C]
    return X_j = X0 + V_j Y_j

Readings: the projection (I - V V^*) is applied twice (classical
Gram-Schmidt, repeated once, equal in exact arithmetic); the rank-revealing
QR is scipy's column-pivoted QR and drops directions with
|R_ii| < rank_tol * |R_00|; the appended block of C uses the new basis block
(V~_{j+1}^* C).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def rrqr(R, rank_tol):
    if R.shape[1] == 0:
        return R[:, :0]
    Q, T, piv = sla.qr(R, mode="economic", pivoting=True)
    d = np.abs(np.diag(T))
    if d.size == 0 or d[0] == 0.0:
        return R[:, :0]
    r = int(np.sum(d > rank_tol * d[0]))
    return Q[:, :r]


def solve_projected(A, Sigma, C):
    """A Y - Y Sigma = C for Hermitian A, Sigma (eigendecompositions)."""
    w, Q = np.linalg.eigh(0.5 * (A + A.conj().T))
    s, U = np.linalg.eigh(0.5 * (Sigma + Sigma.conj().T))
    Ct = Q.conj().T @ C @ U
    Yt = Ct / (w[:, None] - s[None, :])
    return Q @ Yt @ U.conj().T


def fom(applyH, Phi, Sigma, X0, HX0, precond, rtol, maxit=50, rank_tol=1e-7):
    """Returns (X, info) with info = dict(iters, relres, napply (columns), q)."""
    C = Phi - (HX0 - X0 @ Sigma)
    nC = np.linalg.norm(C)
    napply = 0
    V = rrqr(precond(C), rank_tol)
    W = applyH(V)
    napply += V.shape[1]
    A = V.conj().T @ W
    Cj = V.conj().T @ C
    it = 0
    relres = np.inf
    while True:
        it += 1
        Y = solve_projected(A, Sigma, Cj)
        E = C - (W @ Y - V @ Y @ Sigma)
        relres = np.linalg.norm(E) / nC if nC > 0 else 0.0
        if relres <= rtol or it >= maxit:
            break
        Rj = precond(E)
        Rj = Rj - V @ (V.conj().T @ Rj)
        Rj = Rj - V @ (V.conj().T @ Rj)
        Vt = rrqr(Rj, rank_tol)
        if Vt.shape[1] == 0:
            break
        Wt = applyH(Vt)
        napply += Vt.shape[1]
        H12 = V.conj().T @ Wt
        H22 = Vt.conj().T @ Wt
        A = np.block([[A, H12], [H12.conj().T, H22]])
        Cj = np.concatenate([Cj, Vt.conj().T @ C], axis=0)
        V = np.concatenate([V, Vt], axis=1)
        W = np.concatenate([W, Wt], axis=1)
    X = X0 + V @ Y
    return X, dict(iters=it, relres=relres, napply=napply, q=V.shape[1])
