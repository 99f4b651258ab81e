"""Dense self-consistent-field ground state: a pin of the minimisers, and
the oracle of the SCF comparison method (Sec. 5.2), whose GPU form replaces
the dense diagonalisation by a block eigensolver.

Fixed point of rho -> rho[lowest p eigenvectors of the dense H(rho) per k]
(the NLEVP of eq. (1.3) with the Aufbau principle, Sec. 2.1), with Anderson
mixing on the density.  Uses the explicit G-space Hamiltonian of
``hamiltonian.dense_H`` (direct convolution), so it shares no FFT H-apply
with the method's path.
"""
from __future__ import annotations

import numpy as np

from . import hamiltonian as ham


def anderson_next(hist_x, hist_f, beta):
    """Next iterate of Anderson mixing from the history (oldest first) of
    iterates x_i and residuals f_i = g(x_i) - x_i: with dX, dF the differences
    of consecutive entries and gamma the least-squares solution of dF gamma = f,
    x - dX gamma + beta (f - dF gamma); with one entry x + beta f."""
    x, f = hist_x[-1], hist_f[-1]
    if len(hist_f) < 2:
        return x + beta * f
    dF = np.array([hist_f[i + 1] - hist_f[i] for i in range(len(hist_f) - 1)]).T
    dX = np.array([hist_x[i + 1] - hist_x[i] for i in range(len(hist_x) - 1)]).T
    g, *_ = np.linalg.lstsq(dF, f, rcond=None)
    return (x - dX @ g) + beta * (f - dF @ g)


def scf(model, tol=1e-12, maxit=300, beta=0.5, depth=6, rho0=None, Phi0=None):
    if rho0 is None:
        rho0 = ham.density(model, Phi0)
    rho = rho0
    hist_x, hist_f = [], []
    eigs = None
    Phi = None
    res_hist = []
    for it in range(maxit):
        Veff, _ = ham.potentials(model, rho)
        blocks, eigs = [], []
        for ik in range(len(model.bases)):
            H = ham.dense_H(model, ik, Veff)
            w, V = np.linalg.eigh(H)
            blocks.append(V[:, :model.p])
            eigs.append(w)
        Phi = np.concatenate(blocks, axis=0)
        rho_out = ham.density(model, Phi)
        f = rho_out - rho
        res = np.linalg.norm(f) * np.sqrt(model.Omega / model.Ng)
        res_hist.append(res)
        if res < tol:
            break
        hist_x.append(rho.ravel().copy())
        hist_f.append(f.ravel().copy())
        hist_x, hist_f = hist_x[-depth:], hist_f[-depth:]
        rho = anderson_next(hist_x, hist_f, beta).reshape(model.fft)
    E = ham.energy(model, Phi)
    gaps = [float(w[model.p] - w[model.p - 1]) for w in eigs]
    return dict(E=E, Phi=Phi, eigs=eigs, iters=it, res=res, gap=min(gaps), res_hist=res_hist)
