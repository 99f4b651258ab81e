"""Dense self-consistent-field ground state (a pin, not the method).

Fixed point of rho -> rho[lowest p eigenvectors of the dense H(rho) per k]
(the NLEVP of eq. (1.3) with the Aufbau principle, Sec. 2.1), with Anderson
mixing on the density.  Uses the explicit G-space Hamiltonian of
``hamiltonian.dense_H`` (direct convolution), so it shares no FFT H-apply
with the method's path.
"""
from __future__ import annotations

import numpy as np

from . import hamiltonian as ham


def scf(model, tol=1e-12, maxit=300, beta=0.5, depth=6, rho0=None, Phi0=None):
    if rho0 is None:
        rho0 = ham.density(model, Phi0)
    rho = rho0
    hist_x, hist_f = [], []
    eigs = None
    Phi = None
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
        if res < tol:
            break
        hist_x.append(rho.ravel().copy())
        hist_f.append(f.ravel().copy())
        hist_x, hist_f = hist_x[-depth:], hist_f[-depth:]
        if len(hist_f) > 1:
            dF = np.array([hist_f[i + 1] - hist_f[i] for i in range(len(hist_f) - 1)]).T
            dX = np.array([hist_x[i + 1] - hist_x[i] for i in range(len(hist_x) - 1)]).T
            g, *_ = np.linalg.lstsq(dF, f.ravel(), rcond=None)
            xb = rho.ravel() - dX @ g
            fb = f.ravel() - dF @ g
            rho = (xb + beta * fb).reshape(model.fft)
        else:
            rho = rho + beta * f
    E = ham.energy(model, Phi)
    gaps = [float(w[model.p] - w[model.p - 1]) for w in eigs]
    return dict(E=E, Phi=Phi, eigs=eigs, iters=it, res=res, gap=min(gaps))
