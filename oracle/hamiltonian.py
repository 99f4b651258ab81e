"""Kohn-Sham energy and Hamiltonian in the plane-wave basis (FP64).

The paper's energy functional (eq. (1.1)) and Hamiltonian (eq. (1.4)) are
used in the Hartree scaling of its experiments, H = -1/2 Laplacian + V_eff
(Sec. 5.1, TPA paragraph), with doubly occupied orbitals:

    E = sum_k w_k f [ sum_i sum_G |k+G|^2/2 |c_iG|^2 + sum_{i,I} D_I |<beta_I, psi_i>|^2 ]
        + (Omega/N_g) sum_r [ V_ion rho + V_H rho / 2 + e_x(rho) ](r)

    rho(r) = sum_k w_k f sum_i |psi_ik(r)|^2,   psi(r) = Omega^-1/2 sum_G c_G e^{i(k+G).r}

Readings (the model of the experiments is DFTK's LDA; it is replaced by
synthetic analytic terms):
* V_ion(G) = sum_I -4 pi Z_I exp(-|G|^2 r^2/2) / (Omega |G|^2) e^{-i G.R_I},
  G = 0 value sum_I 2 pi Z_I r^2 / Omega (the finite non-Coulomb limit);
* V_H(G) = 4 pi rho^(G) / |G|^2, V_H(0) = 0 (neutralising background);
* Slater exchange e_x = -3/4 (3/pi)^(1/3) rho^(4/3), V_x = -(3 rho/pi)^(1/3);
* one normalised Gaussian s-projector per atom,
  beta_I(k+G) = Omega^-1/2 2^(3/2) pi^(3/4) r_p^(3/2) exp(-|k+G|^2 r_p^2/2) e^{-i(k+G).R_I},
  with coupling D_I;
* on the grid the Bloch factor e^{ik.r} is dropped (it cancels in |psi|^2
  and in the V psi round trip).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from . import basis as _basis
from . import symmetry as _sym

TERM_ION, TERM_HARTREE, TERM_XC, TERM_NONLOCAL = 1, 2, 4, 8


class Model:
    """Static part of a problem: bases per k, V_ion on the grid, projectors."""

    def __init__(self, sysd, workers=None):
        self.sys = sysd
        self.workers = workers
        lat = sysd["lattice"]
        self.lattice = lat
        self.Omega = _basis.volume(lat)
        fft = sysd.get("fft")
        if fft is None or any(int(x) == 0 for x in fft):
            fft = _basis.auto_fft(lat, sysd["kfrac"], sysd["ecut"])
        self.fft = tuple(int(x) for x in fft)
        self.Ng = int(np.prod(self.fft))
        self.kw = np.asarray(sysd["kweight"], float)
        self.occ = float(sysd["occ"])
        self.p = int(sysd["p"])
        self.terms = int(sysd.get("terms", 15))
        self.bases = [_basis.basis(lat, u, sysd["ecut"], self.fft) for u in np.atleast_2d(sysd["kfrac"])]
        self.npw = [len(b["box"]) for b in self.bases]
        self.offsets = np.concatenate([[0], np.cumsum(self.npw)])
        self.Gbox = _basis.box_G(lat, self.fft)
        self.G2 = np.sum(self.Gbox ** 2, axis=-1)
        self.R = np.asarray(sysd["frac"], float) @ np.asarray(lat, float).T
        self.Vion_r = self._vion() if self.terms & TERM_ION else np.zeros(self.fft)
        self.proj = [self._projectors(b) for b in self.bases]
        rot = sysd.get("sym_rot")
        self.sym = [] if rot is None else [(np.asarray(W, dtype=np.int64).reshape(3, 3), np.asarray(t, float))
                                           for W, t in zip(rot, sysd["sym_trans"])]

    # -- static potentials -------------------------------------------------
    def _vion(self):
        r = self.sys["r_loc"]
        Z = self.sys["Z"]
        G2 = self.G2
        Vg = np.zeros(self.fft, dtype=complex)
        nz = G2 > 0
        for I in range(len(Z)):
            phase = np.exp(-1j * (self.Gbox @ self.R[I]))
            f = np.zeros(self.fft)
            f[nz] = -4.0 * np.pi * Z[I] * np.exp(-0.5 * G2[nz] * r * r) / (self.Omega * G2[nz])
            f[~nz] = 2.0 * np.pi * Z[I] * r * r / self.Omega
            Vg += f * phase
        return self.g_to_r_real(Vg)

    def _projectors(self, b):
        if not (self.terms & TERM_NONLOCAL):
            return np.zeros((len(b["box"]), 0), dtype=complex), np.zeros(0)
        rp = self.sys["r_proj"]
        kG = b["kG"]
        q2 = np.sum(kG * kG, axis=1)
        amp = self.Omega ** -0.5 * 2 ** 1.5 * np.pi ** 0.75 * rp ** 1.5 * np.exp(-0.5 * q2 * rp * rp)
        P = amp[:, None] * np.exp(-1j * (kG @ self.R.T))
        D = np.full(len(self.R), self.sys["D_proj"])
        return P, D

    # -- grid transforms -----------------------------------------------------
    def g_to_r_real(self, Vg):
        """V(r) = Re sum_{G in box} V(G) e^{iG.r} on the grid."""
        return np.real(sfft.ifftn(Vg, workers=self.workers)) * self.Ng

    def to_grid(self, ik, c):
        """psi~(r) = sum_G c_G e^{iG.r} for each column of c (unnormalised)."""
        b = self.bases[ik]
        nb = c.shape[1]
        box = np.zeros((nb, self.Ng), dtype=complex)
        box[:, b["box"]] = c.T
        box = box.reshape((nb,) + self.fft)
        return sfft.ifftn(box, axes=(1, 2, 3), workers=self.workers) * self.Ng

    def from_grid(self, ik, f):
        """Coefficients (1/N_g) sum_r f(r) e^{-iG.r} at the basis G's."""
        b = self.bases[ik]
        nb = f.shape[0]
        F = sfft.fftn(f, axes=(1, 2, 3), workers=self.workers) / self.Ng
        return F.reshape(nb, self.Ng)[:, b["box"]].T

    def blocks(self, Phi):
        return [Phi[self.offsets[i]:self.offsets[i + 1]] for i in range(len(self.bases))]


# -- density and potentials ----------------------------------------------------
def density(model, Phi, chunk=None):
    """rho(r_j) = sum_k w_k f sum_i |psi_ik(r_j)|^2 (columns taken `chunk` at a
    time when given, which bounds the memory of the grid values); averaged over
    the symmetry operations when the k-point set is a reduced one (A38)."""
    rho = np.zeros(model.fft)
    for ik, c in enumerate(model.blocks(Phi)):
        step = c.shape[1] if chunk is None else chunk
        for j0 in range(0, c.shape[1], step):
            psi = model.to_grid(ik, c[:, j0:j0 + step])
            rho += model.kw[ik] * model.occ * np.sum(np.abs(psi) ** 2, axis=0) / model.Omega
    if len(model.sym) > 1:
        rho = _sym.symmetrize(rho, model.sym)
    return rho


def slater(rho):
    """(e_x, V_x) of Slater exchange for rho clamped at >= 0."""
    r = np.maximum(rho, 0.0)
    c = (3.0 / np.pi) ** (1.0 / 3.0)
    return -0.75 * c * r ** (4.0 / 3.0), -c * r ** (1.0 / 3.0)


def hartree(model, rho):
    """V_H(r) with V_H(G) = 4 pi rho^(G)/|G|^2, rho^(G) = N_g^-1 sum_r rho e^{-iG.r}."""
    rg = sfft.fftn(rho, workers=model.workers) / model.Ng
    G2 = model.G2
    Vg = np.zeros_like(rg)
    nz = G2 > 0
    Vg[nz] = 4.0 * np.pi * rg[nz] / G2[nz]
    return model.g_to_r_real(Vg)


def potentials(model, rho):
    """(V_eff, parts) with parts = dict(Vion, VH, Vx, ex)."""
    VH = hartree(model, rho) if model.terms & TERM_HARTREE else np.zeros(model.fft)
    if model.terms & TERM_XC:
        ex, Vx = slater(rho)
    else:
        ex, Vx = np.zeros(model.fft), np.zeros(model.fft)
    Veff = model.Vion_r + VH + Vx
    return Veff, dict(Vion=model.Vion_r, VH=VH, Vx=Vx, ex=ex)


# -- Hamiltonian ---------------------------------------------------------------
def apply_H_k(model, ik, Veff, X):
    """(H X)_G = |k+G|^2/2 X_G + [V_eff X](G) + sum_I D_I beta_I(G) <beta_I, X>."""
    b = model.bases[ik]
    out = b["kin"][:, None] * X
    psi = model.to_grid(ik, X)
    out = out + model.from_grid(ik, psi * Veff[None])
    P, D = model.proj[ik]
    if P.shape[1]:
        out = out + P @ (D[:, None] * (P.conj().T @ X))
    return out


def apply_H(model, Veff, X):
    return np.concatenate([apply_H_k(model, ik, Veff, Xk) for ik, Xk in enumerate(model.blocks(X))], axis=0)


def dense_H(model, ik, Veff):
    """Explicit matrix H_GG' = kin delta + V^(G - G') + sum_I D_I beta_I(G) beta_I(G')^*,
    with V^ taken at the box index of m - m' (direct convolution, no FFT of psi)."""
    b = model.bases[ik]
    Vg = sfft.fftn(Veff) / model.Ng
    n = np.array(model.fft)
    dm = np.mod(b["m"][:, None, :] - b["m"][None, :, :], n)
    H = Vg[dm[..., 0], dm[..., 1], dm[..., 2]]
    H = H + np.diag(b["kin"])
    P, D = model.proj[ik]
    if P.shape[1]:
        H = H + (P * D[None, :]) @ P.conj().T
    return H


# -- energy --------------------------------------------------------------------
def energy_terms(model, Phi, rho=None):
    if rho is None:
        rho = density(model, Phi)
    Veff, parts = potentials(model, rho)
    dv = model.Omega / model.Ng
    ekin = 0.0
    enl = 0.0
    for ik, c in enumerate(model.blocks(Phi)):
        b = model.bases[ik]
        wf = model.kw[ik] * model.occ
        ekin += wf * float(np.sum(b["kin"][:, None] * np.abs(c) ** 2))
        P, D = model.proj[ik]
        if P.shape[1]:
            enl += wf * float(np.sum(D[:, None] * np.abs(P.conj().T @ c) ** 2))
    eion = dv * float(np.sum(parts["Vion"] * rho))
    eh = dv * 0.5 * float(np.sum(parts["VH"] * rho))
    exc = dv * float(np.sum(parts["ex"]))
    return dict(kin=ekin, nl=enl, ion=eion, hartree=eh, xc=exc,
                total=ekin + enl + eion + eh + exc), rho, Veff


def energy(model, Phi):
    return energy_terms(model, Phi)[0]["total"]
