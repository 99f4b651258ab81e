"""Plane-wave basis (Sec. 5.1, plane-wave discretization).

Conventions (readings, the paper gives the discretization only in words):

* lattice columns a_i, reciprocal columns b_i with a_i . b_j = 2 pi delta_ij,
  cell volume Omega = |det A|;
* G(m) = B m for integer m, k = B u for fractional u;
* the basis at k is {m : |k + G(m)|^2 / 2 <= Ecut};
* FFT box n = (n1, n2, n3); the box index of m is i_d = m_d mod n_d and the
  linear box index is (i1 * n2 + i2) * n3 + i3;
* canonical order of the basis = ascending linear box index;
* a box index i corresponds to the frequency i for i < (n+1)//2 and i - n
  otherwise (numpy's fftfreq convention).
"""
from __future__ import annotations

import numpy as np


def reciprocal(lattice):
    lattice = np.asarray(lattice, float)
    return 2.0 * np.pi * np.linalg.inv(lattice).T


def volume(lattice):
    return abs(float(np.linalg.det(np.asarray(lattice, float))))


def freq(n):
    i = np.arange(n)
    return np.where(i < (n + 1) // 2, i, i - n)


def smooth_size(nmin):
    """Smallest n >= nmin whose only prime factors are 2, 3 and 5."""
    n = max(int(nmin), 1)
    while True:
        m = n
        for f in (2, 3, 5):
            while m % f == 0:
                m //= f
        if m == 1:
            return n
        n += 1


def auto_fft(lattice, kfrac, ecut):
    """Smallest 2/3/5-smooth n_d >= 4 * max|m_d| + 1 over all basis sets."""
    B = reciprocal(lattice)
    mmax = np.zeros(3, dtype=int)
    for u in np.atleast_2d(kfrac):
        m = _sphere_m(B, B @ u, ecut)
        mmax = np.maximum(mmax, np.abs(m).max(axis=0))
    return tuple(smooth_size(4 * int(x) + 1) for x in mmax)


def _sphere_m(B, k, ecut):
    gmax = np.sqrt(2.0 * ecut)
    # |m_d| is bounded by (gmax + |k|) * |row d of B^-1| ... use a safe cube
    Binv = np.linalg.inv(B)
    lim = [int(np.ceil((gmax + np.linalg.norm(k)) * np.linalg.norm(Binv[d]))) + 1 for d in range(3)]
    r = [np.arange(-l, l + 1) for l in lim]
    M = np.stack(np.meshgrid(*r, indexing="ij"), axis=-1).reshape(-1, 3)
    q = M @ B.T + k[None, :]
    keep = 0.5 * np.sum(q * q, axis=1) <= ecut
    return M[keep]


def basis(lattice, u, ecut, fft):
    """Basis at fractional k-point u.

    Returns dict with integer triples ``m`` (n x 3, canonical order), box
    indices ``box`` (n,), kinetic energies ``kin`` = |k+G|^2/2 and the
    Cartesian ``kG`` = k + G.
    """
    B = reciprocal(lattice)
    k = B @ np.asarray(u, float)
    M = _sphere_m(B, k, ecut)
    n = np.array(fft)
    i = np.mod(M, n[None, :])
    lin = (i[:, 0] * n[1] + i[:, 1]) * n[2] + i[:, 2]
    order = np.argsort(lin, kind="stable")
    M, lin = M[order], lin[order]
    if np.any(np.abs(M) * 2 >= n[None, :]):
        raise ValueError("FFT box too small for the basis")
    kG = M @ B.T + k[None, :]
    kin = 0.5 * np.sum(kG * kG, axis=1)
    return dict(m=M, box=lin, kin=kin, kG=kG, k=k)


def box_G(lattice, fft):
    """Cartesian G vectors for every box index (shape n1 x n2 x n3 x 3)."""
    B = reciprocal(lattice)
    f = [freq(n) for n in fft]
    M = np.stack(np.meshgrid(*f, indexing="ij"), axis=-1)
    return M @ B.T
