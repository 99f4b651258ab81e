"""Crystal symmetry, symmetry-reduced k-point sets and density symmetrisation.

Test infrastructure only: called by tests/ and never by the product path.

The paper takes the number of k-points K as the k_1 k_2 k_3 points of the
grid divided by the symmetries of the lattice (Sec. 5.1, the paragraph on
periodic structures), and works on the product of the Stiefel manifolds of
the remaining k-points.  It does not spell out how the reduction is done.
Readings (also in the design notes, A35-A38):

* A35 a symmetry operation is a pair (W, t) acting on fractional positions as
  x -> W x + t, W an integer matrix with entries in {-1, 0, 1} that preserves
  the metric A^T A of the lattice, t in [0, 1)^3, that maps every atom onto an
  atom of the same valence charge (Cartesian distance <= symprec modulo the
  lattice); the operations kept are those that also map the FFT box onto
  itself (W_ab != 0 only where n_a = n_b, and n_a t_a an integer), so that the
  density on the box can be symmetrised exactly; pure translations (W = I,
  t != 0) of a non-primitive cell are operations too;
* A36 a rotation acts on a fractional k-point as u -> W^T u (over a group the
  images W^{-T} u and W^T u are the same set); time reversal adds -u; two
  points are equivalent when they differ by an integer vector;
* A37 the reduced set keeps, in input order, the first point of every orbit
  of the input set, with the summed weight of the orbit; an input set that is
  not closed under the operations is an error;
* A38 with a reduced set the density is the average over the operations of
  the density of the kept points: rho(x) <- |G|^-1 sum_g rho(W_g x + t_g)
  evaluated on the box (x = i / n), and everything downstream (potentials,
  energy, H) uses the averaged density.  For a symmetric ground state the
  energy and density equal those of the full set.
"""
from __future__ import annotations

import itertools

import numpy as np


def _frac_dist(lattice, d):
    """Cartesian length of the fractional difference d taken modulo the lattice."""
    d = d - np.round(d)
    return np.linalg.norm(np.asarray(lattice, float) @ d)


def lattice_rotations(lattice, tol=1e-8):
    """Integer matrices W (entries -1, 0, 1) with W^T M W = M, M = A^T A."""
    A = np.asarray(lattice, float)
    M = A.T @ A
    out = []
    scale = np.abs(M).max()
    for e in itertools.product((-1, 0, 1), repeat=9):
        W = np.array(e, dtype=np.int64).reshape(3, 3)
        if abs(round(np.linalg.det(W))) != 1:
            continue
        if np.abs(W.T @ M @ W - M).max() <= tol * scale:
            out.append(W)
    return out


def space_group(sysd, fft, symprec=1e-5):
    """List of (W, t) of A35, ordered by W (as read row-major) and then t."""
    lat = np.asarray(sysd["lattice"], float)
    frac = np.asarray(sysd["frac"], float)
    Z = np.asarray(sysd["Z"], float)
    n = np.asarray(fft, dtype=np.int64)
    ops = []
    for W in lattice_rotations(lat):
        if any(W[a, b] != 0 and n[a] != n[b] for a in range(3) for b in range(3)):
            continue
        if len(Z) == 0:
            cands = [np.zeros(3)]
        else:
            cands = [frac[b] - W @ frac[0] for b in range(len(Z)) if Z[b] == Z[0]]
        found = []
        for t in cands:
            t = t - np.floor(t)
            nt = n * t
            if np.abs(nt - np.round(nt)).max() > 1e-6 * n.max():
                continue
            t = np.round(nt) / n
            t = t - np.floor(t)
            ok = True
            for a in range(len(Z)):
                y = W @ frac[a] + t
                if not any(Z[b] == Z[a] and _frac_dist(lat, y - frac[b]) <= symprec for b in range(len(Z))):
                    ok = False
                    break
            if ok and not any(np.abs(t - s).max() < 1e-12 for s in found):
                found.append(t)
        for t in sorted(found, key=lambda v: tuple(v)):
            ops.append((W.copy(), t))
    return ops


class NotClosedError(ValueError):
    pass


def reduce_kpoints(ops, kfrac, kweight, time_reversal=True, tol=1e-8):
    """A36-A37: (kept points, their weights, map input -> index of its kept point)."""
    kfrac = np.atleast_2d(np.asarray(kfrac, float))
    kweight = np.asarray(kweight, float)
    rots = []
    for W, _ in ops:
        if not any(np.array_equal(W, R) for R in rots):
            rots.append(W)
    signs = (1.0, -1.0) if time_reversal else (1.0,)
    nk = len(kfrac)

    def find(u):
        for j in range(nk):
            d = u - kfrac[j]
            if np.abs(d - np.round(d)).max() <= tol:
                return j
        return -1

    owner = np.full(nk, -1, dtype=np.int64)
    kept, weights = [], []
    for i in range(nk):
        if owner[i] >= 0:
            continue
        members = set()
        for W in rots:
            for s in signs:
                j = find(s * (W.T @ kfrac[i]))
                if j < 0:
                    raise NotClosedError(f"k-point {i} maps outside the set")
                members.add(j)
        idx = len(kept)
        for j in members:
            owner[j] = idx
        kept.append(kfrac[i].copy())
        weights.append(float(sum(kweight[j] for j in members)))
    return np.array(kept), np.array(weights), owner


def symmetrize(rho, ops):
    """A38: |G|^-1 sum_g rho(W_g x + t_g) on the box, x = i / n."""
    n = np.array(rho.shape, dtype=np.int64)
    idx = np.indices(rho.shape).reshape(3, -1)
    out = np.zeros(rho.size)
    for W, t in ops:
        sh = np.round(n * t).astype(np.int64)
        # fractional x_a = i_a / n_a; (W x + t)_a n_a = sum_b W_ab i_b (n_a = n_b where W_ab != 0)
        j = (W @ idx + sh[:, None]) % n[:, None]
        out += rho[j[0], j[1], j[2]]
    return (out / len(ops)).reshape(rho.shape)
