"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the method: it only describes crystals
(lattice, atom positions, charges), k-point sets, method constants and seeded
random numbers.  Everything that is computed *from* these inputs (plane-wave
basis, potentials, Hamiltonian, energy, ...) lives separately in the oracle
and in the HIP library.

Crystal recipe (the paper's workloads are diamond-structure semiconductors
with an LDA-type local functional, Sec. 5.3; its DFTK models are not
available, so these synthetic crystals stand in for them):

* conventional cubic diamond cell, 8 atoms, lattice constant 10.26 bohr
  (the silicon constant of Sec. 5.3), valence charge Z = 4 per atom,
* p = 2 * natoms doubly occupied orbitals,
* supercells replicate the cell; atom jitter and lattice strain are drawn
  from ``numpy.random.default_rng(seed)`` in a fixed call order,
* k-points: unreduced Monkhorst-Pack grids u_r = (2r - q - 1) / (2q),
  uniform weights.

Orbital block layout: per k-point a column-major n_k x p complex block
(orbital j contiguous), rows in the canonical plane-wave order, blocks for
successive k-points concatenated.
"""
from __future__ import annotations

import numpy as np

A_DIAMOND = 10.26
DIAMOND_FRAC = np.array([
    [0.00, 0.00, 0.00], [0.00, 0.50, 0.50], [0.50, 0.00, 0.50], [0.50, 0.50, 0.00],
    [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25],
])

# Method constants of the experiments (Sec. 5.2): step-size parameters
# delta, sigma, gamma, eps; shift correction mu; FOM relative tolerance.
# mu_warm / warm_rtol / restarts / rank_tol / maxit values are this
# project's readings for what the paper leaves open (random start instead of
# the paper's SCF start, deflation threshold, iteration caps).
DEFAULT_PARAMS = dict(
    mu=0.01,
    fom_rtol=2.5e-2,
    fom_maxit=50,
    delta=0.05,
    sigma=0.1,
    gamma=0.5,
    eps=1e-12,
    ls_maxit=20,
    tol=1e-8,
    maxit=200,
    mu_warm=1.0,
    warm_rtol=1e-2,
    rank_tol=1e-7,
    method=0,          # 0 EARCG (Algorithm 3), 1 EARGD, 2 L2RCG
    retraction=0,      # 0 polar (eq. (3.1)), 1 qR
    nm_rho=1e-4,       # EARGD, L2RCG: Armijo constant of the non-monotone test
    nm_backtrack=0.5,  # EARGD, L2RCG: backtracking factor
    nm_theta=0.85,     # EARGD, L2RCG: weight of the Zhang-Hager reference energy
)

# SCF comparator: Anderson mixing of the density (damping, history) as in the
# dense SCF of the tests; eig_tol 0 selects the adaptive eigensolver tolerance
DEFAULT_SCF_PARAMS = dict(tol=1e-10, maxit=100, beta=0.5, depth=6, eig_tol=0.0, eig_maxit=100)

# term switches (used by closed-form special cases)
TERM_ION = 1
TERM_HARTREE = 2
TERM_XC = 4
TERM_NONLOCAL = 8
TERMS_ALL = TERM_ION | TERM_HARTREE | TERM_XC | TERM_NONLOCAL


def diamond_cell(a: float = A_DIAMOND):
    """Return (lattice, frac, Z): lattice columns are the lattice vectors."""
    lattice = np.eye(3) * a
    return lattice, DIAMOND_FRAC.copy(), np.full(8, 4.0)


def supercell(lattice, frac, Z, reps):
    reps = tuple(int(r) for r in reps)
    lat = lattice * np.array(reps, dtype=float)[None, :]
    out = []
    for i in range(reps[0]):
        for j in range(reps[1]):
            for k in range(reps[2]):
                out.append((frac + np.array([i, j, k], dtype=float)) / np.array(reps, dtype=float))
    fr = np.concatenate(out, axis=0)
    return lat, fr, np.tile(Z, int(np.prod(reps)))


def jitter(lattice, frac, amp, rng):
    """Displace every atom by U(-amp, amp) per Cartesian component (bohr)."""
    cart = frac @ lattice.T
    cart = cart + rng.uniform(-amp, amp, size=cart.shape)
    return np.linalg.solve(lattice, cart.T).T


def mp_grid(q):
    """Unreduced Monkhorst-Pack grid, u_r = (2r - q - 1)/(2q), r = 1..q."""
    axes = [(2.0 * np.arange(1, qi + 1) - qi - 1) / (2.0 * qi) for qi in q]
    pts = np.array([[x, y, z] for x in axes[0] for y in axes[1] for z in axes[2]])
    w = np.full(len(pts), 1.0 / len(pts))
    return pts, w


def system(lattice, frac, Z, ecut, fft, kfrac=None, kweight=None, p=None,
           occ=2.0, r_loc=0.8, r_proj=0.8, D_proj=1.0, terms=TERMS_ALL):
    if kfrac is None:
        kfrac = np.zeros((1, 3))
        kweight = np.ones(1)
    if p is None:
        p = int(round(float(np.sum(Z)) / occ))
    return dict(lattice=np.asarray(lattice, float), frac=np.asarray(frac, float),
                Z=np.asarray(Z, float), ecut=float(ecut), fft=tuple(int(x) for x in fft),
                kfrac=np.asarray(kfrac, float), kweight=np.asarray(kweight, float),
                p=int(p), occ=float(occ), r_loc=float(r_loc), r_proj=float(r_proj),
                D_proj=float(D_proj), terms=int(terms))


def config(name: str, seed: int | None = None):
    """The synthetic crystals used throughout (sizes in the docstring above)."""
    lat, fr, Z = diamond_cell()
    if name == "si8_gamma_e10":            # 8 atoms, Gamma, Ecut 10 Ha, 32^3
        return system(lat, fr, Z, 10.0, (32, 32, 32))
    if name == "si64_gamma_e20":           # 2x2x2 supercell, jitter 0.05, Ecut 20, 90^3
        rng = np.random.default_rng(2 if seed is None else seed)
        lat2, fr2, Z2 = supercell(lat, fr, Z, (2, 2, 2))
        fr2 = jitter(lat2, fr2, 0.05, rng)
        return system(lat2, fr2, Z2, 20.0, (90, 90, 90))
    if name == "si8_k444_e15":             # 8 atoms, 4x4x4 MP, Ecut 15, 40^3
        k, w = mp_grid((4, 4, 4))
        return system(lat, fr, Z, 15.0, (40, 40, 40), k, w)
    if name == "si216_gamma_e15":          # 3x3x3 supercell, +2% strain, Ecut 15, 120^3
        lat3, fr3, Z3 = supercell(lat, fr, Z, (3, 3, 3))
        return system(lat3 * 1.02, fr3, Z3, 15.0, (120, 120, 120))
    if name == "si8_gamma_e3":             # tiny case for dense checks
        return system(lat, fr, Z, 3.0, (18, 18, 18))
    raise KeyError(name)


def serving_request(rid: int, base_seed: int = 5):
    """One request of the serving stream: supercell n_i in {1,2}, strain +-3%,
    Ecut in {10,15,20} Ha, Gamma or 2x2x2 MP grid."""
    rng = np.random.default_rng(base_seed + rid)
    reps = tuple(int(x) for x in rng.integers(1, 3, size=3))
    strain = rng.uniform(-0.03, 0.03, size=3)
    ecut = float(rng.choice([10.0, 15.0, 20.0]))
    kgrid = bool(rng.integers(0, 2))
    lat, fr, Z = diamond_cell()
    lat, fr, Z = supercell(lat, fr, Z, reps)
    lat = lat @ np.diag(1.0 + strain)
    if kgrid:
        k, w = mp_grid((2, 2, 2))
    else:
        k, w = np.zeros((1, 3)), np.ones(1)
    return dict(lattice=lat, frac=fr, Z=Z, ecut=ecut, kfrac=k, kweight=w, reps=reps)


def gaussian_block(seed: int, npw_per_k, p: int):
    """Seeded complex Gaussian block: Re, Im ~ N(0,1) i.i.d.

    Drawn per k-point in order, as a (2, p, n_k) array of normals; column j of
    k-block b is re[j] + 1j*im[j].  Returns the stacked (sum n_k) x p array.
    """
    rng = np.random.default_rng(seed)
    blocks = []
    for nk in npw_per_k:
        z = rng.standard_normal((2, p, int(nk)))
        blocks.append((z[0] + 1j * z[1]).T)
    return np.ascontiguousarray(np.concatenate(blocks, axis=0))


def gaussian_real(seed: int, shape):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape)
