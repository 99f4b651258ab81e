"""Pins of the oracle's crystal symmetry, k-point reduction and density
symmetrisation (readings A35-A38) against facts fixed independently of it:

* the diamond structure in its cubic cell: the 48 rotations of the cubic
  point group m-3m, of which the 24 of the site group -43m (T_d) need no
  translation, times the 4 face-centring translations = 192 operations when
  the FFT box is a multiple of 4; a box that is not (45^3) keeps only the
  T_d part, and a box that is even but not a multiple of 4 (18^3) keeps T_d
  with the centrings (96); inversion through (1/8, 1/8, 1/8), i.e. x -> -x +
  (1/4, 1/4, 1/4), is one of them; an orthorhombic strain leaves the 8
  rotations of mmm (32 operations), a random jitter the identity alone;
* the set is a group: closed under composition and inverses modulo the
  lattice;
* k-point orbits counted by hand for the cubic group with time reversal: the
  shifted 4x4x4 grid ((2r-5)/8) has 4 classes of sizes 8, 24, 24, 8; the
  Gamma-centred 4x4x4 grid has 10 classes of sizes 1, 1, 3, 3, 6, 6, 8, 12,
  12, 12; the orthorhombic group gives 8 classes of 8; time reversal alone
  pairs u with -u (the shifted 2x2x2 grid: 4 pairs) and fixes the points
  with coordinates in {0, 1/2};
* the ionic potential of the crystal is invariant under symmetrisation, and
  any field symmetrised twice equals it symmetrised once;
* the dense-SCF ground state of the reduced set, with the symmetrised
  density, has the energy of the full grid (to rounding), while the same
  reduced set without the symmetrisation does not.
"""
import numpy as np
import pytest

import workloads as W
from oracle import hamiltonian as ham, manifold as mf, scf, symmetry as S


def diamond(fft=(40, 40, 40), lattice=None, frac=None):
    lat, fr, Z = W.diamond_cell()
    if lattice is not None:
        lat = lattice
    if frac is not None:
        fr = frac
    return W.system(lat, fr, Z, 3.0, fft)


def n_rot(ops):
    return len({tuple(Wm.ravel()) for Wm, _ in ops})


def test_diamond_space_group():
    ops = S.space_group(diamond(), (40, 40, 40))
    assert len(ops) == 192 and n_rot(ops) == 48
    assert n_rot([o for o in ops if not o[1].any()]) == 24
    assert sum(1 for Wm, t in ops if np.array_equal(Wm, np.eye(3, dtype=int))) == 4
    inv = [t for Wm, t in ops if np.array_equal(Wm, -np.eye(3, dtype=int))]
    assert any(np.allclose(t, 0.25) for t in inv)
    for Wm, _ in ops:
        assert abs(round(np.linalg.det(Wm))) == 1
        assert np.array_equal(Wm.T @ Wm, np.eye(3, dtype=int))  # cubic: orthogonal integer matrices


def test_box_compatibility_drops_operations():
    ops45 = S.space_group(diamond((45, 45, 45)), (45, 45, 45))
    assert len(ops45) == 24 and n_rot(ops45) == 24 and all(not t.any() for _, t in ops45)
    ops18 = S.space_group(diamond((18, 18, 18)), (18, 18, 18))
    assert len(ops18) == 96 and n_rot(ops18) == 24


def test_lower_symmetry_cells():
    lat, fr, _ = W.diamond_cell()
    ortho = S.space_group(diamond(lattice=lat @ np.diag([1.01, 0.99, 1.02])), (40, 40, 40))
    assert len(ortho) == 32 and n_rot(ortho) == 8
    assert all(np.array_equal(np.abs(Wm), np.eye(3, dtype=int)) for Wm, _ in ortho)
    jit = W.jitter(lat, fr, 0.05, np.random.default_rng(3))
    ops = S.space_group(diamond(frac=jit), (40, 40, 40))
    assert len(ops) == 1 and np.array_equal(ops[0][0], np.eye(3, dtype=int)) and not ops[0][1].any()


def test_operations_form_a_group():
    ops = S.space_group(diamond(), (40, 40, 40))
    key = {(tuple(Wm.ravel()), tuple(np.round(t * 40).astype(int) % 40)) for Wm, t in ops}

    def k(Wm, t):
        return tuple(Wm.ravel()), tuple(np.round(t * 40).astype(int) % 40)

    for W1, t1 in ops[::7]:
        for W2, t2 in ops:
            assert k(W1 @ W2, W1 @ t2 + t1) in key
        Wi = np.round(np.linalg.inv(W1)).astype(int)
        assert k(Wi, -Wi @ t1) in key


def test_cubic_kpoint_classes():
    ops = S.space_group(diamond(), (40, 40, 40))
    k, w = W.mp_grid((4, 4, 4))
    kk, ww, owner = S.reduce_kpoints(ops, k, w)
    assert len(kk) == 4
    assert sorted(np.round(ww * 64).astype(int)) == [8, 8, 24, 24]
    assert np.isclose(ww.sum(), 1.0)
    for i, j in enumerate(owner):  # every point has the sorted |coordinates| of its class representative
        assert np.allclose(np.sort(np.abs(k[i])), np.sort(np.abs(kk[j])))
    g = np.array([[a, b, c] for a in range(4) for b in range(4) for c in range(4)]) / 4.0
    kk, ww, _ = S.reduce_kpoints(ops, g, np.full(64, 1 / 64))
    assert sorted(np.round(ww * 64).astype(int)) == [1, 1, 3, 3, 6, 6, 8, 12, 12, 12]
    assert np.allclose(kk[0], 0.0)


def test_orthorhombic_and_time_reversal_classes():
    lat, fr, _ = W.diamond_cell()
    ortho = S.space_group(diamond(lattice=lat @ np.diag([1.01, 0.99, 1.02])), (40, 40, 40))
    k, w = W.mp_grid((4, 4, 4))
    kk, ww, _ = S.reduce_kpoints(ortho, k, w)
    assert len(kk) == 8 and np.allclose(ww, 1 / 8)
    ident = [(np.eye(3, dtype=np.int64), np.zeros(3))]
    k2, w2 = W.mp_grid((2, 2, 2))
    kk, ww, owner = S.reduce_kpoints(ident, k2, w2)
    assert len(kk) == 4 and np.allclose(ww, 0.25)
    for i, j in enumerate(owner):
        assert np.allclose(k2[i], kk[j]) or np.allclose(k2[i], -kk[j])
    g = np.array([[a, b, c] for a in range(2) for b in range(2) for c in range(2)]) / 2.0
    kk, ww, _ = S.reduce_kpoints(ident, g, np.full(8, 1 / 8))
    assert len(kk) == 8
    kk, ww, _ = S.reduce_kpoints(ident, k2, w2, time_reversal=False)
    assert len(kk) == 8


def test_set_not_closed_is_an_error():
    ops = S.space_group(diamond(), (40, 40, 40))
    with pytest.raises(S.NotClosedError):
        S.reduce_kpoints(ops, np.array([[0.1, 0.2, 0.3], [-0.1, -0.2, -0.3]]), np.array([0.5, 0.5]))


def test_symmetrisation_invariants():
    # V_ion is sampled from its G-sum over the box, whose even sizes include the
    # frequency -n/2 but not +n/2: a sign-changing operation is exact only up
    # to the Nyquist-plane terms, ~1e-11 at 18^3 and below rounding at 40^3
    for fft, tol in (((40, 40, 40), 1e-13), ((18, 18, 18), 1e-10)):
        sysd = diamond(fft)
        ops = S.space_group(sysd, fft)
        m = ham.Model(sysd)
        V = m.Vion_r
        assert np.abs(S.symmetrize(V, ops) - V).max() <= tol * np.abs(V).max()
        f = np.random.default_rng(4).standard_normal(fft)
        f1 = S.symmetrize(f, ops)
        assert np.abs(S.symmetrize(f1, ops) - f1).max() < 1e-13
        assert abs(f1.mean() - f.mean()) < 1e-13
        assert np.abs(f1 - f).max() > 0.1  # a random field is not invariant
    # a sign error in the translation breaks the invariance of V_ion
    sysd = diamond((40, 40, 40))
    ops = S.space_group(sysd, (40, 40, 40))
    V = ham.Model(sysd).Vion_r
    wrong = [(Wm, (-t) % 1.0) for Wm, t in ops]
    assert np.abs(S.symmetrize(V, wrong) - V).max() > 1e-3 * np.abs(V).max()


def _ground_energy(sysd):
    m = ham.Model(sysd)
    Z0 = W.gaussian_block(1, m.npw, m.p)
    Phi0 = np.concatenate([mf.polar(b)[0] for b in m.blocks(Z0)], axis=0)
    return scf.scf(m, tol=1e-11, Phi0=Phi0)["E"]


def test_reduced_set_has_the_full_grid_ground_energy():
    lat, fr, Z = W.diamond_cell()
    g = np.array([[a, b, c] for a in range(2) for b in range(2) for c in range(2)]) / 2.0
    w = np.full(8, 1 / 8)
    fft = (20, 20, 20)
    full = W.system(lat, fr, Z, 3.0, fft, g, w)
    ops = S.space_group(full, fft)
    kk, ww, _ = S.reduce_kpoints(ops, g, w)
    assert len(kk) == 4
    red = dict(W.system(lat, fr, Z, 3.0, fft, kk, ww), sym_rot=np.array([o[0] for o in ops]),
               sym_trans=np.array([o[1] for o in ops]))
    E_full = _ground_energy(full)
    E_red = _ground_energy(red)
    assert abs(E_red - E_full) <= 1e-12 * abs(E_full)
    E_nosym = _ground_energy(W.system(lat, fr, Z, 3.0, fft, kk, ww))
    assert abs(E_nosym - E_full) > 1e-6 * abs(E_full)
