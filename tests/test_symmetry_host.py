"""The library's host-side symmetry helpers (eahp_symmetry_find,
eahp_kpoints_reduce) against the oracle's (readings A35-A37), bit for bit:
the same operations in the same order (rotations equal, translations equal
as box shifts), the same kept k-points in the same order, the same map, the
weights to rounding.  Host only: no GPU is touched.
"""
import numpy as np
import pytest

import workloads as W
from oracle import basis, symmetry as S


@pytest.fixture(scope="module")
def B():
    from paper_2503_16225_amd import binding
    binding.load_library()
    return binding


def cells():
    lat, fr, Z = W.diamond_cell()
    k4, w4 = W.mp_grid((4, 4, 4))
    yield "cubic40", W.system(lat, fr, Z, 3.0, (40, 40, 40), k4, w4)
    yield "cubic45", W.system(lat, fr, Z, 3.0, (45, 45, 45), k4, w4)
    yield "cubic18", W.system(lat, fr, Z, 3.0, (18, 18, 18))
    yield "cubic_auto", W.system(lat, fr, Z, 4.0, (0, 0, 0), k4, w4)
    yield "ortho", W.system(lat @ np.diag([1.01, 0.99, 1.02]), fr, Z, 3.0, (40, 40, 40))
    yield "ortho_box", W.system(lat @ np.diag([1.01, 0.99, 1.02]), fr, Z, 3.0, (40, 36, 40))
    yield "jitter", W.system(lat, W.jitter(lat, fr, 0.05, np.random.default_rng(3)), Z, 3.0, (40, 40, 40))
    Z2 = Z.copy()
    Z2[4:] = 3.0  # two species on the two sublattices (zinc blende)
    yield "zincblende", W.system(lat, fr, Z2, 3.0, (40, 40, 40))
    yield "empty", dict(W.system(lat, fr[:0], Z[:0], 3.0, (20, 20, 20)), p=4)


@pytest.mark.parametrize("name,sysd", list(cells()))
def test_operations_match_oracle(B, name, sysd):
    fft = sysd["fft"]
    if any(x == 0 for x in fft):
        fft = basis.auto_fft(sysd["lattice"], sysd["kfrac"], sysd["ecut"])
    ops_o = S.space_group(sysd, fft)
    rot, tr = B.symmetry_find(sysd)
    print(name, fft, len(ops_o), len(rot), flush=True)
    assert len(rot) == len(ops_o)
    n = np.array(fft)
    for (Wo, to), Wl, tl in zip(ops_o, rot, tr):
        assert np.array_equal(Wl, Wo)
        assert np.array_equal(np.round(n * tl).astype(int), np.round(n * to).astype(int))
        assert np.abs(n * tl - np.round(n * tl)).max() < 1e-9


def kcases():
    lat, fr, Z = W.diamond_cell()
    cubic = S.space_group(W.system(lat, fr, Z, 3.0, (40, 40, 40)), (40, 40, 40))
    ortho = S.space_group(W.system(lat @ np.diag([1.01, 0.99, 1.02]), fr, Z, 3.0, (40, 40, 40)), (40, 40, 40))
    ident = [(np.eye(3, dtype=np.int64), np.zeros(3))]
    g4 = np.array([[a, b, c] for a in range(4) for b in range(4) for c in range(4)]) / 4.0
    for q in ((4, 4, 4), (6, 6, 6), (3, 3, 3), (2, 2, 2)):
        k, w = W.mp_grid(q)
        yield f"cubic_mp{q[0]}", cubic, k, w, True
    yield "cubic_gamma4", cubic, g4, np.full(64, 1 / 64), True
    k, w = W.mp_grid((4, 4, 4))
    yield "ortho_mp4", ortho, k, w, True
    yield "ortho_mp4_noTR", ortho, k, w, False
    k, w = W.mp_grid((2, 3, 4))
    yield "ident_mp234", ident, k, w, True
    rng = np.random.default_rng(7)
    wr = rng.uniform(0.5, 1.5, 64)
    yield "cubic_gamma4_weights", cubic, g4 + rng.integers(-2, 3, size=g4.shape), wr / wr.sum(), True


@pytest.mark.parametrize("name,ops,k,w,tr", list(kcases()))
def test_kpoint_reduction_matches_oracle(B, name, ops, k, w, tr):
    ko, wo, mo = S.reduce_kpoints(ops, k, w, time_reversal=tr)
    rot = np.array([o[0] for o in ops])
    kl, wl, ml = B.kpoints_reduce(rot, k, w, time_reversal=tr)
    print(name, len(k), "->", len(ko), len(kl), flush=True)
    assert len(kl) == len(ko)
    assert np.array_equal(kl, ko)
    assert np.array_equal(ml, mo)
    assert np.abs(wl - wo).max() <= 1e-15
    assert abs(wl.sum() - w.sum()) <= 1e-14


def test_errors(B):
    lat, fr, Z = W.diamond_cell()
    cubic = S.space_group(W.system(lat, fr, Z, 3.0, (40, 40, 40)), (40, 40, 40))
    rot = np.array([o[0] for o in cubic])
    with pytest.raises(B.EahpError):
        B.kpoints_reduce(rot, np.array([[0.1, 0.2, 0.3], [-0.1, -0.2, -0.3]]), np.array([0.5, 0.5]))
    with pytest.raises(B.EahpError):
        B.symmetry_find(W.system(lat, fr, Z, 3.0, (40, 40, 40)), symprec=0.0)
