"""Pins of the oracle's EARGD (energy-adaptive gradient descent with a
Barzilai-Borwein step and non-monotone backtracking; readings A28-A31).

What they pin: the ground state against the dense SCF (a method-independent
truth), the energy slope used in the acceptance test against finite
differences of the energy along the retraction curve, the Barzilai-Borwein
steps against the exact step of a uniformly scaled quadratic and against
Cauchy-Schwarz, and the invariants of the Zhang-Hager reference energy.
"""
import numpy as np
import pytest

import workloads as W
from oracle import eargd, hamiltonian as ham, manifold as mf, scf


def tiny(k=None):
    lat, fr, Z = W.diamond_cell()
    if k is None:
        s = W.system(lat, fr, Z, 3.0, (0, 0, 0))
    else:
        s = W.system(lat, fr, Z, 3.0, (0, 0, 0), np.array(k), np.full(len(k), 1.0 / len(k)))
    return ham.Model(s)


def start(model, seed=1):
    Z = W.gaussian_block(seed, model.npw, model.p)
    return np.concatenate([mf.polar(b)[0] for b in model.blocks(Z)], axis=0)


@pytest.fixture(scope="module")
def run_tiny():
    m = tiny()
    Phi0 = start(m)
    prm = dict(W.DEFAULT_PARAMS, tol=1e-9, maxit=400)
    Phi, st, stats = eargd.eargd(m, Phi0, prm)
    return m, Phi0, Phi, st, stats, prm


def test_eargd_reaches_the_scf_ground_state(run_tiny):
    m, Phi0, Phi, st, stats, prm = run_tiny
    ref = scf.scf(m, Phi0=Phi0)
    assert ref["gap"] > 0.05
    assert stats["rnorm"][-1] <= 1e-9
    assert st["E"] == pytest.approx(ref["E"], rel=1e-10)
    assert np.allclose(np.linalg.eigvalsh(st["lams"][0]), ref["eigs"][0][:m.p], atol=1e-7)
    assert np.abs(Phi.conj().T @ Phi - np.eye(m.p)).max() < 1e-12


def test_zhang_hager_reference_invariants(run_tiny):
    """Every accepted step passes the non-monotone test; the reference energy
    C_k never increases and never falls below the current energy."""
    m, Phi0, Phi, st, stats, prm = run_tiny
    E, C = np.array(stats["energy"]), np.array(stats["C"])
    for k, (tau, dE) in enumerate(zip(stats["taus"], stats["slopes"])):
        assert dE < 0.0
        assert E[k + 1] <= C[k] + prm["nm_rho"] * tau * dE
        assert C[k + 1] <= C[k] + 1e-15 * abs(C[k])
        assert E[k + 1] <= C[k + 1] + 1e-15 * abs(C[k + 1])
    assert max(stats["trials"]) >= 1


@pytest.mark.parametrize("k", [None, [[0.25, 0.25, 0.25], [-0.25, 0.25, -0.25]]])
def test_energy_slope_is_the_derivative_along_the_retraction(k):
    """dE/dtau at 0 along pf(Phi + tau d), by Richardson-extrapolated central
    differences, equals 2 f sum_k w_k Re tr(R_k^* d_k) (weights included)."""
    m = tiny(k)
    Phi = start(m, 3)
    st = mf.state(m, Phi)
    Z = W.gaussian_block(9, m.npw, m.p)
    d = np.concatenate([Zk - Pk @ (0.5 * (Pk.conj().T @ Zk + Zk.conj().T @ Pk))
                        for Pk, Zk in zip(m.blocks(Phi), m.blocks(Z))], axis=0)
    d /= np.linalg.norm(d)

    def E(t):
        return ham.energy(m, mf.retract(m, Phi, d, t)[0])

    h = 1e-3
    c1 = (E(h) - E(-h)) / (2 * h)
    c2 = (E(h / 2) - E(-h / 2)) / h
    fd = (4 * c2 - c1) / 3
    assert eargd.energy_slope(m, st["R"], d) == pytest.approx(fd, rel=1e-7)


def test_bb_steps_on_scaled_quadratics():
    """For f = c/2 |x|^2 the gradient difference is Y = c S, and both
    Barzilai-Borwein steps equal the exact step 1/c; for a general SPD
    quadratic the long step is at least the short one (Cauchy-Schwarz) and both
    lie in [1/lambda_max, 1/lambda_min]."""
    rng = np.random.default_rng(4)
    S = rng.standard_normal((30, 4)) + 1j * rng.standard_normal((30, 4))
    for c in (0.3, 2.0, 17.0):
        for k in (1, 2, 5, 8):
            assert eargd.bb_step(S, c * S, k, 9.9) == pytest.approx(1.0 / c, rel=1e-14)
    M = rng.standard_normal((30, 30))
    A = M @ M.T + 0.5 * np.eye(30)
    lam = np.linalg.eigvalsh(A)
    Y = A @ S
    long_, short_ = eargd.bb_step(S, Y, 1, 1.0), eargd.bb_step(S, Y, 2, 1.0)
    assert long_ >= short_
    for t in (long_, short_):
        assert 1.0 / lam[-1] * (1 - 1e-12) <= t <= 1.0 / lam[0] * (1 + 1e-12)
    assert eargd.bb_step(S, np.zeros_like(S), 3, 0.7) == 0.7
