"""Pins of the oracle's qR retraction and its differentiated transport (the
alternative retraction the paper names in Sec. 3.1): the Q factor against
LAPACK's Householder QR with the phases of R made positive, the transport
against finite differences of the Q factor and against the tangent-space
condition, and EARCG and EARGD on the qR retraction against the dense SCF
ground state."""
import numpy as np
import pytest

import workloads as W
from oracle import eargd, earcg, hamiltonian as ham, manifold as mf, scf


def rand(seed, n, p):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, p)) + 1j * rng.standard_normal((n, p))


@pytest.mark.parametrize("n,p", [(5, 1), (40, 7), (300, 16)])
def test_qf_is_the_positive_diagonal_qr(n, p):
    A = rand(n + p, n, p)
    Q, R, Rinv = mf.qf(A)
    Qh, Rh = np.linalg.qr(A)
    ph = np.diag(Rh) / np.abs(np.diag(Rh))
    Qh, Rh = Qh * ph[None, :], ph.conj()[:, None] * Rh
    assert np.abs(Q - Qh).max() < 1e-12 * max(1.0, np.abs(Qh).max()) * 10
    assert np.abs(R - Rh).max() < 1e-12 * np.abs(Rh).max() * 10
    assert np.allclose(np.diag(R).imag, 0) and np.all(np.diag(R).real > 0)
    assert np.abs(np.tril(R, -1)).max() == 0.0
    assert np.abs(R @ Rinv - np.eye(p)).max() < 1e-12 * np.linalg.cond(R)


@pytest.mark.parametrize("p", [1, 6])
def test_qr_transport_is_the_derivative_of_qf(p):
    n = 50
    Phi = mf.qf(rand(1, n, p))[0]
    xi, v = 0.3 * rand(2, n, p), rand(3, n, p)

    class One:
        def blocks(self, X):
            return [X]

    m = One()
    Qn, facs = mf.retract_qr(m, Phi, xi, 1.0)
    T = mf.transport_qr(m, Qn, v, facs)
    h = 1e-4

    def q(t):
        return mf.qf(Phi + xi + t * v)[0]

    c1 = (q(h) - q(-h)) / (2 * h)
    c2 = (q(h / 2) - q(-h / 2)) / h
    fd = (4 * c2 - c1) / 3
    assert np.abs(T - fd).max() < 1e-8 * np.abs(fd).max()
    S = Qn.conj().T @ T
    assert np.abs(S + S.conj().T).max() < 1e-12 * np.abs(T).max()


@pytest.mark.parametrize("method", ["earcg", "eargd"])
def test_qr_retraction_reaches_the_scf_ground_state(method):
    lat, fr, Z = W.diamond_cell()
    m = ham.Model(W.system(lat, fr, Z, 3.0, (0, 0, 0)))
    Zb = W.gaussian_block(1, m.npw, m.p)
    Phi0 = np.concatenate([mf.polar(b)[0] for b in m.blocks(Zb)], axis=0)
    ref = scf.scf(m, Phi0=Phi0)
    prm = dict(W.DEFAULT_PARAMS, tol=1e-9, maxit=400, retraction=1)
    run = earcg.earcg if method == "earcg" else eargd.eargd
    Phi, st, stats = run(m, Phi0, prm)
    assert stats["rnorm"][-1] <= 1e-9
    assert st["E"] == pytest.approx(ref["E"], rel=1e-10)
    assert np.abs(Phi.conj().T @ Phi - np.eye(m.p)).max() < 1e-12
