"""Pins of the oracle's L2RCG (unpreconditioned L2-gradient RCG with the
approximated-Hessian step, readings A33-A34): the ground state against the
dense SCF with both retractions; the curvature h against the exact second
derivative of the energy along the polar retraction curve for a model whose
energy is the band energy alone (kinetic only, where the approximation is
exact); the non-monotone acceptance invariants."""
import numpy as np
import pytest

import workloads as W
from oracle import hamiltonian as ham, l2rcg, manifold as mf, scf


def tiny(terms=W.TERMS_ALL):
    lat, fr, Z = W.diamond_cell()
    return ham.Model(W.system(lat, fr, Z, 3.0, (0, 0, 0), terms=terms))


def start(model, seed=1):
    Z = W.gaussian_block(seed, model.npw, model.p)
    return np.concatenate([mf.polar(b)[0] for b in model.blocks(Z)], axis=0)


@pytest.mark.parametrize("retraction", [0, 1])
def test_l2rcg_reaches_the_scf_ground_state(retraction):
    m = tiny()
    Phi0 = start(m)
    ref = scf.scf(m, Phi0=Phi0)
    prm = dict(W.DEFAULT_PARAMS, tol=1e-9, maxit=2000, retraction=retraction)
    Phi, st, stats = l2rcg.l2rcg(m, Phi0, prm)
    assert stats["rnorm"][-1] <= 1e-9
    assert st["E"] == pytest.approx(ref["E"], rel=1e-10)
    assert np.allclose(np.linalg.eigvalsh(st["lams"][0]), ref["eigs"][0][:m.p], atol=1e-7)
    E, C = np.array(stats["energy"]), np.array(stats["C"])
    for k, (tau, dE) in enumerate(zip(stats["taus"], stats["slopes"])):
        assert dE < 0.0
        assert E[k + 1] <= C[k] + prm["nm_rho"] * tau * dE
        assert C[k + 1] <= C[k] + 1e-15 * abs(C[k])


def test_curvature_is_the_second_derivative_of_the_band_energy():
    m = tiny(terms=0)
    Phi = start(m, 2)
    st = mf.state(m, Phi)
    Z = W.gaussian_block(5, m.npw, m.p)
    M = Phi.conj().T @ Z
    eta = Z - Phi @ (0.5 * (M + M.conj().T))
    eta /= np.linalg.norm(eta)
    h = l2rcg.hessian_curvature(m, st["Veff"], Phi, st["lams"], eta)

    def E(t):
        return ham.energy(m, mf.retract(m, Phi, eta, t)[0])

    e0 = E(0.0)
    # second differences with Richardson extrapolation (steps large enough that
    # the rounding of E ~ 55 Ha does not dominate the O(s^2) differences)
    d = [(E(s) - 2 * e0 + E(-s)) / s ** 2 for s in (4e-2, 2e-2)]
    fd = (4 * d[1] - d[0]) / 3
    assert h == pytest.approx(fd, rel=1e-6)
