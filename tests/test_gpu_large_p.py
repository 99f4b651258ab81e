"""p > 128: the dense paths of the p x p problems beyond one work-group
(Householder on several work-groups + divide and conquer in global memory for
the eigendecompositions, the pivoted Cholesky and inverse for larger
matrices) and the projected FOM systems they feed, against the oracle.

The 8-atom cell at Ecut 10 Ha (1647 plane waves, 32^3 box) carries p = 200 or
432 orbitals, so the oracle stays cheap while every p x p matrix has the size
of the 216-atom workload's (p = 432).  Checked: the polar retraction (Gram
eigendecomposition), the transport (its Lyapunov form in that eigenbasis), a
retraction whose Gram matrix has exactly degenerate eigenvalues, Lambda and
the residual, Algorithm 4 at a definite shift (eigendecomposition of Sigma,
the rank-revealing orthonormalisation, projected systems up to q = 3 p) with
equal iteration counts, and the energy-adaptive gradient.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=[200, 432])
def case(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import hamiltonian as ham, manifold as mf
    from paper_2503_16225_amd import Problem
    p = request.param
    sysd = W.system(*W.diamond_cell(), 10.0, (32, 32, 32), p=p)
    log("case p", p)
    om = ham.Model(sysd, workers=8)
    gp = Problem(sysd)
    Z = W.gaussian_block(1, om.npw, p)
    Phi = np.concatenate([mf.polar(b)[0] for b in om.blocks(Z)], axis=0)
    yield p, om, gp, Phi
    gp.close()


def _tangent(om, Phi, seed, scale):
    Zb = W.gaussian_block(seed, om.npw, om.p)
    M = Phi.conj().T @ Zb
    return scale * (Zb - Phi @ (0.5 * (M + M.conj().T)))


def test_retract_transport(case):
    p, om, gp, Phi = case
    from oracle import manifold as mf
    eta = _tangent(om, Phi, 8, 0.05)
    v = _tangent(om, Phi, 9, 1.0)
    tau = 0.7
    Pn_o, facs = mf.retract(om, Phi, eta, tau)
    Pn = gp.to_blocks(gp.retract(gp.to_device(Phi), gp.to_device(eta), tau))
    log("p", p, "retract", rel(Pn, Pn_o))
    assert rel(Pn, Pn_o) < 1e-11
    assert np.abs(Pn.conj().T @ Pn - np.eye(p)).max() < 1e-13
    T_o = mf.transport_general(om, Pn_o, tau * eta, v, facs)
    T = gp.to_blocks(gp.transport(gp.to_device(Phi), gp.to_device(tau * eta), gp.to_device(v)))
    log("p", p, "transport", rel(T, T_o))
    assert rel(T, T_o) < 1e-10


def test_retract_degenerate(case):
    """pf(Phi (I + tau M)) = Phi for Hermitian M with I + tau M positive
    definite; M has five eigenvalues, each of multiplicity about p / 5."""
    p, om, gp, Phi = case
    rng = np.random.default_rng(11)
    U, _ = np.linalg.qr(rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p)))
    m = np.repeat(np.linspace(0.0, 2.0, 5), (p + 4) // 5)[:p]
    M = (U * m) @ U.conj().T
    out = gp.to_blocks(gp.retract(gp.to_device(Phi), gp.to_device(Phi @ M), 0.7))
    log("p", p, "degenerate retract", rel(out, Phi))
    assert rel(out, Phi) < 1e-12


def test_residual_lambda(case):
    p, om, gp, Phi = case
    from oracle import manifold as mf
    st = mf.state(om, Phi)
    R, L, rn, E = gp.residual(gp.to_device(Phi))
    assert abs(E - st["E"]) <= 1e-12 * abs(st["E"])
    assert rel(gp.to_blocks(R), st["R"]) < 1e-11
    assert rel(gp.lambdas(L)[0], st["lams"][0]) < 1e-12


def test_metric_solve_gradient(case):
    """Algorithm 4 at a shift making every H - s_l positive definite: three
    FOM iterations driven at rtol 1e-12 (projected systems q = p, 2p, 3p), and
    the paper's rtol; then the EA gradient of the result."""
    p, om, gp, Phi = case
    from oracle import earcg, manifold as mf
    st = mf.state(om, Phi)
    lam_max = float(np.linalg.eigvalsh(st["lams"][0])[-1])
    mu = lam_max - float(st["Veff"].min()) + 1.0
    for rtol, maxit in ((1e-12, 3), (2.5e-2, 50)):
        prm = dict(W.DEFAULT_PARAMS, fom_rtol=rtol, fom_maxit=maxit)
        X_o, info_o = earcg.metric_solve(om, Phi, st["HPhi"], st["lams"], st["Veff"], mu, prm)
        X, its, rr = gp.metric_solve(gp.to_device(Phi), mu, rtol, maxit)
        X = gp.to_blocks(X)
        log("p", p, "fom", rtol, its, info_o[0]["iters"], info_o[0]["q"], rr, info_o[0]["relres"], rel(X, X_o))
        assert its[0] == info_o[0]["iters"]
        assert abs(rr[0] - info_o[0]["relres"]) <= 1e-8 * info_o[0]["relres"] + 1e-14
        assert rel(X, X_o) < 1e-9
    G_o = mf.ea_gradient(om, Phi, X_o)
    G = gp.to_blocks(gp.ea_gradient(gp.to_device(Phi), gp.to_device(X_o)))
    log("p", p, "gradient", rel(G, G_o))
    assert rel(G, G_o) < 1e-10
