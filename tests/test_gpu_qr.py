"""The qR retraction and its differentiated transport on the GPU
(eahp_retract_qr, eahp_transport_qr, retraction = EAHP_QR in the solvers)
against the oracle's: at Gamma, with two k-points, with an odd p and at the
64-atom size; the solvers on the qR retraction (EARCG trajectory against the
oracle's, EARCG and EARGD converged to the dense-SCF ground state); a Gram
matrix that is not positive definite is reported as EAHP_ENOTPD.
"""
import ctypes as C
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(__file__), "golden")

CASES = {
    "tiny_gamma": lambda: W.system(*W.diamond_cell(), 3.0, (0, 0, 0)),
    "tiny_k2": lambda: W.system(*W.diamond_cell(), 3.0, (0, 0, 0), np.array([[0.25, -0.125, 0.375], [-0.25, 0.25, 0.25]]),
                                np.array([0.5, 0.5])),
    "tiny_p13": lambda: W.system(*W.diamond_cell(), 3.0, (0, 0, 0), p=13),
    "si64_gamma_e20": lambda: W.config("si64_gamma_e20"),
}


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_16225_amd import binding
    return binding


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def tangent(om, Phi, Zb):
    out = []
    for Pk, Zk in zip(om.blocks(Phi), om.blocks(Zb)):
        M = Pk.conj().T @ Zk
        out.append(Zk - Pk @ (0.5 * (M + M.conj().T)))
    return np.concatenate(out, 0)


@pytest.mark.parametrize("name", list(CASES))
def test_retract_and_transport_qr(name):
    B = _lib()
    from oracle import hamiltonian as ham, manifold as mf
    sysd = CASES[name]()
    om = ham.Model(sysd, workers=8)
    gp = B.Problem(sysd)
    Z = W.gaussian_block(1, om.npw, om.p)
    Phi = np.concatenate([mf.polar(b)[0] for b in om.blocks(Z)], axis=0)
    eta = 0.3 * tangent(om, Phi, W.gaussian_block(8, om.npw, om.p))
    v = tangent(om, Phi, W.gaussian_block(9, om.npw, om.p))
    tau = 0.7
    Pn_o, facs = mf.retract_qr(om, Phi, eta, tau)
    Pn = gp.to_blocks(gp.retract(gp.to_device(Phi), gp.to_device(eta), tau, qr=True))
    print(name, "retract_qr", rel(Pn, Pn_o), flush=True)
    assert rel(Pn, Pn_o) < 1e-12
    for Pk in om.blocks(Pn):
        assert np.abs(Pk.conj().T @ Pk - np.eye(om.p)).max() < 1e-13
    T_o = mf.transport_qr(om, mf.retract_qr(om, Phi, tau * eta, 1.0)[0], v,
                          mf.retract_qr(om, Phi, tau * eta, 1.0)[1])
    T = gp.to_blocks(gp.transport(gp.to_device(Phi), gp.to_device(tau * eta), gp.to_device(v), qr=True))
    print(name, "transport_qr", rel(T, T_o), flush=True)
    assert rel(T, T_o) < 1e-11
    gp.close()


def test_not_positive_definite_is_reported():
    B = _lib()
    gp = B.Problem(CASES["tiny_gamma"]())
    from oracle import manifold as mf
    Z = W.gaussian_block(1, gp.npw, gp.p)
    Phi = mf.polar(Z)[0]
    Psi = gp.to_device(Phi)
    out = gp.empty_frame()
    rc = gp.lib.eahp_retract_qr(gp.pb, C.c_void_p(Psi.data_ptr()), C.c_void_p(Psi.data_ptr()), -1.0,
                                C.c_void_p(out.data_ptr()))
    assert rc == -4
    gp.close()


def test_earcg_qr_first_iterates_match_oracle():
    B = _lib()
    from oracle import earcg, hamiltonian as ham, manifold as mf
    sysd = W.config("si8_gamma_e10")
    om = ham.Model(sysd)
    Z = W.gaussian_block(1, om.npw, om.p)
    Phi0 = np.concatenate([mf.polar(b)[0] for b in om.blocks(Z)], axis=0)
    prm = dict(W.DEFAULT_PARAMS, tol=1e-12, retraction=B.EAHP_QR)
    nsteps = 3
    _, st_o, stats_o = earcg.earcg(om, Phi0, prm, maxit=nsteps)
    gp = B.Problem(sysd)
    Psi = gp.to_device(Z)
    sp = B.SolveParams.from_dict(prm)
    sv = C.c_void_p()
    B._check(gp.lib.eahp_solver_create(gp.pb, C.c_void_p(Psi.data_ptr()), C.byref(sp), C.byref(sv)))
    st = B.Stats()
    energies = [stats_o["energy"][0]]
    for _ in range(nsteps):
        B._check(gp.lib.eahp_solver_step(sv, 1, C.byref(st)), allow=(-8,))
        energies.append(st.energy)
    out = gp.empty_frame()
    B._check(gp.lib.eahp_solver_get(sv, C.c_void_p(out.data_ptr()), None, None))
    gp.lib.eahp_solver_destroy(sv)
    print("earcg qr gpu", energies, st.ls_trials, "oracle", stats_o["energy"], sum(stats_o["trials"]), flush=True)
    assert st.ls_trials == sum(stats_o["trials"])
    for a, b in zip(energies[1:], stats_o["energy"][1:]):
        assert abs(a - b) <= 1e-9 * abs(b)
    assert rel(gp.to_blocks(out), st_o["Phi"]) < 1e-8
    gp.close()


@pytest.mark.parametrize("method", [0, 1])
def test_qr_solvers_reach_the_scf_ground_state(method):
    B = _lib()
    with open(os.path.join(GOLD, "si8_gamma_e10.json")) as f:
        g = json.load(f)
    gp = B.Problem(W.config("si8_gamma_e10"))
    Psi = gp.to_device(W.gaussian_block(1, gp.npw, gp.p))
    prm = dict(W.DEFAULT_PARAMS, tol=1e-8, maxit=400, method=method, retraction=B.EAHP_QR)
    st, rc = gp.solve(Psi, prm)
    print("qr method", method, st, flush=True)
    assert st["rnorm"] <= 1e-8
    assert abs(st["energy"] - g["E_scf"]) <= 1e-10 * abs(g["E_scf"])
    Pb = gp.to_blocks(Psi)
    assert np.abs(Pb.conj().T @ Pb - np.eye(gp.p)).max() < 1e-12
    gp.close()
