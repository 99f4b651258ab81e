"""GPU EARCG solves (eahp_solve / the steppable solver) against the oracle.

The converged energy is compared with the dense-SCF ground state stored in
tests/golden/ (written by tests/golden/make_golden.py from the oracle); the
first iterates of the trajectory are compared with the oracle's own EARCG
iterates (beyond the first steps the trajectory is not pinned: different
rounding may change later line-search decisions, only converged results are).
"""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _problem(sysd):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_16225_amd import Problem
    return Problem(sysd)


def test_si8_gamma_converges_to_scf_ground_state():
    with open(os.path.join(GOLD, "si8_gamma_e10.json")) as f:
        g = json.load(f)
    gp = _problem(W.config("si8_gamma_e10"))
    Z = W.gaussian_block(1, gp.npw, gp.p)
    Psi = gp.to_device(Z)
    prm = dict(W.DEFAULT_PARAMS, tol=1e-8, maxit=200)
    st, rc = gp.solve(Psi, prm)
    print("solve stats", st, flush=True)
    assert st["rnorm"] <= 1e-8
    assert abs(st["energy"] - g["E_scf"]) <= 1e-10 * abs(g["E_scf"])
    R, L, rn, E = gp.residual(Psi)
    lam = np.sort(np.linalg.eigvalsh(gp.lambdas(L)[0]))
    assert np.allclose(lam, g["lambda_scf"], atol=1e-7)
    Pb = gp.to_blocks(Psi)
    assert np.abs(Pb.conj().T @ Pb - np.eye(gp.p)).max() < 1e-12
    gp.close()


def test_first_iterates_match_oracle_trajectory():
    with open(os.path.join(GOLD, "si8_gamma_e10.json")) as f:
        g = json.load(f)
    from paper_2503_16225_amd.binding import SolveParams, Stats, _check
    import ctypes as C
    gp = _problem(W.config("si8_gamma_e10"))
    Z = W.gaussian_block(1, gp.npw, gp.p)
    Psi = gp.to_device(Z)
    prm = SolveParams.from_dict(dict(W.DEFAULT_PARAMS, tol=1e-8))
    sv = C.c_void_p()
    _check(gp.lib.eahp_solver_create(gp.pb, C.c_void_p(Psi.data_ptr()), C.byref(prm), C.byref(sv)))
    st = Stats()
    energies = []
    E = C.c_double()
    rn = C.c_double()
    _check(gp.lib.eahp_solver_get(sv, None, C.byref(E), C.byref(rn)))
    energies.append(E.value)
    for _ in range(3):
        gp.lib.eahp_solver_step(sv, 1, C.byref(st))
        energies.append(st.energy)
    gp.lib.eahp_solver_destroy(sv)
    print("gpu", energies, "oracle", g["first_energies"], flush=True)
    for a, b in zip(energies, g["first_energies"]):
        assert abs(a - b) <= 1e-9 * abs(b)
    gp.close()
