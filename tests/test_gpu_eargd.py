"""EARGD on the GPU (eahp_solve_params.method = EAHP_EARGD): the energy-
adaptive gradient with an alternating Barzilai-Borwein step and non-monotone
backtracking (readings A28-A31), against the oracle's EARGD.

* the first iterates (energies, energy evaluations per step and the frame)
  against the oracle's trajectory at 1e-9, at Gamma (si8_gamma_e10) and with
  two k-points of different weights' structure (tiny_k2);
* a converged FP64 solve against the dense-SCF ground state of
  tests/golden/si8_gamma_e10.json (1e-10) and a converged mixed-precision
  solve against it (1e-7, the single-precision metric solve);
* parameters outside their ranges are rejected.
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


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_16225_amd import binding
    return binding


def tiny_k2():
    lat, fr, Z = W.diamond_cell()
    k = np.array([[0.25, 0.25, 0.25], [-0.25, 0.25, -0.25]])
    return W.system(lat, fr, Z, 3.0, (0, 0, 0), k, np.full(2, 0.5))


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("name", ["si8_gamma_e10", "tiny_k2"])
def test_first_iterates_match_oracle(name):
    B = _lib()
    from oracle import eargd, hamiltonian as ham, manifold as mf
    sysd = tiny_k2() if name == "tiny_k2" else W.config(name)
    nsteps = 4
    m = ham.Model(sysd)
    Z = W.gaussian_block(1, m.npw, m.p)
    Phi0 = np.concatenate([mf.polar(b)[0] for b in m.blocks(Z)], axis=0)
    prm = dict(W.DEFAULT_PARAMS, tol=1e-12, method=B.EAHP_EARGD)
    _, st_o, stats_o = eargd.eargd(m, Phi0, prm, maxit=nsteps)
    gp = B.Problem(sysd)
    Psi = gp.to_device(Z)
    sp = B.SolveParams.from_dict(prm)
    sv = C.c_void_p()
    B._check(gp.lib.eahp_solver_create(gp.pb, C.c_void_p(Psi.data_ptr()), C.byref(sp), C.byref(sv)))
    E, rn = C.c_double(), C.c_double()
    B._check(gp.lib.eahp_solver_get(sv, None, C.byref(E), C.byref(rn)))
    energies, trials = [E.value], []
    st = B.Stats()
    for _ in range(nsteps):
        B._check(gp.lib.eahp_solver_step(sv, 1, C.byref(st)), allow=(-8,))
        energies.append(st.energy)
        trials.append(st.ls_trials - sum(trials))
    out = gp.empty_frame()
    B._check(gp.lib.eahp_solver_get(sv, C.c_void_p(out.data_ptr()), None, None))
    gp.lib.eahp_solver_destroy(sv)
    print(name, "gpu", energies, trials, "oracle", stats_o["energy"], stats_o["trials"], flush=True)
    assert trials == stats_o["trials"]
    for a, b in zip(energies, stats_o["energy"]):
        assert abs(a - b) <= 1e-9 * abs(b)
    assert abs(rn.value - stats_o["rnorm"][0]) <= 1e-9 * stats_o["rnorm"][0]
    assert rel(gp.to_blocks(out), st_o["Phi"]) < 1e-8
    gp.close()


@pytest.mark.parametrize("precision,bar", [(0, 1e-10), (1, 1e-7)])
def test_converged_solve_matches_scf_ground_state(precision, bar):
    B = _lib()
    with open(os.path.join(GOLD, "si8_gamma_e10.json")) as f:
        g = json.load(f)
    gp = B.Problem(W.config("si8_gamma_e10"), precision=precision)
    Psi = gp.to_device(W.gaussian_block(1, gp.npw, gp.p))
    prm = dict(W.DEFAULT_PARAMS, tol=1e-8 if precision == 0 else 1e-6, maxit=400, method=B.EAHP_EARGD)
    st, rc = gp.solve(Psi, prm)
    print("eargd precision", precision, st, flush=True)
    assert abs(st["energy"] - g["E_scf"]) <= bar * abs(g["E_scf"])
    R, L, rn, E = gp.residual(Psi)
    lam = np.sort(np.linalg.eigvalsh(gp.lambdas(L)[0]))
    assert np.allclose(lam, g["lambda_scf"], atol=1e-7 if precision == 0 else 1e-5)
    gp.close()


def test_bad_parameters_are_rejected():
    B = _lib()
    gp = B.Problem(W.config("si8_gamma_e3"))
    Psi = gp.to_device(W.gaussian_block(1, gp.npw, gp.p))
    for bad in (dict(method=7), dict(retraction=3), dict(method=1, nm_backtrack=1.5), dict(method=1, nm_rho=0.0)):
        sp = B.SolveParams.from_dict(dict(W.DEFAULT_PARAMS, **bad))
        sv = C.c_void_p()
        assert gp.lib.eahp_solver_create(gp.pb, C.c_void_p(Psi.data_ptr()), C.byref(sp), C.byref(sv)) == -1
    gp.close()
