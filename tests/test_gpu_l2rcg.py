"""L2RCG on the GPU (method = EAHP_L2RCG): CG on the unpreconditioned L2
gradient with the frozen-potential Hessian step and non-monotone
backtracking (readings A33-A34), against the oracle's L2RCG: the first
iterates at 1e-9 (Gamma and two k-points, polar and qR retractions), and a
converged solve at the dense-SCF ground state of tests/golden/si8_gamma_e10.json."""
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


@pytest.mark.parametrize("name,retraction", [("si8_gamma_e10", 0), ("tiny_k2", 0), ("si8_gamma_e10", 1)])
def test_first_iterates_match_oracle(name, retraction):
    B = _lib()
    from oracle import hamiltonian as ham, l2rcg, manifold as mf
    sysd = tiny_k2() if name == "tiny_k2" else W.config(name)
    nsteps = 5
    m = ham.Model(sysd)
    Z = W.gaussian_block(1, m.npw, m.p)
    Phi0 = np.concatenate([mf.polar(b)[0] for b in m.blocks(Z)], axis=0)
    prm = dict(W.DEFAULT_PARAMS, tol=1e-12, method=B.EAHP_L2RCG, retraction=retraction)
    _, st_o, stats_o = l2rcg.l2rcg(m, Phi0, prm, maxit=nsteps)
    gp = B.Problem(sysd)
    Psi = gp.to_device(Z)
    sp = B.SolveParams.from_dict(prm)
    sv = C.c_void_p()
    B._check(gp.lib.eahp_solver_create(gp.pb, C.c_void_p(Psi.data_ptr()), C.byref(sp), C.byref(sv)))
    energies, trials = [], []
    st = B.Stats()
    for _ in range(nsteps):
        B._check(gp.lib.eahp_solver_step(sv, 1, C.byref(st)), allow=(-8,))
        energies.append(st.energy)
        trials.append(st.ls_trials - sum(trials))
    out = gp.empty_frame()
    B._check(gp.lib.eahp_solver_get(sv, C.c_void_p(out.data_ptr()), None, None))
    gp.lib.eahp_solver_destroy(sv)
    print(name, retraction, "gpu", energies, trials, "oracle", stats_o["energy"][1:], stats_o["trials"], flush=True)
    assert trials == stats_o["trials"]
    for a, b in zip(energies, stats_o["energy"][1:]):
        assert abs(a - b) <= 1e-9 * abs(b)
    assert rel(gp.to_blocks(out), st_o["Phi"]) < 1e-8
    gp.close()


def test_converged_solve_matches_scf_ground_state():
    B = _lib()
    with open(os.path.join(GOLD, "si8_gamma_e10.json")) as f:
        g = json.load(f)
    gp = B.Problem(W.config("si8_gamma_e10"))
    Psi = gp.to_device(W.gaussian_block(1, gp.npw, gp.p))
    prm = dict(W.DEFAULT_PARAMS, tol=1e-8, maxit=3000, method=B.EAHP_L2RCG)
    st, rc = gp.solve(Psi, prm)
    print("l2rcg", st, flush=True)
    assert st["rnorm"] <= 1e-8
    assert abs(st["energy"] - g["E_scf"]) <= 1e-10 * abs(g["E_scf"])
    gp.close()
