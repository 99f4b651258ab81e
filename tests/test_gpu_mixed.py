"""Mixed precision (EAHP_MIXED): the metric solve of Algorithm 4 runs in single
precision (Krylov basis, its H-applies, TPA, orthogonalisation and the Gram
products; the small projected Sylvester problem is solved in FP64, except that
its Householder reduction beyond q = 512 stores the trailing matrix in FP32),
everything else in FP64.

Bars: a converged mixed solve matches the dense-SCF ground-state energy to
1e-7 relative and the FP64 solve's orbital subspace to a 1e-5 principal angle;
the single-precision FOM iterate matches the FP64 oracle's FOM iterate to
1e-4 relative (FP32 rounding ~6e-8 amplified by the Krylov recurrence).
"""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_16225_amd import binding
    return binding


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def sin_max_angle(P, Q):
    """sin of the largest principal angle between the column spans of the
    orthonormal P and Q: the spectral norm of Q - P (P^H Q)."""
    return float(np.linalg.norm(Q - P @ (P.conj().T @ Q), 2))


@pytest.mark.parametrize("name", ["si8_gamma_e10", "si64_gamma_e20"])
def test_mixed_metric_solve_matches_oracle(name):
    B = _gpu()
    from oracle import earcg, hamiltonian as ham, manifold as mf
    sysd = W.config(name)
    om = ham.Model(sysd, workers=8)
    gp = B.Problem(sysd, precision=B.EAHP_MIXED)
    Z = W.gaussian_block(1, om.npw, om.p)
    Phi = np.concatenate([mf.polar(b)[0] for b in om.blocks(Z)], axis=0)
    st = mf.state(om, Phi)
    lam_max = max(np.linalg.eigvalsh(L)[-1] for L in st["lams"])
    mu = lam_max - float(st["Veff"].min()) + 1.0
    maxit = 3 if name == "si64_gamma_e20" else 50
    prm = dict(W.DEFAULT_PARAMS, fom_rtol=2.5e-2, fom_maxit=maxit)
    X_o, info_o = earcg.metric_solve(om, Phi, st["HPhi"], st["lams"], st["Veff"], mu, prm)
    X, its, rr = gp.metric_solve(gp.to_device(Phi), mu, 2.5e-2, maxit)
    X = gp.to_blocks(X)
    print(name, "mixed fom", its, [i["iters"] for i in info_o], rr, [i["relres"] for i in info_o], rel(X, X_o),
          flush=True)
    assert its == [i["iters"] for i in info_o]
    for a, i in zip(rr, info_o):
        assert abs(a - i["relres"]) <= 1e-4 * i["relres"]
    assert rel(X, X_o) < 1e-4
    gp.close()


def test_mixed_solve_matches_ground_state_and_fp64_subspace():
    B = _gpu()
    with open(os.path.join(GOLD, "si8_gamma_e10.json")) as f:
        g = json.load(f)
    sysd = W.config("si8_gamma_e10")
    prm = dict(W.DEFAULT_PARAMS, tol=1e-8, maxit=300)
    frames, stats = {}, {}
    for prec in (B.EAHP_FP64, B.EAHP_MIXED):
        gp = B.Problem(sysd, precision=prec)
        Psi = gp.to_device(W.gaussian_block(1, gp.npw, gp.p))
        st, rc = gp.solve(Psi, prm)
        print("precision", prec, st, flush=True)
        frames[prec] = gp.to_blocks(Psi)
        stats[prec] = st
        gp.close()
    sm = stats[B.EAHP_MIXED]
    assert sm["rnorm"] <= 1e-8
    assert sm["napply_fp32"] > 0
    assert abs(sm["energy"] - g["E_scf"]) <= 1e-7 * abs(g["E_scf"])
    P, Q = frames[B.EAHP_FP64], frames[B.EAHP_MIXED]
    assert np.abs(Q.conj().T @ Q - np.eye(Q.shape[1])).max() < 1e-12
    ang = sin_max_angle(P, Q)
    print("subspace angle (mixed vs FP64)", ang, flush=True)
    assert ang < 1e-5
