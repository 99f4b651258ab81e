"""k-point batching at full size: the 8-atom cell on an unreduced 4x4x4
Monkhorst-Pack grid (64 k-points, ragged plane-wave counts 2984-3022, Ecut
15 Ha, 40^3 box, p = 16 per k).  Every k-block is processed in the same
launches (ragged tables); results are compared with the oracle on every
k-point: density, potential and energy, H applied to every column, Lambda
and the residual, the retraction and transport, and the metric solve of
Algorithm 4 (independent stopping per k).  FP64 tolerances as in the other
parity tests.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def k444():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import hamiltonian as ham, manifold as mf
    from paper_2503_16225_amd import Problem
    sysd = W.config("si8_k444_e15")
    om = ham.Model(sysd, workers=8)
    gp = Problem(sysd)
    assert gp.nk == 64 and gp.npw == om.npw and gp.fft == om.fft
    Z = W.gaussian_block(1, om.npw, om.p)
    Phi = np.concatenate([mf.polar(b)[0] for b in om.blocks(Z)], axis=0)
    st = mf.state(om, Phi)
    print("k444 npw", min(om.npw), max(om.npw), "E", st["E"], flush=True)
    yield om, gp, Phi, st
    gp.close()


def test_k444_density_energy_residual(k444):
    om, gp, Phi, st = k444
    from oracle import hamiltonian as ham
    Phid = gp.to_device(Phi)
    rho, veff = gp.density(Phid)
    rho_o = ham.density(om, Phi)
    assert rel(rho.cpu().numpy().reshape(om.fft), rho_o) < 1e-12
    assert rel(veff.cpu().numpy().reshape(om.fft), st["Veff"]) < 1e-12
    E, _ = gp.energy(Phid)
    assert abs(E - st["E"]) <= 1e-11 * abs(st["E"])
    R, L, rn, E2 = gp.residual(Phid)
    assert rel(gp.to_blocks(R), st["R"]) < 1e-10
    for a, b in zip(gp.lambdas(L), st["lams"]):
        assert np.abs(a - b).max() < 1e-10 * np.abs(b).max()
    assert abs(rn - np.linalg.norm(st["R"])) <= 1e-10 * rn


def test_k444_apply_H_every_k(k444):
    om, gp, Phi, st = k444
    from oracle import hamiltonian as ham
    X = W.gaussian_block(3, om.npw, om.p)
    HX = gp.to_blocks(gp.apply_H(gp.to_device(Phi), gp.to_device(X)))
    o = 0
    worst = 0.0
    for k, (n, Xk) in enumerate(zip(om.npw, om.blocks(X))):
        ref = ham.apply_H_k(om, k, st["Veff"], Xk)
        worst = max(worst, rel(HX[o:o + n], ref))
        o += n
    print("k444 apply_H worst rel", worst, flush=True)
    assert worst < 1e-12


def test_k444_retract_transport(k444):
    om, gp, Phi, st = k444
    from oracle import manifold as mf
    G = W.gaussian_block(8, om.npw, om.p)
    eta = np.concatenate([Gk - Pk @ (0.5 * (Pk.conj().T @ Gk + Gk.conj().T @ Pk))
                          for Pk, Gk in zip(om.blocks(Phi), om.blocks(G))], axis=0) * 0.1
    v = W.gaussian_block(9, om.npw, om.p)
    tau = 0.6
    Pn_o, facs = mf.retract(om, Phi, eta, tau)
    Pn = gp.to_blocks(gp.retract(gp.to_device(Phi), gp.to_device(eta), tau))
    assert rel(Pn, Pn_o) < 1e-12
    T_o = mf.transport_general(om, Pn_o, tau * eta, v, facs)
    T = gp.to_blocks(gp.transport(gp.to_device(Phi), gp.to_device(tau * eta), gp.to_device(v)))
    assert rel(T, T_o) < 1e-10


def test_k444_metric_solve_every_k(k444):
    om, gp, Phi, st = k444
    from oracle import earcg
    prm = dict(W.DEFAULT_PARAMS)
    lam_max = max(np.linalg.eigvalsh(L)[-1] for L in st["lams"])
    mu = lam_max - float(st["Veff"].min()) + 1.0
    X_o, info_o = earcg.metric_solve(om, Phi, st["HPhi"], st["lams"], st["Veff"], mu, prm)
    X, its, rr = gp.metric_solve(gp.to_device(Phi), mu, prm["fom_rtol"], prm["fom_maxit"])
    X = gp.to_blocks(X)
    print("k444 fom iterations", sorted(set(its)), "rel", rel(X, X_o), flush=True)
    assert its == [i["iters"] for i in info_o]
    for a, i in zip(rr, info_o):
        assert abs(a - i["relres"]) <= 1e-7 * i["relres"] + 1e-13
    assert rel(X, X_o) < 1e-9


def test_k444_metric_solve_deep_krylov(k444):
    """The metric solve to a relative residual of 1e-6: the k-points need 8
    or 9 FOM iterations, so the projected order q = 16 j crosses 128, where
    the batched tridiagonal reductions of the projected systems (all 64
    k-points in shared cooperative launches) change to their next register
    size."""
    om, gp, Phi, st = k444
    from oracle import earcg
    rtol, maxit = 1e-6, 40
    prm = dict(W.DEFAULT_PARAMS, fom_rtol=rtol, fom_maxit=maxit)
    lam_max = max(np.linalg.eigvalsh(L)[-1] for L in st["lams"])
    mu = lam_max - float(st["Veff"].min()) + 1.0
    X_o, info_o = earcg.metric_solve(om, Phi, st["HPhi"], st["lams"], st["Veff"], mu, prm)
    X, its, rr = gp.metric_solve(gp.to_device(Phi), mu, rtol, maxit)
    X = gp.to_blocks(X)
    print("k444 deep fom iterations", sorted(set(its)), "rel", rel(X, X_o), flush=True)
    assert max(its) * om.p > 128
    assert its == [i["iters"] for i in info_o]
    for a, i in zip(rr, info_o):
        assert abs(a - i["relres"]) <= 1e-7 * i["relres"] + 1e-13
    assert rel(X, X_o) < 1e-9


def test_k444_solver_steps_are_consistent(k444):
    """Two EARCG steps on the GPU (FP64 and mixed): the energy decreases and
    the oracle's energy of the GPU iterate equals the GPU's own."""
    om, gp, Phi, st = k444
    from oracle import manifold as mf
    from paper_2503_16225_amd import binding as B
    import ctypes as C
    for prec in (B.EAHP_FP64, B.EAHP_MIXED):
        p2 = B.Problem(W.config("si8_k444_e15"), precision=prec)
        Psi = p2.to_device(Phi)
        sp = B.SolveParams.from_dict(dict(W.DEFAULT_PARAMS))
        sv = C.c_void_p()
        B._check(p2.lib.eahp_solver_create(p2.pb, C.c_void_p(Psi.data_ptr()), C.byref(sp), C.byref(sv)))
        s = B.Stats()
        E = [st["E"]]
        for _ in range(2):
            B._check(p2.lib.eahp_solver_step(sv, 1, C.byref(s)), allow=(-8,))
            E.append(s.energy)
        out = p2.empty_frame()
        e_, r_ = C.c_double(), C.c_double()
        B._check(p2.lib.eahp_solver_get(sv, C.c_void_p(out.data_ptr()), C.byref(e_), C.byref(r_)))
        p2.lib.eahp_solver_destroy(sv)
        P1 = p2.to_blocks(out)
        E_o = mf.state(om, P1)["E"]
        print("k444 precision", prec, "energies", E, "oracle at iterate", E_o, flush=True)
        assert E[1] < E[0] and E[2] < E[1]
        assert abs(E_o - s.energy) <= 1e-11 * abs(E_o)
        p2.close()
