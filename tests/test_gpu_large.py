"""The largest workload at full size: 3x3x3 supercell of the 8-atom cell,
+2% strain, 216 atoms, p = 432, Ecut 15 Ha, 86119 plane waves, 120^3 box
(its (y, z) planes exceed LDS in FP64 and take the split-plane transforms;
p x p problems exceed the one-work-group kernels and take the general ones).
The oracle computes the density and energy everywhere, H on sampled columns
and the retraction; one mixed-precision solver step is checked for descent
and for the consistency of its energy with the oracle's at the iterate.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def si216():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import hamiltonian as ham, manifold as mf
    sysd = W.config("si216_gamma_e15")
    om = ham.Model(sysd, workers=16)
    Z = W.gaussian_block(1, om.npw, om.p)
    Phi = np.concatenate([mf.polar(b)[0] for b in om.blocks(Z)], axis=0)
    rho_o = ham.density(om, Phi, chunk=16)
    Veff_o, _ = ham.potentials(om, rho_o)
    E_o = ham.energy_terms(om, Phi, rho_o)[0]["total"]
    print("si216 npw", om.npw, "fft", om.fft, "E", E_o, flush=True)
    return sysd, om, Phi, rho_o, Veff_o, E_o


def test_si216_density_energy_apply(si216):
    sysd, om, Phi, rho_o, Veff_o, E_o = si216
    from oracle import hamiltonian as ham
    from paper_2503_16225_amd import Problem
    gp = Problem(sysd)
    assert gp.npw == om.npw and gp.fft == (120, 120, 120)
    Phid = gp.to_device(Phi)
    rho, veff = gp.density(Phid)
    assert rel(rho.cpu().numpy().reshape(om.fft), rho_o) < 1e-12
    assert rel(veff.cpu().numpy().reshape(om.fft), Veff_o) < 1e-12
    E, _ = gp.energy(Phid)
    print("si216 E", E, E_o, flush=True)
    assert abs(E - E_o) <= 1e-11 * abs(E_o)
    X = W.gaussian_block(3, om.npw, om.p)
    HX = gp.to_blocks(gp.apply_H(Phid, gp.to_device(X)))
    cols = [0, 1, 215, 431]
    HX_o = ham.apply_H_k(om, 0, Veff_o, X[:, cols])
    print("si216 apply_H sampled", rel(HX[:, cols], HX_o), flush=True)
    assert rel(HX[:, cols], HX_o) < 1e-12
    gp.close()


def test_si216_retraction(si216):
    sysd, om, Phi, rho_o, Veff_o, E_o = si216
    from oracle import manifold as mf
    from paper_2503_16225_amd import Problem
    gp = Problem(sysd)
    G = W.gaussian_block(8, om.npw, om.p)
    M = Phi.conj().T @ G
    eta = 0.05 * (G - Phi @ (0.5 * (M + M.conj().T)))
    Pn_o, _ = mf.retract(om, Phi, eta, 0.7)
    Pn = gp.to_blocks(gp.retract(gp.to_device(Phi), gp.to_device(eta), 0.7))
    print("si216 retract", rel(Pn, Pn_o), flush=True)
    assert rel(Pn, Pn_o) < 1e-11
    gp.close()


def test_si216_mixed_solver_step(si216):
    sysd, om, Phi, rho_o, Veff_o, E_o = si216
    import ctypes as C

    from oracle import hamiltonian as ham
    from paper_2503_16225_amd import binding as B
    gp = B.Problem(sysd, precision=B.EAHP_MIXED)
    Psi = gp.to_device(Phi)
    sp = B.SolveParams.from_dict(dict(W.DEFAULT_PARAMS))
    sv = C.c_void_p()
    B._check(gp.lib.eahp_solver_create(gp.pb, C.c_void_p(Psi.data_ptr()), C.byref(sp), C.byref(sv)))
    s = B.Stats()
    B._check(gp.lib.eahp_solver_step(sv, 1, C.byref(s)), allow=(-8,))
    out = gp.empty_frame()
    e_, r_ = C.c_double(), C.c_double()
    B._check(gp.lib.eahp_solver_get(sv, C.c_void_p(out.data_ptr()), C.byref(e_), C.byref(r_)))
    gp.lib.eahp_solver_destroy(sv)
    P1 = gp.to_blocks(out)
    rho1 = ham.density(om, P1, chunk=16)
    E1_o = ham.energy_terms(om, P1, rho1)[0]["total"]
    print("si216 mixed step", E_o, "->", s.energy, "oracle at iterate", E1_o, "napply", s.napply, "fp32",
          s.napply_fp32, flush=True)
    assert s.energy < E_o
    assert abs(E1_o - s.energy) <= 1e-11 * abs(E1_o)
    assert s.napply_fp32 > 0
    gp.close()
