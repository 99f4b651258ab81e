"""Frame H-applies replayed as HIP graphs (eahp_problem_set_graphs).

The graph path must give the plain launches' results bit for bit: the same
kernels with the same arguments, reading the frames, V_eff and the
workspaces at replay time.  Every replay is checked against the plain
H-apply, with other work of the program (energies, H-applies of other
frames, host synchronisations) between the replays; a full EARCG solve with
graphs on takes the same iterates as with graphs off; the H-apply is also
checked against the oracle.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _problem(sysd):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_16225_amd import binding as B
    s = torch.cuda.Stream()  # graph capture needs a stream other than the legacy default one
    with torch.cuda.stream(s):
        gp = B.Problem(sysd)
    return B, gp


def _frames(gp, om):
    from oracle import manifold as mf
    Z = W.gaussian_block(1, om.npw, om.p)
    Phi = np.concatenate([mf.polar(b)[0] for b in om.blocks(Z)], axis=0)
    X = W.gaussian_block(7, om.npw, om.p)
    X2 = W.gaussian_block(8, om.npw, om.p)
    return Phi, X, X2


def test_graph_replays_equal_plain_launches():
    from oracle import hamiltonian as ham
    sysd = W.config("si8_gamma_e10")
    om = ham.Model(sysd)
    B, gp = _problem(sysd)
    try:
        Phi, X, X2 = _frames(gp, om)
        Pd, Xd, X2d = gp.to_device(Phi), gp.to_device(X), gp.to_device(X2)
        ref = gp.apply_H(Pd, Xd).clone()
        ref2 = gp.apply_H(Pd, X2d).clone()
        # oracle: H X at the potential of Phi
        rho = ham.density(om, Phi)
        Veff, _ = ham.potentials(om, rho)
        HX_o = ham.apply_H_k(om, 0, Veff, X)
        assert np.abs(gp.to_blocks(ref) - HX_o).max() <= 1e-12 * np.abs(HX_o).max()
        gp.set_graphs(True)
        out, out2 = gp.empty_frame(), gp.empty_frame()
        for rep in range(6):
            out.fill_(float("nan"))
            gp.apply_H(Pd, Xd, out)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), rep
            # other work between the replays: an energy, another frame's H-apply, host copies
            gp.energy(Pd)
            gp.apply_H(Pd, X2d, out2)
            assert torch.equal(out2, ref2), rep
            _ = out2.cpu()
        captured, replays = gp.graph_stats()
        print("graphs captured", captured, "replays", replays, flush=True)
        assert captured >= 2 and replays >= 8
        gp.set_graphs(False)
        gp.apply_H(Pd, Xd, out)
        assert torch.equal(out, ref)
    finally:
        gp.close()


def test_graph_solve_takes_the_same_iterates():
    sysd = W.config("si8_gamma_e10")
    prm = dict(W.DEFAULT_PARAMS, tol=1e-8, maxit=60)
    res = []
    for graphs in (False, True):
        B, gp = _problem(sysd)
        try:
            if graphs:
                gp.set_graphs(True)
            Psi = gp.to_device(W.gaussian_block(1, gp.npw, gp.p))
            st, rc = gp.solve(Psi, prm)
            res.append((st["energy"], st["rnorm"], st["iters"], st["napply"], gp.to_blocks(Psi)))
            if graphs:
                captured, replays = gp.graph_stats()
                print("solve with graphs: captured", captured, "replays", replays, flush=True)
                assert replays > 0
        finally:
            gp.close()
    (e0, r0, i0, n0, P0), (e1, r1, i1, n1, P1) = res
    print("plain", e0, r0, i0, "graphs", e1, r1, i1, flush=True)
    assert (e0, r0, i0, n0) == (e1, r1, i1, n1)
    assert np.array_equal(P0, P1)


def test_graphs_need_a_non_default_stream():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_16225_amd import binding as B
    gp = B.Problem(W.config("si8_gamma_e10"))  # bound to torch's default (legacy) stream
    try:
        if torch.cuda.current_stream().cuda_stream != 0:
            pytest.skip("torch's current stream is not the legacy default stream")
        with pytest.raises(B.EahpError):
            gp.set_graphs(True)
    finally:
        gp.close()
