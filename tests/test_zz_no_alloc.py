"""eahp_ea_gradient_noalloc (no device allocation, a fixed scratch array)
against eahp_ea_gradient through the C ABI: two calls in a row, the second on
a smaller problem (fewer plane waves, fewer orbitals, one k-point instead of
two), each to the FP64 bar of the gradient (1e-13 relative: the same kernels,
with the row split of the Gram product possibly capped differently); a
problem whose p x p products do not fit the array is rejected before any
device work."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _frames(om, seed):
    from oracle import manifold as mf
    Z = W.gaussian_block(seed, om.npw, om.p)
    Phi = np.concatenate([mf.polar(b)[0] for b in om.blocks(Z)], axis=0)
    X = Phi + 0.3 * W.gaussian_block(seed + 1, om.npw, om.p)
    return Phi, X


def test_noalloc_gradient_matches_allocating_entry_point():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import hamiltonian as ham
    from paper_2503_16225_amd import Problem, load_library
    lib = load_library()
    assert lib.eahp_noalloc_scratch_bytes() == 32 << 20
    cases = [
        ("si8 Ecut 10, 2 k-points, p = 200", W.system(*W.diamond_cell(), 10.0, (32, 32, 32),
                                                    np.array([[0.25, 0.25, 0.25], [-0.25, 0.25, 0.0]]),
                                                    np.array([0.5, 0.5]), p=200)),
        ("si8 Ecut 3, Gamma, p = 16", W.system(*W.diamond_cell(), 3.0, (0, 0, 0))),
    ]
    for name, sysd in cases:
        print("case", name, flush=True)
        om = ham.Model(sysd)
        gp = Problem(sysd)
        Phi, X = _frames(om, 21)
        Pd, Xd = gp.to_device(Phi), gp.to_device(X)
        G_ref = gp.to_blocks(gp.ea_gradient(Pd, Xd))
        G = gp.empty_frame()
        G.fill_(float("nan"))
        G = gp.to_blocks(gp.ea_gradient_noalloc(Pd, Xd, G))
        print(name, "noalloc vs allocating", rel(G, G_ref), flush=True)
        assert np.all(np.isfinite(G))
        assert rel(G, G_ref) < 1e-13
        gp.close()


def test_noalloc_rejects_what_does_not_fit():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_16225_amd import EahpError, Problem
    k, w = W.mp_grid((3, 3, 1))
    sysd = W.system(*W.diamond_cell(), 10.0, (32, 32, 32), k, w, p=512)  # 9 x 512^2 x 16 bytes > 32 MiB
    gp = Problem(sysd)
    Pd = gp.empty_frame()
    G = gp.empty_frame()
    with pytest.raises(EahpError) as e:
        gp.ea_gradient_noalloc(Pd, Pd, G)
    assert e.value.status == -1 and "scratch" in str(e.value)
    gp.close()
