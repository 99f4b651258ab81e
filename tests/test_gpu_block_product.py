"""Complex block products (eahp_block_product) in every tile shape.

The products V^* W and V Y of Secs. 5.1 and 5.2 run on the matrix cores in
several tile shapes among which the autotuner chooses.  Every shape
accumulates each output element over the inner dimension in the same order,
so all shapes must give the same bits; shape 0 is compared with the product
in complex128 on the host at a tolerance derived from the precision: the
inner dimension is summed in chunks of 4 inside the MFMA and sequentially
beyond, so the error of an element is bounded by about k u sum |a_i||b_i|
(u the unit roundoff, k the inner length); the inputs are unit Gaussians,
where the observed error is far below that bound, and the tests take
50 sqrt(k) u max|C| (FP64: u = 1.1e-16, FP32: u = 6e-8).
Shapes: ragged edges in every dimension, sizes below one tile, several tiles
with a ragged tail, an empty inner dimension, beta = 0 and beta != 0.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NSHAPES = 8  # candidates of FP32 (FP64 has 5; forcing beyond clamps to the last)

CASES = [  # (op, n, a, b)
    (0, 1000, 37, 70),
    (0, 5003, 300, 433),
    (0, 17, 5, 3),
    (0, 40000, 130, 150),
    (1, 1000, 37, 70),
    (1, 5003, 300, 433),
    (1, 17, 5, 3),
    (1, 3001, 0, 20),
    (1, 20000, 600, 145),
]


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_16225_amd import binding as B
    g = B.Problem(W.config("si8_gamma_e10"))
    yield B, g
    B.autotune_force(-1)
    g.close()


def _cplx(seed, rows, cols):
    """Column-major rows x cols matrix as a (cols, rows) array."""
    if rows * cols == 0:
        return np.zeros((cols, rows), np.complex128)
    re = W.gaussian_real(seed, (cols, rows))
    im = W.gaussian_real(seed + 1000, (cols, rows))
    return re + 1j * im


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("case", CASES)
def test_block_product_all_shapes(gp, case, fp32):
    B, g = gp
    op, n, a, b = case
    ct = torch.complex64 if fp32 else torch.complex128
    A = _cplx(11, n, a)
    Bm = _cplx(12, n, b) if op == 0 else _cplx(12, a, b)
    rows_c = a if op == 0 else n
    C0 = _cplx(13, rows_c, b)
    for beta in (0.0, 0.5):
        # reference in complex128 on the host, from the values the GPU sees
        Ah = A.astype(np.complex64).astype(np.complex128) if fp32 else A
        Bh = Bm.astype(np.complex64).astype(np.complex128) if fp32 else Bm
        Ch = C0.astype(np.complex64).astype(np.complex128) if fp32 else C0
        # arrays are (cols, rows): column-major matrices are their transposes
        Am, Bmat, Cm = Ah.T, Bh.T, Ch.T
        ref = (Am.conj().T @ Bmat if op == 0 else Am @ Bmat) + beta * Cm
        Ad = torch.from_numpy(A).to(ct).cuda()
        Bd = torch.from_numpy(Bm).to(ct).cuda()
        outs = []
        for c in range(NSHAPES):
            B.autotune_force(c)
            Cd = torch.from_numpy(C0).to(ct).cuda()
            g.block_product(op, Ad, Bd, Cd, beta)
            outs.append(Cd.cpu().numpy())
        B.autotune_force(-1)
        for c in range(1, NSHAPES):
            assert np.array_equal(outs[c], outs[0]), (case, fp32, beta, c)
        got = outs[0].T.astype(np.complex128)
        k = n if op == 0 else a
        u = 6e-8 if fp32 else 1.1e-16
        scale = max(np.abs(ref).max(), 1.0)
        err = np.abs(got - ref).max()
        print(case, "fp32" if fp32 else "fp64", "beta", beta, "max err", err, "scale", scale, flush=True)
        assert err <= 50 * np.sqrt(max(k, 1)) * u * scale


def test_tuned_products_identical(gp):
    """With the autotuner on, the chosen shapes give the bits of shape 0
    (products of at least 2e10 flops are tuned)."""
    B, g = gp
    n, a, b = 40000, 600, 145
    A = torch.from_numpy(_cplx(21, n, a)).to(torch.complex64).cuda()
    M = torch.from_numpy(_cplx(22, a, b)).to(torch.complex64).cuda()
    Bn = torch.from_numpy(_cplx(23, n, b)).to(torch.complex64).cuda()
    B.autotune_force(0)
    C1 = torch.zeros((b, n), dtype=torch.complex64, device="cuda")
    G1 = torch.zeros((b, a), dtype=torch.complex64, device="cuda")
    g.block_product(1, A, M, C1)
    g.block_product(0, A, Bn, G1)
    B.autotune_force(-1)
    B.autotune_enable(True)
    try:
        for _ in range(2):  # first call tunes, second takes the kept choice
            C2 = torch.zeros_like(C1)
            G2 = torch.zeros_like(G1)
            g.block_product(1, A, M, C2)
            g.block_product(0, A, Bn, G2)
            assert torch.equal(C1, C2) and torch.equal(G1, G2)
        rep = B.autotune_report()
        print(rep, flush=True)
        assert "gemm_nn f32" in rep and "gemm_hn f32" in rep
    finally:
        B.autotune_enable(False)
