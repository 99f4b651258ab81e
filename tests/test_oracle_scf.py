"""Pins of the oracle's SCF mixing (the oracle of the SCF comparator, A40),
fixed independently of it:

* with one history entry the step is damped simple mixing x + beta f;
* on an affine map g(x) = M x + b in dimension n, Anderson mixing with an
  untruncated history and beta = 1 reaches the fixed point (I - M)^-1 b after
  at most n + 1 steps (its equivalence with GMRES on (I - M) x = b, Walker and
  Ni, SIAM J. Numer. Anal. 49 (2011)); with beta = 1 and depth 2 it is the
  secant method on a scalar affine map, exact after two steps;
* the SCF fixed point of the dense oracle is a point where the density of the
  p lowest eigenvectors of H(rho) is rho (checked in the pins of the
  minimisers against EARCG's converged energy).
"""
import numpy as np

from oracle import scf


def test_single_entry_is_damped_simple_mixing():
    x = np.array([1.0, 2.0, -1.0])
    f = np.array([0.5, -0.25, 0.125])
    assert np.allclose(scf.anderson_next([x], [f], 0.3), x + 0.3 * f)


def run(M, b, x0, beta, depth, steps):
    hx, hf, x = [], [], x0
    for _ in range(steps):
        f = M @ x + b - x
        hx.append(x.copy())
        hf.append(f)
        hx, hf = hx[-depth:], hf[-depth:]
        x = scf.anderson_next(hx, hf, beta)
    return x


def test_affine_map_fixed_point_in_n_plus_one_steps():
    rng = np.random.default_rng(3)
    n = 6
    M = 0.4 * rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    xstar = np.linalg.solve(np.eye(n) - M, b)
    x = run(M, b, np.zeros(n), 1.0, n + 2, n + 1)
    assert np.abs(x - xstar).max() < 1e-10
    x_short = run(M, b, np.zeros(n), 1.0, n + 2, n - 2)
    assert np.abs(x_short - xstar).max() > 1e-8  # not yet there after fewer steps


def test_scalar_secant():
    M, b = np.array([[0.3]]), np.array([1.0])
    x = run(M, b, np.array([5.0]), 1.0, 2, 2)
    assert abs(x[0] - 1.0 / 0.7) < 1e-14
