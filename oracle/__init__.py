"""Plain FP64 CPU oracle for the EARCG hot path (test infrastructure only).

This package is a slow, deliberately straightforward numpy/scipy
implementation of what the HIP library computes.  It exists to check the
library: only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it.  The product path never calls it, and it
shares no code with the library (only the seeded inputs of ``workloads``).

Modules, in the order the method uses them:

* ``basis``       plane-wave basis, FFT box, reciprocal lattice (Sec. 5.1)
* ``hamiltonian`` density, potentials, H-apply through FFTs, dense H,
                  energy (eq. (1.1) energy functional, eq. (1.4) Hamiltonian,
                  in the Hartree scaling of the experiments, Sec. 5.1)
* ``manifold``    Lambda, residual, polar retraction, transports, TPA
                  preconditioner, energy-adaptive gradient (Secs. 2-5)
* ``fom``         preconditioned block FOM for the Sylvester equation
                  (Appendix A, Algorithm 4)
* ``linesearch``  modified secant step size strategy (Algorithm 2)
* ``earcg``       energy-adaptive RCG (Algorithm 3)
* ``eargd``       energy-adaptive gradient descent (Sec. 5.2 comparison)
* ``l2rcg``       L2-gradient RCG (Sec. 5.2 comparison)
* ``symmetry``    crystal symmetry, symmetry-reduced k-sets and density
                  symmetrisation (Sec. 5.1, periodic structures)
* ``scf``         dense SCF ground state: a pin of the minimisers and the
                  oracle of the SCF comparator (Sec. 5.2)

Every function is pinned by the ``-m "not gpu"`` tests against closed forms,
brute force or invariants; none is marked "parity unpinned".
"""
