"""Writes the stored reference values under tests/golden/ (calls only oracle/).

    python tests/golden/make_golden.py

si8_gamma_e10.json: 8-atom diamond cell, Gamma, Ecut 10 Ha, 32^3 box, p = 16,
seeded start (gaussian_block seed 1, polar factor).  Holds the dense-SCF
ground-state energy and Lambda spectrum, the HOMO-LUMO gap, the oracle
EARCG energy at ||R||_F <= 1e-8 and its first iterations (E, ||R||_F, tau).
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import earcg, hamiltonian as ham, manifold as mf, scf  # noqa: E402


def main():
    m = ham.Model(W.config("si8_gamma_e10"), workers=8)
    Z = W.gaussian_block(1, m.npw, m.p)
    Phi0 = np.concatenate([mf.polar(b)[0] for b in m.blocks(Z)], axis=0)
    ref = scf.scf(m, Phi0=Phi0)
    prm = dict(W.DEFAULT_PARAMS, tol=1e-8)
    Phi, st, stats = earcg.earcg(m, Phi0, prm)
    out = dict(
        config="si8_gamma_e10", seed=1, npw=m.npw, fft=list(m.fft), p=m.p,
        E_scf=ref["E"], lambda_scf=[float(x) for x in ref["eigs"][0][:m.p]], gap=ref["gap"],
        E_earcg=st["E"], lambda_earcg=[float(x) for x in np.linalg.eigvalsh(st["lams"][0])],
        rnorm_final=stats["rnorm"][-1], iters=stats["iters"], napply=stats["napply"],
        first_energies=stats["energy"][:4], first_rnorms=stats["rnorm"][:4], first_taus=stats["taus"][:3],
        terms={k: v for k, v in st["terms"].items()},
    )
    with open(os.path.join(HERE, "si8_gamma_e10.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
