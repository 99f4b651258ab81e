"""The C ABI without a GPU: libeahp.so loads, exports every function that
include/eahp.h declares, and its host-only entry points agree with the
oracle (plane-wave counts per k-point and the FFT box of every workload,
computed from the definitions of the basis)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eahp.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(eahp_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2503_16225_amd import load_library
    return load_library()


def test_library_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 30
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    for code in range(0, -10, -1):
        s = lib.eahp_strerror(code).decode()
        assert s and s != "unknown status"
    assert lib.eahp_strerror(-99).decode() == "unknown status"


@pytest.mark.parametrize("name", ["si8_gamma_e10", "si64_gamma_e20", "si8_k444_e15", "si216_gamma_e15",
                                  "si8_gamma_e3"])
def test_layout_matches_oracle_basis(name):
    from oracle import basis
    from paper_2503_16225_amd import layout_estimate
    sysd = W.config(name)
    npw, fft, nbytes = layout_estimate(sysd)
    assert tuple(fft) == tuple(sysd["fft"])
    lat = sysd["lattice"]
    expect = [basis.basis(lat, u, sysd["ecut"], sysd["fft"])["m"].shape[0] for u in sysd["kfrac"]]
    assert npw == expect
    assert nbytes > 16 * sum(npw) * sysd["p"]


def test_layout_auto_box_matches_oracle():
    """fft = 0: the smallest 2/3/5-smooth size that holds every G - G'."""
    from oracle import basis
    from paper_2503_16225_amd import layout_estimate
    for rid in range(6):
        r = W.serving_request(rid)
        sysd = W.system(r["lattice"], r["frac"], r["Z"], r["ecut"], (0, 0, 0), r["kfrac"], r["kweight"])
        npw, fft, _ = layout_estimate(sysd)
        assert tuple(fft) == tuple(basis.auto_fft(sysd["lattice"], sysd["kfrac"], sysd["ecut"]))


def test_invalid_description_is_rejected(lib):
    from paper_2503_16225_amd.binding import SystemDesc
    d = SystemDesc()
    d.nk = 0
    assert lib.eahp_layout_estimate(C.byref(d), None, None, None) == -1
