"""Stored expected values (tests/golden/, written by tests/golden/make_golden.py
without the HIP library): the oracle reproduces them, and the loader used
by the GPU parity tests reads them."""
import os

import numpy as np

import oracle
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
EPS = 2.0 ** -52


def load_golden(name: str) -> dict:
    """Arrays of a fixture file: '# ...' comment lines, then blocks of
    'NAME rows cols' followed by the rows."""
    out, lines = {}, [l for l in open(os.path.join(GOLDEN, name)) if not l.startswith("#")]
    i = 0
    while i < len(lines):
        key, r, c = lines[i].split()
        r, c = int(r), int(c)
        out[key] = np.array([[float(v) for v in lines[i + 1 + k].split()] for k in range(r)]).reshape(r, c)
        i += 1 + r
    return out


def test_tiny_exact_r_is_reproduced_by_the_oracle():
    g = load_golden("tiny_exact_r.txt")
    R = oracle.householder_r(g["X"])
    kappa = np.linalg.cond(g["R"])
    assert oracle.rel_err_r(R, g["R"]) <= 64 * EPS * kappa
    assert np.allclose(g["R"].T @ g["R"], g["X"].T @ g["X"], rtol=1e-14, atol=0)


def test_config1_r_is_the_oracle_value_bit_for_bit():
    g = load_golden("config1_r.txt")
    assert np.array_equal(oracle.householder_r(wl.config1()), g["R"])
