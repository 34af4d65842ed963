"""Stored expected values (tests/golden/, written by tests/golden/make_golden.py from the
oracle only): the oracle must keep reproducing them, and the stored Airy line must stay
within the Simpson rule's error of the paper's closed form (Sec. 5.2.2)."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_golden as MG  # noqa: E402


def _load(name):
    v = np.loadtxt(os.path.join(HERE, "golden", name), comments="#")
    return v[:, 0] + 1j * v[:, 1]


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def test_airy_line_fixture():
    stored = _load("airy_line.txt")
    E, ref = MG.airy_line()
    assert _rel(E, stored[:41]) < 1e-13
    assert _rel(ref, stored[41:]) < 1e-13
    # the stored field is the paper's Airy disk to within Simpson's error at 65 nodes
    assert _rel(stored[:41], stored[41:]) < 1e-6


def test_fresnel_fixture():
    stored = _load("fresnel_q.txt")
    qs, qp = MG.fresnel_q()
    assert _rel(np.concatenate([qs, qp]), stored) < 1e-14
    assert np.all(stored[:9].imag[:4] == 0) and np.any(stored[:9].imag != 0)   # complex past the critical angle


def test_vectorial_psf_fixture():
    stored = _load("psf_vectorial.txt")
    assert _rel(MG.psf_vectorial(), stored) < 1e-13
