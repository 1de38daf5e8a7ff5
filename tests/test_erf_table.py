"""The piecewise-polynomial table of erf(z)/z that the propagation evaluates
for the Shin-Metiu coupling (paper_1805_11169_amd/csrc/erf_table.inc, written
by gen_erf_table.py): read back from the header and evaluated by Horner's rule
in double precision, it agrees with scipy's erf(z)/z to a few units in the last
place on all of [0, 6); beyond 6, erf rounds to 1 in double precision, which is
what lets the kernel take 1/|d| there."""

import pathlib
import re

import numpy as np
from scipy.special import erf

INC = pathlib.Path(__file__).resolve().parents[1] / "paper_1805_11169_amd" / "csrc" / "erf_table.inc"


def _table():
    text = INC.read_text()
    pieces = int(re.search(r"kErfPieces = (\d+);", text).group(1))
    terms = int(re.search(r"kErfTerms = (\d+);", text).group(1))
    body = text[text.index("= {") + 3:text.rindex("};")]
    rows = re.findall(r"\{([^{}]*)\}", body)
    tab = np.array([[float(v) for v in row.split(",") if v.strip()] for row in rows])
    assert tab.shape == (pieces, terms)
    return tab


def _eval(tab, z):
    j = np.minimum((z * 4.0).astype(int), tab.shape[0] - 1)
    s = z - (j + 0.5) * 0.25
    e = tab[j, -1]
    for k in range(tab.shape[1] - 2, -1, -1):
        e = e * s + tab[j, k]
    return e


def test_table_matches_erf_over_z():
    tab = _table()
    z = np.concatenate([np.linspace(1e-6, 6.0, 200001, endpoint=False), np.arange(24) * 0.25 + 1e-12])
    got = _eval(tab, z)
    ref = erf(z) / z
    rel = np.abs(got - ref) / ref
    assert rel.max() < 4 * 2.0 ** -52, rel.max()


def test_table_limit_at_zero():
    tab = _table()
    assert abs(_eval(tab, np.array([0.0]))[0] - 2.0 / np.sqrt(np.pi)) < 2 * 2.0 ** -52


def test_erf_is_one_from_six_on():
    z = np.linspace(6.0, 50.0, 1001)
    assert np.all(erf(z) == 1.0)
    assert erf(5.8) < 1.0   # the table does cover where it is not
