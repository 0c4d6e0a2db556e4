"""Pin of the whole oracle loop to values the paper prints: Section 5.2,
Table 1, n = 5000 rows (Matrix 1 and Matrix 2, P = 1, b = 50, paper p rules).

The printed rank l is forced by the method being near-optimal (the
Eckart-Young minimal ranks are 313 / 497 / 185 / 245, which blocks of 50
round up to the printed l), so a wrong step anywhere in the loop moves l.
eps_opt is a 20-trial mean; one seeded trial is held to +-10% of it, and to
the hard bounds EY(l) <= eps_opt <= eps.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import FarpcaParams, farpca
from paper_2506_03859_amd import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_n5000.json")))
N = 5000


@pytest.fixture(scope="module")
def matrices():
    return {1: (synth.matrix1(N, seed=11), synth.matrix1_sigma(N)),
            2: (synth.matrix2(N, seed=12), synth.matrix2_sigma(N))}


CASES = [(ri, ci) for ri in range(len(GOLD["rows"])) for ci in range(len(GOLD["columns"]))]


@pytest.mark.slow
@pytest.mark.parametrize("ri,ci", CASES)
def test_table1_rank_and_error(matrices, ri, ci):
    row = GOLD["rows"][ri]
    sketch = GOLD["columns"][ci]
    a, sigma = matrices[row["matrix"]]
    r = farpca(a, FarpcaParams(tol=row["eps"], power=1, sketch=sketch, seed=7 + ci))
    assert r.status == 0
    assert r.rank == row["l"][ci]
    eps_opt = np.linalg.norm(a - (r.U * r.S) @ r.V.T) / math.sqrt(r.norm_a2)
    ey = math.sqrt(np.sum(sigma[r.rank:] ** 2) / np.sum(sigma ** 2))
    assert ey <= eps_opt <= row["eps"]
    assert abs(eps_opt / row["eps_opt"][ci] - 1.0) < 0.10
    # the indicator the loop stopped on is the true squared error, up to the
    # FP64 cancellation in ||A||^2 - tr(T Z^{-1}) (Section 2.1: reliable for
    # eps above about 2.1e-7)
    assert abs(r.err_indicator / r.norm_a2 - eps_opt ** 2) < 1e-12
