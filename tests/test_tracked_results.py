"""The tracked campaign rows (results/) agree with the code that computes
their summaries and with the paper's Table 1 (Sec. 4).  No GPU: the rows
hold C(x) and its error per increment, as the campaign wrote them."""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

from paper_2304_03311_amd import analysis

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE1 = {r["L"]: r for r in json.load(open(os.path.join(ROOT, "tests", "golden", "paper_values.json")))[
    "table1_fit_k"]["rows"]}


@pytest.mark.parametrize("name", ["table1_2d_L32", "table1_2d_L32_th40k", "table1_2d_L64", "table1_2d_L64_nt4096",
                                  "table1_2d_L128"])
def test_table1_rows_refit_and_agree_with_the_paper(name):
    rows = json.load(open(os.path.join(ROOT, "results", f"{name}.json")))
    assert len(rows) == 1
    row = rows[0]
    L = row["L"]
    x, C, err = (np.array(row[k]) for k in ("x", "C", "C_err"))
    # one midpoint per increment, x = (l + 1/2) / L
    assert len(x) == L and np.allclose(x, (np.arange(L) + 0.5) / L)
    k, k_err, chi = analysis.fit_k_2d(x, C, err, L)
    assert k == pytest.approx(row["k"], rel=1e-12) and k_err == pytest.approx(row["k_err"], rel=1e-12)
    assert chi == pytest.approx(row["chi2_fit"], rel=1e-12)
    ref = TABLE1[L]
    pull = (k - ref["k"]) / math.hypot(k_err, ref["k_err"])
    print(f"L={L}: k={k:.4f}({k_err:.4f}) paper {ref['k']}({ref['k_err']}) pull {pull:+.2f}, "
          f"chi2/nu {chi:.2f} (paper {ref['chi2_dof']})")
    assert abs(pull) < 2.5
    assert chi < 2.0
