"""CPU checks of the host assembly (S_2 by summation, symmetrised c-function,
2D fit, App. C systematic) against closed forms printed in the paper."""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

from paper_2304_03311_amd import analysis

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def cft_S(l, L, c=0.5, n=2):
    """Sec. 2: S_n(l, L) = (c/6)(1 + 1/n) log((L/pi) sin(pi l/L)) + k_n (k_n = 0 here)."""
    return (c / 6.0) * (1.0 + 1.0 / n) * np.log((L / math.pi) * np.sin(math.pi * np.asarray(l) / L))


def test_cft_c_function_constant_is_one_sixteenth():
    p = json.load(open(GOLDEN))
    assert p["central_charge_2d_ising"]["value"] == 0.5
    # (c/12)(1 + 1/n) at x -> 0 with c = 1/2, n = 2; the fit function's leading term is cos(pi x)/16
    assert analysis.cft_c_function_2d(0.0) == pytest.approx(1.0 / 16.0, rel=1e-15)


def test_renyi_summation():
    dS = np.array([0.3, 0.1, -0.05])
    S, Se = analysis.renyi_from_increments(dS, np.array([0.01, 0.02, 0.02]))
    assert S[0] == 0.0 and np.allclose(S, [0, 0.3, 0.4, 0.35])
    assert Se[-1] == pytest.approx(0.03)


@pytest.mark.parametrize("L", [32, 64, 128])
def test_c_function_of_cft_increments_matches_appendix_c(L):
    """Finite differences of the CFT entropy, placed at the midpoints, give
    cos(pi x)/16 plus the App. C term sin(pi x)/(48 L^2 pi) S'''(x)."""
    l = np.arange(1, L - 1)  # increments l -> l+1 avoiding S(0), S(L)
    dS = cft_S(l + 1, L) - cft_S(l, L)
    x, C = analysis.c_function(dS, L, dim=2, l0=1)
    # S(x) = (1/8) log sin(pi x) + const  =>  S'''(x) = (pi^3/4) cos(pi x) / sin^3(pi x)
    S3 = (math.pi ** 3 / 4.0) * np.cos(np.pi * x) / np.sin(np.pi * x) ** 3
    plain = analysis.cft_c_function_2d(x)
    pred = plain + analysis.discretisation_systematic(x, S3, L, dim=2)
    # near the edges the expansion parameter is 1/l, so the residual does not
    # shrink with L there; the App. C term removes most of it
    assert np.abs(C - pred).max() < np.abs(C - plain).max() / 10
    # in the middle the finite-difference error is O(L^-2) and App. C removes
    # the leading part
    mid = slice(len(x) // 4, 3 * len(x) // 4)
    assert np.abs(C - plain)[mid].max() < 7e-5 * (32.0 / L) ** 2
    assert np.abs(C - pred)[mid].max() < 0.1 * np.abs(C - plain)[mid].max()


def test_fit_recovers_k():
    L = 64
    rng = np.random.default_rng(0)
    x = (np.arange(L) + 0.5) / L
    for k_true in (0.0, 0.138, 0.3):
        C = np.cos(np.pi * x) / 16 + k_true / np.tan(np.pi * x) / (2 * L)
        err = np.full(L, 1e-4)
        k, k_err, chi2 = analysis.fit_k_2d(x, C + rng.normal(0, 1e-4, L), err, L)
        assert abs(k - k_true) < 5 * k_err
        assert 0.5 < chi2 < 2.0


def test_assemble_shapes_and_3d_area():
    dS = np.full(8, 0.01)
    out = analysis.assemble(dS, np.full(8, 0.001), L=8, dim=3, ly=8)
    assert len(out["S"]) == 9 and len(out["C"]) == 8
    x = (np.arange(8) + 0.5) / 8
    assert np.allclose(out["C"], ((8 / math.pi) * np.sin(math.pi * x)) ** 2 * 0.01 / 16)
