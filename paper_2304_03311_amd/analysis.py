"""Host assembly of Renyi entropies and entropic c-functions from the
increments Delta S_2(l) = S_2(l+1) - S_2(l) that the GPU jobs estimate.

* S_2(l) by summation of the increments with S_2(0) = 0 (Sec. 3, increment
  trick; Z_n(0) = Z^n so S_n(0) vanishes).
* Symmetrised entropic c-function (Sec. 2):
      C(l) = [(L/pi) sin(pi l / L)]^(D-1) / |dA| * dS/dl,
  with the finite difference placed at the midpoint x = (l + 1/2)/L of the
  increment l -> l+1 (App. C: mid-point derivative), |dA| = 2 in 2D (Sec. 2)
  and 2 L_y in 3D (two planar boundaries of the slab).
* 2D fit f(x; k) = cos(pi x)/16 + k cot(pi x)/(2L) (Sec. 4), linear in k.
* App. C systematic: sin^(D-1)(pi x) / (48 L^2 pi^(D-1)) * S'''(x).
"""
from __future__ import annotations

import math

import numpy as np


def renyi_from_increments(dS, dS_err=None):
    dS = np.asarray(dS, dtype=np.float64)
    S = np.concatenate([[0.0], np.cumsum(dS)])
    if dS_err is None:
        return S, None
    e = np.asarray(dS_err, dtype=np.float64)
    return S, np.concatenate([[0.0], np.sqrt(np.cumsum(e * e))])


def c_function(dS, L: int, dim: int = 2, ly: int | None = None, l0: int = 0):
    """C at x_l = (l + 1/2)/L for increments l = l0, l0+1, ..."""
    dS = np.asarray(dS, dtype=np.float64)
    l = l0 + np.arange(len(dS))
    x = (l + 0.5) / L
    area = 2.0 if dim == 2 else 2.0 * (ly if ly is not None else L)
    arc = (L / math.pi) * np.sin(math.pi * x)
    return x, arc ** (dim - 1) * dS / area


def cft_c_function_2d(x, c: float = 0.5, n: int = 2):
    """(c/12)(1 + 1/n) cos(pi x): 2D CFT on the cylinder (Sec. 2)."""
    return (c / 12.0) * (1.0 + 1.0 / n) * np.cos(np.pi * np.asarray(x))


def fit_k_2d(x, C, C_err, L: int, drop_edges: int = 0):
    """Weighted least squares of C - cos(pi x)/16 = k cot(pi x)/(2L)."""
    x = np.asarray(x, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    w = 1.0 / np.asarray(C_err, dtype=np.float64) ** 2
    sel = slice(drop_edges, len(x) - drop_edges) if drop_edges else slice(None)
    x, C, w = x[sel], C[sel], w[sel]
    g = 1.0 / np.tan(np.pi * x) / (2.0 * L)
    y = C - np.cos(np.pi * x) / 16.0
    k = float(np.sum(w * g * y) / np.sum(w * g * g))
    k_err = float(1.0 / math.sqrt(np.sum(w * g * g)))
    resid = y - k * g
    dof = max(len(x) - 1, 1)
    return k, k_err, float(np.sum(w * resid * resid) / dof)


def discretisation_systematic(x, S3, L: int, dim: int = 2):
    """App. C: C^MC - C = sin^(D-1)(pi x) / (48 L^2 pi^(D-1)) * d^3 S/dx^3."""
    x = np.asarray(x, dtype=np.float64)
    return np.sin(np.pi * x) ** (dim - 1) / (48.0 * L * L * math.pi ** (dim - 1)) * np.asarray(S3)


def assemble(dS, dS_err, L: int, dim: int = 2, ly: int | None = None) -> dict:
    """S_2(l) for l = 0..len(dS), C_2 at the midpoints, and (2D, all l) the k fit."""
    S, S_err = renyi_from_increments(dS, dS_err)
    x, C = c_function(dS, L, dim, ly)
    out = {"S": S, "S_err": S_err, "x": x, "C": C}
    if dS_err is not None:
        area = 2.0 if dim == 2 else 2.0 * (ly if ly is not None else L)
        C_err = ((L / math.pi) * np.sin(math.pi * x)) ** (dim - 1) * np.asarray(dS_err) / area
        out["C_err"] = C_err
        if dim == 2 and len(dS) == L and np.all(np.isfinite(C_err)) and np.all(C_err > 0):
            k, k_err, chi2 = fit_k_2d(x, C, C_err, L)
            out.update(fit_k=k, fit_k_err=k_err, fit_chi2_dof=chi2)
    return out
