"""Zero-temperature entropic c-function campaign in 2D (Sec. 4, Table 1).

For a spatial size L the campaign runs every increment l -> l+1, l = 0..L-1,
of the 2D Ising model at beta_c on an L_tau = 8L cylinder with n = 2
replicas.  It assembles S_2(l) and the symmetrised c-function C_2(x) at the
midpoints, and reports what Table 1 of the paper reports:

* chi^2/nu of the scaling function cos(pi x)/16 alone, for all points and
  with the two points nearest each edge dropped (Table 1, left);
* the fit cos(pi x)/16 + k cot(pi x)/(2L) with chi^2/nu (Table 1, right).

Errors are the jackknife errors of the increments, with the App. C
finite-difference systematic added in quadrature (as in the paper: error
bars include statistical and systematic parts).  The zero-temperature
check of Sec. 4, C(x) = -C(1-x), is reported as a chi^2 per pair.

Lattices that fit one workgroup's LDS run through the persistent batch;
larger ones (L >= 128 here) run through the HBM-streaming path, one job
after another.

Usage: python -m paper_2304_03311_amd.campaign --L 32 64 128 --n-traj 1024
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import analysis, ee, workloads


def run_increments(L: int, n_traj: int, n_step: int, n_therm: int, lt_factor: int = 8, seed0: int = 1,
                   beta: float = workloads.BETA_C_2D):
    specs = [ee.JobSpec(dim=2, lt=lt_factor * L, lx=L, ly=1, n=2, beta=beta, l=l, n_step=n_step,
                        n_traj=n_traj, seed=seed0 + l) for l in range(L)]
    on_chip = 2 * specs[0].lt * ((L // 2 + 3) // 4) * 4 * 2 <= 160 * 1024 - 256
    t0 = time.perf_counter()
    if on_chip:
        jobs = [ee.Job(s) for s in specs]
        ee.batch_run(jobs, n_therm)
        res = [j.estimate() for j in jobs]
        for j in jobs:
            j.close()
    else:
        res = []
        for s in specs:
            j = ee.Job(s)
            j.thermalize(n_therm)
            j.run_protocol()
            res.append(j.estimate())
            j.close()
    dt = time.perf_counter() - t0
    return specs, res, dt, on_chip


def table1_row(L: int, dS: np.ndarray, dS_err: np.ndarray) -> dict:
    x, C = analysis.c_function(dS, L, dim=2)
    C_stat = (L / math.pi) * np.sin(math.pi * x) * dS_err / 2.0
    # App. C systematic from the CFT third derivative, S = (1/8) log sin(pi x) + const
    S3 = (math.pi ** 3 / 4.0) * np.cos(np.pi * x) / np.sin(np.pi * x) ** 3
    C_sys = np.abs(analysis.discretisation_systematic(x, S3, L, dim=2))
    err = np.sqrt(C_stat ** 2 + C_sys ** 2)
    scal = np.cos(np.pi * x) / 16.0
    chi_all = float(np.sum(((C - scal) / err) ** 2) / len(x))
    inner = slice(2, len(x) - 2)
    chi_inner = float(np.sum(((C[inner] - scal[inner]) / err[inner]) ** 2) / (len(x) - 4))
    k, k_err, chi_fit = analysis.fit_k_2d(x, C, err, L)
    # zero temperature: C(x) = -C(1-x), pairs (l, L-1-l)
    half = len(x) // 2
    pair = C[:half] + C[::-1][:half]
    pair_err = np.sqrt(err[:half] ** 2 + err[::-1][:half] ** 2)
    chi_sym = float(np.mean((pair / pair_err) ** 2))
    S, S_err = analysis.renyi_from_increments(dS, dS_err)
    return {"L": L, "chi2_scaling_all": chi_all, "chi2_scaling_inner": chi_inner, "k": k, "k_err": k_err,
            "chi2_fit": chi_fit, "chi2_symmetry": chi_sym, "S_L": float(S[-1]), "S_L_err": float(S_err[-1]),
            "x": x.tolist(), "C": C.tolist(), "C_err": err.tolist()}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, nargs="+", default=[32, 64])
    ap.add_argument("--n-traj", type=int, default=1024)
    ap.add_argument("--n-step", type=int, default=1000)
    ap.add_argument("--n-therm", type=int, default=1000)
    ap.add_argument("--out", default=None, help="write the rows as JSON here")
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    rows = []
    for L in args.L:
        specs, res, dt, on_chip = run_increments(L, args.n_traj, args.n_step, args.n_therm)
        row = table1_row(L, np.array([r.dS for r in res]), np.array([r.dF_err for r in res]))
        att = sum(r.attempts for r in res)
        row.update(n_traj=args.n_traj, n_step=args.n_step, n_therm=args.n_therm, seconds=dt,
                   attempts_per_ns=att / (dt * 1e9), path="persistent batch" if on_chip else "HBM streaming")
        rows.append(row)
        brief = {k: v for k, v in row.items() if k not in ("x", "C", "C_err")}
        print(json.dumps(brief), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rows, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
