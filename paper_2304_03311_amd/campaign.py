"""Physics campaigns of the paper with this build's estimator.

Table 1 (Sec. 4): the zero-temperature entropic c-function in 2D.

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

Three further checks of the paper (experiment, and its section):

* zero3d (Sec. 5, zero-temperature condition in 3D): every increment of the
  3D Ising model at beta_c on L_tau x L x L with L_tau = L and L_tau = 4L.  At
  zero temperature the state is pure, so S_2(L) = sum_l dS_2(l) vanishes and
  C(x) = -C(1-x); at L_tau = L it does not.
* dirrev (Sec. 4 and 5, direct and reverse realisations; App. A): every
  increment estimated from both ends, Delta F_forward = -Delta F_reverse,
  with chi^2/nu of their sum over all x.
* proto12 (App. B, protocol 2): every increment in 3D with the ramped row
  moved at once (protocol 1) and one row at a time (protocol 2), chi^2/nu of
  their difference over all x.

Usage: python -m paper_2304_03311_amd.campaign --L 32 64 128 --n-traj 1024
       python -m paper_2304_03311_amd.campaign --experiment zero3d --L 8 16 --out results/zero3d.json
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
                   beta: float = workloads.BETA_C_2D, l_range: tuple | None = None):
    """The increments l of a 2D cylinder (all of them, or l in [l_range[0],
    l_range[1])), each job seeded seed0 + l."""
    lo, hi = l_range if l_range is not None else (0, L)
    specs = [ee.JobSpec(dim=2, lt=lt_factor * L, lx=L, ly=1, n=2, beta=beta, l=l, n_step=n_step,
                        n_traj=n_traj, seed=seed0 + l) for l in range(lo, hi)]
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
            print(json.dumps({"L": L, "l": s.l, "dS": res[-1].dS, "dS_err": res[-1].dF_err,
                              "seconds": time.perf_counter() - t0}), flush=True)
    dt = time.perf_counter() - t0
    return specs, res, dt, on_chip


def merge_partials(paths) -> list:
    """Table 1 rows from partial runs (--l-range): every L whose increments
    0 .. L-1 the files hold, each exactly once, with one (n_traj, n_step,
    n_therm)."""
    parts = {}
    for p in paths:
        with open(p) as f:
            for r in json.load(f):
                if r.get("partial"):
                    parts.setdefault(r["L"], []).append(r)
    rows = []
    for L, rs in sorted(parts.items()):
        dS = {}
        for r in rs:
            for l, d, e in zip(r["l"], r["dS"], r["dS_err"]):
                if l in dS:
                    raise ValueError(f"L = {L}: increment {l} appears twice")
                dS[l] = (d, e)
        if sorted(dS) != list(range(L)):
            raise ValueError(f"L = {L}: increments {sorted(set(range(L)) - set(dS))} are missing")
        params = {(r["n_traj"], r["n_step"], r["n_therm"]) for r in rs}
        if len(params) != 1:
            raise ValueError(f"L = {L}: the partial runs differ in (n_traj, n_step, n_therm): {params}")
        n_traj, n_step, n_therm = params.pop()
        row = table1_row(L, np.array([dS[l][0] for l in range(L)]), np.array([dS[l][1] for l in range(L)]))
        sec = sum(r["seconds"] for r in rs)
        row.update(n_traj=n_traj, n_step=n_step, n_therm=n_therm, seconds=sec,
                   attempts_per_ns=sum(r["attempts"] for r in rs) / (sec * 1e9), path=rs[0]["path"],
                   merged_from=len(rs))
        rows.append(row)
    return rows


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


def run_specs(specs, n_therm: int, want_work: bool = False):
    """Results of the jobs: one persistent batch for those on chip, the
    per-job path for the others (with want_work, also each job's integer
    works I_j)."""
    on = [s for s in specs if ee.ee_job_on_chip(s.desc())]
    off = [s for s in specs if not ee.ee_job_on_chip(s.desc())]
    res, work = {}, {}
    if on:
        jobs = [ee.Job(s) for s in on]
        ee.batch_run(jobs, n_therm)
        for s, j in zip(on, jobs):
            res[id(s)] = j.estimate()
            if want_work:
                work[id(s)] = j.work()
            j.close()
    for s in off:
        j = ee.Job(s)
        j.thermalize(n_therm)
        j.run_protocol()
        res[id(s)] = j.estimate()
        if want_work:
            work[id(s)] = j.work()
        j.close()
    out = [res[id(s)] for s in specs]
    return (out, [work[id(s)] for s in specs]) if want_work else out


def _increments(dim: int, L: int, lt: int, beta: float, n_traj: int, n_step: int, seed0: int, **kw):
    return [ee.JobSpec(dim=dim, lt=lt, lx=L, ly=L if dim == 3 else 1, n=2, beta=beta, l=l, n_step=n_step,
                       n_traj=n_traj, seed=seed0 + l,
                       spin_format=ee.EE_SPINS_BITPACKED if dim == 3 else ee.EE_SPINS_INT8, **kw)
            for l in range(L)]


def _symmetry(dS, dS_err, L, dim):
    """S_2(L) with its error, and chi^2 per pair of C(x) + C(1-x) (zero at
    zero temperature), from the increments."""
    S, S_err = analysis.renyi_from_increments(dS, dS_err)
    x, C = analysis.c_function(dS, L, dim=dim)
    area = 2.0 if dim == 2 else 2.0 * L
    C_err = ((L / math.pi) * np.sin(math.pi * x)) ** (dim - 1) * np.asarray(dS_err) / area
    half = len(x) // 2
    pair = C[:half] + C[::-1][:half]
    pair_err = np.sqrt(C_err[:half] ** 2 + C_err[::-1][:half] ** 2)
    return float(S[-1]), float(S_err[-1]), float(np.mean((pair / pair_err) ** 2)), x, C, C_err


def zero_temperature(dim: int, L: int, lt_factor: int, n_traj: int, n_step: int, n_therm: int,
                     beta: float | None = None, seed0: int = 1) -> dict:
    """Every increment l -> l+1 on an L_tau = lt_factor L lattice: S_2(L) and
    the symmetry of C(x) (Sec. 5 zero-temperature condition; Sec. 4 in 2D)."""
    beta = (workloads.BETA_3D if dim == 3 else workloads.BETA_C_2D) if beta is None else beta
    specs = _increments(dim, L, lt_factor * L, beta, n_traj, n_step, seed0)
    t0 = time.perf_counter()
    res = run_specs(specs, n_therm)
    dt = time.perf_counter() - t0
    dS = np.array([r.dS for r in res])
    err = np.array([r.dF_err for r in res])
    S_L, S_L_err, chi_sym, x, C, C_err = _symmetry(dS, err, L, dim)
    return {"experiment": "zero-temperature condition", "dim": dim, "L": L, "L_tau": lt_factor * L,
            "beta": beta, "n_traj": n_traj, "n_step": n_step, "n_therm": n_therm, "S_L": S_L,
            "S_L_err": S_L_err, "S_L_sigmas": S_L / S_L_err, "chi2_symmetry": chi_sym, "seconds": dt,
            "dS": dS.tolist(), "dS_err": err.tolist(), "x": x.tolist(), "C": C.tolist(), "C_err": C_err.tolist()}


def direct_vs_reverse(dim: int, L: int, lt_factor: int, n_traj: int, n_step: int, n_therm: int,
                      beta: float | None = None, seed0: int = 1) -> dict:
    """Every increment from both ends: forward (add column l, A(l) -> A(l+1))
    and reverse (remove it).  Delta F_f = -Delta F_r (App. A); chi^2/nu of
    Delta F_f + Delta F_r over all x (Sec. 4 and 5 compare the two
    realisations the same way)."""
    beta = (workloads.BETA_3D if dim == 3 else workloads.BETA_C_2D) if beta is None else beta
    fwd = _increments(dim, L, lt_factor * L, beta, n_traj, n_step, seed0)
    rev = _increments(dim, L, lt_factor * L, beta, n_traj, n_step, seed0 + 10000, reverse=True)
    t0 = time.perf_counter()
    res = run_specs(fwd + rev, n_therm)
    dt = time.perf_counter() - t0
    f, r = res[:L], res[L:]
    d = np.array([a.dF + b.dF for a, b in zip(f, r)])
    e = np.array([math.hypot(a.dF_err, b.dF_err) for a, b in zip(f, r)])
    return {"experiment": "direct vs reverse", "dim": dim, "L": L, "L_tau": lt_factor * L, "beta": beta,
            "n_traj": n_traj, "n_step": n_step, "n_therm": n_therm, "chi2_per_dof": float(np.mean((d / e) ** 2)),
            "dof": L, "seconds": dt, "dF_forward": [a.dF for a in f], "dF_reverse": [b.dF for b in r],
            "err_forward": [a.dF_err for a in f], "err_reverse": [b.dF_err for b in r]}


def direct_vs_reverse_n(L: int, lt_factor: int, l: int, n_traj: int, n_steps, n_therm: int,
                        beta: float | None = None, seed0: int = 1) -> dict:
    """2D, one increment l -> l+1 at a fixed n_t, forward and reverse, for a
    range of protocol lengths N (Sec. 4, the direct/reverse comparison at
    fixed n_t over N, and the work distributions, which narrow towards the
    quasi-static limit as N grows).  Per N: Delta F forward, Delta F reverse
    (its negative estimates the same quantity), their pull, and the mean and
    variance of the work of both."""
    beta = workloads.BETA_C_2D if beta is None else beta
    lt = lt_factor * L
    specs = []
    for i, N in enumerate(n_steps):
        for rev in (False, True):
            specs.append(ee.JobSpec(dim=2, lt=lt, lx=L, ly=1, n=2, beta=beta, l=l, n_step=N, n_traj=n_traj,
                                    seed=seed0 + 2 * i + int(rev), reverse=rev))
    t0 = time.perf_counter()
    res, works = run_specs(specs, n_therm, want_work=True)
    dt = time.perf_counter() - t0
    rows = []
    for i, N in enumerate(n_steps):
        f, r = res[2 * i], res[2 * i + 1]
        err = math.hypot(f.dF_err, r.dF_err)
        # work distributions W = -(beta/N) I_j (App. A): the forward one and
        # the reverse one mirrored (W -> -W), on one set of 40 bins
        wf = -(beta / N) * works[2 * i].astype(np.float64)
        wr = (beta / N) * works[2 * i + 1].astype(np.float64)
        edges = np.linspace(min(wf.min(), wr.min()), max(wf.max(), wr.max()), 41)
        rows.append({"N": N, "dF_forward": f.dF, "err_forward": f.dF_err, "dF_reverse": r.dF,
                     "err_reverse": r.dF_err, "pull": (f.dF + r.dF) / err if err > 0 else 0.0,
                     "w_mean_forward": f.w_mean, "w_var_forward": f.w_var, "w_mean_reverse": r.w_mean,
                     "w_var_reverse": r.w_var, "hist_edges": edges.tolist(),
                     "hist_forward": np.histogram(wf, edges)[0].tolist(),
                     "hist_reverse_mirrored": np.histogram(wr, edges)[0].tolist()})
    return {"experiment": "direct vs reverse over N", "dim": 2, "L": L, "L_tau": lt, "l": l, "beta": beta,
            "n_traj": n_traj, "n_therm": n_therm, "seconds": dt, "rows": rows}


def thermalisation_scan(L: int, lt_factor: int, l: int, n_traj: int, n_step: int, therms,
                        beta: float | None = None, seed0: int = 1) -> dict:
    """2D, one increment l -> l+1 after each number of thermalisation sweeps
    in therms (the same seed: every run continues the same chains, so the
    estimates drift only as the starting ensemble relaxes)."""
    beta = workloads.BETA_C_2D if beta is None else beta
    rows = []
    t0 = time.perf_counter()
    for nt in therms:
        spec = ee.JobSpec(dim=2, lt=lt_factor * L, lx=L, ly=1, n=2, beta=beta, l=l, n_step=n_step,
                          n_traj=n_traj, seed=seed0 + l)
        r = run_specs([spec], nt)[0]
        rows.append({"n_therm": nt, "dS": r.dS, "dS_err": r.dF_err, "w_mean": r.w_mean, "w_var": r.w_var})
        print(json.dumps({"L": L, "l": l, **rows[-1]}), flush=True)
    return {"experiment": "thermalisation scan", "dim": 2, "L": L, "L_tau": lt_factor * L, "l": l, "beta": beta,
            "n_traj": n_traj, "n_step": n_step, "seconds": time.perf_counter() - t0, "rows": rows}


def protocol1_vs_2(L: int, lt_factor: int, n_traj: int, n_step: int, n_therm: int, beta: float | None = None,
                   seed0: int = 1) -> dict:
    """3D: every increment with the L links of the ramped row moved at once
    (protocol 1) and one row after the other (protocol 2, App. B); chi^2/nu
    of the difference over all x.  n_step must be a multiple of L."""
    beta = workloads.BETA_3D if beta is None else beta
    p1 = _increments(3, L, lt_factor * L, beta, n_traj, n_step, seed0)
    p2 = _increments(3, L, lt_factor * L, beta, n_traj, n_step, seed0 + 20000, subsets=True)
    t0 = time.perf_counter()
    res = run_specs(p1 + p2, n_therm)
    dt = time.perf_counter() - t0
    a, b = res[:L], res[L:]
    d = np.array([u.dF - v.dF for u, v in zip(a, b)])
    e = np.array([math.hypot(u.dF_err, v.dF_err) for u, v in zip(a, b)])
    return {"experiment": "protocol 1 vs protocol 2", "dim": 3, "L": L, "L_tau": lt_factor * L, "beta": beta,
            "n_traj": n_traj, "n_step": n_step, "n_therm": n_therm, "chi2_per_dof": float(np.mean((d / e) ** 2)),
            "dof": L, "seconds": dt, "dF_protocol1": [u.dF for u in a], "dF_protocol2": [v.dF for v in b],
            "err_protocol1": [u.dF_err for u in a], "err_protocol2": [v.dF_err for v in b],
            "w_var_protocol1": [u.w_var for u in a], "w_var_protocol2": [v.w_var for v in b]}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--experiment", default="table1",
                    choices=["table1", "zero", "zero3d", "dirrev", "dirrev_n", "therm", "proto12"])
    ap.add_argument("--dim", type=int, default=2, help="dirrev, zero: lattice dimension")
    ap.add_argument("--L", type=int, nargs="+", default=[32, 64])
    ap.add_argument("--lt-factor", type=int, nargs="+", default=None,
                    help="L_tau / L (table1: 8; zero: 1 2 4 8 in 2D, 1 4 in 3D; zero3d: 1 4; dirrev: 8 in 2D, "
                         "4 in 3D; proto12: 4)")
    ap.add_argument("--n-traj", type=int, default=1024)
    ap.add_argument("--n-step", type=int, default=1000)
    ap.add_argument("--n-steps", type=int, nargs="+", default=[10, 20, 50, 100, 200, 500, 1000, 2000, 5000],
                    help="dirrev_n: the protocol lengths N")
    ap.add_argument("--l", type=int, default=None, help="dirrev_n, therm: the increment l -> l+1 (default L/8 - 1)")
    ap.add_argument("--therms", type=int, nargs="+", default=[2500, 5000, 10000, 20000, 40000, 80000],
                    help="therm: the thermalisation lengths")
    ap.add_argument("--n-therm", type=int, default=1000)
    ap.add_argument("--out", default=None, help="write the rows as JSON here")
    ap.add_argument("--l-range", type=int, nargs=2, default=None, metavar=("LO", "HI"),
                    help="table1: run only the increments l in [LO, HI) and write them as a partial row")
    ap.add_argument("--merge", nargs="+", default=None, metavar="FILE",
                    help="table1: combine partial rows (from --l-range runs) into the rows of their L")
    args = ap.parse_args(argv)
    if args.merge:
        rows = merge_partials(args.merge)
        for row in rows:
            print(json.dumps({k: v for k, v in row.items() if not isinstance(v, list)}), flush=True)
        if args.out:
            with open(args.out, "w") as f:
                json.dump(rows, f)
        return 0
    import torch
    torch.cuda.set_device(0)
    rows = []
    for L in args.L:
        if args.experiment == "table1" and args.l_range is not None:
            specs, res, dt, on_chip = run_increments(L, args.n_traj, args.n_step, args.n_therm,
                                                     l_range=tuple(args.l_range))
            rows.append({"partial": True, "L": L, "l": [s.l for s in specs], "dS": [r.dS for r in res],
                         "dS_err": [r.dF_err for r in res], "attempts": sum(r.attempts for r in res),
                         "seconds": dt, "n_traj": args.n_traj, "n_step": args.n_step, "n_therm": args.n_therm,
                         "path": "persistent batch" if on_chip else "HBM streaming"})
            continue
        if args.experiment == "table1":
            specs, res, dt, on_chip = run_increments(L, args.n_traj, args.n_step, args.n_therm)
            row = table1_row(L, np.array([r.dS for r in res]), np.array([r.dF_err for r in res]))
            att = sum(r.attempts for r in res)
            row.update(n_traj=args.n_traj, n_step=args.n_step, n_therm=args.n_therm, seconds=dt,
                       attempts_per_ns=att / (dt * 1e9), path="persistent batch" if on_chip else "HBM streaming")
            rows.append(row)
            continue
        if args.experiment in ("zero", "zero3d"):
            dim = 3 if args.experiment == "zero3d" else args.dim
            for f in (args.lt_factor or ([1, 2, 4, 8] if dim == 2 else [1, 4])):
                rows.append(zero_temperature(dim, L, f, args.n_traj, args.n_step, args.n_therm))
        elif args.experiment == "therm":
            f = (args.lt_factor or [8])[0]
            rows.append(thermalisation_scan(L, f, max(0, L // 8 - 1) if args.l is None else args.l, args.n_traj,
                                            args.n_step, args.therms))
        elif args.experiment == "dirrev_n":
            f = (args.lt_factor or [8])[0]
            rows.append(direct_vs_reverse_n(L, f, max(0, L // 8 - 1) if args.l is None else args.l, args.n_traj,
                                            args.n_steps, args.n_therm))
        elif args.experiment == "dirrev":
            f = (args.lt_factor or [8 if args.dim == 2 else 4])[0]
            rows.append(direct_vs_reverse(args.dim, L, f, args.n_traj, args.n_step, args.n_therm))
        else:
            f = (args.lt_factor or [4])[0]
            rows.append(protocol1_vs_2(L, f, args.n_traj, args.n_step, args.n_therm))
    for row in rows:
        brief = {k: v for k, v in row.items() if not isinstance(v, list) or k == "rows"}
        print(json.dumps(brief), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rows, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
