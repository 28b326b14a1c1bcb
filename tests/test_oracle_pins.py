"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  The oracle (oracle/ee_oracle.c) is checked
against things that are *not* itself:

* rocRAND's open-source Philox4x32-10 (an independent implementation);
* closed forms of the Metropolis thresholds at the 2D critical point;
* exact partition functions (brute force, transfer matrix, Kaufman's torus
  formula) and exact propagation of the protocol, through which Jarzynski's
  equality must hold for every N;
* the paper's counting of varied links, the beta = 0 limit, the N = 1
  reweighting limit and the estimator's deterministic bounds.

``test_planted_mistakes_are_caught`` compiles copies of the oracle with a
single plausible mistake each and checks that a pin fails for every one.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
import subprocess
from decimal import Decimal, getcontext

import numpy as np
import pytest

from oracle import build as obuild
from oracle import exact as ex
from oracle import oracle as eo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")
BC2 = 0.5 * math.log(1.0 + math.sqrt(2.0))
BC3 = 0.2216546


def _paper():
    with open(GOLDEN) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# Philox
# --------------------------------------------------------------------------

def _rocrand_ref():
    if not os.path.exists(obuild.ROCRAND_REF_SO):
        if obuild.build_rocrand_ref() is None:
            pytest.skip("hipcc not available to build the rocRAND reference")
    L = ctypes.CDLL(obuild.ROCRAND_REF_SO)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    L.ref_philox4x32_10.argtypes = [u32p, u32p, u32p]
    return L


def test_philox_matches_rocrand():
    L = _rocrand_ref()
    rng = np.random.default_rng(12345)
    A = ctypes.c_uint32 * 4
    B = ctypes.c_uint32 * 2
    cases = [((0, 0, 0, 0), (0, 0)), ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2)]
    cases += [(tuple(int(v) for v in rng.integers(0, 2**32, 4)), tuple(int(v) for v in rng.integers(0, 2**32, 2)))
              for _ in range(500)]
    for ctr, key in cases:
        out = A()
        L.ref_philox4x32_10(A(*ctr), B(*key), out)
        assert eo.philox(ctr, key) == tuple(out), (ctr, key)


def test_philox_counter_words_all_matter():
    base = eo.philox((1, 2, 3, 4), (5, 6))
    for i in range(4):
        c = [1, 2, 3, 4]
        c[i] ^= 1
        assert eo.philox(tuple(c), (5, 6)) != base
    assert eo.philox((1, 2, 3, 4), (5, 7)) != base


def test_lazy_decision_equals_32bit_comparison():
    """Accepting on the 16-bit field v and drawing w only on a tie is the
    same decision as u <= U with u = 2^16 v + w."""
    rng = np.random.default_rng(5)
    for _ in range(400):
        t, y, x = int(rng.integers(0, 8)), int(rng.integers(0, 4)), int(rng.integers(0, 12))
        g, j, r = int(rng.integers(0, 1000)), int(rng.integers(0, 50)), int(rng.integers(0, 2))
        v, w, _ = eo.site_fields(3, 8, 12, 4, 2, 99, g, j, r, t, y, x, 0)
        for U in (0, 0xFFFFFFFF, int(rng.integers(0, 2**32)), (v << 16) | w, ((v << 16) | w) - 1,
                  (v << 16) | 0xFFFF, (v << 16), ((v + 1) << 16) & 0xFFFFFFFF):
            U &= 0xFFFFFFFF
            _, _, d = eo.site_fields(3, 8, 12, 4, 2, 99, g, j, r, t, y, x, U)
            assert d == int(((v << 16) | w) <= U), (v, w, U)


def test_sweep_fields_are_philox_halves():
    """v and w are 16-bit halves of Philox4x32-10 words (phases 1 and 2, one
    call per 8 sites of a row)."""
    for (t, y, x) in [(0, 0, 0), (3, 1, 7), (5, 2, 23), (7, 3, 16)]:
        c, h = (t + y + x) & 1, x >> 1
        G8 = (24 // 2 + 7) // 8
        for phase in (1, 2):
            out = eo.philox(((t * 4 + y) * G8 + (h >> 3), 17, 3, (phase << 28) | (1 << 1) | c), (99, 0))
            word = out[(h & 7) >> 1]
            want = (word >> 16) if (h & 1) else (word & 0xFFFF)
            v, w, _ = eo.site_fields(3, 8, 24, 4, 2, 99, 17, 3, 1, t, y, x, 0)
            assert (v, w)[phase - 1] == want


# --------------------------------------------------------------------------
# Thresholds
# --------------------------------------------------------------------------

def _exact_floor_2p32(x: Decimal) -> int:
    return int((x * (Decimal(2) ** 32)).to_integral_value(rounding="ROUND_FLOOR"))


def test_threshold_closed_forms_at_2d_critical_point():
    # beta_c = log(1+sqrt2)/2  =>  exp(-2 beta_c) = sqrt2 - 1,
    # exp(-4 beta_c) = 3 - 2 sqrt2, exp(-8 beta_c) = 17 - 12 sqrt2.
    getcontext().prec = 60
    r2 = Decimal(2).sqrt()
    p4 = Decimal(3) - 2 * r2
    p8 = Decimal(17) - 12 * r2
    for N in (1, 7, 256, 1000):
        # bulk site: K = N * s with s = sigma * sum(neighbours)
        assert eo.threshold(BC2, 2 * N, N) == _exact_floor_2p32(p4) - 1
        assert eo.threshold(BC2, 4 * N, N) == _exact_floor_2p32(p8) - 1


def test_threshold_limits():
    assert eo.threshold(0.0, 5, 3) == 0xFFFFFFFF  # beta = 0 accepts everything
    for K in (0, -1, -4000):
        assert eo.threshold(0.44, K, 1000) == 0xFFFFFFFF  # energy not raised
    vals = [eo.threshold(0.44, K, 10) for K in range(1, 200)]
    assert all(a >= b for a, b in zip(vals, vals[1:]))  # monotone in the energy cost
    assert eo.threshold(50.0, 100, 1) == 0  # exp(-10^4) underflows: accept only u == 0


# --------------------------------------------------------------------------
# Geometry
# --------------------------------------------------------------------------

def test_varied_links_count_matches_paper():
    p = _paper()
    assert p["varied_links_2d_two_replicas"]["value"] == 4
    for (dim, lt, lx, ly, n) in [(2, 16, 16, 1, 2), (2, 8, 6, 1, 3), (3, 8, 6, 6, 2), (3, 4, 4, 8, 3)]:
        L = ly  # spatial extent along the slab (L^(D-2) = Ly in 3D, 1 in 2D)
        expect = 2 * (L ** (dim - 2) if dim == 3 else 1) * n
        for l in (0, 1, lx - 1):
            assert eo.count_ramped_bonds(dim, lt, lx, ly, n, l) == expect
    # 3D with two replicas: 4L couplings (App. B)
    assert eo.count_ramped_bonds(3, 8, 12, 12, 2, 3) == 4 * 12


def test_energy_endpoints_are_geometries():
    """At m = 0 the ramped column is in B, at m = N it is in A: the oracle's
    integer energy must equal the pure-geometry energy of the exact module."""
    rng = np.random.default_rng(3)
    for (dim, lt, lx, ly, n, l) in [(2, 4, 6, 1, 2, 2), (3, 4, 4, 2, 3, 1)]:
        lat0 = ex.Lattice(dim, lt, lx, ly, n, l)
        job = eo.Job(dim, lt, lx, ly, n, 0.3, l, 5, 1, 1)
        for _ in range(5):
            s = rng.choice(np.array([-1, 1], dtype=np.int8), size=lat0.nsites)
            for m, glued in ((0, l), (5, l + 1)):
                b = ex.bonds(lat0, glued_upto=glued, ramp=False)
                e = -sum(int(s[a]) * int(s[c]) for a, c, *_ in b) * 5
                assert eo.energy_units(job, m, s) == e


# --------------------------------------------------------------------------
# Exact partition functions
# --------------------------------------------------------------------------

def test_bruteforce_matches_kaufman():
    for (rows, cols, K) in [(4, 4, BC2), (2, 6, 0.3), (4, 2, 0.7)]:
        lat = ex.Lattice(2, rows, cols, 1, 1, 0)
        assert ex.log_z_bruteforce(lat, K, ramp=False) == pytest.approx(ex.log_z_kaufman(rows, cols, K), rel=1e-13)


def test_transfer_matrix_matches_kaufman_for_unglued_and_fully_glued():
    for (lt, lx, n) in [(8, 4, 2), (6, 2, 3), (16, 4, 2)]:
        lat = ex.Lattice(2, lt, lx, 1, n, 0)
        z0 = ex.log_z_transfer(lat, BC2, ramp=False)
        assert z0 == pytest.approx(n * ex.log_z_kaufman(lt, lx, BC2), rel=1e-13)  # Z_n(0) = Z^n
        zall = ex.log_z_transfer(lat, BC2, glued_upto=lx, ramp=False)
        assert zall == pytest.approx(ex.log_z_kaufman(n * lt, lx, BC2), rel=1e-13)  # one n*Lt torus


def test_transfer_matrix_matches_bruteforce_with_ramp_and_3d():
    cases = [(2, 4, 2, 1, 2, 1, BC2), (2, 2, 4, 1, 2, 2, BC2), (2, 2, 2, 1, 3, 1, 0.5), (3, 2, 2, 2, 2, 1, BC3)]
    for (dim, lt, lx, ly, n, l, beta) in cases:
        lat = ex.Lattice(dim, lt, lx, ly, n, l)
        for m in (0, 1, 3):
            assert ex.log_z_transfer(lat, beta, 3, m) == pytest.approx(ex.log_z_bruteforce(lat, beta, 3, m), rel=1e-13)


def test_renyi_entropy_zero_without_cut_and_symmetric_at_low_temperature():
    # S_2(0) = 0 exactly; S_2(l) ~ S_2(L-l) once Lt >> L (pure state, Sec. 2 / Sec. 4)
    lat = ex.Lattice(2, 48, 4, 1, 2, 0)
    z0 = ex.log_z_transfer(lat, BC2, ramp=False)
    S = [-(ex.log_z_transfer(lat, BC2, glued_upto=l, ramp=False) - z0) for l in range(5)]
    assert S[0] == 0.0
    assert abs(S[4]) < 5e-3 and abs(S[1] - S[3]) < 5e-3
    assert S[2] > S[1] > 0


# --------------------------------------------------------------------------
# Exact protocol: Jarzynski's equality
# --------------------------------------------------------------------------

@pytest.mark.parametrize("case", [
    (2, 2, 4, 1, 2, 0, BC2),
    (2, 2, 4, 1, 2, 2, BC2),
    (3, 2, 2, 2, 2, 0, BC3),
    (2, 2, 2, 1, 3, 0, 0.6),
])
def test_exact_protocol_obeys_jarzynski(case):
    dim, lt, lx, ly, n, l, beta = case
    lat = ex.Lattice(dim, lt, lx, ly, n, l)
    Nb = 2
    dF_exact = -(ex.log_z_bruteforce(lat, beta, Nb, Nb) - ex.log_z_bruteforce(lat, beta, Nb, 0))
    for N in (1, 2):
        v, p = ex.exact_protocol(lat, beta, N)
        assert p.sum() == pytest.approx(1.0, abs=1e-13)
        assert -math.log(ex.jarzynski_average(v, p, beta, N)) == pytest.approx(dF_exact, abs=2e-13)
        # reverse protocol: <exp(-W)>_rev = 1 / <exp(-W)>_dir (App. A)
        v, p = ex.exact_protocol(lat, beta, N, reverse=True)
        assert -math.log(ex.jarzynski_average(v, p, beta, N)) == pytest.approx(-dF_exact, abs=2e-13)


# --------------------------------------------------------------------------
# Oracle Monte Carlo vs the exact work distribution
# --------------------------------------------------------------------------

def _chi2_pvalue(I: np.ndarray, vals: np.ndarray, probs: np.ndarray) -> float:
    from scipy import stats
    n = len(I)
    exp_counts = probs * n
    obs = np.array([np.sum(I == v) for v in vals], dtype=float)
    assert obs.sum() == n, "oracle produced a work value outside the exact support"
    # pool bins with small expectations
    order = np.argsort(exp_counts)
    e_pool, o_pool, acc_e, acc_o = [], [], 0.0, 0.0
    for i in order:
        acc_e += exp_counts[i]
        acc_o += obs[i]
        if acc_e >= 20:
            e_pool.append(acc_e)
            o_pool.append(acc_o)
            acc_e, acc_o = 0.0, 0.0
    if acc_e > 0:
        e_pool[-1] += acc_e
        o_pool[-1] += acc_o
    e_pool, o_pool = np.array(e_pool), np.array(o_pool)
    chi2 = float(np.sum((o_pool - e_pool) ** 2 / e_pool))
    return float(stats.chi2.sf(chi2, max(len(e_pool) - 1, 1)))


MC_CASES = [
    # dim, lt, lx, ly, n, l, beta, N, n_therm, reverse
    (2, 2, 4, 1, 2, 1, BC2, 3, 6, False),
    (2, 2, 4, 1, 2, 0, BC2, 2, 2, True),
    (3, 2, 2, 2, 2, 0, BC3, 2, 3, False),
    (2, 2, 2, 1, 3, 1, 0.6, 3, 2, False),
]


def _oracle_vs_exact(lib_run, case, n_traj=20000, seed=11):
    dim, lt, lx, ly, n, l, beta, N, n_therm, reverse = case
    lat = ex.Lattice(dim, lt, lx, ly, n, l)
    v, p = ex.exact_protocol(lat, beta, N, start="hot", n_therm=n_therm, reverse=reverse)
    job = eo.Job(dim, lt, lx, ly, n, beta, l, N, n_traj, seed, reverse)
    I = lib_run(job, n_therm)
    if not np.all(np.isin(I, v)):
        return 0.0
    return _chi2_pvalue(I, v, p)


@pytest.mark.parametrize("case", MC_CASES)
def test_oracle_work_distribution_matches_exact_propagation(case):
    pval = _oracle_vs_exact(lambda job, nt: eo.run(job, nt)[0], case)
    assert pval > 1e-4, pval


def test_oracle_estimate_close_to_exact_free_energy():
    lat = ex.Lattice(2, 4, 4, 1, 2, 1)
    N = 4
    dF_exact = -(ex.log_z_transfer(lat, BC2, N, N) - ex.log_z_transfer(lat, BC2, N, 0))
    job = eo.Job(2, 4, 4, 1, 2, BC2, 1, N, 4000, 5)
    I, _ = eo.run(job, 50)
    est = eo.estimate(I, BC2, N, 2)
    assert abs(est.dF - dF_exact) < 4 * est.dF_err + 0.5 * est.w_var / len(I)


# --------------------------------------------------------------------------
# Special cases of the method
# --------------------------------------------------------------------------

def test_beta_zero_every_attempt_flips_and_dF_is_zero():
    job = eo.Job(2, 4, 6, 1, 2, 0.0, 2, 5, 3, 9)
    I0, s0 = eo.run(job, 0, n_step_run=0, want_spins=True)  # initial state
    for g in (1, 2, 7):
        _, s = eo.run(job, g, n_step_run=0, want_spins=True)
        assert np.array_equal(s, s0 * (-1) ** g)
    I, _ = eo.run(job, 4)
    est = eo.estimate(I, 0.0, job.n_step, 2)
    assert est.dF == 0.0 and est.w_mean == 0.0


def test_initial_state_is_a_fair_coin():
    job = eo.Job(2, 32, 32, 1, 2, 0.4, 3, 1, 8, 21)
    _, s = eo.run(job, 0, n_step_run=0, want_spins=True)
    frac = np.mean(s == 1)
    assert abs(frac - 0.5) < 4 * 0.5 / math.sqrt(s.size)


def test_work_is_energy_difference_on_state_before_each_sweep():
    """I(k+1) - I(k) = -(E(m_{k+1}) - E(m_k)) evaluated on phi_k (App. A)."""
    for reverse in (False, True):
        job = eo.Job(3, 4, 4, 2, 2, BC3, 1, 6, 3, 4, reverse)
        nt = 5
        for k in range(job.n_step):
            Ik, sk = eo.run(job, nt, n_step_run=k, want_spins=True)
            Ik1, _ = eo.run(job, nt, n_step_run=k + 1)
            mk = job.n_step - k if reverse else k
            mk1 = job.n_step - (k + 1) if reverse else k + 1
            for j in range(job.n_traj):
                dE = eo.energy_units(job, mk1, sk[j]) - eo.energy_units(job, mk, sk[j])
                assert Ik1[j] - Ik[j] == -dE


def test_single_step_is_reweighting():
    """N = 1: W = H_f(phi_0) - H_i(phi_0) on the thermalised state (App. A)."""
    job = eo.Job(2, 6, 6, 1, 2, BC2, 2, 1, 16, 8)
    _, s0 = eo.run(job, 12, n_step_run=0, want_spins=True)
    I, _ = eo.run(job, 12)
    for j in range(job.n_traj):
        assert I[j] == -(eo.energy_units(job, 1, s0[j]) - eo.energy_units(job, 0, s0[j]))


def test_work_bound():
    job = eo.Job(2, 8, 8, 1, 2, 2.0, 3, 7, 64, 2)
    I, _ = eo.run(job, 3)
    assert np.all(np.abs(I) <= 2 * job.n * 1 * job.n_step)


def test_trajectories_are_independent_of_the_range_run():
    job = eo.Job(2, 6, 8, 1, 2, BC2, 3, 9, 10, 77)
    Iall, sall = eo.run(job, 4, want_spins=True)
    Ipart, spart = eo.run(job, 4, 3, 7, want_spins=True)
    assert np.array_equal(Iall[3:7], Ipart) and np.array_equal(sall[3:7], spart)


# --------------------------------------------------------------------------
# Estimator
# --------------------------------------------------------------------------

def test_estimator_bounds_and_closed_forms():
    rng = np.random.default_rng(0)
    beta, N = 0.44, 50
    for _ in range(20):
        I = rng.integers(-400, 400, size=int(rng.integers(2, 300)))
        est = eo.estimate(I, beta, N, 2)
        W = -(beta / N) * I
        assert W.min() - 1e-12 <= est.dF <= W.mean() + 1e-12  # Jensen
        assert est.dF == pytest.approx(-math.log(np.mean(np.exp(-W))), rel=1e-12, abs=1e-12)
        assert est.i_min == I.min() and est.i_max == I.max()
        assert 1.0 <= est.ess <= len(I) + 1e-9
    # constant work: dF = W exactly, zero jackknife error, ESS = n_t
    est = eo.estimate(np.full(10, 37), beta, N, 3)
    assert est.dF == pytest.approx(-(beta / N) * 37, rel=1e-15)
    assert est.dS == pytest.approx(est.dF / 2, rel=1e-15)
    assert est.dF_err == pytest.approx(0.0, abs=1e-14) and est.ess == pytest.approx(10.0)
    # two samples: jackknife of two points, sigma = |dF_(1) - dF_(2)| / 2 * sqrt(... ) closed form
    I = np.array([0, 100])
    est = eo.estimate(I, beta, N, 2)
    d1, d2 = -(beta / N) * 100, 0.0  # leave-one-out values
    assert est.dF_err == pytest.approx(math.sqrt(0.5 * ((d1 - d2) ** 2 / 2)), rel=1e-12)
    assert math.isnan(eo.estimate(np.array([5]), beta, N, 2).dF_err)


def _decimal_estimate(I, beta, N, n_rep):
    """The estimator's outputs from their definitions (App. A: Delta F =
    -log <exp(-W)> over the n_t trajectories, W_j = -(beta/N) I_j; the
    delete-one jackknife; the mean and population variance of W; the
    effective sample size (sum e)^2 / sum e^2 with e_j = exp(-W_j)),
    evaluated in 50-digit decimal arithmetic with no shift or reordering."""
    getcontext().prec = 50
    n = len(I)
    b, NN = Decimal(beta), Decimal(N)
    W = [-(b / NN) * Decimal(int(v)) for v in I]
    e = [(-w).exp() for w in W]
    se = sum(e)
    dF = -(se / n).ln()
    wm = sum(W) / n
    wv = sum((w - wm) ** 2 for w in W) / n
    ess = se * se / sum(x * x for x in e)
    err = None
    if n >= 2:
        loo = [-((se - e[i]) / (n - 1)).ln() for i in range(n)]
        lm = sum(loo) / n
        err = (Decimal(n - 1) / n * sum((v - lm) ** 2 for v in loo)).sqrt()
    return dF, dF / (n_rep - 1), err, wm, wv, ess


ESTIMATOR_CASES = [(5, 0.44, 50, 2, 1), (37, 0.2216546, 2000, 3, 2), (300, 0.7, 256, 2, 3), (1024, BC2, 1000, 2, 4)]


@pytest.mark.parametrize("n,beta,N,n_rep,seed", ESTIMATOR_CASES)
def test_estimator_matches_decimal_definitions(n, beta, N, n_rep, seed):
    """Every output of eo_estimate against its definition in 50-digit decimal
    arithmetic: dF, dS, the jackknife error, the mean and population variance
    of W and the ESS.  The tolerances are the oracle's FP64 rounding (dF and
    the leave-one-out values are sums of terms of size log n_t); a sample
    instead of population variance, a missing square or a dropped term
    misses them by orders of magnitude."""
    rng = np.random.default_rng(seed)
    I = 2 * rng.integers(-3 * N // 4, 3 * N // 4, size=n) // max(1, N // 100)
    est = eo.estimate(I, beta, N, n_rep)
    dF, dS, err, wm, wv, ess = _decimal_estimate(I, beta, N, n_rep)
    scale = abs(beta * float(I.max()) / N) + math.log(n)
    assert abs(est.dF - float(dF)) <= 4e-16 * max(scale, 1.0) * math.sqrt(n)
    assert abs(est.dS - float(dS)) <= 4e-16 * max(scale, 1.0) * math.sqrt(n)
    assert est.w_mean == pytest.approx(float(wm), rel=1e-13, abs=1e-17)
    assert est.w_var == pytest.approx(float(wv), rel=1e-12)
    assert est.ess == pytest.approx(float(ess), rel=1e-13)
    # the leave-one-out values differ from their mean by ~dF_err/n_t, so their
    # FP64 rounding (~1e-16 of log n_t) is amplified by ~n_t log n_t / dF_err
    assert est.dF_err == pytest.approx(float(err), rel=2e-15 * n * math.log(n) / float(err) + 1e-12)


ESTIMATOR_MUTATIONS = {
    "sample variance": ("wv /= n_t;", "wv /= (n_t - 1);"),
    "variance without square": ("wv += d * d;", "wv += d * fabs(d);"),
    "jackknife factor": ("err = sqrt((double)(n_t - 1) / (double)n_t * acc);", "err = sqrt(acc / (double)n_t);"),
    "ess without square": ("out[5] = s * s / s2;", "out[5] = s / s2;"),
    "log n_t dropped": ("double dF = -(shift + log(s) - log((double)n_t));", "double dF = -(shift + log(s));"),
}


def test_planted_estimator_mistakes_are_caught(tmp_path):
    """Each plausible mistake in eo_estimate fails the decimal pin."""
    src = open(os.path.join(os.path.dirname(obuild.ORACLE_SO), "ee_oracle.c")).read()
    rng = np.random.default_rng(11)
    I = 2 * rng.integers(-40, 40, size=23)
    beta, N = 0.44, 50
    dF, dS, err, wm, wv, ess = (float(v) for v in _decimal_estimate(I, beta, N, 2))
    for name, (old, new) in ESTIMATOR_MUTATIONS.items():
        assert src.count(old) == 1, name
        path = tmp_path / (name.replace(" ", "_") + ".c")
        path.write_text(src.replace(old, new))
        so = str(path) + ".so"
        subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-ffp-contract=off", str(path), "-o", so, "-lm"],
                       check=True)
        L = ctypes.CDLL(so)
        L.eo_estimate.argtypes = eo.lib().eo_estimate.argtypes
        L.eo_estimate.restype = ctypes.c_int
        out = np.zeros(8)
        Ic = np.ascontiguousarray(I, dtype=np.int64)
        assert L.eo_estimate(Ic.ctypes.data, len(I), beta, N, 2, out.ctypes.data, None) == 0
        got = dict(dF=out[0], err=out[2], wv=out[4], ess=out[5])
        want = dict(dF=dF, err=err, wv=wv, ess=ess)
        assert any(abs(got[k] - want[k]) > 1e-9 * max(abs(want[k]), 1e-3) for k in got), name


# --------------------------------------------------------------------------
# Planted mistakes
# --------------------------------------------------------------------------

MUTATIONS = {
    "work sign": ("if (I_out) I_out[j - j0] = -work_units;", "if (I_out) I_out[j - j0] = work_units;"),
    "sweep at lambda_k": ("sweep(&G, m_next, g++, (uint32_t)j, s);", "sweep(&G, m_now, g++, (uint32_t)j, s);"),
    "dropped inter bond": ("field += bond_weight(G, G->adj_kind[e], G->adj_y[e], pos) * s[G->adj_nbr[e]];",
                           "field += (G->adj_kind[e] == BOND_INTER ? 0 : bond_weight(G, G->adj_kind[e], G->adj_y[e], pos)) * s[G->adj_nbr[e]];"),
    "glue to r-1": ("add_bond(G, s, site_index(G, (r + 1) % n, 1, y, x), BOND_BULK, y);",
                    "add_bond(G, s, site_index(G, (r + n - 1) % n, 1, y, x), BOND_BULK, y);"),
    "threshold beta": ("double x = (2.0 * beta * (double)K) / (double)N;", "double x = (1.0 * beta * (double)K) / (double)N;"),
    "intra weight": ("if (kind == BOND_INTRA) return (int64_t)(G->S - row_m(G, y, pos));",
                     "if (kind == BOND_INTRA) return (int64_t)(G->S - row_m(G, y, pos) + 1);"),
    "work after sweep": ("work_units += energy_units(&G, m_next, s) - energy_units(&G, m_now, s);\n      sweep(&G, m_next, g++, (uint32_t)j, s);",
                         "sweep(&G, m_next, g++, (uint32_t)j, s);\n      work_units += energy_units(&G, m_next, s) - energy_units(&G, m_now, s);"),
}
# Not listed: the order of the two colours.  The reflection t -> 1-t together
# with r -> -r maps the cut geometry onto itself and swaps the colours, so the
# work distribution cannot see it; it is a convention of the random-number
# streams, checked only by bit-exact parity of the GPU path.


def _build_mutant(tmp_path, name, old, new):
    src = open(os.path.join(os.path.dirname(obuild.ORACLE_SO), "ee_oracle.c")).read()
    assert src.count(old) == 1, f"mutation site for '{name}' not found exactly once"
    path = tmp_path / (name.replace(" ", "_") + ".c")
    path.write_text(src.replace(old, new))
    so = str(path) + ".so"
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-ffp-contract=off", str(path), "-o", so, "-lm"], check=True)
    L = ctypes.CDLL(so)
    L.eo_run.argtypes = eo.lib().eo_run.argtypes
    L.eo_run.restype = ctypes.c_int
    return L


def test_planted_mistakes_are_caught(tmp_path):
    """Each plausible mistake in the oracle makes a pin fail."""
    # n = 3 so that the glue direction matters; the colour-order mutation
    # needs an asymmetric case with N >= 2.
    cases = [(2, 2, 2, 1, 3, 1, 0.6, 3, 2, False), (2, 2, 4, 1, 2, 1, BC2, 3, 2, False)]
    for name, (old, new) in MUTATIONS.items():
        L = _build_mutant(tmp_path, name, old, new)

        def run(job, nt, L=L):
            I = np.zeros(job.n_traj, dtype=np.int64)
            rc = L.eo_run(job.dim, job.lt, job.lx, job.ly, job.n, job.beta, job.l, job.n_step, job.n_traj,
                          job.seed, int(job.reverse), nt, 0, job.n_traj, job.n_step, I.ctypes.data, None)
            assert rc == 0
            return I

        caught = any(_oracle_vs_exact(run, c, n_traj=20000) < 1e-6 for c in cases)
        assert caught, f"planted mistake '{name}' was not detected"


# --------------------------------------------------------------------------
# Protocol 2 (App. B): the rows of the ramped column moved one at a time
# --------------------------------------------------------------------------

def test_protocol2_exact_propagation_obeys_jarzynski():
    lat = ex.Lattice(3, 2, 2, 2, 2, 0)
    dF_exact = -(ex.log_z_bruteforce(lat, BC3, 2, 2) - ex.log_z_bruteforce(lat, BC3, 2, 0))
    for N, rev in ((2, False), (2, True), (4, False)):
        v, p = ex.exact_protocol(lat, BC3, N, subsets=True, reverse=rev)
        S = N // lat.ly
        want = -dF_exact if rev else dF_exact
        assert -math.log(ex.jarzynski_average(v, p, BC3, S)) == pytest.approx(want, abs=2e-13)
    # and it is a different protocol from protocol 1 (different work law)
    v1, p1 = ex.exact_protocol(lat, BC3, 2)
    v2, p2 = ex.exact_protocol(lat, BC3, 2, subsets=True)
    assert not (len(v1) == len(v2) and np.allclose(p1, p2))


@pytest.mark.parametrize("reverse", [False, True])
def test_oracle_protocol2_matches_exact_propagation(reverse):
    lat = ex.Lattice(3, 2, 2, 2, 2, 1)
    N, n_therm = 4, 2
    v, p = ex.exact_protocol(lat, BC3, N, start="hot", n_therm=n_therm, reverse=reverse, subsets=True)
    job = eo.Job(3, 2, 2, 2, 2, BC3, 1, N, 20000, 17, reverse, subsets=True)
    I, _ = eo.run(job, n_therm)
    assert _chi2_pvalue(I, v, p) > 1e-4


def test_protocol2_in_2d_is_protocol1():
    a = eo.Job(2, 8, 8, 1, 2, BC2, 3, 12, 6, 5)
    b = eo.Job(2, 8, 8, 1, 2, BC2, 3, 12, 6, 5, subsets=True)
    Ia, sa = eo.run(a, 4, want_spins=True)
    Ib, sb = eo.run(b, 4, want_spins=True)
    assert np.array_equal(Ia, Ib) and np.array_equal(sa, sb)


def test_protocol2_work_is_energy_difference_and_needs_divisible_N():
    job = eo.Job(3, 4, 4, 4, 2, BC3, 2, 8, 2, 9, False, subsets=True)
    for k in range(job.n_step):
        Ik, sk = eo.run(job, 3, n_step_run=k, want_spins=True)
        Ik1, _ = eo.run(job, 3, n_step_run=k + 1)
        for j in range(job.n_traj):
            dE = eo.energy_units(job, k + 1, sk[j]) - eo.energy_units(job, k, sk[j])
            assert Ik1[j] - Ik[j] == -dE
            # only row k // S moves during step k: its 2n bonds change by one unit each
            assert abs(dE) <= 2 * job.n
    with pytest.raises(ValueError):
        eo.run(eo.Job(3, 4, 4, 4, 2, BC3, 2, 6, 2, 9, False, subsets=True), 1)


# --------------------------------------------------------------------------
# Whole-region protocol (Sec. 3): every cut link of A = {x < l} ramped at
# once, from n decoupled replicas to A(l), so Delta F = (n-1) S_n(l)
# --------------------------------------------------------------------------

def test_whole_region_exact_propagation_gives_renyi_entropy():
    """The exact work law of the whole-region protocol reproduces
    log Z_n(0) - log Z_n(l) (brute force; transfer matrix) for every N, and
    its reverse the inverse."""
    cases = [  # lattice, beta, protocol lengths N, also reversed
        ((2, 2, 2, 1, 2, 1), BC2, (1, 2, 3), True),
        ((2, 2, 2, 1, 2, 2), 0.4, (1, 2, 3), True),   # l = lx: every column
        ((2, 2, 2, 1, 3, 2), 0.5, (1, 2), True),      # three replicas
        ((2, 4, 2, 1, 2, 1), 0.6, (1, 2), False),
        ((3, 2, 2, 2, 2, 2), BC3, (1,), False),
    ]
    for (dim, lt, lx, ly, n, l), beta, Ns, rev in cases:
        lat = ex.Lattice(dim, lt, lx, ly, n, l)
        lz0 = ex.log_z_bruteforce(ex.Lattice(dim, lt, lx, ly, n, 0), beta, ramp=False)
        lzl = ex.log_z_bruteforce(lat, beta, glued_upto=l, ramp=False)
        assert lzl == pytest.approx(ex.log_z_transfer(lat, beta, glued_upto=l, ramp=False), abs=1e-12)
        for N in Ns:
            v, p = ex.exact_protocol(lat, beta, N, whole=True)
            assert -math.log(ex.jarzynski_average(v, p, beta, N)) == pytest.approx(lz0 - lzl, abs=2e-13)
            if rev:
                v, p = ex.exact_protocol(lat, beta, N, whole=True, reverse=True)
                assert -math.log(ex.jarzynski_average(v, p, beta, N)) == pytest.approx(lzl - lz0, abs=2e-13)


def test_whole_region_of_one_column_is_protocol1_from_no_cut():
    """A(0) -> A(1) is both the whole-region protocol with l = 1 and the
    c-function protocol with l = 0: the same geometry, bond for bond."""
    for (dim, lt, lx, ly, n) in [(2, 8, 6, 1, 2), (3, 4, 6, 2, 3)]:
        a = eo.Job(dim, lt, lx, ly, n, 0.44, 1, 12, 5, 7, whole=True)
        b = eo.Job(dim, lt, lx, ly, n, 0.44, 0, 12, 5, 7)
        Ia, sa = eo.run(a, 5, want_spins=True)
        Ib, sb = eo.run(b, 5, want_spins=True)
        assert np.array_equal(Ia, Ib) and np.array_equal(sa, sb)


def test_whole_region_energy_endpoints_are_geometries():
    """At m = 0 the replicas are decoupled, at m = N the columns x < l are
    glued: the oracle's integer energy equals the pure-geometry energy."""
    rng = np.random.default_rng(5)
    for (dim, lt, lx, ly, n, l) in [(2, 4, 6, 1, 2, 3), (2, 4, 6, 1, 3, 6), (3, 4, 4, 2, 2, 2)]:
        lat = ex.Lattice(dim, lt, lx, ly, n, l)
        job = eo.Job(dim, lt, lx, ly, n, 0.3, l, 5, 1, 1, whole=True)
        for _ in range(4):
            s = rng.choice(np.array([-1, 1], dtype=np.int8), size=lat.nsites)
            for m, glued in ((0, 0), (5, l)):
                b = ex.bonds(lat, glued_upto=glued, ramp=False)
                e = -sum(int(s[a]) * int(s[c]) for a, c, *_ in b) * 5
                assert eo.energy_units(job, m, s) == e


@pytest.mark.parametrize("reverse", [False, True])
def test_oracle_whole_region_matches_exact_propagation(reverse):
    lat = ex.Lattice(2, 2, 2, 1, 3, 2)
    N, n_therm = 3, 4
    v, p = ex.exact_protocol(lat, 0.5, N, start="hot", n_therm=n_therm, reverse=reverse, whole=True)
    job = eo.Job(2, 2, 2, 1, 3, 0.5, 2, N, 20000, 19, reverse, whole=True)
    I, _ = eo.run(job, n_therm)
    assert _chi2_pvalue(I, v, p) > 1e-4


def test_whole_region_rejects_bad_l_and_subsets():
    for l in (0, 7):
        with pytest.raises(ValueError):
            eo.run(eo.Job(2, 4, 6, 1, 2, 0.4, l, 3, 1, 1, whole=True), 1)
    with pytest.raises(ValueError):
        eo.run(eo.Job(3, 4, 4, 2, 2, 0.4, 1, 4, 1, 1, whole=True, subsets=True), 1)
    eo.run(eo.Job(2, 4, 6, 1, 2, 0.4, 6, 3, 1, 1, whole=True), 1)  # l = lx: every column


WHOLE_MUTATIONS = {
    "whole: intra link not ramped": (
        "if (whole && t == 0 && x < l) {                                             /* ramped */\n"
        "            add_bond(G, s, site_index(G, r, 1, y, x), BOND_INTRA, y);",
        "if (whole && t == 0 && x < l) {                                             /* ramped */\n"
        "            add_bond(G, s, site_index(G, r, 1, y, x), BOND_BULK, y);"),
    "whole: one column too few": ("if (whole && t == 0 && x < l) {", "if (whole && t == 0 && x < l - 1) {"),
}
# Not listed: gluing to replica r-1 instead of r+1.  With no column glued
# before the ramp, the relabelling r -> -r maps one geometry onto the other
# at every step, so the work law cannot see it; like the colour order, it is
# a convention checked only by bit-exact parity of the GPU path.


def test_planted_whole_region_mistakes_are_caught(tmp_path):
    """Each plausible mistake in the whole-region geometry makes the exact
    work law fail (three replicas so that the inter direction matters)."""
    lat = ex.Lattice(2, 2, 2, 1, 3, 1)
    v, p = ex.exact_protocol(lat, 0.6, 3, start="hot", n_therm=2, whole=True)
    job = eo.Job(2, 2, 2, 1, 3, 0.6, 1, 3, 20000, 23, whole=True)
    for name, (old, new) in WHOLE_MUTATIONS.items():
        L = _build_mutant(tmp_path, name, old, new)
        I = np.zeros(job.n_traj, dtype=np.int64)
        rc = L.eo_run(job.dim, job.lt, job.lx, job.ly, job.n, job.beta, job.l, job.n_step, job.n_traj, job.seed,
                      job.flags, 2, 0, job.n_traj, job.n_step, I.ctypes.data, None)
        assert rc == 0
        caught = (not np.all(np.isin(I, v))) or _chi2_pvalue(I, v, p) < 1e-6
        assert caught, f"planted mistake '{name}' was not detected"
    # the unmutated oracle passes the same check
    I, _ = eo.run(job, 2)
    assert _chi2_pvalue(I, v, p) > 1e-4
