"""The estimator kernel's exp and log (csrc/ee_dd.hpp), built for the host.

The header is plain C++ apart from its host/device qualifiers, so the same
source the kernel uses is compiled here with g++ (contraction off, as in the
library build) and every result is compared with the correctly rounded value
from 60-digit decimal arithmetic.  The constants of the header (ln 2 in three
parts, 1/n!) are checked against their definitions too.
"""
from __future__ import annotations

import math
import os
import random
import re
import subprocess

import pytest
from decimal import Decimal, getcontext

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_2304_03311_amd", "csrc", "ee_dd.hpp")
BC2 = 0.5 * math.log(1.0 + math.sqrt(2.0))

HARNESS = r"""
#include <cstdio>
#include <cstdlib>
#include "ee_dd.hpp"
int main() {
  char op; char buf[64];
  while (scanf(" %c %63s", &op, buf) == 2) {
    const double x = strtod(buf, nullptr);
    printf("%a\n", op == 'e' ? ee::dd::exp_cr(x) : ee::dd::log_cr(x));
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("dd")
    src = d / "h.cpp"
    src.write_text(HARNESS)
    exe = d / "h"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-Wno-unknown-pragmas",
                    "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    return str(exe)


def _run(exe, ops):
    inp = "".join(f"{op} {x.hex()}\n" for op, x in ops)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split()
    return [float.fromhex(v) for v in out]


def _cr_exp(x: float) -> float:
    getcontext().prec = 60
    return float(Decimal(x).exp())


def _cr_log(x: float) -> float:
    getcontext().prec = 60
    return float(Decimal(x).ln())


def test_exp_is_correctly_rounded(harness):
    rng = random.Random(5)
    xs = []
    # the estimator's arguments beta (I_j - I_max) / S for integer works
    for beta, S in ((BC2, 256), (BC2, 1000), (0.2216546, 2000), (0.23, 500), (0.21, 3)):
        xs += [(beta * float(-k)) / float(S) for k in range(0, 3001)]
    xs += [rng.uniform(-708.0, 709.0) for _ in range(20000)]
    xs += [rng.uniform(-1.0, 1.0) * 10.0 ** rng.uniform(-20.0, 0.0) for _ in range(10000)]
    got = _run(harness, [("e", x) for x in xs])
    bad = [(x, y) for x, y in zip(xs, got) if y != _cr_exp(x)]
    assert not bad, bad[:5]


def test_exp_limits(harness):
    xs = [0.0, -0.0, 709.78, 710.0, -745.2, -800.0, float("inf"), float("-inf")]
    got = _run(harness, [("e", x) for x in xs])
    assert got[0] == 1.0 and got[1] == 1.0
    assert got[2] == _cr_exp(709.78)
    assert math.isinf(got[3]) and got[4] == 0.0 and got[5] == 0.0
    assert math.isinf(got[6]) and got[7] == 0.0


def test_log_is_correctly_rounded(harness):
    rng = random.Random(6)
    ss = [float(n) for n in range(1, 65536)]  # log n_t and log (n_t - 1)
    ss += [rng.uniform(1.0, 70000.0) for _ in range(20000)]
    ss += [1.0 + rng.uniform(-1.0, 1.0) * 10.0 ** rng.uniform(-15.0, -1.0) for _ in range(10000)]
    ss += [10.0 ** rng.uniform(-300.0, 300.0) for _ in range(10000)]
    got = _run(harness, [("l", s) for s in ss])
    bad = [(s, y) for s, y in zip(ss, got) if y != _cr_log(s)]
    assert not bad, bad[:5]


def test_log_limits(harness):
    got = _run(harness, [("l", x) for x in (1.0, 0.0, -1.0, float("inf"))])
    assert got[0] == 0.0 and got[1] == -math.inf and math.isnan(got[2]) and got[3] == math.inf


def test_header_constants_match_their_definitions():
    getcontext().prec = 80
    src = open(HEADER).read()
    ln2 = Decimal(2).ln()
    c = {k: float.fromhex(v) for k, v in re.findall(r"constexpr double (k\w+) = (-?0x[0-9a-fp.+-]+);", src)}
    # C1: ln 2 to 42 significant bits; C2, C3: the next doubles of the remainder
    m, e = math.frexp(c["kC1"])
    assert float(m * 2 ** 42).is_integer()
    assert abs(Decimal(c["kC1"]) - ln2) <= Decimal(2) ** (e - 42)
    assert c["kC2"] == float(ln2 - Decimal(c["kC1"]))
    assert c["kC3"] == float(ln2 - Decimal(c["kC1"]) - Decimal(c["kC2"]))
    assert c["kInvLn2"] == float(1 / ln2)
    # 1/n! as (nearest double, nearest double to the remainder)
    pairs = re.findall(r"case (\d+): return DD\{(-?0x[0-9a-fp.+-]+), (-?0x[0-9a-fp.+-]+|0\.0)\};", src)
    pairs += re.findall(r"default: return DD\{(-?0x[0-9a-fp.+-]+), (-?0x[0-9a-fp.+-]+)\};  // n = (\d+)", src)
    seen = set()
    for p in pairs:
        n, h, l = (p[0], p[1], p[2]) if len(p[0]) <= 2 else (p[2], p[0], p[1])
        n = int(n)
        v = Decimal(1) / math.factorial(n)
        hh = float.fromhex(h)
        ll = 0.0 if l == "0.0" else float.fromhex(l)
        assert hh == float(v) and ll == float(v - Decimal(hh)), n
        seen.add(n)
    assert seen == set(range(2, 11))
