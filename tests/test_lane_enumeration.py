"""The row enumeration of the sweep kernels (csrc/ee_lanes.hpp), built for
the host.

The kernels' lanes walk the rows of a trajectory's colour planes in one of
two orders (the lane map, also used by the streaming kernel, and the
parity-major order), from per-lane start states made by make_lane and
make_lane_pm.  Here the same header is compiled with g++ and, for many
lattice shapes and launch shapes (lanes per trajectory), a host walk that
follows the kernels' loop control checks that

* every word of a colour plane is visited exactly once per half-sweep;
* each visited row's storage offset, Philox counter word and neighbour rows
  (t -+ 1 with the periodic wrap, y -+ 1) are those of its (r, t, y);
* in parity-major order, the two rows of a step have the x parities the
  kernel compiles in, and the rows next to the cut carry the offset of their
  glued partner (replica r+1 at t = 1 for t = 0, r-1 at t = 0 for t = 1) and
  the byte masks of the glued columns x < l.
"""
from __future__ import annotations

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2304_03311_amd", "csrc")

HARNESS = r"""
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "ee_internal.hpp"
#include "ee_lanes.hpp"
using namespace ee::lanes;

static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { if (fails < 20) { printf("FAIL %s:%d ", __FILE__, __LINE__); \
  printf(__VA_ARGS__); printf("\n"); } ++fails; } } while (0)

static JP make_jp(int dim, int lt, int lx, int ly, int n, int l) {
  JP P{};
  P.dim = dim; P.n = n; P.lt = lt; P.ly = ly; P.l = l;
  P.H = lx / 2; P.G = (P.H + 3) / 4; P.G8 = (P.H + 7) >> 3; P.R = lt * ly;
  P.traj_words = 2 * n * P.R * P.G;
  ee::Magic mr = ee::make_magic((uint32_t)P.R), my = ee::make_magic((uint32_t)ly);
  P.mR = mr.mul; P.sR = mr.shift; P.mLy = my.mul; P.sLy = my.shift;
  return P;
}

// The lane-map walk of half_sweep (groups: the on-chip grouping; else the
// streaming kernel's storage order).
static void walk_lanemap(const JP& P, int T, int W, bool groups, const char* tag) {
  const int G = P.G, R = P.R, ly = P.ly, lt = P.lt;
  std::vector<int> seen((size_t)P.n * R * G, 0);
  for (int lane = 0; lane < T; ++lane) {
    const Lane ln = make_lane(P, lane, T, W, groups);
    if (!(ln.kstart < ln.kend)) continue;
    int r = ln.r0, t = ln.t0, y = ln.y0, rowbase = ln.rowbase0;
    for (int kk = ln.kstart; kk < ln.kend; kk += ln.kstep) {
      CHECK(r >= 0 && r < P.n && t >= 0 && t < lt && y >= 0 && y < ly, "%s lane %d row out of range r%d t%d y%d",
            tag, lane, r, t, y);
      if (fails) return;
      CHECK(rowbase == (r * R + t * ly + y) * G, "%s lane %d rowbase %d != (r%d t%d y%d)", tag, lane, rowbase, r, t, y);
      for (int q = 0; q < W; ++q) {
        CHECK(ln.w + q < G, "%s lane %d word %d beyond row", tag, lane, ln.w + q);
        seen[(size_t)rowbase + ln.w + q] += 1;
      }
      // neighbour rows as half_sweep forms them (offsets from the row)
      const int LyG = ly * G, ltLyG = lt * LyG;
      const int tpo = LyG - ((t == lt - 1) ? ltLyG : 0);
      const int tmo = -LyG + ((t == 0) ? ltLyG : 0);
      const int ymo = (y == 0) ? (ly - 1) * G : -G;
      const int ypo = (y == ly - 1) ? -(ly - 1) * G : G;
      CHECK(rowbase + tpo == (r * R + ((t + 1) % lt) * ly + y) * G, "%s t+1 row", tag);
      CHECK(rowbase + tmo == (r * R + ((t + lt - 1) % lt) * ly + y) * G, "%s t-1 row", tag);
      CHECK(rowbase + ymo == (r * R + t * ly + (y + ly - 1) % ly) * G, "%s y-1 row", tag);
      CHECK(rowbase + ypo == (r * R + t * ly + (y + 1) % ly) * G, "%s y+1 row", tag);
      const int wl = (ln.w == 0) ? G - 1 : ln.w - 1, wr = (ln.w + W == G) ? 0 : ln.w + W;
      CHECK(ln.wl == wl && ln.wr == wr, "%s lane %d x-neighbour words", tag, lane);
      rowbase += ln.step;
      if (P.dim == 3) {
        y += ln.dy;
        if (y >= ly) { y -= ly; ++t; }
      }
      t += ln.dt;
      if (t >= lt) { t -= lt; r += ln.rinc; rowbase -= ln.wrapadj; }
      r += ln.dr;
    }
  }
  for (size_t i = 0; i < seen.size(); ++i) CHECK(seen[i] == 1, "%s word %zu visited %d times", tag, i, seen[i]);
}

// The parity-major walk of rows_pm for colour C.
template <int DIM, int W>
static void walk_pm(const JP& P, int T, int C, const char* tag) {
  const int G = P.G, R = P.R, ly = P.ly, lt = P.lt;
  std::vector<int> seen((size_t)P.n * R * G, 0);
  for (int lane = 0; lane < T; ++lane) {
    const LanePM lp = make_lane_pm<DIM, W>(P, lane, T);
    int step = 0;
    for (int t = lp.t; t < lt; t += lp.dt, ++step) {
      const int rw = lp.rw + step * lp.dt * ly * G;
      const uint32_t c0 = lp.c0 + (uint32_t)(step * lp.dt * ly * P.G8);
      for (int q = 0; q < 2; ++q) {
        const int tq = (DIM == 2) ? t + q : t;
        const int yq = lp.y[q];
        CHECK(tq < lt && yq >= 0 && yq < ly, "%s lane %d class %d row t%d y%d", tag, lane, q, tq, yq);
        if (fails) return;
        const int off = rw + (q ? lp.d_rw : 0);
        CHECK(off == (lp.r0 * R + tq * ly + yq) * G + lp.w, "%s lane %d class %d offset", tag, lane, q);
        const uint32_t cq = c0 + (q ? lp.d_c0 : 0u);
        CHECK(cq == (uint32_t)((tq * ly + yq) * P.G8 + (lp.w >> 1)), "%s lane %d class %d Philox counter", tag, lane, q);
        // class q rows hold the sites of x parity C ^ q
        CHECK((((C + tq + yq) & 1) ^ C) == q, "%s lane %d class %d parity", tag, lane, q);
        const int ymo = (yq == 0) ? (ly - 1) * G : -G, ypo = (yq == ly - 1) ? -(ly - 1) * G : G;
        CHECK(lp.ymo[q] == ymo && lp.ypo[q] == ypo, "%s lane %d class %d y neighbours", tag, lane, q);
        if (tq <= 1) {
          CHECK(step == 0, "%s lane %d meets the cut after its first step", tag, lane);
          const int rgl = (tq == 0) ? (lp.r0 + 1) % P.n : (lp.r0 + P.n - 1) % P.n;
          CHECK(lp.og[q] == (rgl * R + (1 - tq) * ly + yq) * G + lp.w, "%s lane %d class %d glued row", tag, lane, q);
        }
        for (int i = 0; i < W; ++i) {
          // bytes of word w+i with x < l for sites of parity p: x = 8 (w+i) + 2 b + p
          const int p = C ^ q;
          uint32_t m = 0;
          for (int b = 0; b < 4; ++b)
            if (8 * (lp.w + i) + 2 * b + p < P.l) m |= 0xFFu << (8 * b);
          CHECK(lp.gm[p][i] == m, "%s lane %d glued mask parity %d word %d", tag, lane, p, lp.w + i);
          seen[(size_t)off + i] += 1;
        }
      }
    }
  }
  for (size_t i = 0; i < seen.size(); ++i) CHECK(seen[i] == 1, "%s word %zu visited %d times", tag, i, seen[i]);
}

template <int DIM>
static void walk_pm_any(const JP& P, int T, int W, int C, const char* tag) {
  switch (W) {
    case 4: walk_pm<DIM, 4>(P, T, C, tag); break;
    case 3: walk_pm<DIM, 3>(P, T, C, tag); break;
    case 2: walk_pm<DIM, 2>(P, T, C, tag); break;
    default: walk_pm<DIM, 1>(P, T, C, tag);
  }
}

int main() {
  struct S { int dim, lt, lx, ly, n, l; };
  const S shapes[] = {
    {2, 8, 8, 1, 2, 3}, {2, 16, 16, 1, 2, 4}, {2, 64, 64, 1, 2, 31}, {2, 16, 64, 1, 2, 21}, {2, 8, 24, 1, 2, 17},
    {2, 6, 10, 1, 2, 9}, {2, 2, 2, 1, 2, 1}, {2, 12, 16, 1, 2, 5}, {2, 8, 6, 1, 2, 2}, {2, 8, 12, 1, 3, 0},
    {2, 4, 14, 1, 4, 7}, {2, 10, 70, 1, 2, 33}, {2, 4, 96, 1, 2, 70}, {2, 8, 64, 1, 3, 37}, {2, 256, 32, 1, 2, 11},
    {2, 4, 2048, 1, 2, 1001}, {2, 24, 24, 1, 2, 5}, {2, 96, 96, 1, 2, 40}, {2, 512, 64, 1, 2, 20},
    {3, 8, 8, 8, 2, 3}, {3, 4, 32, 4, 2, 9}, {3, 4, 16, 6, 2, 5}, {3, 4, 24, 4, 3, 10}, {3, 32, 32, 32, 2, 8},
    {3, 4, 6, 2, 2, 5}, {3, 6, 10, 4, 2, 4}, {3, 16, 16, 16, 2, 5}, {3, 24, 24, 24, 2, 11}, {3, 8, 32, 4, 2, 22},
    {3, 64, 16, 16, 2, 7}, {3, 4, 8, 4, 3, 0}, {3, 96, 24, 24, 2, 3},
  };
  int cases = 0;
  char tag[160];
  for (const S& s : shapes) {
    const JP P = make_jp(s.dim, s.lt, s.lx, s.ly, s.n, s.l);
    const int min_T = (P.G + 63) / 64 * 64;
    // on-chip launch shapes: block sizes and trajectories per workgroup
    for (int block : {64, 128, 192, 256, 384, 512, 576, 768, 1024})
      for (int k : {1, 2, 3, 4, 8, 16}) {
        const int T = block / k;
        if (T < P.G || block < min_T) continue;
        const int W = words_per_lane(P, T);
        const bool full = (P.H & 3) == 0;
        if (W > 1 && !full) continue;
        snprintf(tag, sizeof tag, "D%d %dx%dx%d n%d T%d W%d", s.dim, s.lt, s.lx, s.ly, s.n, T, W);
        walk_lanemap(P, T, W, true, tag);
        if (full && use_pm(P, T, W)) {
          for (int C = 0; C < 2; ++C) {
            if (s.dim == 3) walk_pm_any<3>(P, T, W, C, tag); else walk_pm_any<2>(P, T, W, C, tag);
          }
        }
        ++cases;
      }
    // the streaming kernel's map: r rows per lane, storage order
    const int nrows = s.n * P.R;
    const int Ws = ((P.H & 15) == 0) ? 4 : (P.H == 12) ? 3 : ((P.H & 7) == 0) ? 2 : 1;
    for (int r : {1, 2, 4, 7, 16}) {
      const int lanes = ((nrows + r - 1) / r) * (P.G / Ws);
      snprintf(tag, sizeof tag, "stream D%d %dx%dx%d n%d lanes%d W%d", s.dim, s.lt, s.lx, s.ly, s.n, lanes, Ws);
      CHECK(words_per_lane(P, lanes) == Ws, "%s: the runtime's W differs from the kernel's", tag);
      walk_lanemap(P, lanes, Ws, false, tag);
      ++cases;
    }
  }
  printf("cases %d fails %d\n", cases, fails);
  return fails ? 1 : 0;
}
"""


def test_row_enumeration_covers_every_word_once(tmp_path):
    src = tmp_path / "walk.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "walk"
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-Wno-unknown-pragmas", "-I", CSRC,
                    "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "fails 0" in r.stdout
