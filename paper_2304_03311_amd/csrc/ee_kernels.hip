// ee_kernels.hip -- gfx950 kernels of the non-equilibrium Renyi-entropy
// estimator (Bulgarelli & Panero, arXiv:2304.03311).
//
// sweep_kernel: one workgroup holds k trajectories of one job in LDS
//   (int8 spins, colour-separated rows) and runs, entirely on chip, the
//   initial spins, the thermalisation sweeps and the N protocol sweeps with
//   the integer work (Sec. 3 linear protocol; App. A work-then-update).
//   One lane updates W 32-bit words = 4W same-colour sites of a row.  One
//   Philox4x32-10 call gives a 16-bit field to each of 8 sites; a site
//   accepts when its field is below the top half of its uint32 threshold,
//   and only a tie (probability 2^-16) draws the low 16 bits from a second
//   call.  In batch mode the workgroups are persistent and pull work units
//   (job, block of trajectories) from a device queue.
// estimate_kernel: Jarzynski estimator of one job per workgroup (App. A),
//   with wave-shuffle reductions and scans:
//   integer max/min/sum of I_j, FP64 sum of exp(beta (I_j - I_max)/N),
//   log-sum-exp, delete-one jackknife from prefix/suffix sums.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>
#include <vector>

#include "ee_dd.hpp"
#include "ee_internal.hpp"
#include "ee_lanes.hpp"

namespace {

using ee::JobDev;
using ee::Unit;
using namespace ee::lanes;

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename T>
__device__ __forceinline__ T* uni_ptr(T* p) {
  uint64_t v = reinterpret_cast<uint64_t>(p);
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64 products;
// the two xors of each output word are one 3-input bitwise op (table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Philox4x32-10 whose output words 0 and 2 come xored with m: those words
// are the three-input xors of the last round, so m joins its (uniform) key
// at no cost.
__device__ __forceinline__ void philox10_x02(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                             uint32_t k0, uint32_t k1, uint32_t m, uint32_t out[4]) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, (i == 9) ? (k0 ^ m) : k0);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, (i == 9) ? (k1 ^ m) : k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

__device__ __forceinline__ JP load_jp(const JobDev* J) {
  JP P;
  P.dim = uni(J->dim);
  P.n = uni(J->n); P.lt = uni(J->lt); P.ly = uni(J->ly); P.l = uni(J->l); P.N = uni(J->N);
  P.S = uni(J->S); P.subsets = uni(J->subsets); P.whole = uni(J->whole);
  P.H = uni(J->H); P.G = uni(J->G); P.R = uni(J->R); P.traj_words = uni(J->traj_words);
  P.G8 = (P.H + 7) >> 3;
  P.packed_row_words = (P.H + 31) >> 5;
  P.key0 = uni(J->key0); P.key1 = uni(J->key1);
  P.thr0 = uni(J->thr_bulk[0]); P.thr1 = uni(J->thr_bulk[1]); P.thr2 = uni(J->thr_bulk[2]);
  P.reverse = uni(J->reverse); P.spin_format = uni(J->spin_format);
  // Top halves of the bulk thresholds thr[a] (a anti-aligned neighbours;
  // 2^32-1 for a >= dim), offset by 0x8000 so that the unsigned order of
  // 16-bit fields becomes the signed order, as high and low byte tables
  // indexed by a through v_perm_b32 (a <= 7).
  P.pt_hi0 = P.pt_hi1 = P.pt_lo0 = P.pt_lo1 = 0;
  for (int a = 0; a < 8; ++a) {
    const uint32_t th = (a == 0) ? P.thr0 : (a == 1) ? P.thr1 : (a == 2 && P.dim == 3) ? P.thr2 : 0xFFFFFFFFu;
    const uint32_t t16 = (th >> 16) ^ 0x8000u;
    const uint32_t sh = 8u * (uint32_t)(a & 3);
    if (a < 4) {
      P.pt_hi0 |= (t16 >> 8) << sh;
      P.pt_lo0 |= (t16 & 0xFFu) << sh;
    } else {
      P.pt_hi1 |= (t16 >> 8) << sh;
      P.pt_lo1 |= (t16 & 0xFFu) << sh;
    }
  }
  P.mR = uni(J->magic_R); P.sR = uni(J->shift_R); P.mLy = uni(J->magic_Ly); P.sLy = uni(J->shift_Ly);
  P.ramp = uni_ptr(J->ramp_thr);
  P.spins = uni_ptr(J->spins);
  P.work = uni_ptr(J->work);
  return P;
}

// (a ^ b) + c as one v_xad_u32.  Written out because the compiler splits a
// chain of them into separate xors and three-input adds (six instructions
// for the four neighbours of a word instead of four).
__device__ __forceinline__ uint32_t xad_op(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t d;
  asm("v_xad_u32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}

// Ramp position (0..S) of row y when the protocol stands at position pos
// (0..N): every row follows pos, or (subset protocol) row y moves during
// steps [y S, (y+1) S).
__device__ __forceinline__ int row_m(const JP& P, int y, int pos) {
  if (!P.subsets) return pos;
  const int m = pos - y * P.S;
  return m < 0 ? 0 : (m > P.S ? P.S : m);
}

// Output word o (0..3, possibly not a compile-time constant) of a Philox
// result, by selects rather than a dynamically indexed register array.
__device__ __forceinline__ uint32_t pick4(const uint32_t u[4], int o) {
  const uint32_t lo = (o & 1) ? u[1] : u[0];
  const uint32_t hi = (o & 1) ? u[3] : u[2];
  return (o & 2) ? hi : lo;
}

// Two 16-bit lanes per 32-bit word: saturating signed difference a - b, and
// unsigned minimum (v_pk_sub_i16 with clamp, v_pk_min_u16).
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t sub_sat_s16x2(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(s16x2, a),
                                                                    __builtin_bit_cast(s16x2, b)));
}
__device__ __forceinline__ uint32_t min_u16x2(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, a),
                                                                __builtin_bit_cast(u16x2, b)));
}

// The W consecutive words p[0..W-1] of a lane as one 4W-byte access.  Where
// W is 2 or 4, p is 4W-byte aligned (w, the row pitch G and every plane and
// trajectory offset are multiples of W), and the lanes of a wave then cover
// consecutive LDS banks; W separate dword accesses at a lane stride of W
// words would conflict W-fold.  W = 3 (rows of three words, one lane per
// row) reads dwords: an odd lane stride does not conflict.
// GM: p points into device memory (the HBM-streaming path).  The access is
// then made through a global-address-space pointer: a flat access, which is
// what a pointer of unknown space compiles to, also counts against the
// LDS/scalar wait counter, so every LDS or scalar wait would drain the HBM
// loads in flight.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) uint32_t g_u32;
typedef __attribute__((address_space(1))) u32x2 g_u32x2;
typedef __attribute__((address_space(1))) u32x4 g_u32x4;

template <bool GM>
__device__ __forceinline__ uint32_t ld_word(const uint32_t* p) {
  if constexpr (GM) return *(const g_u32*)p;
  else return *p;
}

template <int W, bool GM = false>
__device__ __forceinline__ void ld_words(const uint32_t* p, uint32_t v[W]) {
  if constexpr (GM && W == 4) {
    const u32x4 x = *(const g_u32x4*)p;
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  } else if constexpr (GM && W == 2) {
    const u32x2 x = *(const g_u32x2*)p;
    v[0] = x.x; v[1] = x.y;
  } else if constexpr (W == 4) {
    const uint4 x = *reinterpret_cast<const uint4*>(p);
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  } else if constexpr (W == 2) {
    const uint2 x = *reinterpret_cast<const uint2*>(p);
    v[0] = x.x; v[1] = x.y;
  } else {
#pragma unroll
    for (int q = 0; q < W; ++q) v[q] = ld_word<GM>(p + q);
  }
}
template <int W, bool GM = false>
__device__ __forceinline__ void st_words(uint32_t* p, const uint32_t v[W]) {
  if constexpr (GM && W == 4) {
    *(g_u32x4*)p = u32x4{v[0], v[1], v[2], v[3]};
  } else if constexpr (GM && W == 2) {
    *(g_u32x2*)p = u32x2{v[0], v[1]};
  } else if constexpr (GM) {
#pragma unroll
    for (int q = 0; q < W; ++q) *(g_u32*)(p + q) = v[q];
  } else if constexpr (W == 4) {
    *reinterpret_cast<uint4*>(p) = make_uint4(v[0], v[1], v[2], v[3]);
  } else if constexpr (W == 2) {
    *reinterpret_cast<uint2*>(p) = make_uint2(v[0], v[1]);
  } else {
#pragma unroll
    for (int q = 0; q < W; ++q) p[q] = v[q];
  }
}

// 16-bit half hi (0 low, 1 high) of a Philox output word.
__device__ __forceinline__ uint32_t half16(uint32_t word, int hi) { return hi ? (word >> 16) : (word & 0xFFFFu); }

// The Metropolis update of the sites of one row of colour c that a lane
// owns (words w .. w+W-1 of the row).
//   Lc, Lo  the row's own colour plane and the other one (LDS or HBM)
//   thr     LDS table: thr[a] = threshold of a bulk/glued site with a
//           anti-aligned neighbours (2^32-1 for a >= DIM)
//   (r, t, y)  the row; pC, pO  word w of the row in Lc and in Lo
//   tmo, tpo, ymo, ypo  offsets from pO of the same words in rows t-1,
//           t+1, y-1 and y+1 (periodic)
//   c0, c3  Philox counter words 0 and 3 of the row's first call
//   pos     protocol position of this sweep; dpos  pos minus the previous
//           position (+1 forward, -1 reverse, 0 while thermalising)
// FULL: lx/2 is a multiple of 4 (no pad bytes, x-neighbours by byte
// alignment of two words).  W: consecutive words per lane (2 or 4 need
// FULL and a word count that W divides; 3 needs FULL and rows of exactly
// three words, so that w = 0 and words 0, 1 share a Philox call while word
// 2 takes the next one).  PAR: the row's x parity p = (c + t + y) & 1 when
// the caller knows it at compile time, else -1.  CUT: the code for rows next
// to the cut (t = 0, 1) is compiled in; without it the row must have t > 1.
// XG: the glued partner row is at Lo + og_in (a layout other than the
// colour-plane storage order), with the parity known only at run time.
// LA (lookahead): the row's Philox outputs (phase 1) come in preU, computed
// during the previous half-sweep, and this update computes those of the
// same row in sweep g_next with counter word c3_next into nextU.  They do
// not depend on spins, so that chain overlaps this row's loads and
// decisions instead of lengthening the next half-sweep.
template <int DIM, bool FULL, int W, int PAR, bool CUT, bool XG = false, bool LA = false, bool GM = false>
__device__ __forceinline__ void row_update(const JP& P, const int w, const int wl, const int wr,
                                           uint32_t* __restrict__ Lc, const uint32_t* __restrict__ Lo,
                                           const uint32_t* __restrict__ thr, const int c, const uint32_t g,
                                           const uint32_t j, const int pos, const int dpos, const bool work,
                                           int& dI, const int r, const int t, const int y,
                                           uint32_t* __restrict__ pC, const uint32_t* __restrict__ pO,
                                           const int tmo, const int tpo, const int ymo, const int ypo,
                                           const uint32_t c0, const uint32_t c3, const int og_in = 0,
                                           const uint32_t* gm_in = nullptr, const uint32_t* preU = nullptr,
                                           uint32_t* nextU = nullptr, const uint32_t g_next = 0,
                                           const uint32_t c3_next = 0) {
  static_assert(W == 1 || ((W == 2 || W == 3 || W == 4) && FULL), "several words per lane need whole rows");
  constexpr int NC = (W + 1) / 2;  // Philox calls per row: 8 sites each
  const int G = P.G;
  const int tailsh = 8 * ((P.H - 1) & 3);
  const uint32_t valid = (!FULL && w == G - 1 && tailsh != 24) ? ((1u << (tailsh + 8)) - 1u) : 0xFFFFFFFFu;
  const uint32_t fmask = valid & 0x01010101u;  // bit 0 of every real site's byte
  const uint32_t rshift = (w == G - 1) ? (uint32_t)tailsh : 24u;
  const int p = (PAR >= 0) ? PAR : ((c + t + y) & 1);  // x parity of this row's sites
  uint32_t A[W], B[W], S[W], a[W];
  ld_words<W, GM>(pO, A);
  if (LA) {
#pragma unroll
    for (int k = 0; k < NC; ++k) philox10_x02(c0 + k, g_next, j, c3_next, P.key0, P.key1, 0x80008000u, nextU + 4 * k);
  }
  if (FULL) {
    // the sites' x-1 (p = 0) or x+1 (p = 1) neighbours straddle two words
    const uint32_t E = ld_word<GM>(pO + ((p ? wr : wl) - w));
    const uint32_t sh = p ? 1u : 3u;
#pragma unroll
    for (int q = 0; q < W; ++q) {
      const uint32_t nxt = (q + 1 < W) ? A[q + 1] : E;
      const uint32_t prv = (q > 0) ? A[q - 1] : E;
      B[q] = __builtin_amdgcn_alignbyte(p ? nxt : A[q], p ? A[q] : prv, sh);
    }
  } else {
    const uint32_t nb = ld_word<GM>(pO + ((p ? wr : wl) - w));
    const uint32_t Br = (A[0] >> 8) | ((nb & 0xFFu) << rshift);
    const uint32_t Bl = (A[0] << 8) | ((w == 0) ? ((nb >> tailsh) & 0xFFu) : (nb >> 24));
    B[0] = p ? Br : Bl;
  }
  // t -+ 1 neighbours
  uint32_t Tm[W], Tp[W];
  ld_words<W, GM>(pC, S);
  ld_words<W, GM>(pO + tmo, Tm);
  ld_words<W, GM>(pO + tpo, Tp);
#pragma unroll
  for (int q = 0; q < W; ++q) a[q] = xad_op(A[q], S[q], xad_op(B[q], S[q], xad_op(Tm[q], S[q], Tp[q] ^ S[q])));
  if (DIM == 3) {
    uint32_t Ym[W], Yp[W];
    ld_words<W, GM>(pO + ymo, Ym);
    ld_words<W, GM>(pO + ypo, Yp);
#pragma unroll
    for (int q = 0; q < W; ++q) a[q] = xad_op(Ym[q], S[q], xad_op(Yp[q], S[q], a[q]));
  }
  // Rows next to the cut (t = 0, 1; compiled in with CUT): for glued
  // columns x < l the temporal partner across the cut is in replica r+1
  // (t = 0) or r-1 (t = 1).
  // Tgl: the glued partners' words; Tcu: the own-replica partners across
  // the cut (Tp on t = 0, Tm on t = 1); Tef: the partners counted in a.
  const bool cutrow = CUT && t <= 1;
  uint32_t Tgl[W], Tcu[W], Tef[W];
  // gmq(q): bytes of word q with x < l (precomputed per lane where the
  // caller knows the parity at compile time)
  const auto gmq = [&](int q) { return (PAR >= 0) ? gm_in[q] : glued_mask(P.l - p - 8 * (w + q)); };
  if (cutrow) {
    const int og = (PAR >= 0 || XG) ? og_in : glued_row(P, r, t, y) * G + w;
    ld_words<W, GM>(Lo + og, Tgl);
#pragma unroll
    for (int q = 0; q < W; ++q) {
      Tcu[q] = (t == 0) ? Tp[q] : Tm[q];
      Tef[q] = Tcu[q];
      if (!P.whole) {
        const uint32_t gm = gmq(q);
        Tef[q] = (Tgl[q] & gm) | (Tcu[q] & ~gm);
        a[q] = a[q] - (Tcu[q] ^ S[q]) + (Tef[q] ^ S[q]);
      }
    }
  }
  // Random numbers: one Philox call serves the 8 sites of this row with the
  // same h >> 3; site i of word q uses the 16-bit half (i & 1) of output
  // word ob + 2q + (i >> 1).  The decision u <= U with u = 2^16 v + w is
  // v < U >> 16 unless v equals U >> 16; only then is w (a phase-2 call)
  // needed.  Sites 0, 1 of word q take the halves of one output word and
  // sites 2, 3 those of the next, so both sides are compared two at a time
  // as 16-bit lanes: d = sat(v' - t) with v' = v ^ 0x8000 and
  // t = (U >> 16) ^ 0x8000 has the sign of v - (U >> 16), and d = 0 marks
  // a tie.
  // Call k serves words 2k and 2k+1 of the lane (W >= 2) or, with W = 1,
  // the lane's word alone, whose fields start at output word ob.  The
  // outputs are kept (as v ^ 0x8000 per field) for tied and ramped sites.
  const int ob = (W == 1) ? 2 * (w & 1) : 0;
  uint32_t f[W];
  uint32_t U[NC][4];
  uint32_t dmk[NC];  // per call: minimum of its d's (a zero half marks a tie)
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    // u[0], u[2] arrive as v ^ 0x8000 per field; u[1], u[3] are xored here
    uint32_t u[4];
    if (LA) {
#pragma unroll
      for (int e = 0; e < 4; ++e) u[e] = preU[4 * k + e];
    } else {
      philox10_x02(c0 + k, g, j, c3, P.key0, P.key1, 0x80008000u, u);
    }
    u[1] ^= 0x80008000u;
    u[3] ^= 0x80008000u;
    dmk[k] = 0xFFFFFFFFu;
#pragma unroll
    for (int q = 2 * k; q < 2 * k + 2 && q < W; ++q) {
      // bulk/glued sites: t of site i from the byte tables, selected by byte i of a
      const uint32_t th = __builtin_amdgcn_perm(P.pt_hi1, P.pt_hi0, a[q]);
      const uint32_t tl = __builtin_amdgcn_perm(P.pt_lo1, P.pt_lo0, a[q]);
      const int o = (ob + 2 * q) & 3;
      const uint32_t d01 = sub_sat_s16x2(pick4(u, o), __builtin_amdgcn_perm(th, tl, 0x05010400u));
      const uint32_t d23 = sub_sat_s16x2(pick4(u, o + 1), __builtin_amdgcn_perm(th, tl, 0x07030602u));
      dmk[k] = min_u16x2(dmk[k], min_u16x2(d01, d23));
      // byte i <- the high byte of site i's difference: its bit 7 is the flip
      f[q] = __builtin_amdgcn_perm(d23, d01, 0x07050301u);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) U[k][e] = u[e];
  }
  uint32_t dmin = dmk[0];
#pragma unroll
  for (int k = 1; k < NC; ++k) dmin = min_u16x2(dmin, dmk[k]);
  const auto tied = [](uint32_t d) { return ((d & 0xFFFFu) == 0) | ((d >> 16) == 0); };
  if (__builtin_expect(tied(dmin), 0)) {
    // rare (2^-16 per site): decide the tied sites on u = 2^16 v + w, with
    // the phase-2 call of only the calls that have a tie
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      if (!tied(dmk[k])) continue;
      uint32_t u2[4];
      philox10(c0 + k, g, j, c3 + (1u << 28), P.key0, P.key1, u2);
#pragma unroll
      for (int q = 2 * k; q < 2 * k + 2 && q < W; ++q) {
        const uint32_t a4 = a[q] << 2;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t th = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(thr) +
                                                                 ((a4 >> (8 * i)) & 0xFFu));
          const int o = ((ob + 2 * q) & 3) + (i >> 1);
          if ((half16(pick4(U[k], o), i & 1) ^ 0x8000u) == (th >> 16)) {
            const uint32_t acc = half16(pick4(u2, o), i & 1) <= (th & 0xFFFFu);
            f[q] = (f[q] & ~(0xFFu << (8 * i))) | (acc << (8 * i + 7));
          }
        }
      }
    }
  }
  if (cutrow) {
    // rows next to the cut: the ramped sites (one column, or with the
    // whole-region protocol every column x < l), decided after the bulk
    // and tie decisions, which they replace for their bytes
    const int ramp_w = P.l >> 3;
    const int ramp_sh = 8 * ((P.l >> 1) & 3);
    if (!P.whole && p == (P.l & 1) && (unsigned)(ramp_w - w) < (unsigned)W) {
      // ramped site x = l of a row next to the cut (one lane per row).
      // K = s (S a_fix + (S-m) s_intra + m s_inter) in units of beta/S.
      const int m = row_m(P, y, pos);
#pragma unroll
      for (int q = 0; q < W; ++q) {
        if (w + q != ramp_w) continue;
        const uint32_t fa = ((a[q] - (Tef[q] ^ S[q])) >> ramp_sh) & 0xFFu;
        const uint32_t bb = ((Tcu[q] ^ S[q]) >> ramp_sh) & 1u;
        const uint32_t cc = ((Tgl[q] ^ S[q]) >> ramp_sh) & 1u;
        const uint32_t Ur = P.ramp[m * (8 * DIM) + fa * 4 + bb * 2 + cc];
        const int ri = ramp_sh >> 3;
        const int o = ((ob + 2 * q) & 3) + (ri >> 1);
        const uint32_t vr = half16(pick4(U[q >> 1], o), ri & 1) ^ 0x8000u;
        uint32_t acc = vr < (Ur >> 16);
        if (vr == (Ur >> 16)) {
          uint32_t u2[4];
          philox10(c0 + (q >> 1), g, j, c3 + (1u << 28), P.key0, P.key1, u2);
          acc = half16(pick4(u2, o), ri & 1) <= (Ur & 0xFFFFu);
        }
        f[q] = (f[q] & ~(0xFFu << ramp_sh)) | (acc << (ramp_sh + 7));
        if (work) {
          // the ramped site of colour 0 sees phi_k: its bonds' weights moved
          // by (m - m_prev), so the D_k term is (m - m_prev) 2 (b - c)
          const int dm = m - row_m(P, y, pos - dpos);
          dI += dm * 2 * ((int)bb - (int)cc);
        }
      }
    }
    if (P.whole && 8 * w + p < P.l) {
      // whole-region protocol: every site x < l of a row next to the cut is
      // ramped and none is glued.  Per site K = s (S a_fix + (S-m) s_intra +
      // m s_inter) from the ramp table, replacing the bulk decision.
      const int m = row_m(P, y, pos);
      const uint32_t* __restrict__ Um = P.ramp + m * (8 * DIM);
#pragma unroll
      for (int q = 0; q < W; ++q) {
        const uint32_t rm = gmq(q);  // bytes with x < l
        if (rm == 0) continue;
        const uint32_t bw = Tcu[q] ^ S[q];  // intra partner anti-aligned (bit 0 of each byte)
        const uint32_t cw = Tgl[q] ^ S[q];  // inter partner anti-aligned
        const uint32_t fw = a[q] - bw;      // the 2 dim - 1 fixed neighbours
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (!((rm >> (8 * i)) & 1u)) continue;
          const uint32_t fa = (fw >> (8 * i)) & 0xFFu;
          const uint32_t bb = (bw >> (8 * i)) & 1u;
          const uint32_t cc = (cw >> (8 * i)) & 1u;
          const uint32_t Ur = Um[fa * 4 + bb * 2 + cc];
          const int o = ((ob + 2 * q) & 3) + (i >> 1);
          const uint32_t vr = half16(pick4(U[q >> 1], o), i & 1) ^ 0x8000u;
          uint32_t acc = vr < (Ur >> 16);
          if (vr == (Ur >> 16)) {
            uint32_t u2[4];
            philox10(c0 + (q >> 1), g, j, c3 + (1u << 28), P.key0, P.key1, u2);
            acc = half16(pick4(u2, o), i & 1) <= (Ur & 0xFFFFu);
          }
          f[q] = (f[q] & ~(0xFFu << (8 * i))) | (acc << (8 * i + 7));
        }
        if (work) {
          // colour-0 ramped sites see phi_k; each adds (m - m_prev) 2 (b - c)
          const int dm = m - row_m(P, y, pos - dpos);
          const uint32_t sel = rm & 0x01010101u;
          dI += dm * 2 * (__popc(bw & sel) - __popc(cw & sel));
        }
      }
    }
  }
  uint32_t Snew[W];
#pragma unroll
  for (int q = 0; q < W; ++q) {
    // S ^ ((f >> 7) & fmask) in one three-input op (table 0x78 = a ^ (b & c))
    Snew[q] = __builtin_amdgcn_bitop3_b32(S[q], f[q] >> 7, fmask, 0x78);
  }
  st_words<W, GM>(pC, Snew);
}

// One half-sweep of colour c over the lane's rows of one trajectory, in the
// order of the lane map (any map; the streaming path's and the general
// on-chip one).  L: the trajectory (two colour planes).  UJ: the
// trajectory index is uniform per wave.  GM: L is in device memory (the
// streaming path), accessed through global-address-space pointers.
template <int DIM, bool FULL, bool UJ, int W, bool GM = false>
__device__ __forceinline__ void half_sweep(const JP& P, const Lane& ln, uint32_t* __restrict__ L,
                                           const uint32_t* __restrict__ thr, const int c,
                                           const uint32_t g, uint32_t j, const int pos, const int dpos,
                                           const bool work, int& dI) {
  if (UJ) j = __builtin_amdgcn_readfirstlane(j);
  const int G = P.G;
  const int cw = P.n * P.R * G;  // words per colour plane
  uint32_t* __restrict__ Lc = L + c * cw;
  const uint32_t* __restrict__ Lo = L + (c ^ 1) * cw;
  const int LyG = P.ly * G;
  const int ltLyG = P.lt * LyG;
  const int ywrap = (P.ly - 1) * G;
  const uint32_t ctr3 = (1u << 28) | (uint32_t)c;
  const int w = ln.w;
  int r = ln.r0, t = ln.t0, y = ln.y0;
  int rowbase = ln.rowbase0;
  for (int kk = ln.kstart; kk < ln.kend; kk += ln.kstep) {
    // the periodic wrap in t adds or removes one replica's rows; the one
    // below t = 0 belongs to a row next to the cut (cut variant only)
    const int tpo = LyG - ((t == P.lt - 1) ? ltLyG : 0);
    const int ymo = (y == 0) ? ywrap : -G;
    const int ypo = (y == P.ly - 1) ? -ywrap : G;
    const uint32_t c0 = (uint32_t)((t * P.ly + y) * P.G8 + (w >> 1));
    const auto row = [&](auto cut) {
      const int tmo = -LyG + ((decltype(cut)::value && t == 0) ? ltLyG : 0);
      row_update<DIM, FULL, W, -1, decltype(cut)::value, false, false, GM>(
          P, w, ln.wl, ln.wr, Lc, Lo, thr, c, g, j, pos, dpos, work, dI, r, t, y, Lc + rowbase + w, Lo + rowbase + w,
          tmo, tpo, ymo, ypo, c0, ctr3 | ((uint32_t)r << 1));
    };
    // the code for rows next to the cut runs only where some lane of the
    // wave has such a row
    if (__builtin_amdgcn_ballot_w64(t <= 1) != 0) row(std::true_type{});
    else row(std::false_type{});
    // next row of this lane
    rowbase += ln.step;
    if (DIM == 3) {
      y += ln.dy;
      if (y >= P.ly) { y -= P.ly; ++t; }
    }
    t += ln.dt;
    if (t >= P.lt) {
      t -= P.lt;
      r += ln.rinc;
      rowbase -= ln.wrapadj;
    }
    r += ln.dr;
  }
}

// Rows of colour C of the lane in parity-major order: class 0 (x parity C)
// and class 1 (x parity C ^ 1) in each step.
template <int DIM, int W, int C>
__device__ __forceinline__ void rows_pm(const JP& P, const LanePM& lp, uint32_t* __restrict__ Lc,
                                        const uint32_t* __restrict__ Lo, const uint32_t* __restrict__ thr,
                                        const uint32_t g, const uint32_t j, const int pos, const int dpos,
                                        const bool work, int& dI) {
  const int LyG = P.ly * P.G;
  const int ltLyG = P.lt * LyG;
  const int drw = lp.dt * LyG;
  const uint32_t dc0 = (uint32_t)(lp.dt * P.ly * P.G8);
  const uint32_t c3 = lp.c3 | (uint32_t)C;
  int t = lp.t;
  // The two row addresses as LDS byte addresses, opaque to the compiler at
  // each step (the empty asm statement emits nothing): every access is then
  // one register plus at most one offset, instead of one induction variable
  // per access plus the LDS base.
  typedef __attribute__((address_space(3))) uint32_t lds_u32;
  uint32_t aC = (uint32_t)(uintptr_t)(lds_u32*)(Lc + lp.rw);
  uint32_t aO = (uint32_t)(uintptr_t)(const lds_u32*)(Lo + lp.rw);
  const uint32_t da = 4u * (uint32_t)drw;
  uint32_t c0 = lp.c0;
  for (; t < P.lt; t += lp.dt, aC += da, aO += da, c0 += dc0) {
    asm volatile("" : "+v"(aC), "+v"(aO));
    uint32_t* __restrict__ pC = (uint32_t*)(lds_u32*)(uintptr_t)aC;
    const uint32_t* __restrict__ pO = (const uint32_t*)(const lds_u32*)(uintptr_t)aO;
    // class 0.  2D: t is even, so only the wrap below t = 0 can occur.
    // class 1.  2D: the row t + 1 (odd), whose only possible wrap is above
    // t + 1 = lt - 1; 3D: the same t.  The wrap below t = 0 belongs to a
    // row next to the cut, so only the cut variant has it.
    const int t1 = (DIM == 2) ? t + 1 : t;
    const int wrap_p = (DIM == 3 && t == P.lt - 1) ? ltLyG : 0;
    const int wrap_p1 = (DIM == 3) ? wrap_p : ((t1 == P.lt - 1) ? ltLyG : 0);
    const auto rows = [&](auto cut) {
      constexpr bool CUT = decltype(cut)::value;
      const int wrap_m = (CUT && t == 0) ? ltLyG : 0;
      const int wrap_m1 = (DIM == 3) ? wrap_m : 0;
      row_update<DIM, true, W, C, CUT>(P, lp.w, lp.wl, lp.wr, Lc, Lo, thr, C, g, j, pos, dpos, work, dI, lp.r0,
                                       t, lp.y[0], pC, pO, wrap_m - LyG, LyG - wrap_p, lp.ymo[0], lp.ypo[0], c0,
                                       c3, lp.og[0], lp.gm[C]);
      row_update<DIM, true, W, C ^ 1, CUT>(P, lp.w, lp.wl, lp.wr, Lc, Lo, thr, C, g, j, pos, dpos, work, dI,
                                           lp.r0, t1, lp.y[1], pC + lp.d_rw, pO + lp.d_rw, wrap_m1 - LyG,
                                           LyG - wrap_p1, lp.ymo[1], lp.ypo[1], c0 + lp.d_c0, c3, lp.og[1],
                                           lp.gm[C ^ 1]);
    };
    // Both rows of a step are next to the cut or neither is (t <= 1 implies
    // t1 <= 1 in 2D, t1 = t in 3D).  The code for rows next to the cut runs
    // only in steps where some lane of the wave has such a row.
    if (__builtin_amdgcn_ballot_w64(t <= 1) != 0) rows(std::true_type{});
    else rows(std::false_type{});
  }
}

// half_sweep for lanes that own at most one row (small, latency-bound
// lattices): the row's Philox outputs U were computed during the previous
// half-sweep, and this one computes those of the next (sweep g_next,
// colour c_next) into U.
template <int DIM, bool FULL, bool UJ, int W>
__device__ __forceinline__ void half_sweep_la(const JP& P, const Lane& ln, uint32_t* __restrict__ L,
                                              const uint32_t* __restrict__ thr, const int c, const uint32_t g,
                                              uint32_t j, const int pos, const int dpos, const bool work, int& dI,
                                              uint32_t* U, const uint32_t g_next, const int c_next) {
  if (UJ) j = __builtin_amdgcn_readfirstlane(j);
  if (ln.kstart >= ln.kend) return;
  const int G = P.G;
  const int cw = P.n * P.R * G;  // words per colour plane
  uint32_t* __restrict__ Lc = L + c * cw;
  const uint32_t* __restrict__ Lo = L + (c ^ 1) * cw;
  const int LyG = P.ly * G;
  const int ltLyG = P.lt * LyG;
  const int ywrap = (P.ly - 1) * G;
  const int w = ln.w, r = ln.r0, t = ln.t0, y = ln.y0;
  const int rowbase = ln.rowbase0;
  const int tpo = LyG - ((t == P.lt - 1) ? ltLyG : 0);
  const int ymo = (y == 0) ? ywrap : -G;
  const int ypo = (y == P.ly - 1) ? -ywrap : G;
  const uint32_t c0 = (uint32_t)((t * P.ly + y) * P.G8 + (w >> 1));
  const uint32_t c3 = (1u << 28) | ((uint32_t)r << 1) | (uint32_t)c;
  const uint32_t c3n = (1u << 28) | ((uint32_t)r << 1) | (uint32_t)c_next;
  constexpr int NC = (W + 1) / 2;
  uint32_t Un[4 * NC];
  const auto row = [&](auto cut) {
    const int tmo = -LyG + ((decltype(cut)::value && t == 0) ? ltLyG : 0);
    row_update<DIM, FULL, W, -1, decltype(cut)::value, false, true>(
        P, w, ln.wl, ln.wr, Lc, Lo, thr, c, g, j, pos, dpos, work, dI, r, t, y, Lc + rowbase + w, Lo + rowbase + w,
        tmo, tpo, ymo, ypo, c0, c3, 0, nullptr, U, Un, g_next, c3n);
  };
  if (__builtin_amdgcn_ballot_w64(t <= 1) != 0) row(std::true_type{});
  else row(std::false_type{});
#pragma unroll
  for (int e = 0; e < 4 * NC; ++e) U[e] = Un[e];
}

template <int DIM, bool UJ, int W>
__device__ __forceinline__ void half_sweep_pm(const JP& P, const LanePM& lp, uint32_t* __restrict__ L,
                                              const uint32_t* __restrict__ thr, const int c,
                                              const uint32_t g, uint32_t j, const int pos, const int dpos,
                                              const bool work, int& dI) {
  if (UJ) j = __builtin_amdgcn_readfirstlane(j);
  const int cw = P.n * P.R * P.G;
  uint32_t* __restrict__ Lc = L + c * cw;
  const uint32_t* __restrict__ Lo = L + (c ^ 1) * cw;
  if (c == 0) rows_pm<DIM, W, 0>(P, lp, Lc, Lo, thr, g, j, pos, dpos, work, dI);
  else rows_pm<DIM, W, 1>(P, lp, Lc, Lo, thr, g, j, pos, dpos, work, dI);
}

// Initial spins (phase 0 of the Philox streams): +1 iff u < 2^31.
__device__ void init_spins(const JP& P, uint32_t* L, uint32_t j, int lt_, int T) {
  const int nR = P.n * P.R;
  for (int q = lt_; q < P.traj_words; q += T) {
    const int w = q % P.G;
    const int rowg = q / P.G;
    const int c = rowg / nR;
    const int row = rowg - c * nR;
    const int r = row / P.R;
    const int rho = row - r * P.R;
    uint32_t u[4];
    philox10((uint32_t)(rho * P.G + w), 0u, j, ((uint32_t)r << 1) | (uint32_t)c, P.key0, P.key1, u);
    uint32_t word = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (4 * w + i < P.H) word |= (uint32_t)(u[i] < 0x80000000u) << (8 * i);
    L[q] = word;
  }
}

__device__ void load_spins(const JP& P, uint32_t* L, uint32_t j, int lt_, int T) {
  if (P.spin_format == EE_SPINS_INT8) {
    const uint32_t* src = P.spins + (size_t)j * P.traj_words;
    for (int q = lt_; q < P.traj_words; q += T) L[q] = src[q];
  } else {
    const int PW = P.packed_row_words;
    const uint32_t* src = P.spins + (size_t)j * (2 * P.n * P.R * PW);
    for (int q = lt_; q < P.traj_words; q += T) {
      const int w = q % P.G;
      const int rowg = q / P.G;
      const uint32_t nib = (src[rowg * PW + (w >> 3)] >> (4 * (w & 7))) & 0xFu;
      L[q] = (nib * 0x00204081u) & 0x01010101u;  // 4 bits -> 4 bytes
    }
  }
}

__device__ void store_spins(const JP& P, const uint32_t* L, uint32_t j, int lt_, int T) {
  if (P.spin_format == EE_SPINS_INT8) {
    uint32_t* dst = P.spins + (size_t)j * P.traj_words;
    for (int q = lt_; q < P.traj_words; q += T) dst[q] = L[q];
  } else {
    const int PW = P.packed_row_words;
    const int total = 2 * P.n * P.R * PW;
    uint32_t* dst = P.spins + (size_t)j * total;
    for (int q = lt_; q < total; q += T) {
      const int wb = q % PW;
      const int rowg = q / PW;
      uint32_t packed = 0;
      for (int k = 0; k < 8; ++k) {
        const int w = 8 * wb + k;
        if (w < P.G) packed |= (((L[rowg * P.G + w] * 0x01020408u) >> 24) & 0xFu) << (4 * k);
      }
      dst[q] = packed;
    }
  }
}

// All sweeps of one work unit: k trajectories of one job, one per LDS slot.
// PM: the rows in parity-major order (half_sweep_pm), else in the order of
// the lane map.
template <int DIM, bool FULL, bool UJ, int W, bool PM>
__device__ __forceinline__ void run_unit(const JP& P, uint32_t* lds, int* s_dI, uint32_t* s_thr, int j0,
                                         int cnt, int kslots, uint32_t flags, int n_therm, int g0) {
  static_assert(!PM || FULL, "the parity-major order needs rows of whole words");
  const int tid = threadIdx.x;
  const int T = blockDim.x / kslots;
  const int slot = tid / T;
  const int lt_ = tid - slot * T;
  const bool active = slot < cnt;
  uint32_t* L = lds + (size_t)slot * P.traj_words;
  const uint32_t j = (uint32_t)(j0 + slot);
  if (tid < ee::kMaxSlots) s_dI[tid] = 0;
  if (tid < 8) s_thr[tid] = (tid == 0) ? P.thr0 : (tid == 1) ? P.thr1 : (tid == 2 && DIM == 3) ? P.thr2 : 0xFFFFFFFFu;
  if (active) {
    if (flags & ee::kFlagInit) init_spins(P, L, j, lt_, T);
    else load_spins(P, L, j, lt_, T);
  }
  Lane ln;
  LanePM lp;
  bool on = active;
  if constexpr (PM) {
    lp = make_lane_pm<DIM, W>(P, lt_, T);
  } else {
    ln = make_lane(P, lt_, T, W, true);
    on = active && ln.kstart < ln.kend;
  }
  __syncthreads();

  int dI = 0;
  uint32_t g = (uint32_t)g0;
  const int pos0 = P.reverse ? P.N : 0;
  const auto half = [&](int c, uint32_t gg, int pos, int dpos, bool work) {
    if constexpr (PM) half_sweep_pm<DIM, UJ, W>(P, lp, L, s_thr, c, gg, j, pos, dpos, work, dI);
    else half_sweep<DIM, FULL, UJ, W>(P, ln, L, s_thr, c, gg, j, pos, dpos, work, dI);
  };
  // n_therm sweeps at the starting position, then (protocol) the N sweeps
  // k = 0 .. N-1 at positions k+1 (forward) or N-1-k (reverse); the work
  // is taken at the colour-0 half of each protocol sweep.  One call site
  // of the half-sweep keeps the code to one copy of the row update.
  const bool proto = (flags & ee::kFlagProto) != 0;
  const int n_sweeps = n_therm + (proto ? P.N : 0);
  const int dpos_p = P.reverse ? -1 : 1;
  // Lane-map order with at most one row per lane (uniform, from the shape:
  // the row slots of a replica cover its rows): the Philox outputs of each
  // half-sweep are computed during the one before.
  bool lookahead = false;
  if constexpr (!PM) {
    const int slots = T / (P.G / W);
    lookahead = n_sweeps > 0 && ((slots >= P.n) ? (slots / P.n >= P.R) : (slots >= P.n * P.R));
  }
  if (lookahead) {
    constexpr int NC = (W + 1) / 2;
    uint32_t U[4 * NC];
    if (on) {
      const uint32_t jj = UJ ? __builtin_amdgcn_readfirstlane(j) : j;
      const uint32_t c0 = (uint32_t)((ln.t0 * P.ly + ln.y0) * P.G8 + (ln.w >> 1));
      const uint32_t c3 = (1u << 28) | ((uint32_t)ln.r0 << 1);  // colour 0
#pragma unroll
      for (int k = 0; k < NC; ++k) philox10_x02(c0 + k, g, jj, c3, P.key0, P.key1, 0x80008000u, U + 4 * k);
    }
    for (int s = 0; s < n_sweeps; ++s, ++g) {
      const int k = s - n_therm;
      const bool in_proto = k >= 0;
      const int pos = in_proto ? (P.reverse ? P.N - 1 - k : k + 1) : pos0;
      const int dpos = in_proto ? dpos_p : 0;
#pragma unroll 1
      for (int c = 0; c < 2; ++c) {
        if (on)
          half_sweep_la<DIM, FULL, UJ, W>(P, ln, L, s_thr, c, g, j, pos, dpos, in_proto && c == 0, dI, U,
                                          c == 0 ? g : g + 1, c ^ 1);
        __syncthreads();
      }
    }
  } else {
    for (int s = 0; s < n_sweeps; ++s, ++g) {
      const int k = s - n_therm;
      const bool in_proto = k >= 0;
      const int pos = in_proto ? (P.reverse ? P.N - 1 - k : k + 1) : pos0;
      const int dpos = in_proto ? dpos_p : 0;
#pragma unroll 1
      for (int c = 0; c < 2; ++c) {
        if (on) half(c, g, pos, dpos, in_proto && c == 0);
        __syncthreads();
      }
    }
  }
  if (proto) {
    if (dI != 0) atomicAdd(&s_dI[slot], dI);
    __syncthreads();
    if (active && lt_ == 0) P.work[j] = (int64_t)s_dI[slot];
  }
  if (active) store_spins(P, L, j, lt_, T);
  __syncthreads();
}

template <int DIM, bool UJ, int W>
__device__ __forceinline__ void run_unit_full(const JP& P, uint32_t* lds, int* s_dI, uint32_t* s_thr, int j0,
                                              int cnt, int kslots, uint32_t flags, int n_therm, int g0) {
  if (use_pm(P, blockDim.x / kslots, W))
    run_unit<DIM, true, UJ, W, true>(P, lds, s_dI, s_thr, j0, cnt, kslots, flags, n_therm, g0);
  else
    run_unit<DIM, true, UJ, W, false>(P, lds, s_dI, s_thr, j0, cnt, kslots, flags, n_therm, g0);
}

template <int DIM>
__device__ __forceinline__ void run_unit_dispatch(const JP& P, uint32_t* lds, int* s_dI, uint32_t* s_thr,
                                                  int j0, int cnt, int kslots, uint32_t flags, int n_therm,
                                                  int g0) {
  const int T = blockDim.x / kslots;
  const bool full = (P.H & 3) == 0;
  const bool uj = (T & 63) == 0;
  switch (words_per_lane(P, T)) {
    case 4:
      if (uj) run_unit_full<DIM, true, 4>(P, lds, s_dI, s_thr, j0, cnt, kslots, flags, n_therm, g0);
      else run_unit_full<DIM, false, 4>(P, lds, s_dI, s_thr, j0, cnt, kslots, flags, n_therm, g0);
      return;
    case 3:
      if (uj) run_unit_full<DIM, true, 3>(P, lds, s_dI, s_thr, j0, cnt, kslots, flags, n_therm, g0);
      else run_unit_full<DIM, false, 3>(P, lds, s_dI, s_thr, j0, cnt, kslots, flags, n_therm, g0);
      return;
    case 2:
      if (uj) run_unit_full<DIM, true, 2>(P, lds, s_dI, s_thr, j0, cnt, kslots, flags, n_therm, g0);
      else run_unit_full<DIM, false, 2>(P, lds, s_dI, s_thr, j0, cnt, kslots, flags, n_therm, g0);
      return;
    default:
      if (full && uj) run_unit_full<DIM, true, 1>(P, lds, s_dI, s_thr, j0, cnt, kslots, flags, n_therm, g0);
      else if (full) run_unit_full<DIM, false, 1>(P, lds, s_dI, s_thr, j0, cnt, kslots, flags, n_therm, g0);
      else run_unit<DIM, false, false, 1, false>(P, lds, s_dI, s_thr, j0, cnt, kslots, flags, n_therm, g0);
  }
}

// Per-job mode (units == nullptr): workgroup b runs trajectories
// [b*single_k, b*single_k + single_k) of single_job.  Batch mode: persistent
// workgroups draw units from the queue until it is empty.  The dimension of
// each unit's job selects the 2D or 3D sweep (uniform per workgroup).
// tail: word offset, in the dynamic LDS, of the workgroup's small tables
// (unit index, per-slot work sums, threshold table), which follow the
// trajectory slots.  The kernel has no static LDS, so the slots start at
// LDS address 0 and the row addresses need no base added.
__device__ __forceinline__ void sweep_body(const JobDev* single_job, int single_k, const Unit* units, int n_units,
                                           int* queue, const JobDev* const* jobtab, uint32_t flags, int n_therm,
                                           int g0, int tail) {
  extern __shared__ __align__(16) uint32_t lds_raw[];
  // The LDS base as an opaque scalar register value rather than the
  // (link-time) address of the array: the compiler then folds it into the
  // row address induction variables instead of adding it at every access.
  // The empty asm statement only hides the value's origin; it emits nothing.
  typedef __attribute__((address_space(3))) uint32_t lds_u32;
  uint32_t lds_addr = (uint32_t)(uintptr_t)(lds_u32*)lds_raw;
  asm volatile("" : "+s"(lds_addr));
  uint32_t* const lds = (uint32_t*)(lds_u32*)(uintptr_t)lds_addr;
  int* const s_tab = reinterpret_cast<int*>(lds + tail);
  int& s_unit = s_tab[0];
  int* const s_dI = s_tab + 4;
  uint32_t* const s_thr = reinterpret_cast<uint32_t*>(s_dI + ee::kMaxSlots);
  const int tid = threadIdx.x;
  for (int iter = 0;; ++iter) {
    const JobDev* J;
    int j0, cnt, kslots;
    if (units != nullptr) {
      if (tid == 0) s_unit = atomicAdd(queue, 1);
      __syncthreads();
      const int u = s_unit;
      if (u >= n_units) break;
      const Unit U = units[u];
      J = uni_ptr(jobtab[uni(U.job)]);
      j0 = uni(U.j0);
      cnt = uni(U.count);
      kslots = uni(U.slots);
    } else {
      if (iter > 0) break;
      J = single_job;
      kslots = single_k;
      j0 = blockIdx.x * kslots;
      cnt = min(kslots, J->n_traj - j0);
    }
    const JP P = load_jp(J);
    if (uni(J->dim) == 3)
      run_unit_dispatch<3>(P, lds, s_dI, s_thr, j0, cnt, kslots, flags, n_therm, g0);
    else
      run_unit_dispatch<2>(P, lds, s_dI, s_thr, j0, cnt, kslots, flags, n_therm, g0);
  }
}

// The sweep kernel: up to 4 waves per SIMD (128 VGPRs) and up to four words
// per lane, so that the per-row address and loop work is spread over 16
// sites.
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4, 4)))
sweep_kernel(const JobDev* single_job, int single_k, const Unit* units, int n_units, int* queue,
             const JobDev* const* jobtab, uint32_t flags, int n_therm, int g0, int tail) {
  sweep_body(single_job, single_k, units, n_units, queue, jobtab, flags, n_therm, g0, tail);
}

// ---------------------------------------------------------------------------
// Streaming path: lattices larger than one workgroup's LDS.  The spins stay
// in HBM (INT8 colour planes); one launch updates one colour of every
// trajectory of a job.  Block (x, y) covers lanes of trajectory y; a
// trajectory has `lanes` lanes, each walking its rows as in the on-chip
// path.  The neighbour rows are read through the vector caches, and the
// integer work goes to HBM with 64-bit atomics.
// ---------------------------------------------------------------------------
// Workgroups are dispatched to the XCDs (kXcd of them, each with its own L2)
// in turn by workgroup id.  The grid is one-dimensional, bx blocks per
// trajectory; the physical id is mapped to a logical (trajectory, block)
// such that each XCD gets one contiguous run of logical blocks, i.e. whole
// trajectories and neighbouring rows, which then meet in one L2.  The map
// is a bijection of [0, total), so results do not depend on it.
constexpr int kXcd = 8;
__device__ __forceinline__ void xcd_block(int bx, int total, int& j, int& b) {
  const int id = blockIdx.x;
  const int q = total / kXcd, rem = total - q * kXcd;
  const int x = id % kXcd, k = id / kXcd;
  const int logical = (x < rem) ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
  j = logical / bx;
  b = logical - j * bx;
}

template <int DIM, bool FULL, int W>
__device__ __forceinline__ void stream_half(const JP& P, uint32_t* s_thr, int lanes, int c, uint32_t g, int pos,
                                            int dpos, bool work) {
  const int bx = (lanes + 255) / 256;
  int jj, b;
  xcd_block(bx, (int)gridDim.x, jj, b);
  const int lt_ = b * blockDim.x + threadIdx.x;
  const uint32_t j = (uint32_t)jj;
  uint32_t* L = P.spins + (size_t)j * P.traj_words;
  int dI = 0;
  const Lane ln = make_lane(P, lt_ < lanes ? lt_ : 0, lanes, W, false);
  if (lt_ < lanes && ln.kstart < ln.kend)
    half_sweep<DIM, FULL, true, W, true>(P, ln, L, s_thr, c, g, j, pos, dpos, work, dI);
  if (dI != 0) atomicAdd(reinterpret_cast<unsigned long long*>(&P.work[j]), (unsigned long long)(long long)dI);
}

// Body of the streaming launches: the widest lane width (words per lane)
// that the job's rows allow.
__device__ __forceinline__ void stream_body(const JobDev* J, int lanes, int c, uint32_t g, int pos, int dpos,
                                            int work) {
  __shared__ uint32_t s_thr[8];
  const JP P = load_jp(J);
  const int dim = uni(J->dim);
  if (threadIdx.x < 8)
    s_thr[threadIdx.x] = (threadIdx.x == 0) ? P.thr0 : (threadIdx.x == 1) ? P.thr1
                       : (threadIdx.x == 2 && dim == 3) ? P.thr2 : 0xFFFFFFFFu;
  __syncthreads();
  const bool full = (P.H & 3) == 0;
  const bool w = work != 0;
  switch (words_per_lane(P, lanes)) {
    case 4:
      if (dim == 3) stream_half<3, true, 4>(P, s_thr, lanes, c, g, pos, dpos, w);
      else stream_half<2, true, 4>(P, s_thr, lanes, c, g, pos, dpos, w);
      return;
    case 3:
      if (dim == 3) stream_half<3, true, 3>(P, s_thr, lanes, c, g, pos, dpos, w);
      else stream_half<2, true, 3>(P, s_thr, lanes, c, g, pos, dpos, w);
      return;
    case 2:
      if (dim == 3) stream_half<3, true, 2>(P, s_thr, lanes, c, g, pos, dpos, w);
      else stream_half<2, true, 2>(P, s_thr, lanes, c, g, pos, dpos, w);
      return;
    default:
      if (dim == 3) {
        if (full) stream_half<3, true, 1>(P, s_thr, lanes, c, g, pos, dpos, w);
        else stream_half<3, false, 1>(P, s_thr, lanes, c, g, pos, dpos, w);
      } else {
        if (full) stream_half<2, true, 1>(P, s_thr, lanes, c, g, pos, dpos, w);
        else stream_half<2, false, 1>(P, s_thr, lanes, c, g, pos, dpos, w);
      }
  }
}

// 4 waves per SIMD (128 VGPRs), up to four words per lane.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
stream_sweep_kernel(const JobDev* J, int lanes, int c, uint32_t g, int pos, int dpos, int work) {
  stream_body(J, lanes, c, g, pos, dpos, work);
}

// ---------------------------------------------------------------------------
// Plane-marching streaming path: lattices larger than one workgroup's LDS,
// jobs with enough trajectories to fill the GPU with long marches.  One
// sweep is one launch of march_kernel and one of march_fixup_kernel.
//
// A plane is every site of one replica with one t (all y, both colours).
// A sweep updates colour 0 everywhere with colour 1 unchanged, then colour
// 1 with colour 0 new (the oracle's order; sites of one colour are
// independent).  Workgroup (j, r, s) marches the planes of segment s of
// replica r of trajectory j through a ring of kMarchSlots plane slots in
// LDS: at step p it updates colour 0 of plane p (colour 1 of planes p-1, p,
// p+1 still old) and then colour 1 of plane p-1 (colour 0 of planes p-2,
// p-1, p already new), while plane p+2 is loaded and plane p-2, final,
// written back.  Each plane is read and written once per sweep, 2 B per
// site.  Colour 1 of a segment's first and last plane needs colour 0 of the
// neighbouring segments' planes, so it is left to march_fixup_kernel; the
// main pass only reads colour 1 of the neighbouring segments' boundary
// planes, which nobody writes during it.  Segments cover the unwrapped
// planes [1, lt + 1) (plane lt is t = 0), so planes t = 1 and t = 0, the
// rows next to the cut, are always boundary planes: the main pass updates
// only their colour 0, whose glued partners (colour 1 of replica r +- 1 in
// plane 1 - t) it reads from HBM, unchanged by the main pass.
// ---------------------------------------------------------------------------
constexpr int kMarchSlots = 5;
__device__ __forceinline__ void segment_bounds(int lt, int nseg, int s, int& t0, int& t1) {
  t0 = 1 + (int)((int64_t)lt * s / nseg);
  t1 = 1 + (int)((int64_t)lt * (s + 1) / nseg);
}

// Plane transfers between replica r of the trajectory in HBM (colour-plane
// storage) and a ring slot ([colour][y][word], the rows of the plane in
// storage order, so that slot unit i is simply the i-th unit of the slot).
// A unit is four words when the row length G is a multiple of 4, else one
// word; GV units per row.  The HBM side goes through global-address-space
// pointers: flat accesses would also count against the LDS wait counter, so
// that every LDS wait of the compute phases would wait for the transfers
// in flight.  A 16-byte unit is a native four-word vector.
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
template <typename V>
using gptr = __attribute__((address_space(1))) V*;

// HBM word offset, at t = 0, of unit u of a plane of replica r.
__device__ __forceinline__ int unit_offset(const JP& P, int r, int u, int GV, int uw) {
  const int q = u / GV, wv = u - q * GV;
  const int c = q / P.ly, y = q - c * P.ly;
  return ((c * P.n + r) * P.R + y) * P.G + uw * wv;
}

template <bool TO_LDS, typename V>
__device__ __forceinline__ void plane_copy_v(const JP& P, uint32_t* traj, uint32_t* slot, int r, int t, int i_lo,
                                             int i_hi, int GV) {
  constexpr int UW = sizeof(V) / 4;
  V* sv = reinterpret_cast<V*>(slot);
  const gptr<uint32_t> base = (gptr<uint32_t>)(traj + t * P.ly * P.G);
  for (int i = i_lo + (int)threadIdx.x; i < i_hi; i += blockDim.x) {
    const gptr<V> g = (gptr<V>)(base + unit_offset(P, r, i, GV, UW));
    if (TO_LDS) sv[i] = *g;
    else *g = sv[i];
  }
}

// Copy colours [c_lo, c_hi) of plane t (synchronously: each unit's load or
// store is followed by its use).
template <bool TO_LDS>
__device__ __forceinline__ void plane_copy(const JP& P, uint32_t* traj, uint32_t* slot, int r, int t, int c_lo,
                                           int c_hi) {
  if ((P.G & 3) == 0) {
    const int GV = P.G >> 2;
    plane_copy_v<TO_LDS, v4u>(P, traj, slot, r, t, c_lo * P.ly * GV, c_hi * P.ly * GV, GV);
  } else {
    plane_copy_v<TO_LDS, uint32_t>(P, traj, slot, r, t, c_lo * P.ly * P.G, c_hi * P.ly * P.G, P.G);
  }
}

// This thread's share of the plane transfers: 16-byte units u0 + k T
// (k < 4) of a plane, with their HBM word offsets at t = 0 (the units of
// plane t sit at the same offsets plus t ly G words), computed once per
// launch.  A load is split in two: xfer_fetch() issues the loads into
// registers, xfer_put() writes them to the slot; between the two the loads
// are in flight while the workgroup computes.  Units from 4 T on, and
// planes whose rows are not a multiple of four words, are copied at once.
struct Xfer {
  int o0, o1, o2, o3;  // HBM word offsets (t = 0) of units u0 + k T
  int u0, T, U, U0;    // first unit, stride, units per plane, units of colour 0
  int GV, tw, r;       // units per row, HBM words per plane step (ly G), replica
  bool vec;            // rows of a multiple of four words
};

__device__ __forceinline__ Xfer make_xfer(const JP& P, int r) {
  Xfer X;
  X.vec = (P.G & 3) == 0;
  X.GV = P.G >> 2;
  X.U = 2 * P.ly * X.GV;
  X.U0 = P.ly * X.GV;
  X.T = blockDim.x;
  X.u0 = threadIdx.x;
  X.tw = P.ly * P.G;
  X.r = r;
  const auto off = [&](int u) { return (X.vec && u < X.U) ? unit_offset(P, r, u, X.GV, 4) : 0; };
  X.o0 = off(X.u0);
  X.o1 = off(X.u0 + X.T);
  X.o2 = off(X.u0 + 2 * X.T);
  X.o3 = off(X.u0 + 3 * X.T);
  return X;
}

// Issue the loads of colours [c_lo, 2) of plane t.
__device__ __forceinline__ void xfer_fetch(const Xfer& X, const JP& P, uint32_t* traj, uint32_t* slot, int t,
                                           int c_lo, v4u& v0, v4u& v1, v4u& v2, v4u& v3) {
  if (!X.vec) {
    plane_copy<true>(P, traj, slot, X.r, t, c_lo, 2);
    return;
  }
  const int lo = c_lo * X.U0;
  const gptr<uint32_t> base = (gptr<uint32_t>)(traj + t * X.tw);
  const auto ld = [&](int k, int o, v4u& v) {
    const int u = X.u0 + k * X.T;
    if (u >= lo && u < X.U) v = *(gptr<v4u>)(base + o);
  };
  ld(0, X.o0, v0);
  ld(1, X.o1, v1);
  ld(2, X.o2, v2);
  ld(3, X.o3, v3);
  if (4 * X.T < X.U) plane_copy_v<true, v4u>(P, traj, slot, X.r, t, max(lo, 4 * X.T), X.U, X.GV);
}

__device__ __forceinline__ void xfer_put(const Xfer& X, uint32_t* slot, int c_lo, const v4u& v0, const v4u& v1,
                                         const v4u& v2, const v4u& v3) {
  if (!X.vec) return;
  const int lo = c_lo * X.U0;
  v4u* sv = reinterpret_cast<v4u*>(slot);
  const auto st = [&](int k, const v4u& v) {
    const int u = X.u0 + k * X.T;
    if (u >= lo && u < X.U) sv[u] = v;
  };
  st(0, v0);
  st(1, v1);
  st(2, v2);
  st(3, v3);
}

// Write colours [0, c_hi) of plane t back to HBM.
__device__ __forceinline__ void xfer_store(const Xfer& X, const JP& P, uint32_t* traj, uint32_t* slot, int t,
                                           int c_hi) {
  if (!X.vec) {
    plane_copy<false>(P, traj, slot, X.r, t, 0, c_hi);
    return;
  }
  const int hi = c_hi * X.U0;
  const gptr<uint32_t> base = (gptr<uint32_t>)(traj + t * X.tw);
  const v4u* sv = reinterpret_cast<const v4u*>(slot);
  const auto st = [&](int k, int o) {
    const int u = X.u0 + k * X.T;
    if (u < hi) *(gptr<v4u>)(base + o) = sv[u];
  };
  st(0, X.o0);
  st(1, X.o1);
  st(2, X.o2);
  st(3, X.o3);
  if (4 * X.T < hi) plane_copy_v<false, v4u>(P, traj, slot, X.r, t, 4 * X.T, hi, X.GV);
}

// A row of a plane's colour: y and first word w.
struct RowDesc {
  int y, w;
};

__device__ __forceinline__ RowDesc row_desc(int it, int GW, int W) {
  RowDesc d;
  d.y = it / GW;
  d.w = (it - d.y * GW) * W;
  return d;
}

// Colour c of plane t of replica r (unwrapped plane index p: slots of p-1,
// p, p+1 are sm, s0, sp) from the ring; PW words per slot.  d0: this
// thread's first row (the same in every plane).  Rows next to the cut
// (t <= 1) come here with c = 0 only.
template <int DIM, bool FULL, int W>
__device__ __forceinline__ void march_colour(const JP& P, uint32_t* win, uint32_t* traj, int PW, int sm, int s0,
                                             int sp, int c, int r, int t, const uint32_t* thr, uint32_t g,
                                             uint32_t j, int pos, int dpos, bool work, int& dI, const RowDesc& d0) {
  const int G = P.G, GW = G / W, ly = P.ly;
  uint32_t* own = win + s0 * PW + c * ly * G;
  const uint32_t* oth = win + s0 * PW + (c ^ 1) * ly * G;
  const int tmo = (sm - s0) * PW, tpo = (sp - s0) * PW;
  const uint32_t c3 = (1u << 28) | ((uint32_t)r << 1) | (uint32_t)c;
  const auto rows = [&](auto cut) {
    constexpr bool CUT = decltype(cut)::value;
    // glued partners: colour 1 of replica r+1 in plane 1 (t = 0) or of
    // replica r-1 in plane 0 (t = 1), in HBM
    const int rgl = (t == 0) ? ((r + 1 == P.n) ? 0 : r + 1) : ((r == 0) ? P.n - 1 : r - 1);
    const int ogl = ((P.n + rgl) * P.R + (1 - t) * ly) * G;
    RowDesc d = d0;
    for (int it = threadIdx.x; it < ly * GW;) {
      const int y = d.y, w = d.w;
      const int wl = (w == 0) ? G - 1 : w - 1, wr = (w + W == G) ? 0 : w + W;
      const int ymo = (y == 0) ? (ly - 1) * G : -G, ypo = (y == ly - 1) ? -(ly - 1) * G : G;
      const uint32_t c0 = (uint32_t)((t * ly + y) * P.G8 + (w >> 1));
      row_update<DIM, FULL, W, -1, CUT, true>(P, w, wl, wr, own, traj, thr, c, g, j, pos, dpos, work, dI, r, t, y,
                                              own + y * G + w, oth + y * G + w, tmo, tpo, ymo, ypo, c0, c3,
                                              CUT ? ogl + y * G + w : 0);
      it += blockDim.x;
      if (it < ly * GW) d = row_desc(it, GW, W);
    }
  };
  if (t <= 1) rows(std::true_type{});
  else rows(std::false_type{});
}

template <int DIM, bool FULL, int W>
__device__ __forceinline__ void march_segment(const JP& P, uint32_t* win, const uint32_t* thr, int nseg, uint32_t g,
                                              int pos, int dpos, bool work) {
  int jj, rs;
  xcd_block(P.n * nseg, (int)gridDim.x, jj, rs);
  const int r = rs / nseg, seg = rs - r * nseg;
  const uint32_t j = (uint32_t)jj;
  uint32_t* traj = P.spins + (size_t)j * P.traj_words;
  const int PW = 2 * P.ly * P.G;
  int t0, t1;
  segment_bounds(P.lt, nseg, seg, t0, t1);
  // ring of kMarchSlots slots: plane p in slot (p - t0 + 1) mod kMarchSlots
  const auto slot = [&](int p) { return (p - t0 + 1) % kMarchSlots; };
  const auto phys = [&](int p) { return (p >= P.lt) ? p - P.lt : p; };  // 0 <= p < 2 lt
  const Xfer X = make_xfer(P, r);
  const RowDesc d0 = row_desc(threadIdx.x, P.G / W, W);
  int dI = 0;
  v4u v0 = {}, v1 = {}, v2 = {}, v3 = {};
  // planes t0-1 .. t0+1; a neighbouring segment's boundary plane
  // contributes only its colour 1
  for (int p = t0 - 1; p <= t0 + 1; ++p) {
    const int c_lo = (p < t0 || p >= t1) ? 1 : 0;
    xfer_fetch(X, P, traj, win + slot(p) * PW, phys(p), c_lo, v0, v1, v2, v3);
    xfer_put(X, win + slot(p) * PW, c_lo, v0, v1, v2, v3);
  }
  __syncthreads();
  for (int p = t0; p < t1; ++p) {
    // step p: colour 0 of plane p (planes p-1 .. p+1 in the ring), then
    // colour 1 of plane p-1 (planes p-2 .. p).  Meanwhile plane p+2 is
    // fetched (into registers, then into its slot, free since plane p-3
    // was written back) and the final plane p-2 is written back.
    const bool fetch = p + 2 <= t1;
    const int c_lo = (p + 2 == t1) ? 1 : 0;
    if (fetch) xfer_fetch(X, P, traj, win + slot(p + 2) * PW, phys(p + 2), c_lo, v0, v1, v2, v3);
    march_colour<DIM, FULL, W>(P, win, traj, PW, slot(p - 1), slot(p), slot(p + 1), 0, r, phys(p), thr, g, j, pos,
                               dpos, work, dI, d0);
    __syncthreads();
    // plane p-2 is final (colour 1 of the segment's first plane waits for
    // the fix-up pass)
    if (p - 2 >= t0) xfer_store(X, P, traj, win + slot(p - 2) * PW, phys(p - 2), (p - 2 > t0) ? 2 : 1);
    if (p - 1 >= t0 + 1)
      march_colour<DIM, FULL, W>(P, win, traj, PW, slot(p - 2), slot(p - 1), slot(p), 1, r, phys(p - 1), thr, g, j,
                                 pos, dpos, false, dI, d0);
    if (fetch) xfer_put(X, win + slot(p + 2) * PW, c_lo, v0, v1, v2, v3);
    __syncthreads();
  }
  if (t1 - 2 >= t0) xfer_store(X, P, traj, win + slot(t1 - 2) * PW, phys(t1 - 2), (t1 - 2 > t0) ? 2 : 1);
  xfer_store(X, P, traj, win + slot(t1 - 1) * PW, phys(t1 - 1), 1);
  if (dI != 0) atomicAdd(reinterpret_cast<unsigned long long*>(&P.work[j]), (unsigned long long)(long long)dI);
}

// Colour 1 of each segment's first and last plane, every replica, from HBM
// (block: one plane of one segment of one trajectory).
template <int DIM, bool FULL, int W>
__device__ __forceinline__ void fixup_plane(const JP& P, const uint32_t* thr, int nseg, uint32_t g, int pos,
                                            int dpos) {
  const int b = blockIdx.x;
  const int jj = b / (2 * nseg), rem = b - jj * 2 * nseg, seg = rem >> 1, last = rem & 1;
  int t0, t1;
  segment_bounds(P.lt, nseg, seg, t0, t1);
  if (last && t1 - 1 == t0) return;  // a one-plane segment has one boundary plane
  const int t = (last ? t1 - 1 : t0) % P.lt;
  const uint32_t j = (uint32_t)jj;
  uint32_t* traj = P.spins + (size_t)j * P.traj_words;
  const int G = P.G, GW = G / W, ly = P.ly, R = P.R;
  uint32_t* Lc = traj + P.n * R * G;  // colour 1
  const uint32_t* Lo = traj;          // colour 0
  const int LyG = ly * G, ltLyG = P.lt * LyG;
  const int tpo = LyG - ((t == P.lt - 1) ? ltLyG : 0);
  const int tmo = -LyG + ((t == 0) ? ltLyG : 0);
  int dI = 0;
  const auto rows = [&](auto cut) {
    constexpr bool CUT = decltype(cut)::value;
    for (int it = threadIdx.x; it < P.n * ly * GW; it += blockDim.x) {
      const int rr = it / GW, w = (it - rr * GW) * W;
      const int r = rr / ly, y = rr - r * ly;
      const int wl = (w == 0) ? G - 1 : w - 1, wr = (w + W == G) ? 0 : w + W;
      const int ymo = (y == 0) ? (ly - 1) * G : -G, ypo = (y == ly - 1) ? -(ly - 1) * G : G;
      const int rowbase = (r * R + t * ly + y) * G;
      const uint32_t c0 = (uint32_t)((t * ly + y) * P.G8 + (w >> 1));
      const uint32_t c3 = (1u << 28) | ((uint32_t)r << 1) | 1u;
      row_update<DIM, FULL, W, -1, CUT>(P, w, wl, wr, Lc, Lo, thr, 1, g, j, pos, dpos, false, dI, r, t, y,
                                        Lc + rowbase + w, Lo + rowbase + w, tmo, tpo, ymo, ypo, c0, c3);
    }
  };
  if (t <= 1) rows(std::true_type{});
  else rows(std::false_type{});
}

// Words per lane of the marching kernels: as the on-chip kernel chooses for
// a workgroup of blockDim lanes per plane.
template <bool MAIN>
__device__ __forceinline__ void march_body(const JobDev* J, int nseg, uint32_t g, int pos, int dpos, int work) {
  extern __shared__ __align__(16) uint32_t march_lds[];
  const JP P = load_jp(J);
  const int dim = uni(J->dim);
  const int PW = 2 * P.ly * P.G;
  uint32_t* thr = MAIN ? march_lds + kMarchSlots * PW : march_lds;  // after the ring (main pass) or alone (fix-up)
  if (threadIdx.x < 8)
    thr[threadIdx.x] = (threadIdx.x == 0) ? P.thr0 : (threadIdx.x == 1) ? P.thr1
                     : (threadIdx.x == 2 && dim == 3) ? P.thr2 : 0xFFFFFFFFu;
  __syncthreads();
  const bool full = (P.H & 3) == 0;
  const bool w = work != 0;
  const auto go = [&](auto dimc, auto fullc, auto wc) {
    constexpr int D = decltype(dimc)::value;
    constexpr bool F = decltype(fullc)::value;
    constexpr int WW = decltype(wc)::value;
    if (MAIN) march_segment<D, F, WW>(P, march_lds, thr, nseg, g, pos, dpos, w);
    else fixup_plane<D, F, WW>(P, thr, nseg, g, pos, dpos);
  };
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  using T_ = std::true_type;
  using F_ = std::false_type;
  switch (words_per_lane(P, (int)blockDim.x)) {
    case 4:
      if (dim == 3) go(I3{}, T_{}, std::integral_constant<int, 4>{});
      else go(I2{}, T_{}, std::integral_constant<int, 4>{});
      return;
    case 3:
      if (dim == 3) go(I3{}, T_{}, std::integral_constant<int, 3>{});
      else go(I2{}, T_{}, std::integral_constant<int, 3>{});
      return;
    case 2:
      if (dim == 3) go(I3{}, T_{}, std::integral_constant<int, 2>{});
      else go(I2{}, T_{}, std::integral_constant<int, 2>{});
      return;
    default:
      if (dim == 3) {
        if (full) go(I3{}, T_{}, std::integral_constant<int, 1>{});
        else go(I3{}, F_{}, std::integral_constant<int, 1>{});
      } else {
        if (full) go(I2{}, T_{}, std::integral_constant<int, 1>{});
        else go(I2{}, F_{}, std::integral_constant<int, 1>{});
      }
  }
}

__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4, 4)))
march_kernel(const JobDev* J, int nseg, uint32_t g, int pos, int dpos, int work) {
  march_body<true>(J, nseg, g, pos, dpos, work);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
march_fixup_kernel(const JobDev* J, int nseg, uint32_t g, int pos, int dpos) {
  march_body<false>(J, nseg, g, pos, dpos, 0);
}

// Initial spins of every trajectory, written straight to HBM.
__global__ void __launch_bounds__(256) stream_init_kernel(const JobDev* J, int lanes) {
  const JP P = load_jp(J);
  const uint32_t j = blockIdx.y;
  const int lt_ = blockIdx.x * blockDim.x + threadIdx.x;
  if (lt_ < lanes) init_spins(P, P.spins + (size_t)j * P.traj_words, j, lt_, lanes);
}

__global__ void zero_work_kernel(const JobDev* J) {
  const int n = J->n_traj;
  int64_t* w = J->work;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) w[i] = 0;
}

__global__ void queue_reset_kernel(int* queue) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0;
}

// ---------------------------------------------------------------------------
// Estimator (App. A, Jarzynski's equality), one workgroup per job.
//
// Every floating-point result is formed by the same operations in the same
// order as the plain definition: the n_t exponentials e_j are summed one
// after the other in ascending j, each leave-one-out sum is its own
// ascending sum over j != i, and the mean and variance of W are sums of the
// terms -(beta/S) I_j in ascending j.  exp and log are the correctly
// rounded ones of ee_dd.hpp.  The order costs no time worth counting: the
// long sums are a few thousand dependent FP64 adds, each done by one lane
// while other waves do the others, and the leave-one-out sums run one per
// lane (n_t^2 adds in all, e_j broadcast from LDS tiles).
// ---------------------------------------------------------------------------
#pragma clang fp contract(off)
constexpr int kEstThreads = ee::kEstimateThreads;
constexpr int kEstWaves = kEstThreads / 64;
constexpr int kEstTile = 4096;  // e_j per LDS tile (32 KiB)
constexpr int kEstAcc = 8;      // leave-one-out sums per lane and pass

// Integer reduction over the block: butterfly shuffles within each 64-lane
// wave, then the wave results through LDS (sh: kEstWaves entries).
template <typename Op>
__device__ long long block_reduce_ll(long long v, long long* sh, Op op) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = op(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  long long r = sh[0];
#pragma unroll
  for (int k = 1; k < kEstWaves; ++k) r = op(r, sh[k]);
  __syncthreads();
  return r;
}

// Visit load(0), load(1), ... load(n-1) in order with add(), loading
// kEstGroup values ahead of their adds.
constexpr int kEstGroup = 16;
template <typename Load, typename Add>
__device__ __forceinline__ void for_groups(int n, Load load, Add add) {
  int j = 0;
  for (; j + kEstGroup <= n; j += kEstGroup) {
    double v[kEstGroup];
#pragma unroll
    for (int k = 0; k < kEstGroup; ++k) v[k] = load(j + k);
#pragma unroll
    for (int k = 0; k < kEstGroup; ++k) add(v[k]);
  }
  for (; j < n; ++j) add(load(j));
}

__global__ void __launch_bounds__(kEstThreads) estimate_kernel(const JobDev* const* jobtab) {
  __shared__ double tile[kEstTile];
  __shared__ long long shl[kEstWaves];
  __shared__ double shd[4];
  const JobDev* J = jobtab[blockIdx.x];
  const int tid = threadIdx.x;
  const int n = J->n_traj;
  const int64_t* I = J->work;
  const double beta = J->beta;
  const double N = (double)J->S;  // W_j = -(beta/S) I_j
  ee_result* res = J->result;
  double* e = reinterpret_cast<double*>(J->work + n);  // n doubles: e_j
  double* loo = e + n;                                 // n doubles: leave-one-out estimates

  long long mx = LLONG_MIN, mn = LLONG_MAX;
  for (int i = tid; i < n; i += kEstThreads) {
    const long long v = I[i];
    mx = v > mx ? v : mx;
    mn = v < mn ? v : mn;
  }
  const long long imax = block_reduce_ll(mx, shl, [](long long a, long long b) { return a > b ? a : b; });
  const long long imin = block_reduce_ll(mn, shl, [](long long a, long long b) { return a < b ? a : b; });
  for (int i = tid; i < n; i += kEstThreads) e[i] = ee::dd::exp_cr((beta * (double)(I[i] - imax)) / N);
  __syncthreads();

  // The sums in ascending j, each by one lane of its own wave.  The loads of
  // a group of kEstGroup terms are issued before its adds, which stay in
  // order: one memory latency per group instead of one per term.
  if (tid == 0) {
    double s = 0.0;
    for_groups(n, [&](int j) { return e[j]; }, [&](double v) { s += v; });
    shd[0] = s;
  } else if (tid == 64) {
    double s2 = 0.0;
    for_groups(n, [&](int j) { return e[j]; }, [&](double v) { s2 += v * v; });
    shd[1] = s2;
  } else if (tid == 128) {
    double wm = 0.0;
    for_groups(n, [&](int j) { return (double)I[j]; }, [&](double v) { wm += -(beta / N) * v; });
    wm /= n;
    double wv = 0.0;
    for_groups(n, [&](int j) { return (double)I[j]; }, [&](double v) {
      const double d = -(beta / N) * v - wm;
      wv += d * d;
    });
    wv /= n;
    shd[2] = wm;
    shd[3] = wv;
  }
  __syncthreads();
  const double s = shd[0];
  const double shift = (beta * (double)imax) / N;
  const double dF = -(shift + ee::dd::log_cr(s) - ee::dd::log_cr((double)n));

  if (n >= 2) {
    // leave-one-out sums S_i = sum_{j != i} e_j, ascending j: lane t takes
    // i = t, t + T, ... in passes of A sums; adding +0.0 for j = i leaves a
    // sum of non-negative terms unchanged, so it stands for skipping j.
    const double log_n1 = ee::dd::log_cr((double)(n - 1));
    const int per_lane = (n + kEstThreads - 1) / kEstThreads;
    const auto passes = [&](auto acount) {
      constexpr int A = decltype(acount)::value;
      for (int p0 = 0; p0 < per_lane; p0 += A) {
        double acc[A];
        int idx[A];
#pragma unroll
        for (int a = 0; a < A; ++a) {
          acc[a] = 0.0;
          idx[a] = tid + (p0 + a) * kEstThreads;
        }
        for (int t0 = 0; t0 < n; t0 += kEstTile) {
          const int len = min(kEstTile, n - t0);
          __syncthreads();
          for (int q = tid; q < len; q += kEstThreads) tile[q] = e[t0 + q];
          __syncthreads();
          for (int q = 0; q < len; ++q) {
            const double v = tile[q];
            const int j = t0 + q;
#pragma unroll
            for (int a = 0; a < A; ++a) acc[a] += (j == idx[a]) ? 0.0 : v;
          }
        }
#pragma unroll
        for (int a = 0; a < A; ++a)
          if (idx[a] < n) loo[idx[a]] = -(shift + ee::dd::log_cr(acc[a]) - log_n1);
      }
    };
    if (per_lane <= 1) passes(std::integral_constant<int, 1>{});
    else if (per_lane <= 2) passes(std::integral_constant<int, 2>{});
    else if (per_lane <= 4) passes(std::integral_constant<int, 4>{});
    else passes(std::integral_constant<int, kEstAcc>{});
    __syncthreads();
  }
  if (tid == 0) {
    double err = __builtin_nan("");
    if (n >= 2) {
      double mean = 0.0;
      for_groups(n, [&](int i) { return loo[i]; }, [&](double v) { mean += v; });
      mean /= n;
      double acc = 0.0;
      for_groups(n, [&](int i) { return loo[i]; }, [&](double v) { acc += (v - mean) * (v - mean); });
      err = sqrt((double)(n - 1) / (double)n * acc);
    }
    res->dF = dF;
    res->dS = dF / (double)(J->n - 1);
    res->dF_err = err;
    res->w_mean = shd[2];
    res->w_var = shd[3];
    res->ess = s * s / shd[1];
    res->i_min = imin;
    res->i_max = imax;
    res->n_traj = n;
  }
}

}  // namespace

// Fixed device scratch of the allocation-free batch entry point: the queue
// counter, the job table and the work units of one launch.  Each GPU holds
// its own copy until the process ends.  In host code the array's name is
// only a stand-in: its device address comes from hipGetSymbolAddress.
constexpr size_t kScratchBytes = size_t(2) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

extern "C" {

int ee_k_max_lds_bytes() { return 160 * 1024 - 256; }

size_t ee_k_scratch_bytes() { return kScratchBytes; }

// Device address of the current device's copy of the scratch array, looked
// up once per device (with that device current) and kept.
int ee_k_scratch_ptr(void** out) {
  static std::mutex mu;
  static std::vector<void*> ptrs;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)ptrs.size() <= dev) ptrs.resize(dev + 1, nullptr);
  if (ptrs[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    ptrs[dev] = p;
  }
  *out = ptrs[dev];
  return 0;
}

static hipError_t set_lds_attr(const void* fn) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                             ee_k_max_lds_bytes() + ee::kSweepTailBytes);
}

int ee_k_sweep_kernel_ptr(const void** fn) {
  *fn = reinterpret_cast<const void*>(&sweep_kernel);
  return (int)set_lds_attr(*fn);
}
int ee_k_queue_reset_ptr(const void** fn) {
  *fn = reinterpret_cast<const void*>(&queue_reset_kernel);
  return 0;
}
int ee_k_estimate_ptr(const void** fn) {
  *fn = reinterpret_cast<const void*>(&estimate_kernel);
  return 0;
}

int ee_k_launch_sweep(const ee::JobDev* single_job, int single_k, const ee::Unit* units, int n_units, int* queue,
                      const ee::JobDev* const* jobtab, uint32_t flags, int n_therm, int g0, int grid, int block,
                      int lds_bytes, void* stream) {
  const void* fn = nullptr;
  hipError_t e = (hipError_t)ee_k_sweep_kernel_ptr(&fn);
  if (e != hipSuccess) return (int)e;
  const int tail = ee::sweep_tail_words(lds_bytes);
  const int bytes = lds_bytes + ee::kSweepTailBytes;
  hipLaunchKernelGGL(sweep_kernel, dim3(grid), dim3(block), bytes, (hipStream_t)stream, single_job, single_k, units,
                     n_units, queue, jobtab, flags, n_therm, g0, tail);
  return (int)hipGetLastError();
}

int ee_k_launch_stream_sweep(const ee::JobDev* job, int n_traj, int lanes, int c, uint32_t g, int pos, int dpos,
                             int work, void* stream) {
  const int bx = (lanes + 255) / 256;
  // one-dimensional grid: bx blocks per trajectory, remapped per XCD in the kernel
  hipLaunchKernelGGL(stream_sweep_kernel, dim3(bx * n_traj), dim3(256), 0, (hipStream_t)stream, job, lanes, c, g,
                     pos, dpos, work);
  return (int)hipGetLastError();
}

int ee_k_march_lds_bytes(int plane_words) { return kMarchSlots * plane_words * 4 + 32; }

int ee_k_launch_march(const ee::JobDev* job, int n_traj, int n_replicas, int nseg, int block, int plane_words,
                      uint32_t g, int pos, int dpos, int work, void* stream) {
  const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&march_kernel),
                                              hipFuncAttributeMaxDynamicSharedMemorySize, ee_k_max_lds_bytes());
  if (attr != hipSuccess) return (int)attr;
  hipLaunchKernelGGL(march_kernel, dim3(n_traj * n_replicas * nseg), dim3(block), ee_k_march_lds_bytes(plane_words),
                     (hipStream_t)stream, job, nseg, g, pos, dpos, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  hipLaunchKernelGGL(march_fixup_kernel, dim3(n_traj * nseg * 2), dim3(256), 32, (hipStream_t)stream, job, nseg, g,
                     pos, dpos);
  return (int)hipGetLastError();
}

int ee_k_launch_stream_init(const ee::JobDev* job, int n_traj, int lanes, void* stream) {
  const int bx = (lanes + 255) / 256;
  hipLaunchKernelGGL(stream_init_kernel, dim3(bx, n_traj), dim3(256), 0, (hipStream_t)stream, job, lanes);
  return (int)hipGetLastError();
}

int ee_k_launch_zero_work(const ee::JobDev* job, int n_traj, void* stream) {
  const int bx = (n_traj + 255) / 256;
  hipLaunchKernelGGL(zero_work_kernel, dim3(bx), dim3(256), 0, (hipStream_t)stream, job);
  return (int)hipGetLastError();
}

int ee_k_launch_queue_reset(int* queue, void* stream) {
  hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, queue);
  return (int)hipGetLastError();
}

int ee_k_launch_estimate(const ee::JobDev* const* jobtab, int count, void* stream) {
  hipLaunchKernelGGL(estimate_kernel, dim3(count), dim3(kEstThreads), 0, (hipStream_t)stream, jobtab);
  return (int)hipGetLastError();
}

}  // extern "C"
