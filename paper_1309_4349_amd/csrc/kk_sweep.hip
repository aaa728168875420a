// kk_sweep.hip -- the Kawasaki sweep kernel (the hot loop).
//
// One launch performs complete sweeps (8 class phases each) on LDS-resident
// tiles of the lattice, stored one bit per site.  Each 32-bit LDS word holds
// 32 consecutive sites of a row; a phase touches every 4th bit of every
// other row, and the 8 centres of a word are decided together with bitwise
// (SWAR) logic against the word's 12 bit-sliced random planes.
//
// Two tile modes:
//  * halo tiles (hx = 1 word, hy = 16 rows on each side): one sweep per
//    launch.  A phase's dependency radius is 2 sites, so after 8 phases the
//    interior is exact while the outermost 16 rows / 16 bits of the halo
//    may be stale; the counter-based random numbers make the redundant halo
//    work reproduce exactly what the neighbouring tile computes.
//  * cyclic tile (whole lattice, L % 32 == 0): rows and words wrap inside
//    LDS, so no halo exists and any number of sweeps runs in one launch.
//
// Within a phase all chosen pairs are at L1 distance >= 2 from one another
// (classes 2*((x - y) mod 4) + (y mod 2)), so no pair writes a site that
// another pair reads: the LDS updates are xor-flips of disjoint bits issued
// with ds_xor, and a workgroup barrier separates phases.
#include "kk_common.hpp"
#include "kk_kernels.hpp"

namespace kk {

namespace {

__device__ __forceinline__ uint32_t sel4(uint32_t d1, uint32_t d0, uint32_t v0, uint32_t v1, uint32_t v2,
                                         uint32_t v3) {
  // direction (d1 d0): 0 -> v0 (+x), 1 -> v1 (-x), 2 -> v2 (+y), 3 -> v3 (-y), per bit
  const uint32_t lo = (d0 & v1) | (~d0 & v0);
  const uint32_t hi = (d0 & v3) | (~d0 & v2);
  return (d1 & hi) | (~d1 & lo);
}

__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) {
  return (a & b) | (a & c) | (b & c);
}

// Pack 32 bytes (each 0 or 1) into one word, byte b -> bit b.
__device__ __forceinline__ uint32_t pack4(uint32_t d) {
  return (d | (d >> 7) | (d >> 14) | (d >> 21)) & 0xFu;
}

// Spread 4 bits into 4 bytes (bit b -> byte b, value 0/1).
__device__ __forceinline__ uint32_t spread4(uint32_t n) {
  return (n * 0x00204081u) & 0x01010101u;
}

template <int LAYOUT>
__device__ uint32_t load_word(const SweepParams& p, int yv, int Xw) {
  const int L = p.L;
  const int y = imod(yv, L);
  if (LAYOUT == kLayoutBits) {
    const int xw = imod(Xw, L);  // a multiple of 32: the bit-packed layout needs L % 32 == 0
    return static_cast<const uint32_t*>(p.src)[(size_t)y * p.wpr + (xw >> 5)];
  } else {
    const uint8_t* row = static_cast<const uint8_t*>(p.src) + (size_t)y * L;
    if (Xw >= 0 && Xw + 32 <= L) {
      uint32_t v = 0;
      if ((L & 15) == 0) {
        const uint4* d = reinterpret_cast<const uint4*>(row + Xw);
        const uint4 a = d[0], b = d[1];
        v = pack4(a.x) | (pack4(a.y) << 4) | (pack4(a.z) << 8) | (pack4(a.w) << 12) | (pack4(b.x) << 16) |
            (pack4(b.y) << 20) | (pack4(b.z) << 24) | (pack4(b.w) << 28);
      } else {
        const uint32_t* d = reinterpret_cast<const uint32_t*>(row + Xw);
#pragma unroll
        for (int k = 0; k < 8; ++k) v |= pack4(d[k]) << (4 * k);
      }
      return v;
    }
    uint32_t v = 0;
    for (int b = 0; b < 32; ++b) v |= (uint32_t)(row[imod(Xw + b, L)] & 1u) << b;
    return v;
  }
}

// Store the low `nbits` sites of word v at true coordinates (x0, y).
template <int LAYOUT>
__device__ void store_word(const SweepParams& p, int y, int x0, uint32_t v, int nbits) {
  if (LAYOUT == kLayoutBits) {
    static_cast<uint32_t*>(p.dst)[(size_t)y * p.wpr + (x0 >> 5)] = v;
  } else {
    uint8_t* row = static_cast<uint8_t*>(p.dst) + (size_t)y * p.L;
    if (nbits == 32) {
      if ((p.L & 15) == 0) {
        uint4* d = reinterpret_cast<uint4*>(row + x0);
        d[0] = make_uint4(spread4(v & 0xFu), spread4((v >> 4) & 0xFu), spread4((v >> 8) & 0xFu),
                          spread4((v >> 12) & 0xFu));
        d[1] = make_uint4(spread4((v >> 16) & 0xFu), spread4((v >> 20) & 0xFu), spread4((v >> 24) & 0xFu),
                          spread4(v >> 28));
      } else {
        uint32_t* d = reinterpret_cast<uint32_t*>(row + x0);
#pragma unroll
        for (int k = 0; k < 8; ++k) d[k] = spread4((v >> (4 * k)) & 0xFu);
      }
    } else {
      // a ragged last word: nbits is a multiple of 4 (x0 and L are)
      uint32_t* d = reinterpret_cast<uint32_t*>(row + x0);
      for (int k = 0; k < nbits / 4; ++k) d[k] = spread4((v >> (4 * k)) & 0xFu);
    }
  }
}

// The 12 random planes of the 32 virtual sites starting at virtual x = Xw in
// virtual row yv for sweep t.  Segment-aligned windows take the three Philox
// blocks of their segment directly; windows that straddle the periodic wrap
// of an L % 32 != 0 lattice (or L < 32) gather from the segments they cover.
__device__ void gen_planes(const SweepParams& p, int yv, int Xw, uint64_t t, uint32_t* pl) {
  const int L = p.L;
  const uint32_t y = (uint32_t)imod(yv, L);
  const uint32_t tl = (uint32_t)t, thi = ctr_hi(t, kTagSweep);
  const int x0 = imod(Xw, L);
  if ((x0 & 31) == 0 && x0 + 32 <= L) {
    const uint32_t g4 = (uint32_t)(x0 >> 5) * 4u;
    const Philox4 a = philox10(y, g4 + 0u, tl, thi, p.k0, p.k1);
    const Philox4 b = philox10(y, g4 + 1u, tl, thi, p.k0, p.k1);
    const Philox4 c = philox10(y, g4 + 2u, tl, thi, p.k0, p.k1);
    pl[0] = a.x; pl[1] = a.y; pl[2] = a.z; pl[3] = a.w;
    pl[4] = b.x; pl[5] = b.y; pl[6] = b.z; pl[7] = b.w;
    pl[8] = c.x; pl[9] = c.y; pl[10] = c.z; pl[11] = c.w;
    return;
  }
#pragma unroll
  for (int k = 0; k < kPlanes; ++k) pl[k] = 0u;
  int b = 0;
  while (b < 32) {
    const int x = imod(Xw + b, L);
    const int off = x & 31;
    int len = 32 - off;
    if (L - x < len) len = L - x;
    if (32 - b < len) len = 32 - b;
    const uint32_t g4 = (uint32_t)(x >> 5) * 4u;
    const Philox4 q0 = philox10(y, g4 + 0u, tl, thi, p.k0, p.k1);
    const Philox4 q1 = philox10(y, g4 + 1u, tl, thi, p.k0, p.k1);
    const Philox4 q2 = philox10(y, g4 + 2u, tl, thi, p.k0, p.k1);
    const uint32_t P[12] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
    const uint32_t m = (len == 32) ? 0xFFFFFFFFu : ((1u << len) - 1u);
#pragma unroll
    for (int k = 0; k < kPlanes; ++k) pl[k] |= ((P[k] >> off) & m) << b;
    b += len;
  }
}


// Bit-packed or int8 word at true row y, 32 sites from true x0 (which may
// straddle the periodic wrap only when L % 32 != 0 or L < 32).
template <int LAYOUT>
__device__ __forceinline__ uint32_t load_word_at(const SweepParams& p, int y, int x0) {
  if (LAYOUT == kLayoutBits) return static_cast<const uint32_t*>(p.src)[(size_t)y * p.wpr + (x0 >> 5)];
  const int L = p.L;
  const uint8_t* row = static_cast<const uint8_t*>(p.src) + (size_t)y * L;
  if (x0 + 32 <= L) {
    uint32_t v = 0;
    if ((L & 15) == 0) {
      const uint4* d = reinterpret_cast<const uint4*>(row + x0);
      const uint4 a = d[0], b = d[1];
      v = pack4(a.x) | (pack4(a.y) << 4) | (pack4(a.z) << 8) | (pack4(a.w) << 12) | (pack4(b.x) << 16) |
          (pack4(b.y) << 20) | (pack4(b.z) << 24) | (pack4(b.w) << 28);
    } else {
      const uint32_t* d = reinterpret_cast<const uint32_t*>(row + x0);
#pragma unroll
      for (int k = 0; k < 8; ++k) v |= pack4(d[k]) << (4 * k);
    }
    return v;
  }
  // the word passes the end of the row: eight 4-byte pieces, each inside the
  // row (x0 and L are multiples of 4), the start of each wrapped; the loads
  // are independent, so they are all in flight at once
  uint32_t v = 0;
  int x = x0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v |= pack4(*reinterpret_cast<const uint32_t*>(row + x)) << (4 * k);
    x += 4;
    if (x >= L) x -= L;
  }
  return v;
}

// Layout chosen at run time (LAYOUT == 0) or at compile time.
template <int LAYOUT>
__device__ __forceinline__ uint32_t load_word_any(const SweepParams& p, int y, int x0) {
  if constexpr (LAYOUT == 0)
    return p.layout == kLayoutBits ? load_word_at<kLayoutBits>(p, y, x0) : load_word_at<kLayoutInt8>(p, y, x0);
  else
    return load_word_at<LAYOUT>(p, y, x0);
}

template <int LAYOUT>
__device__ __forceinline__ void store_word_any(const SweepParams& p, int y, int x0, uint32_t v, int nbits) {
  if constexpr (LAYOUT == 0) {
    if (p.layout == kLayoutBits) store_word<kLayoutBits>(p, y, x0, v, nbits);
    else store_word<kLayoutInt8>(p, y, x0, v, nbits);
  } else {
    store_word<LAYOUT>(p, y, x0, v, nbits);
  }
}

// Random planes of the 32 sites starting at true column x0 of true row y.
__device__ __forceinline__ void gen_planes_at(const SweepParams& p, int y, int x0, int Xw, uint64_t t, uint32_t* pl) {
  if ((x0 & 31) == 0 && x0 + 32 <= p.L) {
    const uint32_t tl = (uint32_t)t, thi = ctr_hi(t, kTagSweep);
    const uint32_t g4 = (uint32_t)(x0 >> 5) * 4u;
    const Philox4 a = philox10((uint32_t)y, g4 + 0u, tl, thi, p.k0, p.k1);
    const Philox4 b = philox10((uint32_t)y, g4 + 1u, tl, thi, p.k0, p.k1);
    const Philox4 c = philox10((uint32_t)y, g4 + 2u, tl, thi, p.k0, p.k1);
    pl[0] = a.x; pl[1] = a.y; pl[2] = a.z; pl[3] = a.w;
    pl[4] = b.x; pl[5] = b.y; pl[6] = b.z; pl[7] = b.w;
    pl[8] = c.x; pl[9] = c.y; pl[10] = c.z; pl[11] = c.w;
    return;
  }
  gen_planes(p, y, Xw, t, pl);
}

// Three-input bitwise function with a truth table built from the operand
// patterns a = 0xF0, b = 0xCC, c = 0xAA (one v_bitop3_b32).
#define KK_TA 0xF0u
#define KK_TB 0xCCu
#define KK_TC 0xAAu
#define KK_TT(expr) ((unsigned)((expr) & 0xFFu))
template <unsigned TT>
__device__ __forceinline__ uint32_t bop3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, TT);
}
// a ? b : c, per bit
__device__ __forceinline__ uint32_t bsel(uint32_t a, uint32_t b, uint32_t c) {
  return bop3<KK_TT((KK_TA & KK_TB) | (~KK_TA & KK_TC))>(a, b, c);
}
constexpr unsigned kXor3 = KK_TT(KK_TA ^ KK_TB ^ KK_TC);
constexpr unsigned kMaj3 = KK_TT((KK_TA & KK_TB) | (KK_TA & KK_TC) | (KK_TB & KK_TC));

// 10-bit (u < K) and (u == K) over bit-sliced u, planes[2] = MSB .. planes[11] = LSB,
// for a K that is the same on every lane.  Less-than is the borrow chain of
// u - K from the least significant bit, lt' = maj(~u_k, K_k, lt), one
// three-input op per bit; equality is the AND of u_k XNOR K_k, one XNOR per bit
// and a tree of three-input ANDs.
__device__ __forceinline__ void cmp10(const uint32_t* pl, uint32_t K, uint32_t& lt, uint32_t& eq,
                                      uint32_t bin = 0u, uint32_t em = 0xFFFFFFFFu) {
  constexpr unsigned kBorrow = KK_TT((~KK_TA & KK_TB) | (~KK_TA & KK_TC) | (KK_TB & KK_TC));
  constexpr unsigned kAnd3 = KK_TT(KK_TA & KK_TB & KK_TC);
  uint32_t l = bin, x[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    const uint32_t u = pl[11 - k];
    const uint32_t kb = 0u - ((K >> k) & 1u);
    l = bop3<kBorrow>(u, kb, l);
    x[k] = ~(u ^ kb);
  }
  lt = l;
  eq = bop3<kAnd3>(bop3<kAnd3>(bop3<kAnd3>(x[0], x[1], x[2]), bop3<kAnd3>(x[3], x[4], x[5]),
                                bop3<kAnd3>(x[6], x[7], x[8])),
                   x[9], em);
}

template <bool CYC>
__device__ __forceinline__ unsigned sweep_item(uint32_t* S, const SweepParams& p, int stride, int r, int w,
                                               const uint32_t* pl, uint32_t cmask, uint32_t intmask, int yv,
                                               int Xw, uint64_t t) {
  int rn, rs, rnn, rss, wl, wr;
  if (CYC) {
    const int R = p.R, C = p.C;
    rn = (r == 0) ? R - 1 : r - 1;
    rs = (r + 1 == R) ? 0 : r + 1;
    rnn = (rn == 0) ? R - 1 : rn - 1;
    rss = (rs + 1 == R) ? 0 : rs + 1;
    wl = (w == 0) ? C - 1 : w - 1;
    wr = (w + 1 == C) ? 0 : w + 1;
  } else {
    rn = r - 1;
    rs = r + 1;
    rnn = r - 2;
    rss = r + 2;
    wl = w - 1;  // the pad words at -1 and C are never part of a result
    wr = w + 1;
  }
#define KK_AT(rr, ww) S[(rr) * stride + (ww) + 1]
  const uint32_t c0 = KK_AT(r, w), cL = KK_AT(r, wl), cR = KK_AT(r, wr);
  const uint32_t n0 = KK_AT(rn, w), nL = KK_AT(rn, wl), nR = KK_AT(rn, wr);
  const uint32_t s0 = KK_AT(rs, w), sL = KK_AT(rs, wl), sR = KK_AT(rs, wr);
  const uint32_t nn = KK_AT(rnn, w), ss = KK_AT(rss, w);

  // value of the site at x+1 / x-1 / x+2 / x-2, aligned to bit x
  const uint32_t cE = __builtin_amdgcn_alignbit(cR, c0, 1);
  const uint32_t cW = __builtin_amdgcn_alignbit(c0, cL, 31);
  const uint32_t cE2 = __builtin_amdgcn_alignbit(cR, c0, 2);
  const uint32_t cW2 = __builtin_amdgcn_alignbit(c0, cL, 30);
  const uint32_t nE = __builtin_amdgcn_alignbit(nR, n0, 1);
  const uint32_t nW = __builtin_amdgcn_alignbit(n0, nL, 31);
  const uint32_t sE = __builtin_amdgcn_alignbit(sR, s0, 1);
  const uint32_t sW = __builtin_amdgcn_alignbit(s0, sL, 31);

  const uint32_t d0 = pl[0], d1 = pl[1];
  // partner b: +x east, -x west, +y the row below (y+1), -y the row above
  const uint32_t B = sel4(d1, d0, cE, cW, s0, n0);
  const uint32_t A = (c0 ^ B) & cmask;  // centres of this class whose partner is unlike

  // m = n + 1 = (unlike neighbours of c, partner included) + (neighbours of b
  // other than c that equal c, i.e. are unlike b)
  const uint32_t o1 = sel4(d1, d0, cE2, cW2, ss, nn);
  const uint32_t o2 = sel4(d1, d0, nE, nW, sW, nW);
  const uint32_t o3 = sel4(d1, d0, sE, sW, sE, nE);
  const uint32_t uE = c0 ^ cE, uW = c0 ^ cW, uN = c0 ^ n0, uS = c0 ^ s0;
  const uint32_t e1 = ~(c0 ^ o1), e2 = ~(c0 ^ o2), e3 = ~(c0 ^ o3);
  const uint32_t s1 = uE ^ uW ^ uN, c1 = maj3(uE, uW, uN);
  const uint32_t s2 = uS ^ e1 ^ e2, c2 = maj3(uS, e1, e2);
  const uint32_t m0 = s1 ^ s2 ^ e3, c3 = maj3(s1, s2, e3);
  const uint32_t m1 = c1 ^ c2 ^ c3, m2 = maj3(c1, c2, c3);

  uint32_t F = A;  // accepted exchanges
  if (p.acc.restricted) {
    uint32_t lt0, eq0, lt1, eq1, lt2, eq2;
    if (p.acc.hi[0] < 1024u) cmp10(pl, p.acc.hi[0], lt0, eq0); else { lt0 = 0xFFFFFFFFu; eq0 = 0u; }
    if (p.acc.hi[1] < 1024u) cmp10(pl, p.acc.hi[1], lt1, eq1); else { lt1 = 0xFFFFFFFFu; eq1 = 0u; }
    if (p.acc.hi[2] < 1024u) cmp10(pl, p.acc.hi[2], lt2, eq2); else { lt2 = 0xFFFFFFFFu; eq2 = 0u; }
    const uint32_t rm = ~(m2 ^ p.acc.negmask) & (m0 | m1);  // m in the rejectable range
    const uint32_t ltsel = (m1 & ((m0 & lt2) | (~m0 & lt1))) | (~m1 & lt0);
    const uint32_t eqsel = (m1 & ((m0 & eq2) | (~m0 & eq1))) | (~m1 & eq0);
    F = A & (~rm | ltsel);
    uint32_t tie = A & rm & eqsel;
    while (tie) {  // u10 equals the threshold prefix: draw the low 32 bits
      const int bp = __builtin_ctz(tie);
      tie &= tie - 1u;
      const uint32_t x = (uint32_t)imod(Xw + bp, p.L), y = (uint32_t)imod(yv, p.L);
      const Philox4 e = philox10(y, x >> 2, (uint32_t)t, ctr_hi(t, kTagExt), p.k0, p.k1);
      const uint32_t xs = x & 3u;
      const uint32_t ext = xs == 0 ? e.x : xs == 1 ? e.y : xs == 2 ? e.z : e.w;
      const uint32_t j = ((((m1 >> bp) & 1u) << 1) | ((m0 >> bp) & 1u)) - 1u;
      const uint32_t lo = j == 0 ? p.acc.lo[0] : j == 1 ? p.acc.lo[1] : p.acc.lo[2];
      if (ext < lo) F |= 1u << bp;
    }
  }

  const uint32_t Fpx = F & ~d1 & ~d0, Fmx = F & ~d1 & d0;
  const uint32_t Fpy = F & d1 & ~d0, Fmy = F & d1 & d0;
  const uint32_t flip = F ^ (Fpx << 1) ^ (Fmx >> 1);
  if (flip) atomicXor(&KK_AT(r, w), flip);
  if (Fpx >> 31) atomicXor(&KK_AT(r, wr), 1u);
  if (Fmx & 1u) atomicXor(&KK_AT(r, wl), 0x80000000u);
  if (Fpy) atomicXor(&KK_AT(rs, w), Fpy);
  if (Fmy) atomicXor(&KK_AT(rn, w), Fmy);
#undef KK_AT
  return (unsigned)__builtin_popcount(F & intmask);
}

template <int LAYOUT, bool CYC, int KU>
__global__ __launch_bounds__(KU == 1 ? 1024 : 768) void sweep_kernel(SweepParams p) {
  extern __shared__ uint32_t S[];
  const int stride = p.C + 2;
  const int tile = blockIdx.x;
  const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
  const int X0 = tx * p.tww * 32, Y0 = ty * p.th;
  const int XL = X0 - 32 * p.hx;  // virtual x of LDS word 0
  const int YT = Y0 - p.hy;       // virtual y of LDS row 0
  const int xend = min(X0 + p.tww * 32, p.L);  // interior is [X0, xend) x [Y0, yend)
  const int yend = min(Y0 + p.th, p.L);

  // stage the tile (with halo) into LDS, one bit per site
  for (int i = threadIdx.x; i < p.R * stride; i += blockDim.x) {
    const int r = i / stride, w = i - r * stride - 1;
    S[i] = (w >= 0 && w < p.C) ? load_word<LAYOUT>(p, YT + r, XL + 32 * w) : 0u;
  }

  // units owned by this thread: (row pair q, word w); rows r0 = row0 + 2q and r0 + 1
  int ur0[KU], uw[KU];
  bool uok[KU];
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    const int u = threadIdx.x + k * blockDim.x;
    uok[k] = u < p.nunits;
    const int q = uok[k] ? u / p.C : 0;
    uw[k] = uok[k] ? u - q * p.C : 0;
    ur0[k] = p.row0 + 2 * q;
  }
  // interior bit masks of each owned word (for counting accepted moves)
  uint32_t imask[KU][2];
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    const int Xw = XL + 32 * uw[k];
    uint32_t wm = 0u;
    if (Xw + 32 <= X0 || Xw >= xend) wm = 0u;
    else {
      const int lo = max(Xw, X0), hi = min(Xw + 32, xend);
      const int n = hi - lo, sh = lo - Xw;
      wm = (n == 32 ? 0xFFFFFFFFu : ((1u << n) - 1u)) << sh;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int yv = YT + ur0[k] + h;
      imask[k][h] = (uok[k] && yv >= Y0 && yv < yend) ? wm : 0u;
    }
  }

  unsigned count = 0;
  for (int s = 0; s < p.nsweeps; ++s) {
    const uint64_t t = p.t0 + (uint64_t)s;
    uint32_t pl[KU][2][kPlanes];
#pragma unroll
    for (int k = 0; k < KU; ++k) {
      if (!uok[k]) continue;
#pragma unroll
      for (int h = 0; h < 2; ++h) gen_planes(p, YT + ur0[k] + h, XL + 32 * uw[k], t, pl[k][h]);
    }
    const uint32_t perm = class_order(p.k0, p.k1, t);
    __syncthreads();  // staging (or the previous sweep) complete
    for (int ph = 0; ph < 8; ++ph) {
      const uint32_t cls = (perm >> (4 * ph)) & 0xFu;
      const int a = (int)(cls >> 1);
      // Every unit starts on an even virtual row (tiles start on even rows and
      // the halo is even), so the active row of the pair is row r0 + (class
      // parity): uniform over the workgroup, which keeps the plane arrays in
      // registers.
      if ((cls & 1u) == 0u) {
#pragma unroll
        for (int k = 0; k < KU; ++k) {
          if (!uok[k]) continue;
          const int yv = YT + ur0[k];
          count += sweep_item<CYC>(S, p, stride, ur0[k], uw[k], pl[k][0], 0x11111111u << ((a + yv) & 3),
                                   imask[k][0], yv, XL + 32 * uw[k], t);
        }
      } else {
#pragma unroll
        for (int k = 0; k < KU; ++k) {
          if (!uok[k]) continue;
          const int yv = YT + ur0[k] + 1;
          count += sweep_item<CYC>(S, p, stride, ur0[k] + 1, uw[k], pl[k][1], 0x11111111u << ((a + yv) & 3),
                                   imask[k][1], yv, XL + 32 * uw[k], t);
        }
      }
      __syncthreads();
    }
  }

  // write the interior back
  const int iw = (xend - X0 + 31) / 32, ih = yend - Y0;
  for (int i = threadIdx.x; i < iw * ih; i += blockDim.x) {
    const int rr = i / iw, ww = i - rr * iw;
    const int x0 = X0 + 32 * ww;
    const int nb = min(32, xend - x0);
    const uint32_t v = S[(p.hy + rr) * stride + p.hx + ww + 1];
    store_word<LAYOUT>(p, Y0 + rr, x0, nb == 32 ? v : (v & ((1u << nb) - 1u)), nb);
  }

  // Accepted-move count: reduce over the workgroup, then one plain
  // read-modify-write of this tile's own partial sum.  (One device-scope
  // atomic per wave on a single address serialises across the XCDs and
  // cost more than the sweep itself.)
  unsigned c = count;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
  unsigned* red = reinterpret_cast<unsigned*>(S + p.R * stride);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) tot += red[wv];
    p.accepted[tile] += tot;
  }
}


// Per-row random state for one sweep: the two direction planes and, for each
// of the three rejectable classes of moves (slot j), the plane of sites whose
// 42-bit uniform U = u10 * 2^32 + ext32 lies below the slot's threshold T_j.
// The 10-bit prefix decides every site whose u10 differs from T_j's top bits;
// for the others (about 3 sites in 1024 per slot) the low word ext32 is drawn
// here, once per sweep, so the phases decide with bitwise logic alone and
// never branch on a tie.
struct RowRand {
  uint32_t d0, d1, acc0, acc1, acc2;
};

// The threshold prefixes pass through an empty asm so that their per-bit masks
// are rebuilt (a few scalar ops) at every use instead of being hoisted and
// kept live across the kernel, which overflows the scalar registers.
__device__ __forceinline__ uint32_t opaque_sgpr(uint32_t v) {
  asm volatile("" : "+s"(v));
  return v;
}

// Ties: u10 equals a threshold prefix, and the low 32 bits of U decide.  eq[j]
// holds the tied sites of slot j among the 32 sites from true column xtrue of
// true row ytrue (xtrue + b may pass the wrap only for L % 32 != 0 or L < 32);
// the tied sites that lie below the threshold join lt[j].
__device__ __forceinline__ void resolve_ties(const SweepParams& p, int ytrue, int xtrue, uint64_t t,
                                             const uint32_t* eq, uint32_t* lt) {
  uint32_t tie = eq[0] | eq[1] | eq[2];
  while (tie) {
    const int bp = __builtin_ctz(tie);
    tie &= tie - 1u;
    int x = xtrue + bp;
    if (x >= p.L) x = imod(x, p.L);
    const Philox4 e = philox10((uint32_t)ytrue, (uint32_t)x >> 2, (uint32_t)t, ctr_hi(t, kTagExt), p.k0, p.k1);
    const uint32_t xs = (uint32_t)x & 3u;
    const uint32_t ext = xs == 0 ? e.x : xs == 1 ? e.y : xs == 2 ? e.z : e.w;
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (((eq[j] >> bp) & 1u) && ext < p.acc.lo[j]) lt[j] |= 1u << bp;
  }
}

// pl: the 12 random planes of 32 sites of true row ytrue from true column
// xtrue (xtrue + b may pass the wrap only for L % 32 != 0 or L < 32).
__device__ __forceinline__ void row_rand(const uint32_t* pl, const SweepParams& p, int ytrue, int xtrue, uint64_t t,
                                         RowRand& q) {
  q.d0 = pl[0];
  q.d1 = pl[1];
  uint32_t lt[3], eq[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (p.acc.hi[j] < 1024u) cmp10(pl, opaque_sgpr(p.acc.hi[j]), lt[j], eq[j]);
    else {
      lt[j] = 0xFFFFFFFFu;
      eq[j] = 0u;
    }
  }
  resolve_ties(p, ytrue, xtrue, t, eq, lt);
  q.acc0 = lt[0];
  q.acc1 = lt[1];
  q.acc2 = lt[2];
}

// N Philox4x32-10 blocks at once, round by round across the blocks: the
// multiplies of different blocks are independent and issue back to back
// instead of waiting on one block's chain.  c0..c3: counters in, outputs out.
template <int N>
__device__ __forceinline__ void philox10_n(uint32_t* c0, uint32_t* c1, uint32_t* c2, uint32_t* c3, uint32_t k0,
                                           uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
#pragma unroll
    for (int n = 0; n < N; ++n) {
      const uint64_t p0 = (uint64_t)c0[n] * 0xD2511F53u;
      const uint64_t p1 = (uint64_t)c2[n] * 0xCD9E8D57u;
      const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1[n], k0, 0x96);
      const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3[n], k1, 0x96);
      c1[n] = (uint32_t)p1;
      c3[n] = (uint32_t)p0;
      c0[n] = n0;
      c2[n] = n2;
    }
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Ties of NR rows on the segment grid (no site index wraps): each pass takes
// the next tied site of every row and draws the NR extension words together,
// so the passes follow the largest per-row tie count in the wave (one or two)
// rather than the sum over rows, and the NR Philox chains overlap.
template <int NR>
__device__ __forceinline__ void resolve_ties_grid(const SweepParams& p, const int* y, const int* x, uint64_t t,
                                                  const uint32_t (*eq)[3], uint32_t (*lt)[3]) {
  uint32_t tie[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) tie[i] = eq[i][0] | eq[i][1] | eq[i][2];
  const uint32_t tl = (uint32_t)t, th = ctr_hi(t, kTagExt);
  for (;;) {
    uint32_t left = 0u;
#pragma unroll
    for (int i = 0; i < NR; ++i) left |= tie[i];
    if (!left) break;
    uint32_t c0[NR], c1[NR], c2[NR], c3[NR], bit[NR], xs[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const uint32_t m = tie[i];
      bit[i] = m & (0u - m);  // the next tied site (none: 0, and the draw below is unused)
      tie[i] = m & (m - 1u);
      const uint32_t xsite = (uint32_t)x[i] + (uint32_t)(31 - __clz((int)bit[i]));
      xs[i] = xsite & 3u;
      c0[i] = (uint32_t)y[i];
      c1[i] = xsite >> 2;
      c2[i] = tl;
      c3[i] = th;
    }
    philox10_n<NR>(c0, c1, c2, c3, p.k0, p.k1);
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      // word xs of the block, by bitwise selects (a branch here would split
      // the NR chains again)
      const uint32_t s1 = 0u - (xs[i] & 1u), s2 = 0u - (xs[i] >> 1);
      const uint32_t ext = bsel(s2, bsel(s1, c3[i], c2[i]), bsel(s1, c1[i], c0[i]));
#pragma unroll
      for (int j = 0; j < 3; ++j)
        if (ext < p.acc.lo[j]) lt[i][j] |= eq[i][j] & bit[i];
    }
  }
}

// Random state of NR rows whose words sit on the 32-site segment grid
// (x % 32 == 0 and x + 32 <= L): the 3 NR Philox blocks are drawn together,
// then the 3 NR compares, then the rare ties.  A slot whose threshold prefix is 1024 or more accepts
// every site: its compare runs with a borrow-in (u < 1023 + 1) and an empty
// equality mask instead of a branch.
template <int NR>
__device__ __forceinline__ void rand_rows_grid(const SweepParams& p, uint64_t t, const int* y, const int* x,
                                               RowRand* q) {
  const uint32_t tl = (uint32_t)t, thi = ctr_hi(t, kTagSweep);
  uint32_t c0[NR * 3], c1[NR * 3], c2[NR * 3], c3[NR * 3];
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const uint32_t g4 = (uint32_t)(x[i] >> 5) * 4u;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      c0[3 * i + b] = (uint32_t)y[i];
      c1[3 * i + b] = g4 + (uint32_t)b;
      c2[3 * i + b] = tl;
      c3[3 * i + b] = thi;
    }
  }
  philox10_n<NR * 3>(c0, c1, c2, c3, p.k0, p.k1);
  uint32_t pl[NR][kPlanes];
#pragma unroll
  for (int i = 0; i < NR; ++i) {
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      pl[i][4 * b] = c0[3 * i + b];
      pl[i][4 * b + 1] = c1[3 * i + b];
      pl[i][4 * b + 2] = c2[3 * i + b];
      pl[i][4 * b + 3] = c3[3 * i + b];
    }
  }
  // The compares run bit by bit across the rows: each bit of a threshold
  // prefix becomes one all-zeros / all-ones scalar mask (a signed one-bit
  // field extract), shared by the rows' borrow chains (u < K) and equality
  // chains (u == K), one three-input op per bit and chain.
  constexpr unsigned kBorrow = KK_TT((~KK_TA & KK_TB) | (~KK_TA & KK_TC) | (KK_TB & KK_TC));
  constexpr unsigned kEqStep = KK_TT(KK_TA & ~(KK_TB ^ KK_TC));
  uint32_t lt[NR][3], eq[NR][3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const uint32_t hi = p.acc.hi[j];
    const bool all = hi >= 1024u;
    const uint32_t K = opaque_sgpr(all ? 1023u : hi);
    const uint32_t bin = all ? 0xFFFFFFFFu : 0u, em = all ? 0u : 0xFFFFFFFFu;
    uint32_t l[NR], e[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      l[i] = bin;
      e[i] = em;
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      const uint32_t kb = (uint32_t)((int32_t)(K << (31 - k)) >> 31);
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const uint32_t u = pl[i][11 - k];  // planes 2 .. 11: bits 9 .. 0 of u10
        l[i] = bop3<kBorrow>(u, kb, l[i]);
        e[i] = bop3<kEqStep>(e[i], u, kb);
      }
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      lt[i][j] = l[i];
      eq[i][j] = e[i];
    }
  }
  // one test for all rows, so that no Philox block sinks past a tie loop
  uint32_t anytie = 0u;
#pragma unroll
  for (int i = 0; i < NR; ++i) anytie |= eq[i][0] | eq[i][1] | eq[i][2];
  if (anytie) resolve_ties_grid<NR>(p, y, x, t, eq, lt);
#pragma unroll
  for (int i = 0; i < NR; ++i) q[i] = RowRand{pl[i][0], pl[i][1], lt[i][0], lt[i][1], lt[i][2]};
}


// Decide the exchanges of the centres in `cmask` of one 32-site word.
// v: the word (0), its west/east neighbours (1, 2), the same three in the
// row above (3..5) and below (6..8), and the words two rows above / below
// (9, 10).  Returns the accepted centres.
__device__ __forceinline__ uint32_t decide_word(const uint32_t* v, const RowRand& q, const SweepParams& p,
                                                uint32_t cmask) {
  const uint32_t c0 = v[0], n0 = v[3], s0 = v[6];
  const uint32_t cE = __builtin_amdgcn_alignbit(v[2], c0, 1);
  const uint32_t cW = __builtin_amdgcn_alignbit(c0, v[1], 31);
  const uint32_t cE2 = __builtin_amdgcn_alignbit(v[2], c0, 2);
  const uint32_t cW2 = __builtin_amdgcn_alignbit(c0, v[1], 30);
  const uint32_t nE = __builtin_amdgcn_alignbit(v[5], n0, 1);
  const uint32_t nW = __builtin_amdgcn_alignbit(n0, v[4], 31);
  const uint32_t sE = __builtin_amdgcn_alignbit(v[8], s0, 1);
  const uint32_t sW = __builtin_amdgcn_alignbit(s0, v[7], 31);
  const uint32_t d0 = q.d0, d1 = q.d1;
  // direction (d1 d0): 0 +x east, 1 -x west, 2 +y the row below, 3 -y the row above.
  // B: the partner; o1..o3: the partner's neighbours other than the centre.
  const uint32_t B = bsel(d1, bsel(d0, n0, s0), bsel(d0, cW, cE));
  const uint32_t o1 = bsel(d1, bsel(d0, v[9], v[10]), bsel(d0, cW2, cE2));
  const uint32_t o2 = bsel(bop3<KK_TT(KK_TA & ~KK_TB)>(d1, d0, d0), sW, bsel(d0, nW, nE));
  const uint32_t o3 = bsel(d0, bsel(d1, nE, sW), sE);
  const uint32_t A = bop3<KK_TT(KK_TA & (KK_TB ^ KK_TC))>(cmask, c0, B);  // active: unlike partner
  // m = n + 1 = #(neighbours of c unlike c, partner included) + #(o_i equal to c),
  // summed by a bit-sliced 7 -> 3 counter written relative to c so the xors with c cancel
  const uint32_t X1 = bop3<kXor3>(cE, cW, n0);
  const uint32_t M1 = bop3<kMaj3>(cE, cW, n0);
  const uint32_t X2 = bop3<kXor3>(s0, o1, o2);
  const uint32_t M2 = bop3<KK_TT((KK_TA & ~KK_TB) | (KK_TA & ~KK_TC) | (~KK_TB & ~KK_TC))>(s0, o1, o2);
  const uint32_t M3 = bop3<KK_TT((KK_TA & KK_TB) | (KK_TA & ~KK_TC) | (KK_TB & ~KK_TC))>(X1, X2, o3);
  const uint32_t m0 = ~(bop3<kXor3>(X1, X2, o3) ^ c0);
  const uint32_t m1 = bop3<kXor3>(M1, M2, M3) ^ c0;
  const uint32_t m2 = bop3<kMaj3>(M1, M2, M3) ^ c0;
  // rejectable: m in {1,2,3} for omega > 0 (dU = 6,4,2), {5,6,7} for omega < 0;
  // slot j = (m & 3) - 1 holds the acceptance plane of that move class.  No
  // branch on omega == 0: there every slot's plane is all ones.  (A branch
  // here split the neighbourhood reads into two LDS round trips per unit.)
  const uint32_t rm = bop3<KK_TT(~KK_TA & (KK_TB | KK_TC))>(m2 ^ p.acc.negmask, m0, m1);
  const uint32_t accsel = bsel(m1, bsel(m0, q.acc2, q.acc1), q.acc0);
  return bop3<KK_TT(KK_TA & (~KK_TB | KK_TC))>(A, rm, accsel);
}

template <int TWW>
struct HaloGeom {
  static constexpr int C = TWW + 2;  // LDS words per row: the tile plus one halo word each side
  // Row stride: at least C + 2 (one pad word each side), and congruent to
  // C/2 modulo 32 so that the words a phase touches (every other row,
  // consecutive words) fall in consecutive LDS banks.
  static constexpr int ST = (C % 2 == 0) ? (C / 2 + 32) : 34;
};

// One phase of the halo kernel for the thread's units, active row = r0 + H.
// Branch-free over the units: a unit beyond the tile reads a valid word and
// has an empty centre mask, so it decides nothing and writes nothing.
template <int ST, int KU, int H>
__device__ __forceinline__ unsigned halo_phase(uint32_t* S, const SweepParams& p, const int* base0, const int* yrow,
                                               const int* xw, const uint32_t* okm, const RowRand (*rr)[2],
                                               const uint32_t (*imask)[2], int a, uint64_t t) {
  uint32_t v[KU][11];
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    const int b = base0[k] + H * ST;
    v[k][0] = S[b];
    v[k][1] = S[b - 1];
    v[k][2] = S[b + 1];
    v[k][3] = S[b - ST];
    v[k][4] = S[b - ST - 1];
    v[k][5] = S[b - ST + 1];
    v[k][6] = S[b + ST];
    v[k][7] = S[b + ST - 1];
    v[k][8] = S[b + ST + 1];
    v[k][9] = S[b - 2 * ST];
    v[k][10] = S[b + 2 * ST];
  }
  uint32_t F[KU];
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    // class mask: the unit's base pattern rotated left by a (its period is 4)
    const uint32_t cmask = __builtin_amdgcn_alignbit(okm[k * 2 + H], okm[k * 2 + H], (32 - a) & 31);
    F[k] = decide_word(v[k], rr[k][H], p, cmask);
  }
  unsigned count = 0;
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    const uint32_t d0 = rr[k][H].d0, d1 = rr[k][H].d1;
    const uint32_t f = F[k];
    const uint32_t Fpx = bop3<KK_TT(KK_TA & ~KK_TB & ~KK_TC)>(f, d1, d0);
    const uint32_t Fmx = bop3<KK_TT(KK_TA & ~KK_TB & KK_TC)>(f, d1, d0);
    const uint32_t Fpy = bop3<KK_TT(KK_TA & KK_TB & ~KK_TC)>(f, d1, d0);
    const uint32_t Fmy = bop3<KK_TT(KK_TA & KK_TB & KK_TC)>(f, d1, d0);
    const int b = base0[k] + H * ST;
    // centres of one class sit 4 sites apart, so f, Fpx << 1 and Fmx >> 1
    // never share a bit and their xor is their or.  Zero masks are harmless:
    // every update goes out unconditionally (the two carries into the
    // neighbouring words are mostly zero, but a masked store costs more issue
    // slots than an xor with zero, and skipping a wave's carries when none is
    // set measured slower: 16.45 against 16.1 us per 4096^2 sweep)
    atomicXor(&S[b], (Fpx << 1) | f | (Fmx >> 1));
    atomicXor(&S[b + ST], Fpy);
    atomicXor(&S[b - ST], Fmy);
    atomicXor(&S[b + 1], Fpx >> 31);
    atomicXor(&S[b - 1], Fmx << 31);
    count += (unsigned)__builtin_popcount(f & imask[k][H]);
  }
  return count;
}

// Sum over a wavefront of a per-lane count below 256, from eight ballots
// (scalar popcounts; no LDS round trip).
__device__ __forceinline__ unsigned wave_sum8(unsigned c) {
  unsigned s = 0;
#pragma unroll
  for (int b = 0; b < 8; ++b) s += (unsigned)__popcll(__ballot((c >> b) & 1u)) << b;
  return s;
}

// Halo-tile sweep with a compile-time tile width: the LDS row stride is a
// constant, so every neighbour of a unit is an immediate offset from one
// base address.  Each thread owns KU (row pair, word) units; their random
// state lives in registers for the whole sweep.  In a phase the thread reads
// the neighbourhoods of all its units before issuing any exchange (the
// conflict-free schedule makes that reordering exact), so the LDS latency of
// the second unit hides behind the first.
// One sweep of tile `tile` of the lattice described by p (halo mode).
// Returns the workgroup's accepted count for the tile interior (the same in
// every thread).

template <int LAYOUT, int TWW, int KU>
__device__ __forceinline__ unsigned halo_tile_sweep(uint32_t* S, const SweepParams& p, int tile) {
  constexpr int C = HaloGeom<TWW>::C;
  constexpr int ST = HaloGeom<TWW>::ST;
  const int CP = C + 2;       // staged words per row (the pads included)
  constexpr int NSTG = 6;     // staged global words per thread
  const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
  constexpr int TW = TWW;
  const int X0 = tx * TW * 32, Y0 = ty * p.th;
  const int XL = X0 - 32, YT = Y0 - 16;
  const int xend = min(X0 + TW * 32, p.L), yend = min(Y0 + p.th, p.L);
  const int total = p.R * CP;
  const uint64_t t = p.t0;
  // LDS words that can reach the interior: the left halo word, the interior
  // words and one halo word past them.  In a ragged last tile the words after
  // that behave like the zero pad of a full tile: they are neither loaded nor
  // computed (for L % 32 != 0 they would also sit off the 32-site segment grid).
  const int wneed = min(C, (xend - X0 + 31) / 32 + 2);
  // true (wrapped) row of every LDS row and true column of every LDS word
  int* ytab = reinterpret_cast<int*>(S + p.R * ST + 16);
  int* xtab = ytab + p.R;
  for (int i = threadIdx.x; i < p.R + C; i += blockDim.x) {
    if (i < p.R) ytab[i] = imod(YT + i, p.L);
    else xtab[i - p.R] = imod(XL + 32 * (i - p.R), p.L);
  }
  // the workgroup's accepted count, in the gap between the rows and the tables
  uint32_t* acc_total = S + p.R * ST;
  if (threadIdx.x == 0) *acc_total = 0u;
  __syncthreads();

  // global loads first; they complete while the random state is computed
  uint32_t stg[NSTG];
#pragma unroll
  for (int j = 0; j < NSTG; ++j) {
    const int i = threadIdx.x + j * blockDim.x;
    const int r = i / CP, w = i - r * CP - 1;
    stg[j] = (i < total && w >= 0 && w < wneed) ? load_word_at<LAYOUT>(p, ytab[r], xtab[w]) : 0u;
  }
  for (int i = threadIdx.x + NSTG * blockDim.x; i < total; i += blockDim.x) {
    const int r = i / CP, w = i - r * CP - 1;
    S[r * ST + w + 1] = (w >= 0 && w < wneed) ? load_word_at<LAYOUT>(p, ytab[r], xtab[w]) : 0u;
  }

  int base0[KU], yrow[KU * 2], xw[KU];  // LDS base; true row of each of the pair's rows; true x of bit 0
  uint32_t okm[KU * 2];                 // class-0 centre pattern of each row (0 for a unit beyond the tile)
  uint32_t imask[KU][2];
  RowRand rr[KU][2];
  int ry[KU * 2], rx[KU * 2];  // true row and column of each of the thread's rows
  bool okk[KU];
  const bool grid = (p.L & 31) == 0;
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    const int u = threadIdx.x + k * blockDim.x;
    const bool in = u < p.nunits;
    int q, wu;
    if ((p.L & 31) == 0) {
      q = in ? u / C : 0;
      wu = in ? u - q * C : 0;
    } else {
      // off-grid lattices: the two edge words of every row gather their random
      // planes from two or three segments; numbering them after all inner
      // words confines that slower path to the last waves
      const int nin = p.npairs * (C - 2);
      if (u < nin) {
        q = u / (C - 2);
        wu = 1 + (u - q * (C - 2));
      } else {
        const int e = in ? u - nin : 0;
        q = e >> 1;
        wu = (e & 1) ? C - 1 : 0;
      }
    }
    const bool ok = in && wu < wneed;
    const int w = ok ? wu : 0;
    const int r0 = 2 + 2 * q;
    base0[k] = r0 * ST + w + 1;
    yrow[2 * k] = ytab[r0];
    yrow[2 * k + 1] = ytab[r0 + 1];
    xw[k] = xtab[w];
    // class a = 0 centres of a row with virtual y sit at x = y (mod 4); the
    // virtual x of bit 0 is a multiple of 32
    okm[2 * k] = ok ? (0x11111111u << ((YT + r0) & 3)) : 0u;
    okm[2 * k + 1] = ok ? (0x11111111u << ((YT + r0 + 1) & 3)) : 0u;
    const int Xw = XL + 32 * w;
    uint32_t wm = 0u;
    if (Xw + 32 > X0 && Xw < xend) {
      const int lo = max(Xw, X0), hi = min(Xw + 32, xend);
      const int n = hi - lo;
      wm = (n == 32 ? 0xFFFFFFFFu : ((1u << n) - 1u)) << (lo - Xw);
    }
    okk[k] = ok;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int yv = YT + r0 + h;
      imask[k][h] = (ok && yv >= Y0 && yv < yend) ? wm : 0u;
      ry[2 * k + h] = ytab[r0 + h];
      rx[2 * k + h] = xtab[w];
      if (!grid) {
        if (ok) {
          uint32_t pl[kPlanes];
          gen_planes_at(p, ytab[r0 + h], xtab[w], Xw, t, pl);
          row_rand(pl, p, ytab[r0 + h], xtab[w], t, rr[k][h]);
        } else {
          rr[k][h] = RowRand{0u, 0u, 0u, 0u, 0u};
        }
      }
    }
  }
  if (grid) {
    // row by row (a unit beyond the tile draws for a valid row and decides
    // nothing: its centre masks are empty); a wave whose units of one index
    // all lie beyond the tile skips them.  Drawing more rows at once, to
    // overlap more Philox chains, measured slower: 16.3 us per 4096^2 sweep
    // for a unit's two rows, 18.7 us for all four rows of a thread, against
    // 16.2 us row by row.
    RowRand rq[KU * 2];
#pragma unroll
    for (int k = 0; k < KU; ++k) {
      if (k == 0 || __any(okk[k])) {
        rand_rows_grid<1>(p, t, ry + 2 * k, rx + 2 * k, rq + 2 * k);
        rand_rows_grid<1>(p, t, ry + 2 * k + 1, rx + 2 * k + 1, rq + 2 * k + 1);
      } else {
        rq[2 * k] = rq[2 * k + 1] = RowRand{0u, 0u, 0u, 0u, 0u};
      }
    }
#pragma unroll
    for (int k = 0; k < KU; ++k) {
      rr[k][0] = rq[2 * k];
      rr[k][1] = rq[2 * k + 1];
    }
  }
  // the class order is the same for the whole workgroup: the first wave
  // computes it into the word after the column table
  uint32_t* perm_slot = reinterpret_cast<uint32_t*>(xtab + C);
  if (threadIdx.x < 64) {
    const uint32_t pm = class_order(p.k0, p.k1, t);
    if (threadIdx.x == 0) *perm_slot = pm;
  }
#pragma unroll
  for (int j = 0; j < NSTG; ++j) {
    const int i = threadIdx.x + j * blockDim.x;
    const int r = i / CP, w = i - r * CP;
    if (i < total) S[r * ST + w] = stg[j];
  }
  __syncthreads();
  const uint32_t perm = *perm_slot;

  unsigned count = 0;
#pragma unroll 1
  for (int ph = 0; ph < 8; ++ph) {
    const uint32_t cls = (perm >> (4 * ph)) & 0xFu;
    const int a = (int)(cls >> 1);
    // pairs start on even rows, so the active row of every pair is the class
    // parity: a uniform branch keeps each row's random state in registers
    if (cls & 1u) count += halo_phase<ST, KU, 1>(S, p, base0, yrow, xw, okm, rr, imask, a, t);
    else count += halo_phase<ST, KU, 0>(S, p, base0, yrow, xw, okm, rr, imask, a, t);
    if (ph == 7) {  // each wave adds its count before the last barrier
      const unsigned ws = wave_sum8(count);
      if ((threadIdx.x & 63) == 0) atomicAdd(acc_total, ws);
    }
    __syncthreads();
  }

  // write the interior back (a full-width tile divides by a constant)
  const int iw = (xend - X0 + 31) / 32, ih = yend - Y0;
  if (xend - X0 == TW * 32) {
    for (int i = threadIdx.x; i < TW * ih; i += blockDim.x) {
      const int rr2 = i / TW, ww = i - rr2 * TW;
      store_word<LAYOUT>(p, Y0 + rr2, X0 + 32 * ww, S[(16 + rr2) * ST + 1 + ww + 1], 32);
    }
  } else {
    for (int i = threadIdx.x; i < iw * ih; i += blockDim.x) {
      const int rr2 = i / iw, ww = i - rr2 * iw;
      const int x0 = X0 + 32 * ww;
      const int nb = min(32, xend - x0);
      const uint32_t val = S[(16 + rr2) * ST + 1 + ww + 1];
      store_word<LAYOUT>(p, Y0 + rr2, x0, nb == 32 ? val : (val & ((1u << nb) - 1u)), nb);
    }
  }

  return *acc_total;
}

// Block-wide sum of the per-thread accepted counts, added to *dst by thread 0.
__device__ __forceinline__ void add_block_count(uint32_t* red_lds, unsigned count, unsigned long long* dst) {
  unsigned c = count;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red_lds[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) tot += red_lds[wv];
    // one workgroup per address: an add without a returned value does not wait
    // for a read of the old sum at the end of the kernel
    atomicAdd(dst, tot);
  }
}

template <int LAYOUT, int TWW, int KU>
__global__ __launch_bounds__(KU == 1 ? 1024 : 768)
__attribute__((amdgpu_waves_per_eu(KU == 1 ? 4 : 3, KU == 1 ? 4 : 3))) void halo_kernel(SweepParams p) {
  extern __shared__ uint32_t S[];
  const unsigned total = halo_tile_sweep<LAYOUT, TWW, KU>(S, p, xcd_tile((int)blockIdx.x, (int)gridDim.x));
  // one workgroup per address: an add without a returned value does not wait
  // for a read of the old sum at the end of the kernel
  if (threadIdx.x == 0) atomicAdd(p.accepted + blockIdx.x, (unsigned long long)total);
}

// ---------------------------------------------------------------------------
// Cyclic whole-lattice tile (L % 32 == 0, C = L/32 words per row).  The
// lattice rows -2..L+1 and words -1..C are all present in LDS: the ones
// outside 0..L-1 / 0..C-1 are mirror copies of the wrapped sites, so every
// neighbour read is an immediate offset as in the halo kernel.  Every
// exchange is written to all LDS copies of the sites it flips; a unit near
// the wrap carries a small descriptor of which of its targets have a copy.
// ---------------------------------------------------------------------------
template <int C>
struct CycGeom {
  static constexpr int ST = (C % 2 == 0) ? (C / 2 + 32) : 34;  // see HaloGeom
};

// Row copy delta (in LDS rows) of lattice row x in [-2, R+1]: +R, -R or 0.
__device__ __forceinline__ int row_copy(int x, int R) { return x <= 1 ? R : (x >= R - 2 ? -R : 0); }
// Word copy delta of word x in [-1, C] (C >= 2): +C, -C or 0.
template <int C>
__device__ __forceinline__ int word_copy(int x) { return x <= 0 ? C : (x >= C - 1 ? -C : 0); }

__device__ __forceinline__ void xor_copies(uint32_t* S, int idx, uint32_t m, int dr, int dw) {
  if (!m) return;
  if (dr) atomicXor(&S[idx + dr], m);
  if (dw) atomicXor(&S[idx + dw], m);
  if (dr && dw) atomicXor(&S[idx + dr + dw], m);
}

template <int C, int KU, int H>
__device__ __forceinline__ unsigned cyc_phase(uint32_t* S, const SweepParams& p, const int* base0, const int* yrow,
                                              const int* xw, const uint32_t* okm, const RowRand (*rr)[2],
                                              const int* ur, const int* uw, int a, uint64_t t) {
  constexpr int ST = CycGeom<C>::ST;
  uint32_t v[KU][11];
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    const int b = base0[k] + H * ST;
    v[k][0] = S[b];
    v[k][1] = S[b - 1];
    v[k][2] = S[b + 1];
    v[k][3] = S[b - ST];
    v[k][4] = S[b - ST - 1];
    v[k][5] = S[b - ST + 1];
    v[k][6] = S[b + ST];
    v[k][7] = S[b + ST - 1];
    v[k][8] = S[b + ST + 1];
    v[k][9] = S[b - 2 * ST];
    v[k][10] = S[b + 2 * ST];
  }
  uint32_t F[KU];
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    const uint32_t cmask = __builtin_amdgcn_alignbit(okm[k * 2 + H], okm[k * 2 + H], (32 - a) & 31);
    F[k] = decide_word(v[k], rr[k][H], p, cmask);
  }
  unsigned count = 0;
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    const uint32_t d0 = rr[k][H].d0, d1 = rr[k][H].d1;
    const uint32_t f = F[k];
    const uint32_t Fpx = bop3<KK_TT(KK_TA & ~KK_TB & ~KK_TC)>(f, d1, d0);
    const uint32_t Fmx = bop3<KK_TT(KK_TA & ~KK_TB & KK_TC)>(f, d1, d0);
    const uint32_t Fpy = bop3<KK_TT(KK_TA & KK_TB & ~KK_TC)>(f, d1, d0);
    const uint32_t Fmy = bop3<KK_TT(KK_TA & KK_TB & KK_TC)>(f, d1, d0);
    const int b = base0[k] + H * ST;
    const uint32_t main = f ^ (Fpx << 1) ^ (Fmx >> 1);
    const uint32_t cr = Fpx >> 31, cl = (Fmx & 1u) << 31;
    atomicXor(&S[b], main);
    atomicXor(&S[b + ST], Fpy);
    atomicXor(&S[b - ST], Fmy);
    if (cr) atomicXor(&S[b + 1], cr);
    if (cl) atomicXor(&S[b - 1], cl);
    const int r = ur[k] + H, w = uw[k];
    if (f && (r <= 2 || r >= p.R - 3 || w <= 1 || w >= C - 2)) {  // some target has a mirror copy
      const int R = p.R;
      const int dr0 = row_copy(r, R) * ST, drp = row_copy(r + 1, R) * ST, drm = row_copy(r - 1, R) * ST;
      const int dw0 = word_copy<C>(w), dwp = word_copy<C>(w + 1), dwm = word_copy<C>(w - 1);
      xor_copies(S, b, main, dr0, dw0);
      xor_copies(S, b + ST, Fpy, drp, dw0);
      xor_copies(S, b - ST, Fmy, drm, dw0);
      xor_copies(S, b + 1, cr, dr0, dwp);
      xor_copies(S, b - 1, cl, dr0, dwm);
    }
    count += (unsigned)__builtin_popcount(f & okm[k * 2 + H + 2 * KU]);
  }
  return count;
}

// Whole lattice in one workgroup, p.nsweeps sweeps from p.t0.  Returns the
// thread's accepted count.
template <int LAYOUT, int C, int KU>
__device__ __forceinline__ unsigned cyc_sweeps(uint32_t* S, const SweepParams& p, uint32_t* perm_slot) {
  constexpr int ST = CycGeom<C>::ST;
  const int R = p.R;  // == L
  const int L = p.L;
  // stage rows -2..R+1, words -1..C (the copies included)
  const int rows = R + 4, cols = C + 2;
  for (int i = threadIdx.x; i < rows * cols; i += blockDim.x) {
    const int rr = i / cols, ww = i - rr * cols;
    int y = rr - 2, x = ww - 1;
    y = y < 0 ? y + R : (y >= R ? y - R : y);
    x = x < 0 ? x + C : (x >= C ? x - C : x);
    S[rr * ST + ww] = load_word_any<LAYOUT>(p, y, 32 * x);
  }
  int base0[KU], yrow[KU * 2], xw[KU], ur[KU], uw[KU];
  uint32_t okm[KU * 4];  // [0, 2KU): class-0 pattern per row; [2KU, 4KU): count mask per row
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    const int u = threadIdx.x + k * blockDim.x;
    const bool ok = u < p.nunits;
    const int q = ok ? u / C : 0, w = ok ? u - q * C : 0;
    const int r0 = 2 * q;  // lattice row of the pair's first row
    base0[k] = (r0 + 2) * ST + w + 1;
    ur[k] = r0;
    uw[k] = w;
    yrow[2 * k] = r0;
    yrow[2 * k + 1] = r0 + 1;
    xw[k] = 32 * w;
    okm[2 * k] = ok ? (0x11111111u << (r0 & 3)) : 0u;
    okm[2 * k + 1] = ok ? (0x11111111u << ((r0 + 1) & 3)) : 0u;
    okm[2 * KU + 2 * k] = ok ? 0xFFFFFFFFu : 0u;
    okm[2 * KU + 2 * k + 1] = ok ? 0xFFFFFFFFu : 0u;
  }
  (void)L;
  unsigned count = 0;
#pragma unroll 1
  for (int s = 0; s < p.nsweeps; ++s) {
    const uint64_t t = p.t0 + (uint64_t)s;
    // every word sits on the segment grid (L % 32 == 0); a unit beyond the
    // lattice draws for row 0 and decides nothing
    RowRand rr[KU][2];
#pragma unroll
    for (int k = 0; k < KU; ++k)
#pragma unroll
      for (int h = 0; h < 2; ++h) rand_rows_grid<1>(p, t, yrow + 2 * k + h, xw + k, &rr[k][h]);
    // one wave computes the sweep's class order; every wave has read the
    // previous one (right after the previous sweep's first barrier)
    if (threadIdx.x < 64) {
      const uint32_t pm = class_order(p.k0, p.k1, t);
      if (threadIdx.x == 0) *perm_slot = pm;
    }
    __syncthreads();  // staging or the previous sweep complete
    const uint32_t perm = *perm_slot;
#pragma unroll 1
    for (int ph = 0; ph < 8; ++ph) {
      const uint32_t cls = (perm >> (4 * ph)) & 0xFu;
      const int a = (int)(cls >> 1);
      if (cls & 1u) count += cyc_phase<C, KU, 1>(S, p, base0, yrow, xw, okm, rr, ur, uw, a, t);
      else count += cyc_phase<C, KU, 0>(S, p, base0, yrow, xw, okm, rr, ur, uw, a, t);
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < R * C; i += blockDim.x) {
    const int y = i / C, x = i - y * C;
    store_word_any<LAYOUT>(p, y, 32 * x, S[(y + 2) * ST + x + 1], 32);
  }
  return count;
}

template <int LAYOUT, int C, int KU>
__global__ __launch_bounds__(KU == 1 ? 1024 : 768) void cyc_kernel(SweepParams p) {
  extern __shared__ uint32_t S[];
  const unsigned count = cyc_sweeps<LAYOUT, C, KU>(S, p, S + (p.R + 4) * CycGeom<C>::ST + 16);
  add_block_count(S + (p.R + 4) * CycGeom<C>::ST, count, p.accepted);
}


// ---------------------------------------------------------------------------
// Batch kernels
// ---------------------------------------------------------------------------
// Sweep hand-off of the batch kernels, which a captured graph replays: ctl[0]
// holds the run sweep at which the current chunk of the graph starts; a tile
// launch adds its own position in the chunk (a kernel argument), a resident
// launch runs the whole chunk, and a one-thread kernel at the end of each
// branch advances ctl[0] by the chunk for the next replay.  Stream order and
// the kernel boundaries order every step, so no workgroup touches a shared
// counter.
__global__ void batch_advance_kernel(unsigned* ctl, unsigned step) { ctl[0] += step; }

// KU = 2: tiles of up to 1024 units; KU = 1: up to 512 units, twice the
// waves per unit, which hides more latency when small tiles spread a batch
// over many workgroups.
// Two workgroups per CU: four waves per SIMD, at most 128 VGPRs each.
template <int KU>
__global__ __launch_bounds__(kBatchTileThreads) __attribute__((amdgpu_waves_per_eu(4)))
void batch_tile_kernel(const SweepParams* reps, const BatchTileJob* jobs, const unsigned* ctl, unsigned rel) {
  extern __shared__ uint32_t S[];
  // the sweep index and the job are independent loads; the replica's
  // parameters (sweep count and both buffers included) follow the job
  const unsigned s = __hip_atomic_load(&ctl[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + rel;
  const BatchTileJob job = jobs[blockIdx.x];
  SweepParams p = reps[job.rep];
  if (s < (unsigned)p.nsweeps) {
    if (s & 1u) {  // p.src holds the lattice at the start of the run, p.dst the other buffer
      const void* t = p.src;
      p.src = p.dst;
      p.dst = const_cast<void*>(t);
    }
    p.t0 += s;
    // compile-time tile width (8 or 16 words: immediate, bank-conflict-free
    // LDS offsets) chosen per replica by a uniform switch; a replica's last
    // tile column may be ragged
    unsigned count;
    if (p.layout == kLayoutBits) {
      if (p.tww == 8) count = halo_tile_sweep<kLayoutBits, 8, KU>(S, p, job.tile);
      else count = halo_tile_sweep<kLayoutBits, 16, KU>(S, p, job.tile);
    } else {
      if (p.tww == 8) count = halo_tile_sweep<kLayoutInt8, 8, KU>(S, p, job.tile);
      else count = halo_tile_sweep<kLayoutInt8, 16, KU>(S, p, job.tile);
    }
    if (threadIdx.x == 0) atomicAdd(p.accepted + job.tile, (unsigned long long)count);
  }
}

// All resident replicas in one launch, one workgroup each: the width is a
// uniform run-time switch over per-width instantiations (disjoint code regions
// share one register allocation) and the layout is a run-time branch of the
// staging and the final store.  The reduction area sits past the largest
// resident lattice (rows L+4, stride <= 36).
__global__ __launch_bounds__(kBatchThreads) void batch_resident_all_kernel(const SweepParams* reps, const int* ids,
                                                                           const unsigned* ctl) {
  extern __shared__ uint32_t S[];
  const unsigned s = __hip_atomic_load(&ctl[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  SweepParams p = reps[ids[blockIdx.x]];
  if (s < (unsigned)p.nsweeps) {  // this launch: up to kBatchChunk sweeps from run sweep s
    p.t0 += s;
    p.nsweeps = min(kBatchChunk, p.nsweeps - (int)s);
    uint32_t* slot = S + (p.R + 4) * 36 + 16;  // past the reduction area
    unsigned count;
    switch (p.C) {
      case 2: count = cyc_sweeps<0, 2, 2>(S, p, slot); break;
      case 3: count = cyc_sweeps<0, 3, 2>(S, p, slot); break;
      case 4: count = cyc_sweeps<0, 4, 2>(S, p, slot); break;
      case 5: count = cyc_sweeps<0, 5, 2>(S, p, slot); break;
      case 6: count = cyc_sweeps<0, 6, 2>(S, p, slot); break;
      case 7: count = cyc_sweeps<0, 7, 2>(S, p, slot); break;
      case 8: count = cyc_sweeps<0, 8, 2>(S, p, slot); break;
      default: count = cyc_sweeps<0, 9, 2>(S, p, slot); break;
    }
    add_block_count(S + (p.R + 4) * 36, count, p.accepted);
  }
}

// Small resident replicas (L <= 32 * kResidentSmallMaxC: at most 512 units)
// in 256-thread workgroups, three per CU.
__global__ __launch_bounds__(kResidentSmallThreads, 3) void batch_resident_small_kernel(const SweepParams* reps,
                                                                                       const int* ids,
                                                                                       const unsigned* ctl) {
  extern __shared__ uint32_t S[];
  const unsigned s = __hip_atomic_load(&ctl[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  SweepParams p = reps[ids[blockIdx.x]];
  if (s < (unsigned)p.nsweeps) {
    p.t0 += s;
    p.nsweeps = min(kBatchChunk, p.nsweeps - (int)s);
    uint32_t* slot = S + (p.R + 4) * 36 + 16;
    unsigned count;
    switch (p.C) {
      case 2: count = cyc_sweeps<0, 2, 2>(S, p, slot); break;
      case 3: count = cyc_sweeps<0, 3, 2>(S, p, slot); break;
      case 4: count = cyc_sweeps<0, 4, 2>(S, p, slot); break;
      default: count = cyc_sweeps<0, 5, 2>(S, p, slot); break;
    }
    add_block_count(S + (p.R + 4) * 36, count, p.accepted);
  }
}

}  // namespace

hipError_t launch_sweep(const SweepParams& p, int layout, bool cyclic, int ku, int threads, hipStream_t stream) {
  const int tiles_y = (p.L + p.th - 1) / p.th;
  const dim3 grid(p.tiles_x * tiles_y), block(threads);
  const size_t lds = (size_t)p.R * (p.C + 2) * sizeof(uint32_t) + 16 * sizeof(unsigned);
  if (cyclic && p.C >= 2 && p.C <= 11) {
#define KK_CYC(LY, CC)                                                                            \
  do {                                                                                            \
    const size_t cl = ((size_t)(p.R + 4) * CycGeom<CC>::ST + 17) * sizeof(uint32_t);              \
    if (ku == 1) hipLaunchKernelGGL((cyc_kernel<LY, CC, 1>), grid, block, cl, stream, p);         \
    else hipLaunchKernelGGL((cyc_kernel<LY, CC, 2>), grid, block, cl, stream, p);                 \
  } while (0)
#define KK_CYC_C(LY)                                                                                          \
  do {                                                                                                        \
    switch (p.C) {                                                                                            \
      case 2: KK_CYC(LY, 2); break;   case 3: KK_CYC(LY, 3); break;   case 4: KK_CYC(LY, 4); break;           \
      case 5: KK_CYC(LY, 5); break;   case 6: KK_CYC(LY, 6); break;   case 7: KK_CYC(LY, 7); break;           \
      case 8: KK_CYC(LY, 8); break;   case 9: KK_CYC(LY, 9); break;   case 10: KK_CYC(LY, 10); break;         \
      default: KK_CYC(LY, 11); break;                                                                         \
    }                                                                                                         \
  } while (0)
    if (layout == kLayoutBits) KK_CYC_C(kLayoutBits);
    else KK_CYC_C(kLayoutInt8);
#undef KK_CYC_C
#undef KK_CYC
    return hipGetLastError();
  }
  if (!cyclic && (p.tww == 1 || p.tww == 2 || p.tww == 4 || p.tww == 8 || p.tww == 16)) {
#define KK_HALO(LY, TW)                                                                                  \
  do {                                                                                                   \
    const size_t hl = ((size_t)p.R * HaloGeom<TW>::ST + 17 + p.R + HaloGeom<TW>::C) * sizeof(uint32_t);  \
    if (ku == 1) hipLaunchKernelGGL((halo_kernel<LY, TW, 1>), grid, block, hl, stream, p);               \
    else hipLaunchKernelGGL((halo_kernel<LY, TW, 2>), grid, block, hl, stream, p);                       \
  } while (0)
#define KK_HALO_W(LY)                          \
  do {                                         \
    switch (p.tww) {                           \
      case 1: KK_HALO(LY, 1); break;           \
      case 2: KK_HALO(LY, 2); break;           \
      case 4: KK_HALO(LY, 4); break;           \
      case 8: KK_HALO(LY, 8); break;           \
      default: KK_HALO(LY, 16); break;         \
    }                                          \
  } while (0)
    if (layout == kLayoutBits) KK_HALO_W(kLayoutBits);
    else KK_HALO_W(kLayoutInt8);
#undef KK_HALO_W
#undef KK_HALO
    return hipGetLastError();
  }
#define KK_LAUNCH(LY, CY, KUV) hipLaunchKernelGGL((sweep_kernel<LY, CY, KUV>), grid, block, lds, stream, p)
  if (layout == kLayoutBits) {
    if (cyclic) { if (ku == 1) KK_LAUNCH(kLayoutBits, true, 1); else KK_LAUNCH(kLayoutBits, true, 2); }
    else { if (ku == 1) KK_LAUNCH(kLayoutBits, false, 1); else KK_LAUNCH(kLayoutBits, false, 2); }
  } else {
    if (cyclic) { if (ku == 1) KK_LAUNCH(kLayoutInt8, true, 1); else KK_LAUNCH(kLayoutInt8, true, 2); }
    else { if (ku == 1) KK_LAUNCH(kLayoutInt8, false, 1); else KK_LAUNCH(kLayoutInt8, false, 2); }
  }
#undef KK_LAUNCH
  return hipGetLastError();
}

}  // namespace kk

namespace kk {

size_t batch_tile_lds_bytes() {
  const int R = kBatchTh + 32;  // the widest tile has the largest stride
  return ((size_t)R * HaloGeom<kBatchMaxTww>::ST + 17 + R + kBatchMaxTww + 2) * sizeof(uint32_t);
}

size_t batch_resident_lds_bytes(int L) { return ((size_t)(L + 4) * 36 + 17) * sizeof(uint32_t); }

hipError_t launch_batch_tiles(const SweepParams* reps, const BatchTileJob* jobs, int njobs, const unsigned* ctl,
                              unsigned rel, int ku, hipStream_t stream) {
  if (ku == 1)
    hipLaunchKernelGGL(batch_tile_kernel<1>, dim3(njobs), dim3(kBatchTileThreads), batch_tile_lds_bytes(), stream,
                       reps, jobs, ctl, rel);
  else
    hipLaunchKernelGGL(batch_tile_kernel<2>, dim3(njobs), dim3(kBatchTileThreads), batch_tile_lds_bytes(), stream,
                       reps, jobs, ctl, rel);
  return hipGetLastError();
}

hipError_t launch_batch_advance(unsigned* ctl, unsigned step, hipStream_t stream) {
  hipLaunchKernelGGL(batch_advance_kernel, dim3(1), dim3(1), 0, stream, ctl, step);
  return hipGetLastError();
}

hipError_t launch_batch_resident(const SweepParams* reps, const int* ids, int n, size_t lds_bytes, bool small,
                                 const unsigned* ctl, hipStream_t stream) {
  if (small)
    hipLaunchKernelGGL(batch_resident_small_kernel, dim3(n), dim3(kResidentSmallThreads), lds_bytes, stream, reps,
                       ids, ctl);
  else
    hipLaunchKernelGGL(batch_resident_all_kernel, dim3(n), dim3(kBatchThreads), lds_bytes, stream, reps, ids, ctl);
  return hipGetLastError();
}

}  // namespace kk
