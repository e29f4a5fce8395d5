// Exactly rounded sums of FP32 or FP64 values, independent of the order of
// the additions.
//
// Every finite FP32 value is an integer multiple of 2^-149 (FP64: 2^-1074),
// the format's smallest subnormal: x = m 2^(b + UNIT_EXP) with an integer
// mantissa m (24 bits; FP64 53) and a bit offset b in [0, 253] (FP64
// [0, 2045]).  A sum of such values is therefore an integer number of units,
// below 2^308 for FP32 (2^2129 for FP64) for fewer than 2^31 terms.  It is
// held as NL signed 64-bit limbs, limb k weighing 2^(32 k) units: a value adds
// m << (b mod 32) to limb b / 32 (FP64: its mantissa in two parts of 27 and 26
// bits, each added to its own limb), integer additions are exact and
// associative, so every order of the terms gives the same integer, and one
// final rounding to FP64 (nearest, ties to even) gives the exactly rounded
// sum.  `xs_normalise` carries every limb but the top one into [0, 2^32),
// which keeps the limbs far from overflow: between two normalisations a limb
// may take up to XS_ADDS_FP32 (FP64: XS_ADDS_FP64) further terms.
//
// Plain C++ apart from the __host__ / __device__ / __forceinline__ markers,
// which the includer defines (HIP's runtime header in the library; empty
// definitions in the CPU tests, which check the rounding against exact
// rational sums).  Inputs must be finite.
#pragma once

#include <cmath>
#include <cstdint>
#include <cstring>

namespace krr {

template <typename TX>
struct ExactSum;

template <>
struct ExactSum<float> {
  static constexpr int NL = 9;            // 8 digit limbs + the signed top one (bits 256 .. 307)
  static constexpr int UNIT_EXP = -149;
  static constexpr int ADDS = 128;        // terms per limb between normalisations: 2^32 + 128 * 2^55 < 2^63
};

template <>
struct ExactSum<double> {
  static constexpr int NL = 66;           // 65 digit limbs + the signed top one (bits 2080 .. 2128)
  static constexpr int UNIT_EXP = -1074;
  static constexpr int ADDS = 8;          // rows per normalisation: 2^32 + 8 * (2^58 + 2^57) < 2^63
};

// The terms one value adds: limb index and amount (a second term for FP64).
struct XsTerms {
  int l0, l1;
  int64_t c0, c1;
};

__host__ __device__ __forceinline__ XsTerms xs_terms(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  const int e = (int)((u >> 23) & 0xffu);
  int64_t m = (int64_t)(u & 0x7fffffu) | (e != 0 ? (int64_t)0x800000 : 0);
  const int b = e != 0 ? e - 1 : 0;   // x = m 2^(b - 149)
  if (u >> 31) m = -m;
  XsTerms t;
  t.l0 = b >> 5;
  t.c0 = m * ((int64_t)1 << (b & 31));   // |c0| < 2^55
  t.l1 = 0;
  t.c1 = 0;
  return t;
}

__host__ __device__ __forceinline__ XsTerms xs_terms(double x) {
  uint64_t u;
  memcpy(&u, &x, 8);
  const int e = (int)((u >> 52) & 0x7ffu);
  const int64_t m = (int64_t)(u & 0xfffffffffffffull) | (e != 0 ? ((int64_t)1 << 52) : 0);
  const int b = e != 0 ? e - 1 : 0;   // x = m 2^(b - 1074)
  const bool neg = (u >> 63) != 0;
  const int64_t lo = m & (((int64_t)1 << 27) - 1), hi = m >> 27;   // m = hi 2^27 + lo
  XsTerms t;
  t.l0 = b >> 5;
  t.c0 = lo * ((int64_t)1 << (b & 31));   // < 2^58
  t.l1 = (b + 27) >> 5;
  t.c1 = hi * ((int64_t)1 << ((b + 27) & 31));   // < 2^57
  if (neg) {
    t.c0 = -t.c0;
    t.c1 = -t.c1;
  }
  return t;
}

// Carries limbs 0 .. NL - 2 into [0, 2^32) (floor division, so negative
// limbs borrow from the next one); the top limb keeps the signed rest.
template <int NL, typename Get, typename Set>
__host__ __device__ __forceinline__ void xs_normalise(Get get, Set set) {
  int64_t carry = 0;
  for (int k = 0; k < NL - 1; ++k) {
    const int64_t v = get(k) + carry;
    carry = v >> 32;   // arithmetic shift: floor(v / 2^32)
    set(k, v - carry * ((int64_t)1 << 32));
  }
  set(NL - 1, get(NL - 1) + carry);
}

// The FP64 value nearest to the integer sum held in the limbs (ties to even),
// times 2^UNIT_EXP.  `limb` is overwritten (normalised, and negated for a
// negative sum).  An exact zero gives +0.
template <typename TX>
__host__ __device__ inline double xs_round(int64_t* limb) {
  constexpr int NL = ExactSum<TX>::NL;
  auto get = [&](int k) { return limb[k]; };
  auto set = [&](int k, int64_t v) { limb[k] = v; };
  xs_normalise<NL>(get, set);
  const bool neg = limb[NL - 1] < 0;
  if (neg) {
    for (int k = 0; k < NL; ++k) limb[k] = -limb[k];
    xs_normalise<NL>(get, set);   // the top limb is now >= 0
  }
  int kh = NL - 1;
  while (kh >= 0 && limb[kh] == 0) --kh;
  if (kh < 0) return 0.0;
  // digit view: limbs 0 .. NL - 2 are 32-bit digits, the top limb (< 2^62)
  // spans two more digits
  auto digit = [&](int k) -> uint64_t {
    if (k < 0) return 0;
    if (k < NL - 1) return (uint64_t)limb[k];
    if (k == NL - 1) return (uint64_t)limb[NL - 1] & 0xffffffffull;
    if (k == NL) return (uint64_t)limb[NL - 1] >> 32;
    return 0;
  };
  const int hb = 32 * kh + 63 - __builtin_clzll((unsigned long long)limb[kh]);   // highest set bit
  if (hb <= 52) {   // below 2^53 units: exact
    const uint64_t v = digit(0) | (digit(1) << 32);
    const double r = ldexp((double)v, ExactSum<TX>::UNIT_EXP);
    return neg ? -r : r;
  }
  // bits [sh - 1, sh + 63): the round bit, then the 53-bit mantissa
  const int sh = hb - 52, lo = sh - 1;
  const int a = lo >> 5, r = lo & 31;
  uint64_t w = digit(a) >> r;
  w |= digit(a + 1) << (32 - r);
  if (r > 0) w |= digit(a + 2) << (64 - r);
  bool sticky = (digit(a) & ((1ull << r) - 1)) != 0;
  for (int k = 0; k < a && !sticky; ++k) sticky = limb[k] != 0;
  uint64_t mant = (w >> 1) & ((1ull << 53) - 1);
  if ((w & 1) && (sticky || (mant & 1))) ++mant;   // mant may reach 2^53: still exact in FP64
  const double res = ldexp((double)mant, sh + ExactSum<TX>::UNIT_EXP);
  return neg ? -res : res;
}

}  // namespace krr
