// Host checks of the index helpers of the kernels:
//  * fastdiv(n, make_fastdiv(d)) against n / d over divisors 1..4096, every
//    power of two and its neighbours, and large divisors, at numerators near 0,
//    near multiples of d and near 2^31;
//  * xcd_order(b, nt, m0) is a bijection on [0, nt) that lists the blocks of
//    each XCD class ((m0 + b) mod 8) contiguously.
// Prints the number of mismatches.
#include <stdint.h>
#include <stdio.h>

#include <vector>

#include "pasd_internal.hpp"

static long check(uint32_t d) {
  const pasd::FastDiv f = pasd::make_fastdiv(d);
  long bad = 0;
  auto one = [&](uint64_t n) {
    if (n >= (uint64_t(1) << 31)) return;
    if (pasd::fastdiv((uint32_t)n, f) != (uint32_t)(n / d)) ++bad;
  };
  for (uint64_t n = 0; n < 4096; ++n) one(n);
  for (uint64_t k = 1; k < 4096; ++k) {
    const uint64_t base = k * d;
    one(base - 1); one(base); one(base + 1);
  }
  const uint64_t top = (uint64_t(1) << 31) - 1;
  for (uint64_t n = top - 4096; n <= top; ++n) one(n);
  const uint64_t q = top / d;
  for (uint64_t k = (q > 64 ? q - 64 : 0); k <= q; ++k) {
    one(k * d - 1); one(k * d); one(k * d + d - 1);
  }
  return bad;
}

int main() {
  long bad = 0, cases = 0;
  for (uint32_t d = 1; d <= 4096; ++d, ++cases) bad += check(d);
  for (int e = 12; e < 31; ++e)
    for (int64_t o = -3; o <= 3; ++o, ++cases) bad += check((uint32_t)((int64_t(1) << e) + o));
  uint64_t x = 88172645463325252ull;  // xorshift64 for arbitrary divisors
  for (int t = 0; t < 2000; ++t, ++cases) {
    x ^= x << 13; x ^= x >> 7; x ^= x << 17;
    bad += check((uint32_t)(1 + x % ((uint64_t(1) << 31) - 1)));
  }
  long obad = 0;
  for (int nt = 1; nt <= 700; ++nt)
    for (int m0 = 0; m0 < 24; ++m0) {
      std::vector<int> seen(nt, 0), at(nt, -1);
      for (int b = 0; b < nt; ++b) {
        const int p = pasd::xcd_order(b, nt, m0);
        if (p < 0 || p >= nt || seen[p]++) { ++obad; continue; }
        at[p] = b;
      }
      int runs = 0;  // class changes along the order: at most kXcds - 1
      for (int p = 1; p < nt; ++p)
        if (at[p] >= 0 && at[p - 1] >= 0 &&
            (m0 + at[p]) % pasd::kXcds != (m0 + at[p - 1]) % pasd::kXcds) ++runs;
      if (runs > pasd::kXcds - 1) ++obad;
    }
  printf("divisors %ld mismatches %ld\n", cases, bad);
  printf("xcd orders mismatches %ld\n", obad);
  return bad == 0 && obad == 0 ? 0 : 1;
}
