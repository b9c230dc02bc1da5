// Host check of the 16-byte-slot quotient map's key mix (qmix2): for prefix widths of 57..128
// bits and 2^10..2^22 slots, distinct keys (random, and structured: small counters) give distinct
// (home slot, remainder) pairs, the home fits its slot bits and the remainder its field.  The
// exactness of the map's lookups rests on this: a slot's home and remainder identify its key.
#include <cstdio>
#include <cstdint>
#include <random>
#include <set>
#include <tuple>
#include "ig_internal.h"
using namespace ig;
int main() {
  std::mt19937_64 rng(7);
  int bad = 0;
  for (uint32_t w : {57u, 64u, 65u, 72u, 96u, 120u, 128u})
    for (uint32_t sbits : {10u, 16u, 22u}) {
      const uint32_t qbits = w - sbits;
      std::set<std::tuple<uint64_t, uint64_t, uint64_t>> seen;
      std::set<std::pair<uint64_t, uint64_t>> keys;
      for (int i = 0; i < 200000; i++) {
        uint64_t lo = rng(), hi = rng();
        if (w < 64) lo &= (1ull << w) - 1;
        if (w <= 64) hi = 0;
        else if (w < 128) hi &= (1ull << (w - 64)) - 1;
        // also structured keys: small counters in the low word
        if (i % 2) { lo = (uint64_t)i; if (w > 64) hi = (uint64_t)(i % 7); }
        if (!keys.insert({lo, hi}).second) continue;
        uint64_t home, rl, rh;
        qmix2(lo, hi, w, sbits, &home, &rl, &rh);
        if (home >> sbits) { bad++; }
        if (qbits < 64) { if (rh || (rl >> qbits)) bad++; }
        else if (qbits < 128 && (rh >> (qbits - 64))) bad++;
        if (!seen.insert({home, rl, rh}).second) bad++;
      }
      std::printf("w=%u sbits=%u keys=%zu images=%zu\n", w, sbits, keys.size(), seen.size());
    }
  std::printf("bad=%d\n", bad);
  return bad != 0;
}
