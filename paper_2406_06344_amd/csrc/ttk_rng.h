// splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) and the keyed streams of the cross algorithm.
//   next():   state += 0x9E3779B97F4A7C15; z = state;
//             z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9;
//             z = (z ^ (z >> 27)) * 0x94D049BB133111EB;  return z ^ (z >> 31)
//   key:      s = seed; for each part p: s = mix((s ^ p) + 0x9E3779B97F4A7C15)
//   below(m): high 64 bits of next() * m;  bit(): top bit of next()
//   floyd(M, k): k distinct values of [0, M) (Floyd's algorithm), sorted
//   (floyd_unsorted: the same values in generation order).
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

namespace ttk {

enum : uint64_t { RNG_TAG_INIT = 1, RNG_TAG_UPDATE = 2, RNG_TAG_TEST = 3 };

class SplitMix64 {
 public:
  static constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
  static uint64_t mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  explicit SplitMix64(uint64_t state) : s_(state) {}
  template <class... P>
  static SplitMix64 keyed(uint64_t seed, P... parts) {
    uint64_t s = seed;
    for (uint64_t p : {static_cast<uint64_t>(parts)...}) s = mix((s ^ p) + kGolden);
    return SplitMix64(s);
  }
  uint64_t next() { s_ += kGolden; return mix(s_); }
  uint64_t below(uint64_t m) {
    return static_cast<uint64_t>((static_cast<unsigned __int128>(next()) * m) >> 64);
  }
  int bit() { return static_cast<int>(next() >> 63); }
  std::vector<int64_t> floyd(int64_t M, int64_t k) {
    std::vector<int64_t> out = floyd_unsorted(M, k);
    std::sort(out.begin(), out.end());
    return out;
  }
  // The same k values in the order Floyd's algorithm produces them.
  std::vector<int64_t> floyd_unsorted(int64_t M, int64_t k) {
    // membership in an open-addressing table (linear probing, load <= 1/4)
    size_t cap = 16;
    while (cap < static_cast<size_t>(k) * 4) cap <<= 1;
    std::vector<int64_t> table(cap, -1);
    const int shift = 64 - __builtin_ctzll(cap);
    auto insert = [&](int64_t v) {   // true if v was not present
      size_t h = static_cast<size_t>((static_cast<uint64_t>(v) * kGolden) >> shift);
      while (true) {
        if (table[h] == v) return false;
        if (table[h] < 0) { table[h] = v; return true; }
        h = (h + 1) & (cap - 1);
      }
    };
    std::vector<int64_t> out;
    out.reserve(static_cast<size_t>(k));
    for (int64_t j = M - k; j < M; ++j) {
      const int64_t t = static_cast<int64_t>(below(static_cast<uint64_t>(j + 1)));
      if (insert(t)) out.push_back(t);
      else { insert(j); out.push_back(j); }
    }
    return out;
  }

 private:
  uint64_t s_;
};

}  // namespace ttk
