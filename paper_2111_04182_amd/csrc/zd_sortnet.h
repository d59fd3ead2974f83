// zd_sortnet.h -- compile-time sorting networks for the register candidate
// sets (plain C++17, no device code: the host tests compile it with g++).
//
// Batcher's odd-even merge sort (Batcher, "Sorting networks and their
// applications", AFIPS 1968) on the next power of two P >= N, keeping only
// the comparators whose both wires lie in [0, N).  This is a sorting
// network for N wires: read the input as P wires whose last P - N hold +inf;
// every comparator of the full network puts the smaller value on its lower
// wire, so one that touches a wire >= N leaves both wires unchanged (the
// +inf stays on the upper wire), and dropping it changes nothing.
#pragma once

namespace zd {

struct CmpEx {
  int lo, hi;  // wires, lo < hi: the smaller value ends on lo
};

constexpr int kMaxCmpEx = 256;

struct SortNet {
  CmpEx v[kMaxCmpEx];
  int n;
};

constexpr SortNet make_sort_net(int N) {
  SortNet s{};
  s.n = 0;
  int P = 1;
  while (P < N) P *= 2;
  // merge runs of length p into runs of 2p; k is the comparator distance
  for (int p = 1; p < P; p *= 2)
    for (int k = p; k >= 1; k /= 2)
      for (int j = k % p; j + k < P; j += 2 * k)
        for (int i = 0; i < k && i + j + k < P; ++i)
          if ((i + j) / (2 * p) == (i + j + k) / (2 * p) && i + j + k < N) {
            if (s.n < kMaxCmpEx) s.v[s.n] = CmpEx{i + j, i + j + k};
            ++s.n;
          }
  return s;
}

// The network for N wires (N <= 32 stays within kMaxCmpEx).
template <int N>
struct SortNetFor {
  static constexpr SortNet net = make_sort_net(N);
  static_assert(net.n <= kMaxCmpEx, "sorting network larger than its table");
};

}  // namespace zd
