"""Host check of the compile-time sorting networks that fill the register
candidate sets (no GPU): the header is plain C++17, compiled here with g++.
By the 0-1 principle (Knuth, TAOCP vol. 3, 5.3.4) a comparator network
sorts every input iff it sorts every 0-1 input; the program tries all 2^N
0-1 inputs, 64 at a time as bit lanes, for each register bucket N."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2111_04182_amd", "csrc")
BUCKETS = (1, 2, 4, 8, 10, 12, 16, 20, 24)

PROG = r"""
#include <cstdint>
#include <cstdio>
#include "zd_sortnet.h"

template <int N>
int check() {
  constexpr zd::SortNet net = zd::SortNetFor<N>::net;
  // wire w of input x is bit w of x; lane b of a 64-bit word carries input
  // x = base + b
  for (uint64_t base = 0; base < (1ull << N); base += 64) {
    uint64_t w[N];
    for (int i = 0; i < N; ++i) {
      w[i] = 0;
      for (int b = 0; b < 64; ++b)
        if ((((base + b) >> i) & 1) && base + b < (1ull << N)) w[i] |= 1ull << b;
    }
    for (int c = 0; c < net.n; ++c) {
      const uint64_t lo = w[net.v[c].lo], hi = w[net.v[c].hi];
      if (net.v[c].lo >= net.v[c].hi || net.v[c].hi >= N) return 2;
      w[net.v[c].lo] = lo & hi;  // min of 0-1 values
      w[net.v[c].hi] = lo | hi;  // max
    }
    for (int i = 0; i + 1 < N; ++i)
      if (w[i] & ~w[i + 1]) return 1;  // a 1 above a 0
  }
  std::printf("%d %d\n", N, net.n);
  return 0;
}

int main() {
  return BUCKETS_CALLS;
}
"""


def test_sorting_networks_sort_every_0_1_input(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("needs g++")
    calls = " | ".join(f"check<{n}>()" for n in BUCKETS)
    src = tmp_path / "net.cpp"
    src.write_text(PROG.replace("BUCKETS_CALLS", calls))
    exe = tmp_path / "net"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    sizes = dict(tuple(int(x) for x in line.split()) for line in r.stdout.split("\n") if line)
    assert sorted(sizes) == sorted(BUCKETS)
    # Batcher's network on 16 wires has 63 comparators; pruned to 10, 32
    assert sizes[16] == 63 and sizes[10] == 32 and sizes[1] == 0


def test_a_broken_network_is_caught(tmp_path):
    """The checker itself: dropping one comparator of the 10-wire network
    must leave some 0-1 input unsorted."""
    if not shutil.which("g++"):
        pytest.skip("needs g++")
    src = tmp_path / "net.cpp"
    prog = PROG.replace("constexpr zd::SortNet net = zd::SortNetFor<N>::net;",
                        "zd::SortNet net = zd::SortNetFor<N>::net;\n  net.n -= 1;")
    src.write_text(prog.replace("BUCKETS_CALLS", "check<10>()"))
    exe = tmp_path / "net"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    assert subprocess.run([str(exe)], capture_output=True, timeout=60).returncode == 1
