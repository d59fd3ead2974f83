// zd_knn_impl.h -- the exact k-NN search kernels (templates; instantiated per
// dimension and k bucket in zd_knn_all_d{2,3}.hip and zd_knn_ext_d{2,3}.hip).
//
// Algorithm 3 (searchUp) scans the query's leaf, then climbs while the ball
// of the current k-th distance leaves the current node's box, searching each
// sibling subtree with Algorithm 2 (searchDown): a child is visited iff its
// box distance is <= the k-th squared distance, nearer child first.
//
// On gfx950 a wavefront answers 64 queries that are consecutive in Morton
// order (all-points rows in tree order; external queries after a Morton
// presort, Section 3.1) with ONE shared walk:
//   * the start node is the lowest common ancestor G of the group's leaves;
//     searchDown runs over G's subtree, then the searchUp climb from G;
//   * a child is visited when ANY lane's ball reaches it (a ballot of
//     box distance <= that lane's k-th d2), and the climb stops once every
//     lane's ball is inside the current box.  Each lane therefore sees a
//     superset of the points its own search would see; since a lane only
//     keeps its k smallest (d2, id), the rows are exact;
//   * the nearer child is taken first (Algorithm 2's order heuristic), judged
//     by the side of the split holding the Morton cell of the group's middle
//     query: one integer test per node instead of two box-centre distances;
//   * node records are read at wave-uniform addresses, and a visited leaf's
//     points are staged once in LDS and broadcast to all lanes, so the walk
//     itself never diverges;
//   * for all-points rows, each lane first scores the group's own points and
//     the 32 sorted positions on either side (its Morton neighbours), which
//     tightens every lane's k-th distance before the walk starts; those
//     positions are skipped later.
// For all-points rows at k > 16 a team of 4 or 8 lanes shares one query
// (TeamSet): a wavefront then answers its 64 positions as groups of 16 or
// 8 queries, one shared walk each.
#pragma once

#include "zd_internal.h"
#include "zd_sortnet.h"

#include <climits>
#include <type_traits>
#include <utility>

namespace zd {

// The candidate set N of Algorithms 2-3: the k best (d2, id) pairs so far,
// ascending, in the LAST k of K registers; the first K-k hold (-inf, INT_MIN)
// and never move.  So the k-th entry is always register K-1 and insertion is
// a branch-free shift with static indices (no dynamic register indexing).
// While fewer than k candidates have arrived the k-th entry is (+inf,
// INT_MAX): distance(p, N, k) is infinite and every candidate enters.  A lane
// without a query holds (-inf, INT_MIN) everywhere: nothing ever enters and
// no box is ever within its k-th distance, so it needs no test of its own.
template <int K>
struct Heap {
  static_assert(K <= 16, "one lane per query serves k <= 16; larger k run in lane teams");
  double d[K];
  int32_t id[K];

  __device__ __forceinline__ void init(int k, bool live) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const bool used = live && j >= K - k;
      d[j] = used ? INFINITY : -INFINITY;
      id[j] = used ? INT_MAX : INT_MIN;
    }
  }

  __device__ __forceinline__ double kth() const { return d[K - 1]; }

  // insert(N, q, k) of Algorithms 2-3: enters iff it precedes the k-th entry.
  // The first test is one compare; a tie with the k-th distance falls through
  // to the exact (d2, id) comparisons, which then change nothing if the
  // candidate does not precede it.
  template <bool kSplit = false>
  __device__ __forceinline__ void offer(double dd, int32_t q) {
    if (!(dd <= d[K - 1])) return;
    if constexpr (kSplit && K >= 8) {
      offer_split(dd, q);
    } else {
      bool lt[K];
#pragma unroll
      for (int j = 0; j < K; ++j) lt[j] = cand_lt(dd, q, d[j], id[j]);
#pragma unroll
      for (int j = K - 1; j > 0; --j) {
        // slot j takes its left neighbour if the candidate precedes that
        // neighbour, else the candidate if it precedes slot j, else stays
        const double nd = lt[j - 1] ? d[j - 1] : (lt[j] ? dd : d[j]);
        const int32_t ni = lt[j - 1] ? id[j - 1] : (lt[j] ? q : id[j]);
        d[j] = nd;
        id[j] = ni;
      }
      if (lt[0]) {
        d[0] = dd;
        id[0] = q;
      }
    }
  }

  // The same shift in two halves, for external queries and for the
  // all-points walk at k >= 16, whose entries mostly arrive near the end of
  // the sorted set: the upper half [H, K)
  // always, taking slot H-1's old entry if the candidate precedes it; the
  // lower half [0, H) only when some lane's candidate does.
  __device__ __forceinline__ void offer_split(double dd, int32_t q) {
    constexpr int H = K / 2;
    bool lt[K];
#pragma unroll
    for (int j = H; j < K; ++j) lt[j] = cand_lt(dd, q, d[j], id[j]);
    const bool low = cand_lt(dd, q, d[H - 1], id[H - 1]);
    const double cd = d[H - 1];
    const int32_t ci = id[H - 1];
#pragma unroll
    for (int j = K - 1; j > H; --j) {
      const double nd = lt[j - 1] ? d[j - 1] : (lt[j] ? dd : d[j]);
      const int32_t ni = lt[j - 1] ? id[j - 1] : (lt[j] ? q : id[j]);
      d[j] = nd;
      id[j] = ni;
    }
    {
      const double nd = low ? cd : (lt[H] ? dd : d[H]);
      const int32_t ni = low ? ci : (lt[H] ? q : id[H]);
      d[H] = nd;
      id[H] = ni;
    }
    if (__ballot(low) != 0) {
#pragma unroll
      for (int j = 0; j < H; ++j) lt[j] = cand_lt(dd, q, d[j], id[j]);
#pragma unroll
      for (int j = H - 1; j > 0; --j) {
        const double nd = lt[j - 1] ? d[j - 1] : (lt[j] ? dd : d[j]);
        const int32_t ni = lt[j - 1] ? id[j - 1] : (lt[j] ? q : id[j]);
        d[j] = nd;
        id[j] = ni;
      }
      if (lt[0]) {
        d[0] = dd;
        id[0] = q;
      }
    }
  }

  // An empty set (k = K) that takes K candidates in a row ends up holding
  // them in ascending (d2, id) order.  The caller stores them unsorted in
  // the K slots and sorts them with a merge network: a compare-exchange
  // per comparator (32 for K = 10) instead of K full insertion shifts.
  template <int A, int B>
  __device__ __forceinline__ void cmp_ex() {
    const bool sw = cand_lt(d[B], id[B], d[A], id[A]);
    const double x = d[A], y = d[B];
    const int32_t i = id[A], j = id[B];
    d[A] = sw ? y : x;
    d[B] = sw ? x : y;
    id[A] = sw ? j : i;
    id[B] = sw ? i : j;
  }
  template <int... I>
  __device__ __forceinline__ void run_net(std::integer_sequence<int, I...>) {
    (cmp_ex<SortNetFor<K>::net.v[I].lo, SortNetFor<K>::net.v[I].hi>(), ...);
  }
  __device__ __forceinline__ void sort_slots() {
    run_net(std::make_integer_sequence<int, SortNetFor<K>::net.n>{});
  }

  __device__ __forceinline__ void write(int k, int32_t *out_ids, double *out_d2) const {
#pragma unroll
    for (int j = 0; j < K; ++j)
      if (j >= K - k) {
        const int o = j - (K - k);
        out_ids[o] = id[j] == INT_MAX ? -1 : id[j];
        out_d2[o] = d[j];
      }
  }
};

// Moves within each team of T = 4 or 8 consecutive lanes (every lane of the
// wavefront is active wherever these run).  T = 4: DPP quad permutations;
// T = 8: a swizzle that reads lane (l & ~7) | R, and a DPP row shift by one.
template <int T, int R>
__device__ __forceinline__ int32_t team_bcast(int32_t v) {
  static_assert(T == 4 || T == 8, "teams of 4 or 8 lanes");
  if constexpr (T == 4)
    return __builtin_amdgcn_mov_dpp(v, R | (R << 2) | (R << 4) | (R << 6), 0xf, 0xf, false);
  else
    return __builtin_amdgcn_ds_swizzle(v, (R << 5) | 0x18);
}
template <int T, int R>
__device__ __forceinline__ double team_bcast(double v) {
  const int64_t b = __double_as_longlong(v);
  const int32_t lo = team_bcast<T, R>((int32_t)b), hi = team_bcast<T, R>((int32_t)(b >> 32));
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}
// lane i of each team takes lane i - 1's value (the team's first lane gets
// some other value, which the caller ignores)
template <int T>
__device__ __forceinline__ int32_t team_prev(int32_t v) {
  if constexpr (T == 4)
    return __builtin_amdgcn_mov_dpp(v, 0 | (0 << 2) | (1 << 4) | (2 << 6), 0xf, 0xf, false);
  else
    return __builtin_amdgcn_update_dpp(v, v, 0x111, 0xf, 0xf, false);  // row_shr:1
}
template <int T>
__device__ __forceinline__ double team_prev(double v) {
  const int64_t b = __double_as_longlong(v);
  const int32_t lo = team_prev<T>((int32_t)b), hi = team_prev<T>((int32_t)(b >> 32));
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

// For the all-points rows at large k, T = 4 or 8 lanes (a team) answer one
// query, so a wavefront answers 64 / T, and hold its candidate set
// together: team lane `sub` holds the sorted slots [S sub, S sub + S),
// S = ceil(K / T), the k best in the last k of the T S slots as in Heap.
// Each lane scores every T-th point of every list of points, and the team
// takes its lanes' candidates one after the other: every lane of the team
// compares the candidate with its S slots and shifts them, the lowest slot
// taking the previous lane's old last entry across the lane boundary.  One
// insertion costs O(k / T) per lane instead of the O(k) shift of one lane's
// whole set, all teams insert at once, and the registers hold 1/T of the
// set; the wavefront's shared walk covers 64 / T queries' balls instead of
// 64.
template <int K, int T_>
struct TeamSet {
  static constexpr int T = T_;
  static constexpr int S = (K + T - 1) / T;
  static constexpr int KT = S * T;
  double d[S];
  int32_t id[S];
  double kd;  // the team's k-th entry (slot KT - 1, held by team lane T - 1)
  int32_t ki;
  int sub;

  __device__ __forceinline__ void init(int k, bool live) {
    sub = threadIdx.x & (T - 1);
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const bool used = live && sub * S + j >= KT - k;
      d[j] = used ? INFINITY : -INFINITY;
      id[j] = used ? INT_MAX : INT_MIN;
    }
    kd = live ? INFINITY : -INFINITY;
    ki = live ? INT_MAX : INT_MIN;
  }

  __device__ __forceinline__ double kth() const { return kd; }

  // team lane R's candidate, offered to the whole team
  template <int R>
  __device__ __forceinline__ void take(double dd, int32_t q) {
    const double cd = team_bcast<T, R>(dd);
    const int32_t cq = team_bcast<T, R>(q);
    const bool cw = cand_lt(cd, cq, kd, ki);
    if (__ballot(cw) == 0) return;
    // slot by slot from the top, with only the masks of two neighbouring
    // slots live (an array of S lane masks would crowd the scalar registers):
    // slot j takes slot j-1's entry if the candidate precedes that entry,
    // else the candidate if it precedes slot j, else keeps its own
    bool hi = cw & cand_lt(cd, cq, d[S - 1], id[S - 1]);
    // the previous lane's last slot, and whether the candidate precedes it
    // (the moves run on every lane: a lane left out of a DPP move is left
    // out as its source too)
    const double pd = team_prev<T>(d[S - 1]);
    const int32_t pi = team_prev<T>(id[S - 1]);
    const int32_t pl = team_prev<T>((int32_t)hi);
    const bool plt = (pl != 0) & (sub > 0);
#pragma unroll
    for (int j = S - 1; j > 0; --j) {
      const bool lo = cw & cand_lt(cd, cq, d[j - 1], id[j - 1]);
      const double nd = lo ? d[j - 1] : (hi ? cd : d[j]);
      const int32_t ni = lo ? id[j - 1] : (hi ? cq : id[j]);
      d[j] = nd;
      id[j] = ni;
      hi = lo;
    }
    const double nd = plt ? pd : (hi ? cd : d[0]);
    const int32_t ni = plt ? pi : (hi ? cq : id[0]);
    d[0] = nd;
    id[0] = ni;
    kd = team_bcast<T, T - 1>(d[S - 1]);
    ki = team_bcast<T, T - 1>(id[S - 1]);
  }

  // every lane offers one candidate (+inf, INT_MAX for none); a team
  // inserts its lanes' candidates in lane order, each tested against the
  // k-th entry as it stands after the ones before
  __device__ __forceinline__ void offer_team(double dd, int32_t q) {
    const bool w = dd <= kd;
    if (__ballot(w) == 0) return;
    take_all(dd, q, std::make_integer_sequence<int, T>{});
  }
  template <int... R>
  __device__ __forceinline__ void take_all(double dd, int32_t q, std::integer_sequence<int, R...>) {
    (take<R>(dd, q), ...);
  }

  // each lane writes its slots' part of the row
  __device__ __forceinline__ void write(int k, int32_t *out_ids, double *out_d2) const {
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const int g = sub * S + j;
      if (g >= KT - k) {
        const int o = g - (KT - k);
        out_ids[o] = id[j] == INT_MAX ? -1 : id[j];
        out_d2[o] = d[j];
      }
    }
  }
};

// Lanes per query of the all-points rows, per k bucket (0: one lane per
// query).  10M points, rows identical: teams of 8 at k = 64 and 100 took
// 75.7 and 138.6 ms on uniform points (62.6 and 116.7 on sphere surfaces)
// against 83.3 and 192.8 (71.6 and 156.7) for teams of 4, whose 25 slots
// per lane at k = 100 left one wavefront per SIMD; at k = 50 the two sizes
// split (uniform 62.7 against 60.2 ms, spheres 50.8 against 53.4).
template <int K>
constexpr int team_size() {
  return K > 50 ? 8 : (K > 16 ? 4 : 0);
}
// The same for external queries, whose sparse sets gain from teams from
// k = 8 on (1M queries into 10M uniform points, rows identical: k = 8 / 10
// / 12 / 16 in 4.30 / 4.65 / 5.00 / 6.55 ms against 4.46 / 5.19 / 5.99 /
// 8.53 ms with one lane per query; k = 4: 3.58 against 3.12 ms); see
// launch_knn_ext for the choice at k = 8-16.
template <int K>
constexpr int ext_team_size() {
  return K > 16 ? team_size<K>() : (K >= 8 ? 4 : 0);
}

// Per k bucket with one lane per query (k <= 16): the candidate set, and
// whether the set is filled by a sorting network (not k = 12, where the
// fill adds two spilled dwords under the 96-VGPR cap and the query
// measured 20% slower, while k = 8-16 otherwise gain 1-3%).
template <int K>
struct HeapFor {
  using type = Heap<K>;
  static constexpr bool sorted_fill = K != 12;
};

// withinBox(C, p, -r) of Algorithm 3, squared: p in the box and every face
// strictly farther than the k-th d2 (never true while N holds fewer than k,
// because the k-th d2 is then +inf).
template <int D>
__device__ __forceinline__ bool ball_inside(double px, double py, double pz, const double *lo,
                                            const double *hi, double kth) {
  const double p[3] = {px, py, pz};
#pragma unroll
  for (int c = 0; c < D; ++c) {
    if (p[c] < lo[c] || p[c] > hi[c]) return false;
    const double a = p[c] - lo[c], b = hi[c] - p[c];
    if (!(a * a > kth) || !(b * b > kth)) return false;
  }
  return true;
}

__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// sorted positions scored on either side of a query group before its walk
// (all-points rows), per k bucket: 48 for k > 50, 32 elsewhere (in lane
// teams 32, 48 and 64 measured within 1% of each other at k = 32, 50 and
// 100)
template <int K>
constexpr int64_t prescore_reach() {
  return K >= 64 ? 48 : 32;
}

// maximum of v over the wavefront (every lane gets it)
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return __builtin_amdgcn_readfirstlane(v);
}

// one staged candidate point (32 bytes: two 16-byte LDS reads)
struct Cand {
  double x, y, z;
  int32_t id;
  int32_t pad;
};

// The per-lane state of one wavefront's shared search.
template <int D, int K, bool kExt = false, bool kPool = false, bool kTeam = false>
struct WaveSearch {
  const TreeView &t;
  Cand *stage;                   // this wavefront's 64-entry LDS slice (candidates)
  double px, py, pz;             // this lane's query
  int32_t self;                  // excluded id (-1 for external queries)
  bool valid;                    // lane holds a query
  int32_t skip_lo, skip_hi;      // sorted positions already scored (all lanes)
  int32_t own_lo, own_n;         // external queries: this lane's scored leaf
  int32_t own_pool = -1;         // pool entry of this lane's query (never its own neighbour)
  int64_t budget;                // walk bound (never reached on a valid tree)
  bool gave_up = false;          // the walk stopped before it finished
  uint64_t key_ref;              // Morton key of the group's middle query (child order)
  // lanes per query in teams
  static constexpr int kTS = kExt ? ext_team_size<K>() : team_size<K>();
  static constexpr int kT = kTS > 0 ? kTS : 4;
  std::conditional_t<kTeam, TeamSet<K, kT>, typename HeapFor<K>::type> h;
  __device__ __forceinline__ WaveSearch(const TreeView &t_, Cand *stage_) : t(t_), stage(stage_) {}

  __device__ __forceinline__ bool wants(const double *lo, const double *hi) const {
    const bool w = box_dist2<D>(px, py, pz, lo, hi) <= h.kth();
    return __ballot(w) != 0;
  }

  // Every lane scores the sorted positions [a, b] around its group (the
  // walk then skips them), each in its own order: lane l (own position
  // a + o) takes at step s the position a + ((o + m) mod cnt) for s odd and
  // a + ((o - m) mod cnt) for s even, m = (s + 1) / 2, so it meets its
  // Morton neighbours first and every other position of [a, b] exactly
  // once.  Its k-th distance tightens sooner than in the shared order, and
  // fewer later candidates enter.  The stage holds the whole window.
  // For the register sets, the first min(k, cnt - 1) steps fill the empty
  // set without insertions: each lane stores those candidates in its slots
  // and sorts them (Heap::sort_slots), which leaves the set as that many
  // insertions would.
  __device__ __forceinline__ void prescore_near_first(int64_t a, int64_t b, int64_t own, int k) {
    const int lane = threadIdx.x & 63;
    const int cnt = (int)(b - a + 1);  // <= 64 + 2 prescore_reach<K>() entries of the stage
    for (int j = lane; j < cnt; j += 64) {
      Cand q;
      q.x = t.X[a + j];
      q.y = t.Y[a + j];
      q.z = D == 3 ? t.Z[a + j] : 0.0;
      q.id = t.id[a + j];
      q.pad = 0;
      stage[j] = q;
    }
    __builtin_amdgcn_wave_barrier();
    const int o = valid ? (int)(own - a) : 0;
    int s0 = 1;
    if constexpr (HeapFor<K>::sorted_fill) {
      // f = min(k, cnt - 1) candidates: slot s - 1 takes step s's candidate
      // for s <= f, an empty entry (+inf, INT_MAX) for f < s <= k and the
      // padding (-inf, INT_MIN) for s > k.  Sorted, the slots hold what
      // init and f insertions leave: the padding, the candidates ascending,
      // then the empty entries.  (Ids are distinct, so the order is total.)
      const int f = min(k, cnt - 1);
#pragma unroll
      for (int s = 1; s <= K; ++s) {
        const int m = (s + 1) >> 1;
        int j = (s & 1) ? o + m : o - m;
        j = j >= cnt ? j - cnt : (j < 0 ? j + cnt : j);
        const Cand q = stage[s <= f ? j : 0];
        const double dd = dist2<D>(px, py, pz, q.x, q.y, q.z);
        // a deleted point still in its slot (NaN) fills as an empty entry:
        // the network needs ordered values
        const bool real = s <= f && !isnan(dd);
        if (valid) {
          h.d[s - 1] = real ? dd : (s <= k ? INFINITY : -INFINITY);
          h.id[s - 1] = real ? q.id : (s <= k ? INT_MAX : INT_MIN);
        }
      }
      h.sort_slots();
      s0 = f + 1;
    }
    for (int s = s0; s < cnt; ++s) {
      const int m = (s + 1) >> 1;
      int j = (s & 1) ? o + m : o - m;
      j = j >= cnt ? j - cnt : (j < 0 ? j + cnt : j);
      const Cand q = stage[j];
      const double dd = dist2<D>(px, py, pz, q.x, q.y, q.z);
      h.offer(dd, q.id);
    }
    __builtin_amdgcn_wave_barrier();
    skip_lo = uni((int32_t)a);
    skip_hi = uni((int32_t)b);
  }

  // prescore_near_first for lane teams: the team's kT lanes take the steps
  // of its query's near-first order in turns (lane `sub` takes steps
  // 1 + sub, 1 + kT + sub, ...), each round offering kT candidates to the
  // team.
  __device__ __forceinline__ void prescore_team(int64_t a, int64_t b, int64_t own) {
    const int lane = threadIdx.x & 63;
    const int sub = lane & (kT - 1);
    const int cnt = (int)(b - a + 1);  // <= 64 / kT + 2 prescore_reach<K>() entries of the stage
    for (int j = lane; j < cnt; j += 64) {
      Cand q;
      q.x = t.X[a + j];
      q.y = t.Y[a + j];
      q.z = D == 3 ? t.Z[a + j] : 0.0;
      q.id = t.id[a + j];
      q.pad = 0;
      stage[j] = q;
    }
    __builtin_amdgcn_wave_barrier();
    const int o = valid ? (int)(own - a) : 0;
    for (int s0 = 1; s0 < cnt; s0 += kT) {
      const int s = s0 + sub;
      const int m = (s + 1) >> 1;
      int j = (s & 1) ? o + m : o - m;
      j = j >= cnt ? j - cnt : (j < 0 ? j + cnt : j);
      const bool in = s < cnt;
      const Cand q = stage[in ? j : 0];
      const double dd = dist2<D>(px, py, pz, q.x, q.y, q.z);
      h.offer_team(in ? dd : INFINITY, in ? q.id : INT_MAX);
    }
    __builtin_amdgcn_wave_barrier();
    skip_lo = uni((int32_t)a);
    skip_hi = uni((int32_t)b);
  }

  // scan_leaf for lane teams: the team's lanes score every kT-th point of
  // each staged chunk and the team takes them kT at a time
  __device__ __forceinline__ void scan_leaf_team(int32_t leaf) {
    const int lane = threadIdx.x & 63;
    const int sub = lane & (kT - 1);
    const int32_t b = uni(t.leaf_begin[leaf]), e = uni(t.leaf_begin[leaf + 1]);
    int32_t pn = 0, pb = 0;
    if constexpr (kPool) {
      pn = uni(t.ovf_cnt[leaf]);
      pb = pn > 0 ? uni(t.ovf_blk[leaf]) * kOvfBlock : 0;
    }
    const int32_t ev = e + pn;
    const int32_t skip_end = kPool ? min(skip_hi + 1, e) : skip_hi + 1;
    for (int32_t c = b; c < ev; c += 64) {
      const int32_t j = c + lane;
      if (j < e) {
        Cand q;
        q.x = t.X[j];
        q.y = t.Y[j];
        q.z = D == 3 ? t.Z[j] : 0.0;
        q.id = t.id[j];
        q.pad = 0;
        stage[lane] = q;
      } else if (kPool && j < ev) {
        const int32_t x = pb + (j - e);
        Cand q;
        q.x = t.pX[x];
        q.y = t.pY[x];
        q.z = D == 3 ? t.pZ[x] : 0.0;
        q.id = t.pid[x];
        q.pad = 0;
        stage[lane] = q;
      }
      __builtin_amdgcn_wave_barrier();
      const int32_t cnt = min(64, ev - c);
      // skipped local range [sa, sb) (empty when sa >= sb)
      const int32_t sa = max(skip_lo - c, 0);
      const int32_t sb = min(skip_end - c, cnt);
      for (int32_t j0 = 0; j0 < cnt; j0 += kT) {
        if (j0 >= sa && j0 + kT <= sb) continue;  // kT skipped points
        const int32_t jj = j0 + sub;
        bool in = jj < cnt && !(jj >= sa && jj < sb);
        if constexpr (kExt) {
          // a point of the query's own leaf was scored before the walk; a
          // pool query never scores its own entry
          const int32_t pos = c + jj;
          const bool seen = !kPool || pos < e ? (uint32_t)(pos - own_lo) < (uint32_t)own_n
                                              : pb + (pos - e) == own_pool;
          in = in && !seen;
        }
        const Cand q = stage[in ? jj : 0];
        const double dd = dist2<D>(px, py, pz, q.x, q.y, q.z);
        h.offer_team(in ? dd : INFINITY, in ? q.id : INT_MAX);
      }
      __builtin_amdgcn_wave_barrier();
    }
  }

  // every lane scores every point of the leaf, except the sorted positions
  // [skip_lo, skip_hi] already scored by all lanes (for all-points rows they
  // hold every lane's own point, so no self test is needed here) and, for
  // external queries, the lane's own leaf
  __device__ __forceinline__ void scan_leaf(int32_t leaf) {
    if constexpr (kTeam)
      scan_leaf_team(leaf);
    else
      scan_leaf_lanes(leaf);
  }

  __device__ __forceinline__ void scan_leaf_lanes(int32_t leaf) {
    const int lane = threadIdx.x & 63;
    const int32_t b = uni(t.leaf_begin[leaf]), e = uni(t.leaf_begin[leaf + 1]);
    // points placed in this leaf by small inserts follow as virtual
    // positions [e, e + pn) (pool entries pb ...); they are never in the
    // skip range, and a deleted one has a NaN x and never enters
    int32_t pn = 0, pb = 0;
    if constexpr (kPool) {
      pn = uni(t.ovf_cnt[leaf]);
      pb = pn > 0 ? uni(t.ovf_blk[leaf]) * kOvfBlock : 0;
    }
    const int32_t ev = e + pn;
    const int32_t skip_end = kPool ? min(skip_hi + 1, e) : skip_hi + 1;
    for (int32_t c = b; c < ev; c += 64) {
      const int32_t j = c + lane;
      if (j < e) {
        Cand q;
        q.x = t.X[j];
        q.y = t.Y[j];
        q.z = D == 3 ? t.Z[j] : 0.0;
        q.id = t.id[j];
        q.pad = 0;
        stage[lane] = q;
      } else if (kPool && j < ev) {
        const int32_t x = pb + (j - e);
        Cand q;
        q.x = t.pX[x];
        q.y = t.pY[x];
        q.z = D == 3 ? t.pZ[x] : 0.0;
        q.id = t.pid[x];
        q.pad = 0;
        stage[lane] = q;
      }
      __builtin_amdgcn_wave_barrier();
      const int32_t cnt = min(64, ev - c);
      // skipped local range [sa, sb); sa = cnt when it is empty
      int32_t sa = max(skip_lo - c, 0);
      const int32_t sb = min(skip_end - c, cnt);
      if (sa >= sb) sa = cnt;
      for (int32_t jj = 0; jj < cnt; ++jj) {
        if (jj == sa) {
          jj = sb;
          if (jj >= cnt) break;
        }
        const Cand q = stage[jj];
        const double dd = dist2<D>(px, py, pz, q.x, q.y, q.z);
        if constexpr (kExt) {
          // a point of the lane's own leaf was scored before the walk; a
          // pool query never scores its own entry
          const int32_t pos = c + jj;
          const bool seen = !kPool || pos < e ? (uint32_t)(pos - own_lo) < (uint32_t)own_n
                                              : pb + (pos - e) == own_pool;
          h.template offer<true>(seen ? INFINITY : dd, seen ? INT_MAX : q.id);
        } else {
          // (the split shift pays off in the walk for k >= 16)
          h.template offer<(K >= 16)>(dd, q.id);
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
  }

  // searchDown (Algorithm 2) below internal node `top`, whose own box the
  // caller has already tested.  The walk is the same on every lane, so its
  // stack of pending (node, side) links is one VGPR holding entry i in lane
  // i (a lane select to push, readlane to pop: no memory traffic).  Each
  // step tests one child box with the current k-th distance; entering an
  // internal node pushes its farther child and tests the nearer one first.  Split bits strictly
  // decrease downwards and lie in [0, 64) below a tree or cloud root, so a
  // path holds at most 64 internal nodes and the stack at most 64 entries;
  // a deeper stack only occurs on a corrupted tree and ends the walk, like
  // the step budget.
  __device__ __forceinline__ void search_down(int32_t top) {
    int32_t stk = 0;
    int32_t sp = 0;
    int32_t n = top;
    int s = -1;  // -1: entering n, child order not chosen yet
    while (--budget > 0) {
      const INode *N = &t.inode[n];
      if (s < 0) {
        // nearer child first: the side of the split holding the reference
        // point's cell (an order heuristic only; it never changes the rows)
        const int bit = uni(N->bit);
        const int first = bit < 64 ? (int)((key_ref >> bit) & 1) : 0;
        if (sp >= 64) {
          gave_up = true;
          return;
        }
        if ((int)(threadIdx.x & 63) == sp) stk = (n << 1) | (1 - first);
        ++sp;
        s = first;
      }
      if (wants(N->lo[s], N->hi[s])) {
        const int32_t ch = uni(N->child[s]);
        if (ch >= 0) {
          n = ch;
          s = -1;
          continue;
        }
        scan_leaf(~ch);
      }
      if (sp == 0) return;
      --sp;
      const int32_t e = __builtin_amdgcn_readlane(stk, sp);
      n = e >> 1;
      s = e & 1;
    }
  }

  // the subtree of G (internal node, or leaf ~G), then the climb from G
  __device__ __forceinline__ void run_from(int32_t G) {
    int32_t link;
    if (G < 0) {
      scan_leaf(~G);
      link = uni(t.leaf_parent[~G]);
    } else {
      search_down(G);
      link = uni(t.inode[G].parent);
    }
    while (link >= 0 && --budget > 0) {
      const int32_t p = link >> 1;
      const int side = link & 1;
      const INode *P = &t.inode[p];
      if (uni(P->bit) >= 64) break;  // a forest's cloud boundary: never cross it
      const bool out = valid && !ball_inside<D>(px, py, pz, P->lo[side], P->hi[side], h.kth());
      if (__ballot(out) == 0) break;
      const int os = 1 - side;
      if (wants(P->lo[os], P->hi[os])) {
        const int32_t ch = uni(P->child[os]);
        if (ch < 0) scan_leaf(~ch);
        else search_down(ch);
      }
      link = uni(P->parent);
    }
    if (budget <= 0) gave_up = true;
  }

  // A search that gave up (a corrupted tree, or the step limit a test sets)
  // is counted where the next synchronising call of the library reads it:
  // its rows are not exact, and the tree is reported broken.
  __device__ __forceinline__ void report() const {
    if (gave_up && (threadIdx.x & 63) == 0) atomicAdd(t.walk_err, 1);
  }
};

// Workgroups are dealt to the chip's 8 XCDs round-robin (workgroup h runs on
// XCD h mod 8), and every XCD has its own L2.  This maps hardware workgroup h
// to a logical one so that each XCD takes one contiguous run of logical
// workgroups: neighbouring query groups share most of their nodes and
// leaves, which then stay in one L2 instead of being fetched by all eight.
// The map is a bijection on [0, nb): XCD x owns nb/8 logical workgroups,
// plus one if x < nb mod 8.  (Used for all-points rows, where it cuts the
// query's L2-miss traffic about fourfold; external queries measured slower
// with it and keep the plain order.)
__device__ __forceinline__ uint32_t xcd_block(uint32_t h, uint32_t nb) {
  constexpr uint32_t kXcd = 8;
  const uint32_t x = h % kXcd, local = h / kXcd, q = nb / kXcd, r = nb % kXcd;
  return x * q + min(x, r) + local;
}

// All-points rows: wavefront w answers sorted positions [64w, 64w + 64).
// LDS per wavefront: the candidate stage, which holds the whole prescore
// window (the group and prescore_reach<K>() positions on either side).
template <int K>
constexpr size_t wave_lds_bytes() {
  return (64 + 2 * prescore_reach<K>()) * sizeof(Cand);
}

// All-points rows in lane teams (TeamSet) for these buckets; their LDS is
// the candidate stage only.  10M uniform points, rows identical: k = 20 /
// 24 / 32 / 40 / 50 / 64 / 100 in 24.3 / 29.8 / 36.0 / 53.1 / 67.3 / 112 /
// 336 ms against 26.3 / 32.8 / 49.2 / 76.4 / 101.6 / 231 / 489 ms with a
// set per lane (before the register caps below); k = 16 slower in teams
// (21.7 against 17.6 ms).
template <int K>
constexpr bool all_team() {
  return team_size<K>() > 0;
}
template <int K>
constexpr size_t all_lds_bytes() {
  return wave_lds_bytes<K>();
}

// Wavefronts per workgroup of a query launch: the requested 1, 2 or 4,
// halved while the workgroup's LDS would exceed one CU's 160 KiB (a stage
// of at most 160 candidates, 5 KB per wavefront, never comes near it).
template <int K, bool kAll = false>
int fit_waves(int want) {
  const size_t per = kAll ? all_lds_bytes<K>() : wave_lds_bytes<K>();
  int w = want == 2 || want == 4 ? want : 1;
  while (w > 1 && (size_t)w * per > 160 * 1024) w >>= 1;
  return w;
}

template <int D, int K, bool E, bool P, bool TM>
__device__ __forceinline__ void bind_lds(WaveSearch<D, K, E, P, TM> &s, char *smem, int w) {
  char *base = smem + (size_t)w * (TM ? all_lds_bytes<K>() : wave_lds_bytes<K>());
  s.stage = reinterpret_cast<Cand *>(base);
}

// Register budget of the all-points kernel.  At k = 10 it needs 85 VGPRs
// (5 wavefronts per SIMD); capped at 80 it keeps 6 resident and spills 7
// dwords to scratch (reloaded once per node or leaf step, never inside the
// insertion), which measured 3-4% faster.  At k = 12, 98 VGPRs (4 per SIMD)
// capped at 96 gives 5 and measured 7% faster.  The lane-team buckets
// (k >= 17) trade a few spilled dwords for occupancy, 10M uniform points:
// k = 20 at 80 VGPRs (6 per SIMD) 24.3 -> 23.4 ms, k = 24, 32 and 40 at 96
// (5) 29.8 -> 27.3, 36.0 -> 33.9 and 53.1 -> 45.2 ms, k = 50 at 128 (4)
// 67.3 -> 60.2 ms; in teams of 8, k = 64 at 96 (5) 81.3 -> 75.7 ms and
// k = 100 at 128 (4) 157.0 -> 138.6 ms.  Other buckets keep the compiler's
// choice (caps that spill inside the insertion, k = 12 at 80 or k = 16 at
// 96, run up to twice as long).
template <int K>
constexpr int knn_all_min_waves() {
  return K == 10 || K == 20 ? 6
         : K == 12 || K == 24 || K == 32 || K == 40 ? 5
         : K == 64 ? 5
         : K == 50 || K == 100 ? 4
                               : 1;
}

// The all-points rows of sorted positions [g0, last] (at most 64), which
// lie in the cloud [c_lo, c_hi] (the whole tree for a single tree), one
// query per lane.  `smem` is the workgroup's dynamic LDS, w the wavefront's
// index in the workgroup.
template <int D, int K, bool kPool>
__device__ __forceinline__ void all_points_lanes(const TreeView &t, int k,
                                                 int32_t *__restrict__ out_ids,
                                                 double *__restrict__ out_d2, int64_t g0,
                                                 int64_t last, int64_t c_lo, int64_t c_hi,
                                                 char *smem, int w) {
  const int lane = threadIdx.x & 63;
  const int64_t i = min(g0 + lane, last);
  WaveSearch<D, K, false, kPool> s(t, nullptr);
  bind_lds(s, smem, w);
  s.px = t.X[i];
  s.py = t.Y[i];
  s.pz = D == 3 ? t.Z[i] : 0.0;
  // (a point deleted by a small batch keeps its slot with a NaN x: no query)
  s.valid = g0 + lane <= last && !isnan(s.px);
  s.self = t.id[i];
  const int mid = (int)((last - g0) / 2);
  s.budget = t.walk_limit > 0 ? t.walk_limit : 4 * t.n + 256;
  s.key_ref = uni((int32_t)(t.key[g0 + mid] >> 32));
  s.key_ref = (s.key_ref << 32) | (uint32_t)uni((int32_t)t.key[g0 + mid]);
  s.h.init(k, s.valid);
  // score first the sorted positions around the group, within its cloud:
  // the group's own points and prescore_reach<K>() on either side (Morton neighbours
  // of every lane).  This tightens every lane's k-th distance before the
  // walk, which then skips these positions.
  s.prescore_near_first(max(c_lo, g0 - prescore_reach<K>()),
                        min(c_hi, last + prescore_reach<K>()), g0 + lane, k);
  // lowest common ancestor of the group's leaves
  const int32_t lf = uni(t.leaf_of[g0]), ll = uni(t.leaf_of[last]);
  int32_t G = ~lf;
  if (lf != ll) {
    int32_t x = uni(t.leaf_parent[lf]) >> 1;
    for (int guard = 0; guard < 130 && uni(t.inode[x].last_leaf) < ll; ++guard) {
      const int32_t par = uni(t.inode[x].parent);
      if (par < 0) break;
      x = par >> 1;
    }
    G = x;
  }
  s.run_from(G);
  s.report();
  if (s.valid) s.h.write(k, out_ids + (int64_t)s.self * k, out_d2 + (int64_t)s.self * k);
}

// The same rows in lane teams (TeamSet): sorted positions [g0, last], at
// most 64 / T, one query per T lanes.
template <int D, int K, bool kPool>
__device__ __forceinline__ void all_points_team(const TreeView &t, int k,
                                                int32_t *__restrict__ out_ids,
                                                double *__restrict__ out_d2, int64_t g0,
                                                int64_t last, int64_t c_lo, int64_t c_hi,
                                                char *smem, int w) {
  constexpr int T = team_size<K>();
  const int lane = threadIdx.x & 63;
  const int64_t i = min(g0 + lane / T, last);
  WaveSearch<D, K, false, kPool, true> s(t, nullptr);
  bind_lds(s, smem, w);
  s.px = t.X[i];
  s.py = t.Y[i];
  s.pz = D == 3 ? t.Z[i] : 0.0;
  s.valid = g0 + lane / T <= last && !isnan(s.px);
  s.self = t.id[i];
  const int mid = (int)((last - g0) / 2);
  s.budget = t.walk_limit > 0 ? t.walk_limit : 4 * t.n + 256;
  s.key_ref = uni((int32_t)(t.key[g0 + mid] >> 32));
  s.key_ref = (s.key_ref << 32) | (uint32_t)uni((int32_t)t.key[g0 + mid]);
  s.h.init(k, s.valid);
  s.prescore_team(max(c_lo, g0 - prescore_reach<K>()), min(c_hi, last + prescore_reach<K>()), i);
  const int32_t lf = uni(t.leaf_of[g0]), ll = uni(t.leaf_of[last]);
  int32_t G = ~lf;
  if (lf != ll) {
    int32_t x = uni(t.leaf_parent[lf]) >> 1;
    for (int guard = 0; guard < 130 && uni(t.inode[x].last_leaf) < ll; ++guard) {
      const int32_t par = uni(t.inode[x].parent);
      if (par < 0) break;
      x = par >> 1;
    }
    G = x;
  }
  s.run_from(G);
  s.report();
  if (s.valid) s.h.write(k, out_ids + (int64_t)s.self * k, out_d2 + (int64_t)s.self * k);
}

// One wavefront answers the all-points rows of sorted positions [g0, last]
// (at most 64) of the cloud [c_lo, c_hi]: in one group of 64 lanes, or,
// for the team buckets, in groups of 64 / T queries one after the other.
template <int D, int K, bool kPool>
__device__ __forceinline__ void all_points_group(const TreeView &t, int k,
                                                 int32_t *__restrict__ out_ids,
                                                 double *__restrict__ out_d2, int64_t g0,
                                                 int64_t last, int64_t c_lo, int64_t c_hi,
                                                 char *smem, int w) {
  if constexpr (all_team<K>()) {
    constexpr int Q = 64 / team_size<K>();  // queries per team group
    for (int64_t sg = g0; sg <= last; sg += Q)
      all_points_team<D, K, kPool>(t, k, out_ids, out_d2, sg, min(sg + Q - 1, last), c_lo, c_hi,
                                   smem, w);
  } else {
    all_points_lanes<D, K, kPool>(t, k, out_ids, out_d2, g0, last, c_lo, c_hi, smem, w);
  }
}

template <int D, int K, bool kPool>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(knn_all_min_waves<K>())))
k_knn_all(TreeView t, int k, int32_t *__restrict__ out_ids,
                                                 double *__restrict__ out_d2,
                                                 const int4 *__restrict__ groups, int64_t ngroups) {
  extern __shared__ __align__(16) char smem[];
  const int w = threadIdx.x >> 6;
  const int64_t gw = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + w;
  int64_t g0, last, c_lo, c_hi;  // the group, and the cloud that holds it
  if (groups) {
    if (gw >= ngroups) return;
    g0 = uni(groups[gw].x);
    last = uni(groups[gw].y);
    c_lo = uni(groups[gw].z);
    c_hi = uni(groups[gw].w);
  } else {
    g0 = gw * 64;
    if (g0 >= t.n) return;
    last = min(g0 + 63, t.n - 1);
    c_lo = 0;
    c_hi = t.n - 1;
  }
  all_points_group<D, K, kPool>(t, k, out_ids, out_d2, g0, last, c_lo, c_hi, smem, w);
}

// External rows: wavefront w answers the Morton-sorted queries
// order[64w .. 64w + 64); row r of the output belongs to query r.
// Register budget of the external-query and root-based kernels: in lane
// teams the all-points kernel's caps; with one lane per query, k = 16
// capped at 128 VGPRs (4 wavefronts per SIMD instead of 3) measured 9-12%
// faster, and the other buckets keep the compiler's choice.
template <int K>
constexpr int knn_root_min_waves() {
  return K == 16 ? 4 : 1;
}
template <int K, bool kTeam>
constexpr int knn_ext_min_waves() {
  return kTeam ? knn_all_min_waves<K>() : knn_root_min_waves<K>();
}

// One wavefront's external rows for the Morton-sorted queries
// order[g0 .. last]: up to 64 with one lane per query, or up to 64 / T in
// lane teams (kTeam).
template <int D, int K, bool kPool, bool kTeam>
__device__ __forceinline__ void ext_group(const TreeView &t, const double *__restrict__ q,
                                          int64_t qs, const uint64_t *__restrict__ qkey,
                                          const int32_t *__restrict__ order, int64_t g0,
                                          int64_t last, int k, int32_t *__restrict__ out_ids,
                                          double *__restrict__ out_d2,
                                          const int32_t *__restrict__ row_ids, char *smem, int w) {
  using Search = WaveSearch<D, K, true, kPool, kTeam>;
  constexpr int T = kTeam ? Search::kT : 1;
  const int lane = threadIdx.x & 63;
  const int sub = lane % T;
  const int64_t i = min(g0 + lane / T, last);
  const int32_t r = order[i];
  Search s(t, nullptr);
  bind_lds(s, smem, w);
  s.px = q[r];
  s.py = q[qs + r];
  s.pz = D == 3 ? q[2 * qs + r] : 0.0;
  s.valid = g0 + lane / T <= last;
  // row_ids: the queries are the tree's own pool entries (points of small
  // inserts): row = the point's id, the entry itself excluded, a deleted
  // entry (NaN) answers nothing
  int64_t row = r;
  if (row_ids) {
    row = row_ids[r];
    s.own_pool = r;
    s.valid = s.valid && !isnan(s.px);
  }
  s.self = -1;
  const int mid = (int)((last - g0) / 2);
  s.budget = t.walk_limit > 0 ? t.walk_limit : 4 * t.n + 256;
  s.skip_lo = 1;
  s.skip_hi = 0;
  s.key_ref = uni((int32_t)(qkey[g0 + mid] >> 32));
  s.key_ref = (s.key_ref << 32) | (uint32_t)uni((int32_t)qkey[g0 + mid]);
  s.h.init(k, s.valid);
  int32_t node = uni(t.meta[kMetaRoot]);
  if (node != kNoRoot) {
    // descend by the Morton bits (the bit-based search of Section 2) with the
    // group's first and last keys; where they part, every key of the sorted
    // group is below: that node is the group's common ancestor
    const uint64_t k0 = qkey[g0], k1 = qkey[last];
    for (int guard = 0; node >= 0 && guard < 66; ++guard) {
      const INode *N = &t.inode[node];
      const int bit = uni(N->bit);
      const int b0 = (int)((k0 >> bit) & 1), b1 = (int)((k1 >> bit) & 1);
      if (b0 != b1) break;
      node = uni(N->child[b0]);
    }
    // every query first scores the leaf its own key leads to (the bit-based
    // descent of Section 2, per query), which gives it a k-th distance from
    // its own neighbourhood before the shared walk; the walk skips those
    // points for that query (a team's lanes take every T-th of them)
    {
      const uint64_t myk = qkey[i];
      int32_t x = node;
      for (int guard = 0; x >= 0 && guard < 66; ++guard) {
        const INode *N = &t.inode[x];
        const int bit = N->bit;
        x = N->child[(int)((myk >> bit) & 1)];
      }
      // (x >= 0 here only on a corrupted tree: nothing is scored then, and
      // the search is reported as given up)
      if (__ballot(s.valid && x >= 0) != 0) s.gave_up = true;
      const int32_t lb = x < 0 ? t.leaf_begin[~x] : 0, le = x < 0 ? t.leaf_begin[~x + 1] : 0;
      s.own_lo = lb;
      s.own_n = s.valid ? le - lb : 0;
      const int rounds = wave_max((s.own_n + T - 1) / T);
      for (int rr = 0; rr < rounds; ++rr) {
        const int jj = rr * T + sub;
        const bool in = jj < s.own_n;
        const int64_t j = lb + (in ? jj : 0);
        const double dd = dist2<D>(s.px, s.py, s.pz, t.X[j], t.Y[j], D == 3 ? t.Z[j] : 0.0);
        const int32_t q = t.id[j];
        if constexpr (kTeam)
          s.h.offer_team(in ? dd : INFINITY, in ? q : INT_MAX);
        else
          s.h.template offer<true>(in ? dd : INFINITY, in ? q : INT_MAX);
      }
    }
    s.run_from(node);
    s.report();
  }
  if (s.valid) s.h.write(k, out_ids + row * k, out_d2 + row * k);
}

template <int D, int K, bool kPool, bool kTeam>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(knn_ext_min_waves<K, kTeam>())))
k_knn_ext(TreeView t, const double *__restrict__ q, int64_t qs,
                                                 const uint64_t *__restrict__ qkey,
                                                 const int32_t *__restrict__ order, int64_t m,
                                                 int k, int32_t *__restrict__ out_ids,
                                                 double *__restrict__ out_d2,
                                                 const int32_t *__restrict__ row_ids) {
  extern __shared__ __align__(16) char smem[];
  const int w = threadIdx.x >> 6;
  const int64_t g0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + w) * 64;
  if (g0 >= m) return;
  const int64_t last = min(g0 + 63, m - 1);
  if constexpr (kTeam) {
    constexpr int Q = 64 / WaveSearch<D, K, true, kPool, true>::kT;  // queries per team group
    for (int64_t sg = g0; sg <= last; sg += Q)
      ext_group<D, K, kPool, true>(t, q, qs, qkey, order, sg, min(sg + Q - 1, last), k, out_ids,
                                   out_d2, row_ids, smem, w);
  } else {
    ext_group<D, K, kPool, false>(t, q, qs, qkey, order, g0, last, k, out_ids, out_d2, row_ids,
                                  smem, w);
  }
}

// Root-based rows (Section 2): Algorithm 2 from the root with an empty
// candidate set and no climb, the variant the paper contrasts with the
// leaf- and bit-based starts.  q == nullptr: all-points rows, wavefront w
// answering sorted positions [64w, 64w + 64) with each lane's own point
// excluded (a one-point "own" range of the external-query scan); otherwise
// Morton-presorted external queries as in k_knn_ext.  The shared walk is the
// same as everywhere else; only its start differs.

// One wavefront's root-based rows for positions [g0, last] (sorted tree
// positions, or Morton-sorted external queries): up to 64 with one lane per
// query, or up to 64 / T in lane teams (kTeam).
template <int D, int K, bool kPool, bool kTeam>
__device__ __forceinline__ void root_group(const TreeView &t, const double *__restrict__ q,
                                           int64_t qs, const uint64_t *__restrict__ qkey,
                                           const int32_t *__restrict__ order, int64_t g0,
                                           int64_t last, int k, int32_t *__restrict__ out_ids,
                                           double *__restrict__ out_d2,
                                           const int32_t *__restrict__ row_ids, char *smem, int w) {
  using Search = WaveSearch<D, K, true, kPool, kTeam>;
  constexpr int T = kTeam ? Search::kT : 1;
  const int lane = threadIdx.x & 63;
  const int64_t i = min(g0 + lane / T, last);
  const int mid = (int)((last - g0) / 2);
  Search s(t, nullptr);
  bind_lds(s, smem, w);
  s.valid = g0 + lane / T <= last;
  int64_t row;
  uint64_t kref;
  if (q) {
    const int32_t r = order[i];
    s.px = q[r];
    s.py = q[qs + r];
    s.pz = D == 3 ? q[2 * qs + r] : 0.0;
    s.own_lo = 0;
    s.own_n = 0;
    row = r;
    if (row_ids) {  // the tree's pool entries as queries (see k_knn_ext)
      row = row_ids[r];
      s.own_pool = r;
      s.valid = s.valid && !isnan(s.px);
    }
    kref = qkey[g0 + mid];
  } else {
    s.px = t.X[i];
    s.py = t.Y[i];
    s.pz = D == 3 ? t.Z[i] : 0.0;
    s.valid = s.valid && !isnan(s.px);
    s.own_lo = (int32_t)i;
    s.own_n = s.valid ? 1 : 0;
    row = t.id[i];
    kref = t.key[g0 + mid];
  }
  s.self = -1;
  s.budget = t.walk_limit > 0 ? t.walk_limit : 4 * t.n + 256;
  s.skip_lo = 1;
  s.skip_hi = 0;
  s.key_ref = uni((int32_t)(kref >> 32));
  s.key_ref = (s.key_ref << 32) | (uint32_t)uni((int32_t)kref);
  s.h.init(k, s.valid);
  const int32_t root = uni(t.meta[kMetaRoot]);
  if (root != kNoRoot) {
    // (the root's own box needs no test: the candidate set is empty)
    if (root < 0) s.scan_leaf(~root);
    else s.search_down(root);
    if (s.budget <= 0) s.gave_up = true;
    s.report();
  }
  if (s.valid) s.h.write(k, out_ids + row * k, out_d2 + row * k);
}

// Root-based rows in lane teams at k > 16, as the leaf-based all-points rows.
template <int D, int K, bool kPool>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    team_size<K>() > 0 ? knn_all_min_waves<K>() : knn_root_min_waves<K>())))
k_knn_root(TreeView t, const double *__restrict__ q, int64_t qs, const uint64_t *__restrict__ qkey,
           const int32_t *__restrict__ order, int64_t m, int k, int32_t *__restrict__ out_ids,
           double *__restrict__ out_d2, const int32_t *__restrict__ row_ids) {
  extern __shared__ __align__(16) char smem[];
  const int w = threadIdx.x >> 6;
  const int64_t g0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + w) * 64;
  if (g0 >= m) return;
  const int64_t last = min(g0 + 63, m - 1);
  if constexpr (team_size<K>() > 0) {
    constexpr int Q = 64 / WaveSearch<D, K, true, kPool, true>::kT;  // queries per team group
    for (int64_t sg = g0; sg <= last; sg += Q)
      root_group<D, K, kPool, true>(t, q, qs, qkey, order, sg, min(sg + Q - 1, last), k, out_ids,
                                    out_d2, row_ids, smem, w);
  } else {
    root_group<D, K, kPool, false>(t, q, qs, qkey, order, g0, last, k, out_ids, out_d2, row_ids,
                                   smem, w);
  }
}

template <int D, int K>
hipError_t launch_knn_root(const TreeView &t, const double *q, int64_t qs, const uint64_t *qkey,
                           const int32_t *order, int64_t m, int k, int32_t *ids, double *d2,
                           const int32_t *row_ids, hipStream_t s, int query_waves) {
  constexpr bool kTeam = team_size<K>() > 0;
  const int64_t waves = (m + 63) / 64;
  const int wpb = fit_waves<K, kTeam>(query_waves);
  const size_t lds = wpb * (kTeam ? all_lds_bytes<K>() : wave_lds_bytes<K>());
  // (the variant that scans leaves' side blocks only while small inserts are pending)
  const dim3 grid((unsigned)((waves + wpb - 1) / wpb)), block(64 * wpb);
  if (t.ovf_cnt)
    k_knn_root<D, K, true><<<grid, block, lds, s>>>(t, q, qs, qkey, order, m, k, ids, d2, row_ids);
  else
    k_knn_root<D, K, false><<<grid, block, lds, s>>>(t, q, qs, qkey, order, m, k, ids, d2, row_ids);
  return hipGetLastError();
}

template <int D, int K>
hipError_t launch_knn_all(const TreeView &t, int k, int32_t *ids, double *d2, hipStream_t s,
                          const int4 *groups, int64_t ngroups, int query_waves) {
  const int64_t waves = groups ? ngroups : (t.n + 63) / 64;
  const int wpb = fit_waves<K, true>(query_waves);
  const dim3 grid((unsigned)((waves + wpb - 1) / wpb)), block(64 * wpb);
  if (t.ovf_cnt)
    k_knn_all<D, K, true><<<grid, block, wpb * all_lds_bytes<K>(), s>>>(t, k, ids, d2, groups,
                                                                        ngroups);
  else
    k_knn_all<D, K, false><<<grid, block, wpb * all_lds_bytes<K>(), s>>>(t, k, ids, d2, groups,
                                                                         ngroups);
  return hipGetLastError();
}

template <int D, int K, bool kTeam>
hipError_t launch_knn_ext_as(const TreeView &t, const double *q, int64_t qs, const uint64_t *qkey,
                             const int32_t *order, int64_t m, int k, int32_t *ids, double *d2,
                             const int32_t *row_ids, hipStream_t s, int query_waves) {
  const int64_t waves = (m + 63) / 64;
  const int wpb = fit_waves<K, kTeam>(query_waves);
  const size_t lds = wpb * (kTeam ? all_lds_bytes<K>() : wave_lds_bytes<K>());
  const dim3 grid((unsigned)((waves + wpb - 1) / wpb)), block(64 * wpb);
  if (t.ovf_cnt)
    k_knn_ext<D, K, true, kTeam>
        <<<grid, block, lds, s>>>(t, q, qs, qkey, order, m, k, ids, d2, row_ids);
  else
    k_knn_ext<D, K, false, kTeam>
        <<<grid, block, lds, s>>>(t, q, qs, qkey, order, m, k, ids, d2, row_ids);
  return hipGetLastError();
}

// External queries run in lane teams from k = 17 on, and at k = 8-16 when
// they are sparse next to the tree (at most a quarter as many queries as
// points): a 64-query group of sparse queries spans many leaves, which the
// teams' 16-query groups cut, while dense queries (the tree's own points as
// queries, 10M into 10M) ran slower in teams at k <= 16 (uniform k = 10:
// 22.6 against 18.4 ms; Plummer 24.0 against 17.3; at k = 20: 29.2
// against 36.1 and 30.5 against 34.2 ms).
template <int D, int K>
hipError_t launch_knn_ext(const TreeView &t, const double *q, int64_t qs, const uint64_t *qkey,
                          const int32_t *order, int64_t m, int k, int32_t *ids, double *d2,
                          const int32_t *row_ids, hipStream_t s, int query_waves) {
  if constexpr (ext_team_size<K>() == 0)
    return launch_knn_ext_as<D, K, false>(t, q, qs, qkey, order, m, k, ids, d2, row_ids, s,
                                          query_waves);
  else if constexpr (K > 16)
    return launch_knn_ext_as<D, K, true>(t, q, qs, qkey, order, m, k, ids, d2, row_ids, s,
                                         query_waves);
  else if (4 * m <= t.n)
    return launch_knn_ext_as<D, K, true>(t, q, qs, qkey, order, m, k, ids, d2, row_ids, s,
                                         query_waves);
  else
    return launch_knn_ext_as<D, K, false>(t, q, qs, qkey, order, m, k, ids, d2, row_ids, s,
                                          query_waves);
}

// K buckets: a k between two buckets runs in the larger one (the padding
// slots cost registers, not correctness)
#define ZD_FOR_EACH_K(X) X(1) X(2) X(4) X(8) X(10) X(12) X(16) X(20) X(24) X(32) X(40) X(50) X(64) X(100)

inline int k_bucket(int k) {
  const int b[] = {1, 2, 4, 8, 10, 12, 16, 20, 24, 32, 40, 50, 64, 100};
  for (int x : b)
    if (k <= x) return x;
  return 100;
}

}  // namespace zd
