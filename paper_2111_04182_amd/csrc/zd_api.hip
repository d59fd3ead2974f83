// zd_api.hip -- the C ABI of libzd (see include/zd.h): argument checks, tree
// storage, and the order of the device passes behind each call.
#include "zd_internal.h"

#include <cmath>
#include <cstring>
#include <new>
#include <algorithm>
#include <mutex>
#include <queue>
#include <vector>

using namespace zd;

namespace {

// Point-side storage of one tree generation, all sized for n points.  An
// update builds the next generation from the current one and then releases
// the current one (stream-ordered), so no array ever needs slack.
struct Store {
  int64_t n = 0;
  uint64_t *key = nullptr;
  int32_t *id = nullptr;
  double *X = nullptr, *Y = nullptr, *Z = nullptr;
  int32_t *leaf_of = nullptr;
  int32_t *leaf_begin = nullptr;
  int32_t *leaf_parent = nullptr;
  INode *inode = nullptr;
};

hipError_t store_alloc(Store &s, int64_t n, int dim, hipStream_t st) {
  s.n = n;
  hipError_t e = dev_alloc_n(&s.key, n, st);
  if (e == hipSuccess) e = dev_alloc_n(&s.id, n, st);
  if (e == hipSuccess) e = dev_alloc_n(&s.X, n, st);
  if (e == hipSuccess) e = dev_alloc_n(&s.Y, n, st);
  if (e == hipSuccess) e = dim == 3 ? dev_alloc_n(&s.Z, n, st) : hipSuccess;
  if (e == hipSuccess) e = dev_alloc_n(&s.leaf_of, n, st);
  if (e == hipSuccess) e = dev_alloc_n(&s.leaf_begin, n + 1, st);
  if (e == hipSuccess) e = dev_alloc_n(&s.leaf_parent, n, st);
  if (e == hipSuccess) e = dev_alloc_n(&s.inode, n, st);
  return e;
}

void store_release(Store &s, hipStream_t st) {
  dev_release(s.key, st);
  dev_release(s.id, st);
  dev_release(s.X, st);
  dev_release(s.Y, st);
  dev_release(s.Z, st);
  dev_release(s.leaf_of, st);
  dev_release(s.leaf_begin, st);
  dev_release(s.leaf_parent, st);
  dev_release(s.inode, st);
  s = Store{};
}

uint64_t splitmix64(uint64_t seed, uint64_t i) {
  // the published SplitMix64 mixer (Steele, Lea, Flood 2014) at seed + i*gamma
  uint64_t z = seed + i * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

zd_status to_status(hipError_t e) {
  if (e == hipSuccess) return ZD_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return ZD_ENOMEM;
  return ZD_EDEVICE;
}

}  // namespace

struct zd_tree_s {
  int dim = 0, L = 0;
  int qwaves = 1;  // wavefronts per workgroup of the query launches
  Geometry geo{};
  double hi[3] = {0, 0, 0};
  int64_t cap = 0;   // id capacity
  int64_t icap = 0;  // allocated length of the id arrays
  hipStream_t stream = nullptr;
  bool broken = false;
  int64_t walk_limit = 0;  // test hook: steps a search may take (0: unbounded in practice)
  Store st;
  int32_t *slot_of = nullptr;  // [icap] id -> sorted position, -1 if dead
  int32_t *mark = nullptr;     // [icap] zero between calls
  int32_t *meta = nullptr;     // [kMetaCount]
  double *root_box = nullptr;  // [6]
  int64_t live = 0;            // live points (sorted arrays and pool, minus deleted)
  // Small batches applied in place since the last relink (zd_update.hip):
  // the side pool of leaf blocks and the count of deleted points that still
  // hold their slot.
  struct Pending {
    int32_t *ovf_blk = nullptr;  // [nleaf] pool block of each leaf, -1: none
    int32_t *ovf_cnt = nullptr;  // [nleaf] points in it
    int64_t nleaf = 0;
    double *pxyz = nullptr;      // [dim][pcap] pool coordinates (NaN: unused or deleted)
    int32_t *pid = nullptr;      // [pcap]
    int32_t *blocks = nullptr;   // device count of blocks handed out
    int64_t pcap = 0;            // pool entries (blocks * kOvfBlock)
    int64_t nblocks = 0;         // blocks handed out (host mirror)
    int64_t n_pool = 0;          // points placed in the pool
    int64_t n_tomb = 0;          // deleted points holding their slot
    bool any() const { return n_pool > 0 || n_tomb > 0; }
  } pend;

  TreeView view() const {
    TreeView v;
    v.key = st.key;
    v.id = st.id;
    v.X = st.X;
    v.Y = st.Y;
    v.Z = st.Z;
    v.leaf_of = st.leaf_of;
    v.leaf_begin = st.leaf_begin;
    v.leaf_parent = st.leaf_parent;
    v.inode = st.inode;
    v.meta = meta;
    v.walk_err = meta + kMetaWalkErr;
    v.n = st.n;
    v.walk_limit = walk_limit;
    const bool pool = pend.n_pool > 0;
    v.ovf_blk = pool ? pend.ovf_blk : nullptr;
    v.ovf_cnt = pool ? pend.ovf_cnt : nullptr;
    v.pX = pend.pxyz;
    v.pY = pend.pxyz ? pend.pxyz + pend.pcap : nullptr;
    v.pZ = pend.pxyz && dim == 3 ? pend.pxyz + 2 * pend.pcap : nullptr;
    v.pid = pend.pid;
    return v;
  }

  BuildBuffers buffers(int32_t *flag) const {
    BuildBuffers b;
    b.key = st.key;
    b.id = st.id;
    b.X = st.X;
    b.Y = st.Y;
    b.Z = st.Z;
    b.leaf_of = st.leaf_of;
    b.leaf_begin = st.leaf_begin;
    b.leaf_parent = st.leaf_parent;
    b.inode = st.inode;
    b.meta = meta;
    b.root_box = root_box;
    b.flag = flag;
    return b;
  }
};

namespace {

// Order all later work of the tree after what was enqueued on its previous
// stream, then make `s` the tree's stream.
hipError_t bind_stream(zd_tree t, hipStream_t s) {
  if (s == t->stream) return hipSuccess;
  hipEvent_t ev;
  hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e != hipSuccess) return e;
  e = hipEventRecord(ev, t->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);
  (void)hipEventDestroy(ev);
  if (e == hipSuccess) t->stream = s;
  return e;
}

// Order a query on stream `s` after the tree's pending work on its own stream,
// and the tree's later work (updates, release) after the query, without
// changing the tree: concurrent queries on other streams only read it.
hipError_t join_query_stream(zd_tree t, hipStream_t s, bool after) {
  if (s == t->stream) return hipSuccess;
  hipEvent_t ev;
  hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e != hipSuccess) return e;
  e = after ? hipEventRecord(ev, s) : hipEventRecord(ev, t->stream);
  if (e == hipSuccess) e = after ? hipStreamWaitEvent(t->stream, ev, 0) : hipStreamWaitEvent(s, ev, 0);
  (void)hipEventDestroy(ev);
  return e;
}

void pending_release(zd_tree t) {
  hipStream_t s = t->stream;
  dev_release(t->pend.ovf_blk, s);
  dev_release(t->pend.ovf_cnt, s);
  dev_release(t->pend.pxyz, s);
  dev_release(t->pend.pid, s);
  dev_release(t->pend.blocks, s);
  t->pend = zd_tree_s::Pending{};
}

// Relink the tree over the points of t->st (keys sorted, coordinates and
// slot map in place).  A forest passes the cloud of every position and the
// leaf size of every cloud.
hipError_t relink(zd_tree t, const int32_t *seg = nullptr, const int32_t *seg_leaf = nullptr,
                  int32_t max_leaf = 0) {
  // leaves and nodes are renumbered: the per-leaf state of in-place small
  // batches goes (every caller has folded their points in, or has none)
  pending_release(t);
  hipStream_t s = t->stream;
  int32_t *flag = nullptr;
  hipError_t e = dev_alloc_n(&flag, t->st.n, s);
  if (e != hipSuccess) return e;
  BuildBuffers b = t->buffers(flag);
  b.seg = seg;
  b.seg_leaf = seg_leaf;
  b.max_leaf = max_leaf;
  e = build_tree_links(t->dim, t->L, t->st.n, b, s);
  dev_release(flag, s);
  return e;
}

// Grow the id arrays to hold `need` ids (old entries kept, new slots dead).
hipError_t grow_ids(zd_tree t, int64_t need) {
  if (need <= t->icap) return hipSuccess;
  hipStream_t s = t->stream;
  int64_t ncap = t->icap > 0 ? t->icap : 1024;
  while (ncap < need) ncap += ncap / 2 + 1;
  int32_t *slot = nullptr, *mark = nullptr;
  hipError_t e = dev_alloc_n(&slot, ncap, s);
  if (e == hipSuccess) e = dev_alloc_n(&mark, ncap, s);
  if (e == hipSuccess) e = fill_i32(slot, -1, ncap, s);
  if (e == hipSuccess) e = fill_i32(mark, 0, ncap, s);
  if (e == hipSuccess && t->cap > 0)
    e = hipMemcpyAsync(slot, t->slot_of, sizeof(int32_t) * (size_t)t->cap,
                       hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) {
    dev_release(slot, s);
    dev_release(mark, s);
    return e;
  }
  dev_release(t->slot_of, s);
  dev_release(t->mark, s);
  t->slot_of = slot;
  t->mark = mark;
  t->icap = ncap;
  return hipSuccess;
}

bool valid_query_waves(int32_t w) { return w == 0 || w == 1 || w == 2 || w == 4; }

bool finite3(const double *v, int dim) {
  for (int c = 0; c < dim; ++c)
    if (!std::isfinite(v[c])) return false;
  return true;
}


void destroy(zd_tree t) {
  if (!t) return;
  pending_release(t);
  hipStream_t s = t->stream;
  store_release(t->st, s);
  dev_release(t->slot_of, s);
  dev_release(t->mark, s);
  dev_release(t->meta, s);
  dev_release(t->root_box, s);
  delete t;
}

// `count` int32 words from device memory (count <= 16), read on stream s
// through the thread's pinned buffer (a pageable destination costs a staged
// copy).
hipError_t read_i32s(const int32_t *dptr, int32_t *out, int count, hipStream_t s) {
  int32_t *h = host_flag();
  hipError_t e =
      hipMemcpyAsync(h ? h : out, dptr, sizeof(int32_t) * count, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && h)
    for (int i = 0; i < count; ++i) out[i] = h[i];
  return e;
}

hipError_t read_i32(const int32_t *dptr, int32_t *out, hipStream_t s) {
  return read_i32s(dptr, out, 1, s);
}

// Read the tree's meta words (synchronises its stream).  A corrupted climb
// in the build or a search that gave up marks the tree broken: ZD_EDEVICE.
zd_status read_meta(zd_tree t, int32_t *meta) {
  hipError_t e = read_i32s(t->meta, meta, kMetaCount, t->stream);
  if (e != hipSuccess) {
    t->broken = true;
    return to_status(e);
  }
  if (meta[kMetaBuildErr] != 0 || meta[kMetaWalkErr] != 0) {
    t->broken = true;
    return ZD_EDEVICE;
  }
  return ZD_OK;
}

constexpr int64_t kMaxIds = (int64_t)INT32_MAX - 1;  // ids are int32, -1 pads

// Fold the small batches applied in place, and an optional batch of new
// points (ids id_base, id_base + 1, ...), back into the sorted arrays and
// relink: the tree then equals a fresh build of the live points again.
// Streaming passes as in an insert: the live sorted points compact in
// order, the live pool points and the batch are keyed and sorted by
// (key, id), and the two sorted lists merge.
hipError_t rebuild_live(zd_tree t, const double *bxyz, int64_t nb, int32_t id_base) {
  hipStream_t s = t->stream;
  const int dim = t->dim;
  zd_tree_s::Pending &pd = t->pend;
  const int64_t n = t->st.n, np = pd.nblocks * kOvfBlock;
  // 1. live flags of the sorted slots and pool entries, their positions,
  // and the counts: all live (total) and live sorted (na)
  int32_t *scan = nullptr;
  hipError_t e = dev_alloc_n(&scan, n + np + 1, s);
  if (e == hipSuccess) e = count_live(t->st.X, n, pd.pxyz, np, scan, scan + n + np, s);
  int32_t *h = host_flag();
  int32_t cnt[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(h ? h : cnt, scan + n + np, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && np > 0)
    e = hipMemcpyAsync(h ? h + 1 : cnt + 1, scan + n, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    dev_release(scan, s);
    return e;
  }
  if (h) {
    cnt[0] = h[0];
    cnt[1] = h[1];
  }
  const int64_t total = cnt[0], na = np > 0 ? cnt[1] : total;
  const int64_t ne = total - na + nb, n2 = total + nb;
  // 2. the compacted sorted points, 3. the extra points sorted by (key, id)
  uint64_t *ka = nullptr, *ekey = nullptr, *ktmp = nullptr;
  int32_t *ia = nullptr, *eid = nullptr, *eidx = nullptr, *itmp = nullptr, *mscr = nullptr,
          *src = nullptr;
  double *xa = nullptr, *tmp = nullptr;
  Store next;
  e = dev_alloc_n(&ka, na, s);
  if (e == hipSuccess) e = dev_alloc_n(&ia, na, s);
  if (e == hipSuccess) e = dev_alloc_n(&xa, na * dim, s);
  if (e == hipSuccess) e = dev_alloc_n(&tmp, ne * dim, s);
  if (e == hipSuccess) e = dev_alloc_n(&ekey, ne, s);
  if (e == hipSuccess) e = dev_alloc_n(&eid, ne, s);
  if (e == hipSuccess) e = dev_alloc_n(&eidx, ne, s);
  if (e == hipSuccess) e = dev_alloc_n(&ktmp, ne, s);
  if (e == hipSuccess) e = dev_alloc_n(&itmp, ne, s);
  if (e == hipSuccess) e = dev_alloc_n(&mscr, 2 * n2, s);
  if (e == hipSuccess) e = dev_alloc_n(&src, n2, s);
  if (e == hipSuccess) e = store_alloc(next, n2, dim, s);
  if (e == hipSuccess)
    e = fold_main(dim, scan, n, t->st.key, t->st.id, t->st.X, t->st.Y, t->st.Z, ka, ia, xa,
                  xa + na, dim == 3 ? xa + 2 * na : nullptr, s);
  if (e == hipSuccess)
    e = fold_extra(dim, scan, n, np, na, pd.pxyz, pd.pcap, pd.pid, bxyz, nb, id_base, ne, tmp,
                   eid, s);
  uint64_t *k2 = nullptr;
  int32_t *i2 = nullptr;
  if (e == hipSuccess) e = dev_alloc_n(&k2, ne, s);
  if (e == hipSuccess) e = dev_alloc_n(&i2, ne, s);
  if (e == hipSuccess) e = encode_keys(t->geo, tmp, ne, ne, 0, ekey, eidx, s);
  if (e == hipSuccess) e = sort_key_id(ekey, eid, ne, dim * t->geo.B, ktmp, itmp, k2, i2, s);
  dev_release(k2, s);
  dev_release(i2, s);
  // 4. merge, gather
  if (e == hipSuccess) e = merge_sorted(ka, ia, na, ekey, eid, ne, mscr, next.key, next.id, src, s);
  if (e == hipSuccess)
    e = fold_gather(dim, src, n2, na, xa, xa + na, dim == 3 ? xa + 2 * na : nullptr, pd.pxyz,
                    pd.pcap, bxyz, nb, id_base, next.id, next.X, next.Y, next.Z, t->slot_of, s);
  for (void *q : {(void *)scan, (void *)ka, (void *)ia, (void *)xa, (void *)tmp, (void *)ekey,
                  (void *)eid, (void *)eidx, (void *)ktmp, (void *)itmp, (void *)mscr,
                  (void *)src})
    dev_release(q, s);
  if (e != hipSuccess) {
    store_release(next, s);
    return e;
  }
  store_release(t->st, s);
  t->st = next;
  t->live = n2;
  return relink(t);  // (releases the pool after the gather, in stream order)
}

// Most points a small insert may place in the pool at once, and the most
// deleted points left in their slots before the tree is rebuilt.
int64_t pool_blocks_for(int64_t n) { return std::max<int64_t>(64, n / 64); }
int64_t tomb_limit(int64_t n) { return std::max<int64_t>(16, n / 16); }

// Algorithm 4 in place for a small batch (zd_update.hip), in two halves
// around the one synchronisation of zd_insert_batch.  prepare: key and sort
// the batch and locate every point's leaf by its key bits, counting the
// points that cannot join their leaf in place and the leaves that need a
// pool block (meta[kMetaLocal], meta[kMetaBlocks]); nothing of the tree
// changes.  commit (after the read): place the points and expand the boxes
// on their paths.
struct SmallInsert {
  uint64_t *bk = nullptr, *bk2 = nullptr;
  int32_t *bi = nullptr, *bi2 = nullptr, *leaf = nullptr, *path = nullptr, *depth = nullptr;
};

void small_release(zd_tree t, SmallInsert &w) {
  hipStream_t s = t->stream;
  dev_release(w.bk, s);
  dev_release(w.bi, s);
  dev_release(w.bk2, s);
  dev_release(w.bi2, s);
  dev_release(w.leaf, s);
  dev_release(w.path, s);
  dev_release(w.depth, s);
  w = SmallInsert{};
}

hipError_t insert_small_prepare(zd_tree t, const double *xyz, int64_t m, SmallInsert &w) {
  hipStream_t s = t->stream;
  const int dim = t->dim;
  zd_tree_s::Pending &pd = t->pend;
  hipError_t e = hipSuccess;
  if (!pd.ovf_blk) {
    // the leaf count of the current tree (its last relink), read with
    // whatever came before on the stream
    int32_t I = 0;
    e = read_i32(t->meta + kMetaInternal, &I, s);
    if (e != hipSuccess) return e;
    pd.nleaf = (int64_t)I + 1;
    pd.pcap = pool_blocks_for(t->st.n) * kOvfBlock;
    e = dev_alloc_n(&pd.ovf_blk, pd.nleaf, s);
    if (e == hipSuccess) e = dev_alloc_n(&pd.ovf_cnt, pd.nleaf, s);
    if (e == hipSuccess) e = dev_alloc_n(&pd.pxyz, pd.pcap * dim, s);
    if (e == hipSuccess) e = dev_alloc_n(&pd.pid, pd.pcap, s);
    if (e == hipSuccess) e = dev_alloc_n(&pd.blocks, 1, s);
    if (e == hipSuccess) e = fill_i32(pd.ovf_blk, -1, pd.nleaf, s);
    if (e == hipSuccess) e = fill_i32(pd.ovf_cnt, 0, pd.nleaf, s);
    if (e == hipSuccess) e = fill_f64(pd.pxyz, NAN, pd.pcap * dim, s);
    if (e == hipSuccess) e = fill_i32(pd.blocks, 0, 1, s);
    if (e != hipSuccess) return e;
  }
  e = dev_alloc_n(&w.bk, m, s);
  if (e == hipSuccess) e = dev_alloc_n(&w.bi, m, s);
  if (e == hipSuccess) e = dev_alloc_n(&w.leaf, m, s);
  if (e == hipSuccess) e = dev_alloc_n(&w.path, m * kMaxPath, s);
  if (e == hipSuccess) e = dev_alloc_n(&w.depth, m, s);
  if (e == hipSuccess && m <= kSmallSortKeys)
    // box check, keys, sort, descent and room check in one launch
    return insert_in_place_prepare(t->geo, t->geo.lo, t->hi, xyz, m, (int32_t)t->cap,
                                   t->st.inode, t->st.key, t->st.leaf_begin, t->meta,
                                   pd.ovf_blk, pd.ovf_cnt, w.bk, w.bi, w.leaf, w.path, w.depth,
                                   s);
  if (e == hipSuccess) e = dev_alloc_n(&w.bk2, m, s);
  if (e == hipSuccess) e = dev_alloc_n(&w.bi2, m, s);
  if (e == hipSuccess) e = fill_i32(t->meta + kMetaCheck, 0, 1, s);
  if (e == hipSuccess)
    e = count_outside_box(dim, xyz, m, t->geo.lo, t->hi, t->meta + kMetaCheck, s);
  if (e == hipSuccess) e = encode_keys(t->geo, xyz, m, m, (int32_t)t->cap, w.bk, w.bi, s);
  if (e == hipSuccess) e = radix_sort_pairs(w.bk, w.bi, w.bk2, w.bi2, m, dim * t->geo.B, s);
  if (e == hipSuccess) e = fill_i32(t->meta + kMetaLocal, 0, 2, s);
  if (e == hipSuccess)
    e = insert_in_place_locate(t->st.inode, t->st.key, t->st.leaf_begin, t->meta, w.bk, m,
                               pd.ovf_blk, pd.ovf_cnt, w.leaf, w.path, w.depth,
                               t->meta + kMetaLocal, t->meta + kMetaBlocks, s);
  return e;
}

bool small_fits(const zd_tree t, const int32_t *meta) {
  return meta[kMetaLocal] == 0 && t->pend.nblocks + meta[kMetaBlocks] <= t->pend.pcap / kOvfBlock;
}

hipError_t insert_small_commit(zd_tree t, const double *xyz, int64_t m, const SmallInsert &w,
                               const int32_t *meta, int32_t *out_new_ids) {
  hipStream_t s = t->stream;
  zd_tree_s::Pending &pd = t->pend;
  hipError_t e = grow_ids(t, t->cap + m);
  if (e == hipSuccess)
    e = insert_in_place_commit(t->dim, w.leaf, m, w.path, w.depth, w.bi, xyz, (int32_t)t->cap,
                               pd.ovf_blk, pd.ovf_cnt, pd.blocks, pd.pxyz, pd.pcap, pd.pid,
                               t->slot_of, t->st.inode, t->root_box, out_new_ids, s);
  if (e == hipSuccess) {
    pd.nblocks += meta[kMetaBlocks];
    pd.n_pool += m;
    t->live += m;
    t->cap += m;
  }
  return e;
}

}  // namespace

extern "C" {

const char *zd_status_str(zd_status status) {
  switch (status) {
    case ZD_OK: return "ok";
    case ZD_EINVAL: return "invalid argument";
    case ZD_EBOUNDS: return "point outside the declared box";
    case ZD_EID: return "id out of range, deleted, or repeated";
    case ZD_ENOMEM: return "device allocation failed";
    case ZD_EDEVICE: return "device error";
    case ZD_EKMAX: return "k exceeds ZD_KMAX";
    case ZD_ELIMIT: return "size beyond the fixed scratch of the allocation-free call";
  }
  return "unknown status";
}

zd_status zd_build(const zd_params *p, const double *xyz, int64_t n, void *stream,
                   zd_tree *out) {
  if (!p || !out) return ZD_EINVAL;
  const int dim = p->dim;
  if ((dim != 2 && dim != 3) || p->leaf_size < 1 || n < 0 || n > kMaxLive) return ZD_EINVAL;
  if (!valid_query_waves(p->query_waves)) return ZD_EINVAL;
  if (n > 0 && !xyz) return ZD_EINVAL;
  if ((p->box_lo == nullptr) != (p->box_hi == nullptr)) return ZD_EINVAL;
  if (n == 0 && !p->box_lo) return ZD_EINVAL;
  const int B = 64 / dim;
  if (p->box_lo) {
    if (!finite3(p->box_lo, dim) || !finite3(p->box_hi, dim)) return ZD_EINVAL;
    for (int c = 0; c < dim; ++c)
      if (!(p->box_hi[c] > p->box_lo[c])) return ZD_EINVAL;
  }
  if (p->shift)
    for (int c = 0; c < dim; ++c)
      if (p->shift[c] >> (B - 1)) return ZD_EINVAL;

  zd_tree t = new (std::nothrow) zd_tree_s();
  if (!t) return ZD_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  t->stream = s;
  t->dim = dim;
  t->L = p->leaf_size;
  t->qwaves = p->query_waves ? p->query_waves : 1;
  t->geo.dim = dim;
  t->geo.B = B;
  for (int c = 0; c < dim; ++c)
    t->geo.shift[c] = p->shift ? p->shift[c]
                               : (splitmix64(p->shift_seed, (uint64_t)c + 1) &
                                  ((uint64_t(1) << (B - 1)) - 1));

  hipError_t e = dev_alloc_n(&t->meta, kMetaCount, s);
  if (e == hipSuccess) e = dev_alloc_n(&t->root_box, 6, s);
  if (e == hipSuccess) e = fill_i32(t->meta, 0, kMetaCount, s);
  if (e == hipSuccess) e = fill_f64(t->root_box, 0.0, 6, s);
  if (e == hipSuccess) {
    if (p->box_lo) {
      for (int c = 0; c < dim; ++c) {
        t->geo.lo[c] = p->box_lo[c];
        t->hi[c] = p->box_hi[c];
        t->geo.S[c] = std::ldexp(1.0, B - 1) / (t->hi[c] - t->geo.lo[c]);
      }
    } else {
      // the bounding cube of the data: one read-back
      double *d = nullptr;
      double h[6];
      double *ph = reinterpret_cast<double *>(host_flag());  // 64 pinned bytes, or null
      e = dev_alloc_n(&d, 6, s);
      if (e == hipSuccess) e = box_reduce(dim, xyz, n, d, s);
      if (e == hipSuccess) e = hipMemcpyAsync(ph ? ph : h, d, sizeof(h), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e == hipSuccess && ph)
        for (int c = 0; c < 6; ++c) h[c] = ph[c];
      dev_release(d, s);
      if (e == hipSuccess) {
        double side = 0.0;
        for (int c = 0; c < dim; ++c)
          if (h[3 + c] - h[c] > side) side = h[3 + c] - h[c];
        if (!(side > 0.0)) side = 1.0;
        for (int c = 0; c < dim; ++c) {
          t->geo.lo[c] = h[c];
          t->hi[c] = h[c] + side;
          t->geo.S[c] = std::ldexp(1.0, B - 1) / side;
        }
        if (!finite3(t->geo.lo, dim) || !std::isfinite(side)) {
          destroy(t);
          return ZD_EINVAL;
        }
      }
    }
  }
  if (e == hipSuccess) e = grow_ids(t, n);
  if (e == hipSuccess) e = store_alloc(t->st, n, dim, s);
  uint64_t *ktmp = nullptr;
  int32_t *itmp = nullptr;
  double *aos = nullptr;  // the points as records, for the gather after the sort
  if (e == hipSuccess && n > 1) e = dev_alloc_n(&ktmp, n, s);
  if (e == hipSuccess && n > 1) e = dev_alloc_n(&itmp, n, s);
  if (e == hipSuccess && n > 0) e = dev_alloc_n(&aos, n * (dim == 3 ? 4 : 2), s);
  if (e == hipSuccess) e = encode_keys(t->geo, xyz, n, n, 0, t->st.key, t->st.id, s, aos);
  if (e == hipSuccess) e = radix_sort_pairs(t->st.key, t->st.id, ktmp, itmp, n, dim * B, s);
  dev_release(ktmp, s);
  dev_release(itmp, s);
  if (e == hipSuccess)
    e = gather_points(dim, xyz, n, t->st.id, n, t->st.X, t->st.Y, t->st.Z, t->slot_of, s, aos);
  dev_release(aos, s);
  if (e == hipSuccess) e = relink(t);
  if (e != hipSuccess) {
    destroy(t);
    return to_status(e);
  }
  t->cap = n;
  t->live = n;
  *out = t;
  return ZD_OK;
}

// All-points rows of a tree with pending small inserts: the points in the
// pool answer as queries of their own, their own entry excluded.
static hipError_t pool_rows(zd_tree t, int k, int32_t *out_ids, double *out_d2, hipStream_t s,
                            bool root) {
  if (t->pend.n_pool <= 0) return hipSuccess;
  return knn_pool_rows(t->dim, t->view(), t->geo, t->pend.pxyz, t->pend.pcap, t->pend.pid,
                       t->pend.nblocks * kOvfBlock, k, out_ids, out_d2, s, t->qwaves, root);
}

zd_status zd_knn(zd_tree t, const double *q_xyz, int64_t m, int32_t k, int32_t *out_ids,
                 double *out_d2, void *stream) {
  if (!t || m < 0 || k < 1) return ZD_EINVAL;
  if (k > ZD_KMAX) return ZD_EKMAX;
  if (t->broken) return ZD_EDEVICE;
  if (m > 0 && (!out_ids || !out_d2)) return ZD_EINVAL;
  if (!q_xyz && m != t->cap) return ZD_EINVAL;
  if (q_xyz && m > kMaxLive) return ZD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = join_query_stream(t, s, false);
  if (e == hipSuccess && m > 0) {
    if (!q_xyz) {
      if (t->cap > t->live) e = fill_dead_rows(t->slot_of, t->cap, k, out_ids, out_d2, s);
      if (e == hipSuccess)
        e = knn_all_points(t->dim, t->view(), k, out_ids, out_d2, s, t->qwaves);
      if (e == hipSuccess) e = pool_rows(t, k, out_ids, out_d2, s, false);
    } else {
      e = knn_external(t->dim, t->view(), t->geo, q_xyz, m, k, out_ids, out_d2, s, t->qwaves);
    }
  }
  if (e == hipSuccess) e = join_query_stream(t, s, true);
  if (e != hipSuccess) {
    // (a failed query leaves the tree as it was; only the caller's stream
    // state is in doubt, so the tree is not marked broken here)
    return to_status(e);
  }
  return ZD_OK;
}

zd_status zd_knn_backward_tree(zd_tree t, int32_t k, const int32_t *ids,
                               const double *grad_d2, double *grad_xyz, void *stream) {
  if (!t || k < 1) return ZD_EINVAL;
  if (k > ZD_KMAX) return ZD_EKMAX;
  if (t->broken) return ZD_EDEVICE;
  if (t->cap > 0 && (!ids || !grad_d2 || !grad_xyz)) return ZD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = join_query_stream(t, s, false);
  // (the side pool's entries, while small inserts are pending in place)
  const int64_t pcap = t->pend.n_pool > 0 ? t->pend.pcap : 0;
  if (e == hipSuccess && t->cap > 0)
    e = knn_backward_tree(t->dim, t->view(), t->slot_of, t->cap, pcap, k, ids, grad_d2, grad_xyz,
                          s);
  if (e == hipSuccess) e = join_query_stream(t, s, true);
  return to_status(e);
}

zd_status zd_knn_root(zd_tree t, const double *q_xyz, int64_t m, int32_t k, int32_t *out_ids,
                      double *out_d2, void *stream) {
  if (!t || m < 0 || k < 1) return ZD_EINVAL;
  if (k > ZD_KMAX) return ZD_EKMAX;
  if (t->broken) return ZD_EDEVICE;
  if (m > 0 && (!out_ids || !out_d2)) return ZD_EINVAL;
  if (!q_xyz && m != t->cap) return ZD_EINVAL;
  if (q_xyz && m > kMaxLive) return ZD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = join_query_stream(t, s, false);
  if (e == hipSuccess && m > 0) {
    if (!q_xyz && t->cap > t->live)
      e = fill_dead_rows(t->slot_of, t->cap, k, out_ids, out_d2, s);
    if (e == hipSuccess)
      e = knn_root_based(t->dim, t->view(), t->geo, q_xyz, m, k, out_ids, out_d2, s, t->qwaves);
    if (e == hipSuccess && !q_xyz) e = pool_rows(t, k, out_ids, out_d2, s, true);
  }
  if (e == hipSuccess) e = join_query_stream(t, s, true);
  return to_status(e);
}

zd_status zd_insert_batch(zd_tree t, const double *xyz, int64_t m, int32_t *out_new_ids,
                          void *stream) {
  if (!t || m < 0) return ZD_EINVAL;
  if (t->broken) return ZD_EDEVICE;
  if (m == 0) return ZD_OK;
  if (!xyz || t->cap + m > kMaxIds || t->live + m > kMaxLive) return ZD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int dim = t->dim;
  hipError_t e = bind_stream(t, s);
  // 1. validate the whole batch against the declared box; a small batch is
  // also keyed, sorted and located in the same pass, so that one
  // synchronisation reads the box check, the tree's error counts and
  // whether the batch can go into its leaves in place
  const bool small = t->st.n > 0 && m <= pool_blocks_for(t->st.n);
  SmallInsert w;
  int32_t meta[kMetaCount];
  if (e == hipSuccess && small) {
    e = insert_small_prepare(t, xyz, m, w);  // (checks the box too)
  } else {
    if (e == hipSuccess) e = fill_i32(t->meta + kMetaCheck, 0, 1, s);
    if (e == hipSuccess)
      e = count_outside_box(dim, xyz, m, t->geo.lo, t->hi, t->meta + kMetaCheck, s);
  }
  if (e != hipSuccess) {
    small_release(t, w);
    t->broken = true;
    return to_status(e);
  }
  const zd_status ms = read_meta(t, meta);
  if (ms != ZD_OK || meta[kMetaCheck]) {
    small_release(t, w);
    return ms != ZD_OK ? ms : ZD_EBOUNDS;
  }
  const int32_t first_id = (int32_t)t->cap;
  // 2a. a small batch goes into its leaves in place (Algorithm 4 without
  // rewriting the sorted arrays) when every point's leaf has room
  if (small && small_fits(t, meta)) {
    e = insert_small_commit(t, xyz, m, w, meta, out_new_ids);  // (writes the new ids too)
    small_release(t, w);
    if (e != hipSuccess) {
      t->broken = true;
      return to_status(e);
    }
    return ZD_OK;
  }
  small_release(t, w);
  // 2b. with small batches pending, rebuild from the live points and the batch
  if (t->pend.any()) {
    e = grow_ids(t, t->cap + m);
    if (e == hipSuccess) e = rebuild_live(t, xyz, m, first_id);
    if (e == hipSuccess && out_new_ids) e = iota_i32(out_new_ids, first_id, m, s);
    if (e != hipSuccess) {
      t->broken = true;
      return to_status(e);
    }
    t->cap += m;
    return ZD_OK;
  }
  // 2c. key and sort the batch (Algorithm 4 starts from a shifted, sorted
  // batch) and merge it into the sorted points
  const int64_t n = t->st.n, n2 = n + m;
  uint64_t *bk = nullptr, *bk2 = nullptr;
  int32_t *bi = nullptr, *bi2 = nullptr, *src = nullptr, *scratch = nullptr;
  Store next;
  e = dev_alloc_n(&bk, m, s);
  if (e == hipSuccess) e = dev_alloc_n(&bi, m, s);
  if (e == hipSuccess) e = dev_alloc_n(&bk2, m, s);
  if (e == hipSuccess) e = dev_alloc_n(&bi2, m, s);
  if (e == hipSuccess) e = dev_alloc_n(&src, n2, s);
  if (e == hipSuccess) e = dev_alloc_n(&scratch, 2 * n2, s);
  if (e == hipSuccess) e = store_alloc(next, n2, dim, s);
  if (e == hipSuccess) e = grow_ids(t, t->cap + m);
  if (e != hipSuccess) {
    // nothing changed yet: release and report
    dev_release(bk, s); dev_release(bi, s); dev_release(bk2, s); dev_release(bi2, s);
    dev_release(src, s); dev_release(scratch, s);
    store_release(next, s);
    return to_status(e);
  }
  e = encode_keys(t->geo, xyz, m, m, (int32_t)t->cap, bk, bi, s);
  if (e == hipSuccess) e = radix_sort_pairs(bk, bi, bk2, bi2, m, dim * t->geo.B, s);
  // 3. merge into the Morton-ordered points, 4. gather, 5. relink
  if (e == hipSuccess)
    e = merge_sorted(t->st.key, t->st.id, n, bk, bi, m, scratch, next.key, next.id, src, s);
  if (e == hipSuccess)
    e = gather_merged(dim, src, n2, t->st.X, t->st.Y, t->st.Z, xyz, m, (int32_t)t->cap, next.id,
                      next.X, next.Y, next.Z, t->slot_of, s);
  if (e == hipSuccess && out_new_ids) e = iota_i32(out_new_ids, (int32_t)t->cap, m, s);
  dev_release(bk, s); dev_release(bi, s); dev_release(bk2, s); dev_release(bi2, s);
  dev_release(src, s); dev_release(scratch, s);
  if (e == hipSuccess) {
    store_release(t->st, s);
    t->st = next;
    t->cap += m;
    t->live += m;
    e = relink(t);
  } else {
    store_release(next, s);
  }
  if (e != hipSuccess) {
    t->broken = true;
    return to_status(e);
  }
  return ZD_OK;
}

zd_status zd_delete_batch(zd_tree t, const int32_t *ids, int64_t m, void *stream) {
  if (!t || m < 0) return ZD_EINVAL;
  if (t->broken) return ZD_EDEVICE;
  if (m == 0) return ZD_OK;
  if (!ids) return ZD_EINVAL;
  if (m > t->live) return ZD_EID;
  hipStream_t s = (hipStream_t)stream;
  const int dim = t->dim;
  hipError_t e = bind_stream(t, s);
  // 1. validate: every id in range, live, and unique in the batch (the
  // tree's error counts are read with the same synchronisation)
  int32_t meta[kMetaCount];
  if (e == hipSuccess) e = fill_i32(t->meta + kMetaCheck, 0, 1, s);
  if (e == hipSuccess)
    e = validate_delete(ids, m, t->cap, t->slot_of, t->mark, t->meta + kMetaCheck, s);
  if (e != hipSuccess) {
    t->broken = true;
    return to_status(e);
  }
  const zd_status ms = read_meta(t, meta);
  if (ms != ZD_OK) return ms;
  const int32_t bad = meta[kMetaCheck];
  if (bad) e = unmark_ids(ids, m, t->cap, t->mark, s);
  if (e != hipSuccess) {
    t->broken = true;
    return to_status(e);
  }
  if (bad) return ZD_EID;
  // 2a. a small batch (or any batch while small batches are pending) leaves
  // its points' slots in place, with a NaN coordinate; past the bound on
  // such slots the tree is rebuilt from the live points
  if (t->pend.any() || m <= tomb_limit(t->st.n)) {
    e = tombstone_ids(ids, m, t->slot_of, t->mark, t->st.X, t->pend.pxyz, s);
    if (e == hipSuccess) {
      t->live -= m;
      t->pend.n_tomb += m;
      if (t->pend.n_tomb > tomb_limit(t->st.n)) e = rebuild_live(t, nullptr, 0, 0);
    }
    if (e != hipSuccess) {
      t->broken = true;
      return to_status(e);
    }
    return ZD_OK;
  }
  // 2b. remove, 3. compact the survivors in Morton order, 4. relink
  const int64_t n = t->st.n, n2 = n - m;
  int32_t *dead = nullptr, *scan = nullptr;
  Store next;
  e = dev_alloc_n(&dead, n, s);
  if (e == hipSuccess) e = dev_alloc_n(&scan, n, s);
  if (e == hipSuccess) e = store_alloc(next, n2, dim, s);
  if (e != hipSuccess) {
    (void)unmark_ids(ids, m, t->cap, t->mark, s);
    dev_release(dead, s); dev_release(scan, s);
    store_release(next, s);
    return to_status(e);
  }
  e = fill_i32(dead, 0, n, s);
  if (e == hipSuccess) e = kill_ids(ids, m, t->slot_of, t->mark, dead, s);
  if (e == hipSuccess)
    e = compact_live(dim, dead, n, scan, t->st.key, t->st.id, t->st.X, t->st.Y, t->st.Z,
                     next.key, next.id, next.X, next.Y, next.Z, t->slot_of, s);
  dev_release(dead, s);
  dev_release(scan, s);
  if (e == hipSuccess) {
    store_release(t->st, s);
    t->st = next;
    t->live -= m;
    e = relink(t);
  } else {
    store_release(next, s);
  }
  if (e != hipSuccess) {
    t->broken = true;
    return to_status(e);
  }
  return ZD_OK;
}

// Bring a tree with pending small batches back to its canonical shape.
static zd_status canonical(zd_tree t) {
  if (!t->pend.any()) return ZD_OK;
  hipError_t e = rebuild_live(t, nullptr, 0, 0);
  if (e != hipSuccess) {
    t->broken = true;
    return to_status(e);
  }
  return ZD_OK;
}

zd_status zd_free(zd_tree t) {
  destroy(t);
  return ZD_OK;
}

zd_status zd_info(zd_tree t, int64_t *n_live, int64_t *id_capacity, int64_t *n_leaves,
                  int64_t *n_internal, int32_t *depth) {
  if (!t) return ZD_EINVAL;
  if (t->broken) return ZD_EDEVICE;
  zd_status st = canonical(t);
  if (st != ZD_OK) return st;
  int32_t meta[kMetaCount];
  st = read_meta(t, meta);
  if (st != ZD_OK) return st;
  const int32_t I = t->st.n > 0 ? meta[kMetaInternal] : 0;
  int32_t dep = 0;
  if (depth && t->st.n > 0) {
    hipError_t e = tree_depth(t->st.leaf_parent, t->st.inode, (int64_t)I + 1,
                              t->meta + kMetaDepth, t->stream);
    if (e == hipSuccess) e = read_i32(t->meta + kMetaDepth, &dep, t->stream);
    if (e != hipSuccess) {
      t->broken = true;
      return to_status(e);
    }
  }
  if (n_live) *n_live = t->live;
  if (id_capacity) *id_capacity = t->cap;
  if (n_leaves) *n_leaves = t->st.n > 0 ? (int64_t)I + 1 : 0;
  if (n_internal) *n_internal = I;
  if (depth) *depth = dep;
  return ZD_OK;
}

zd_status zd_pending(zd_tree t, int64_t *in_place_points, int64_t *dead_slots) {
  if (!t) return ZD_EINVAL;
  if (in_place_points) *in_place_points = t->pend.n_pool;
  if (dead_slots) *dead_slots = t->pend.n_tomb;
  return ZD_OK;
}

zd_status zd_check(zd_tree t) {
  if (!t) return ZD_EINVAL;
  if (t->broken) return ZD_EDEVICE;
  int32_t meta[kMetaCount];
  return read_meta(t, meta);
}

zd_status zd_set_walk_limit(zd_tree t, int64_t steps) {
  if (!t || steps < 0) return ZD_EINVAL;
  t->walk_limit = steps;
  return ZD_OK;
}

zd_status zd_export(zd_tree t, uint64_t *keys, int32_t *ids, int64_t *leaf_count,
                    double *leaf_lo, double *leaf_hi, int32_t *int_bit, double *int_lo,
                    double *int_hi, double *params_out, uint64_t *shift_out) {
  if (!t) return ZD_EINVAL;
  const int dim = t->dim;
  if (params_out)
    for (int c = 0; c < dim; ++c) {
      params_out[c] = t->geo.lo[c];
      params_out[dim + c] = t->hi[c];
      params_out[2 * dim + c] = t->geo.S[c];
    }
  if (shift_out)
    for (int c = 0; c < dim; ++c) shift_out[c] = t->geo.shift[c];
  if (t->broken) return ZD_EDEVICE;
  const zd_status cs = canonical(t);
  if (cs != ZD_OK) return cs;
  const int64_t n = t->st.n;
  if (n == 0) return ZD_OK;
  hipStream_t s = t->stream;
  int32_t meta[kMetaCount];
  const zd_status ms = read_meta(t, meta);
  if (ms != ZD_OK) return ms;
  const int32_t I = meta[kMetaInternal];
  hipError_t e = hipSuccess;
  const int64_t nl = (int64_t)I + 1;
  std::vector<int32_t> lb(nl + 1), lp(nl);
  std::vector<INode> in((size_t)I);
  double rb[6];
  if (keys) e = hipMemcpyAsync(keys, t->st.key, sizeof(uint64_t) * n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && ids)
    e = hipMemcpyAsync(ids, t->st.id, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(lb.data(), t->st.leaf_begin, sizeof(int32_t) * (nl + 1),
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(lp.data(), t->st.leaf_parent, sizeof(int32_t) * nl, hipMemcpyDeviceToHost,
                       s);
  if (e == hipSuccess && I > 0)
    e = hipMemcpyAsync(in.data(), t->st.inode, sizeof(INode) * (size_t)I, hipMemcpyDeviceToHost,
                       s);
  if (e == hipSuccess) e = hipMemcpyAsync(rb, t->root_box, sizeof(rb), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return to_status(e);
  auto put_box = [&](double *lo, double *hi, int64_t row, int32_t link) {
    for (int c = 0; c < dim; ++c) {
      if (link < 0) {
        if (lo) lo[row * dim + c] = rb[c];
        if (hi) hi[row * dim + c] = rb[3 + c];
      } else {
        const INode &P = in[link >> 1];
        if (lo) lo[row * dim + c] = P.lo[link & 1][c];
        if (hi) hi[row * dim + c] = P.hi[link & 1][c];
      }
    }
  };
  for (int64_t j = 0; j < nl; ++j) {
    if (leaf_count) leaf_count[j] = lb[j + 1] - lb[j];
    put_box(leaf_lo, leaf_hi, j, lp[j]);
  }
  for (int64_t x = 0; x < I; ++x) {
    if (int_bit) int_bit[x] = in[x].bit;
    put_box(int_lo, int_hi, x, in[x].parent);
  }
  return ZD_OK;
}

zd_status zd_knn_backward(int32_t dim, const double *xyz, int64_t stride, int64_t rows,
                          int32_t k, const int32_t *ids, const double *grad_d2, double *grad_xyz,
                          void *stream) {
  if ((dim != 2 && dim != 3) || stride < 0 || rows < 0 || rows > stride || k < 1) return ZD_EINVAL;
  if (stride > 0 && (!xyz || !grad_xyz)) return ZD_EINVAL;
  if (rows > 0 && (!ids || !grad_d2)) return ZD_EINVAL;
  return to_status(
      knn_backward(dim, xyz, stride, rows, k, ids, grad_d2, grad_xyz, (hipStream_t)stream));
}

zd_status zd_knn_backward_det(int32_t dim, const double *xyz, int64_t stride, int64_t rows,
                              int32_t k, const int32_t *ids, const double *grad_d2,
                              double *grad_xyz, void *stream) {
  if ((dim != 2 && dim != 3) || stride < 0 || rows < 0 || rows > stride || k < 1) return ZD_EINVAL;
  if (stride > kMaxIds || rows * (int64_t)k > kMaxIds) return ZD_EINVAL;
  if (stride > 0 && (!xyz || !grad_xyz)) return ZD_EINVAL;
  if (rows > 0 && (!ids || !grad_d2)) return ZD_EINVAL;
  return to_status(
      knn_backward_det(dim, xyz, stride, rows, k, ids, grad_d2, grad_xyz, (hipStream_t)stream));
}

}  // extern "C"

// ---------------------------------------------------------------------------
// k-NN queries without any allocation: scratch in a fixed device array
// ---------------------------------------------------------------------------

namespace {

// The external-query path's scratch (query keys and order, their sort
// buffers, digit counts and scan partials) for up to kNoAllocMaxQueries
// queries, one copy per GPU for the life of the process.  In host code the
// name `scratch` is only a stand-in: its device address, per device, comes
// from hipGetSymbolAddress and is the only form passed to kernels.
constexpr int64_t kNoAllocMaxQueries = int64_t(1) << 20;
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kScratchDevs = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevs] = {};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// An upper bound of what knn_external takes from the arena for m queries:
// four arrays of m keys / ids, the sort's 256 digit counts per 4,096-key
// tile, and per pass (at most 8) the scan's partial sums at up to two levels.
size_t noalloc_need(int64_t m) {
  const size_t tiles = (size_t)((m + kSortTileKeys - 1) / kSortTileKeys);
  const size_t counts = 256 * tiles;
  const size_t sums = (counts + 4095) / 4096;
  return 2 * align256(8 * (size_t)m) + 2 * align256(4 * (size_t)m) + align256(4 * counts) +
         8 * 2 * align256(4 * sums + 4);
}
static_assert((size_t)(int64_t(1) << 20) * 24 + (size_t(2) << 20) <= kNoAllocScratchBytes,
              "the largest allowed query batch fits the scratch");

// This device's copy of `scratch` (looked up once per device, with that
// device current).
hipError_t scratch_on_device(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kScratchDevs) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

zd_status zd_knn_noalloc(zd_tree t, const double *q_xyz, int64_t m, int32_t k, int32_t *out_ids,
                         double *out_d2, void *stream) {
  if (!t || m < 0 || k < 1) return ZD_EINVAL;
  if (k > ZD_KMAX) return ZD_EKMAX;
  if (t->broken) return ZD_EDEVICE;
  if (m > 0 && (!out_ids || !out_d2)) return ZD_EINVAL;
  if (!q_xyz && m != t->cap) return ZD_EINVAL;
  if (q_xyz && m > kNoAllocMaxQueries) return ZD_ELIMIT;
  if (q_xyz && noalloc_need(m) > kNoAllocScratchBytes) return ZD_ELIMIT;
  const int64_t mp = t->pend.nblocks * kOvfBlock;  // pool entries queried for all-points rows
  if (!q_xyz && t->pend.n_pool > 0 && (mp > kNoAllocMaxQueries || noalloc_need(mp) > kNoAllocScratchBytes))
    return ZD_ELIMIT;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (m > 0) {
    if (!q_xyz) {
      // all-points rows use no scratch
      if (t->cap > t->live) e = fill_dead_rows(t->slot_of, t->cap, k, out_ids, out_d2, s);
      if (e == hipSuccess)
        e = knn_all_points(t->dim, t->view(), k, out_ids, out_d2, s, t->qwaves);
      if (e == hipSuccess && t->pend.n_pool > 0) {
        // rows of points placed by small inserts: their presort takes scratch
        void *base = nullptr;
        e = scratch_on_device(&base);
        if (e == hipSuccess) {
          Arena a{static_cast<char *>(base), kNoAllocScratchBytes, 0};
          arena_activate(&a);
          e = pool_rows(t, k, out_ids, out_d2, s, false);
          arena_activate(nullptr);
        }
      }
    } else {
      void *base = nullptr;
      e = scratch_on_device(&base);
      if (e == hipSuccess) {
        Arena a{static_cast<char *>(base), kNoAllocScratchBytes, 0};
        arena_activate(&a);
        e = knn_external(t->dim, t->view(), t->geo, q_xyz, m, k, out_ids, out_d2, s, t->qwaves);
        arena_activate(nullptr);
      }
    }
  }
  return to_status(e);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched forest
// ---------------------------------------------------------------------------

struct zd_forest_s {
  zd_tree t = nullptr;          // all clouds in one tree whose top separates them
  int32_t C = 0;
  const double *xyz = nullptr;  // the caller's points (read by every build)
  bool have_box = false;
  bool built = false;           // a build has been issued (a plan: its first run)
  double box_lo[3] = {0, 0, 0}, box_hi[3] = {0, 0, 0};
  int64_t *offsets = nullptr;   // device [C+1]
  int32_t *seg = nullptr;       // device [n]: cloud of each position
  double *seg_lo = nullptr;     // device [C][3]
  double *seg_S = nullptr;      // device [C][3]
  int32_t *seg_leaf = nullptr;  // device [C] or null (one leaf size)
  int32_t max_leaf = 0;         // the largest leaf size of any cloud
  int4 *tiles = nullptr;        // sort tiles, none spanning two clouds
  int ntiles = 0;
  int4 *groups = nullptr;       // query groups (first, last, cloud first, cloud last)
  int64_t ngroups = 0;
  // one persistent launch (zd_forest_plan_persistent): clouds in build
  // order, query groups in that order, ready flags, counters, scratch
  bool persistent = false;
  int32_t *p_order = nullptr;
  int4 *p_groups = nullptr;
  int64_t p_ngroups = 0;
  int32_t *p_ready = nullptr;
  int32_t *p_ctl = nullptr;
  uint64_t *p_key2 = nullptr;
  int32_t *p_id2 = nullptr;
  int8_t *p_sb = nullptr;
  // captured build + query
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  Arena arena{nullptr, 0, 0};
};

namespace {

void forest_destroy(zd_forest f) {
  if (!f) return;
  hipStream_t s = f->t ? f->t->stream : nullptr;
  if (f->exec || f->arena.base) (void)hipStreamSynchronize(s);
  if (f->exec) (void)hipGraphExecDestroy(f->exec);
  if (f->graph) (void)hipGraphDestroy(f->graph);
  if (f->arena.base) (void)hipFree(f->arena.base);
  if (f->cap) (void)hipStreamDestroy(f->cap);
  dev_release(f->offsets, s);
  dev_release(f->seg, s);
  dev_release(f->seg_lo, s);
  dev_release(f->seg_S, s);
  dev_release(f->seg_leaf, s);
  dev_release(f->tiles, s);
  dev_release(f->groups, s);
  dev_release(f->p_order, s);
  dev_release(f->p_groups, s);
  dev_release(f->p_ready, s);
  dev_release(f->p_ctl, s);
  dev_release(f->p_key2, s);
  dev_release(f->p_id2, s);
  dev_release(f->p_sb, s);
  destroy(f->t);
  delete f;
}

// Validate the cloud bounds, allocate everything a forest needs and upload
// the tile and group tables (synchronous copies: plan-time only).
zd_status forest_setup(const zd_params *p, const double *xyz, int64_t n, const int64_t *offsets,
                       int32_t C, const int32_t *leaf_sizes, hipStream_t s, zd_forest *out) {
  if (!p || !out || !offsets || C < 1) return ZD_EINVAL;
  const int dim = p->dim;
  if ((dim != 2 && dim != 3) || p->leaf_size < 1 || n < 0 || n > kMaxLive) return ZD_EINVAL;
  if (!valid_query_waves(p->query_waves)) return ZD_EINVAL;
  if (n > 0 && !xyz) return ZD_EINVAL;
  if ((p->box_lo == nullptr) != (p->box_hi == nullptr)) return ZD_EINVAL;
  if (offsets[0] != 0 || offsets[C] != n) return ZD_EINVAL;
  for (int32_t c = 0; c < C; ++c)
    if (offsets[c + 1] < offsets[c]) return ZD_EINVAL;
  if (leaf_sizes)
    for (int32_t c = 0; c < C; ++c)
      if (leaf_sizes[c] < 1) return ZD_EINVAL;
  const int B = 64 / dim;
  if (p->box_lo) {
    if (!finite3(p->box_lo, dim) || !finite3(p->box_hi, dim)) return ZD_EINVAL;
    for (int c = 0; c < dim; ++c)
      if (!(p->box_hi[c] > p->box_lo[c])) return ZD_EINVAL;
  }
  if (p->shift)
    for (int c = 0; c < dim; ++c)
      if (p->shift[c] >> (B - 1)) return ZD_EINVAL;

  zd_forest f = new (std::nothrow) zd_forest_s();
  zd_tree t = new (std::nothrow) zd_tree_s();
  if (!f || !t) {
    delete f;
    delete t;
    return ZD_ENOMEM;
  }
  f->t = t;
  f->C = C;
  f->xyz = xyz;
  f->max_leaf = p->leaf_size;
  if (leaf_sizes)
    for (int32_t c = 0; c < C; ++c) f->max_leaf = std::max(f->max_leaf, leaf_sizes[c]);
  t->stream = s;
  t->dim = dim;
  t->L = p->leaf_size;
  t->qwaves = p->query_waves ? p->query_waves : 1;
  t->geo.dim = dim;
  t->geo.B = B;
  for (int c = 0; c < dim; ++c)
    t->geo.shift[c] = p->shift ? p->shift[c]
                               : (splitmix64(p->shift_seed, (uint64_t)c + 1) &
                                  ((uint64_t(1) << (B - 1)) - 1));
  if (p->box_lo) {
    f->have_box = true;
    for (int c = 0; c < dim; ++c) {
      f->box_lo[c] = p->box_lo[c];
      f->box_hi[c] = p->box_hi[c];
    }
  }
  // tile and group tables
  std::vector<int4> tiles;
  std::vector<int4> groups;
  for (int32_t c = 0; c < C; ++c) {
    const int64_t a = offsets[c], b = offsets[c + 1], m = b - a;
    const int nts = (int)((m + kSortTileKeys - 1) / kSortTileKeys);
    const int first = (int)tiles.size();
    for (int lt = 0; lt < nts; ++lt) {
      const int64_t st = a + (int64_t)lt * kSortTileKeys;
      tiles.push_back(make_int4((int)st, (int)std::min<int64_t>(kSortTileKeys, b - st),
                                256 * first + lt, nts));
    }
    for (int64_t g = a; g < b; g += 64)
      groups.push_back(make_int4((int)g, (int)std::min<int64_t>(g + 63, b - 1), (int)a, (int)(b - 1)));
  }
  f->ntiles = (int)tiles.size();
  f->ngroups = (int64_t)groups.size();
  hipError_t e = dev_alloc_n(&t->meta, kMetaCount, s);
  if (e == hipSuccess) e = dev_alloc_n(&t->root_box, 6, s);
  if (e == hipSuccess) e = fill_i32(t->meta, 0, kMetaCount, s);
  if (e == hipSuccess) e = grow_ids(t, n);
  if (e == hipSuccess) e = store_alloc(t->st, n, dim, s);
  if (e == hipSuccess) e = dev_alloc_n(&f->offsets, C + 1, s);
  if (e == hipSuccess) e = dev_alloc_n(&f->seg, n, s);
  if (e == hipSuccess) e = dev_alloc_n(&f->seg_lo, (int64_t)C * 3, s);
  if (e == hipSuccess) e = dev_alloc_n(&f->seg_S, (int64_t)C * 3, s);
  if (e == hipSuccess && leaf_sizes) e = dev_alloc_n(&f->seg_leaf, C, s);
  if (e == hipSuccess) e = dev_alloc_n(&f->tiles, f->ntiles, s);
  if (e == hipSuccess) e = dev_alloc_n(&f->groups, f->ngroups, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess)
    e = hipMemcpy(f->offsets, offsets, sizeof(int64_t) * (C + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess && leaf_sizes)
    e = hipMemcpy(f->seg_leaf, leaf_sizes, sizeof(int32_t) * C, hipMemcpyHostToDevice);
  if (e == hipSuccess && f->ntiles)
    e = hipMemcpy(f->tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && f->ngroups)
    e = hipMemcpy(f->groups, groups.data(), sizeof(int4) * groups.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    forest_destroy(f);
    return to_status(e);
  }
  t->cap = n;
  *out = f;
  return ZD_OK;
}

// Build all clouds (stream-ordered, no host synchronisation, no allocator
// call when an arena is active).
hipError_t forest_build_pass(zd_forest f, hipStream_t s) {
  zd_tree t = f->t;
  const int64_t n = t->st.n;
  t->stream = s;
  hipError_t e = forest_geometry(t->dim, f->xyz, n, f->offsets, f->C, t->geo.B,
                                 f->have_box ? f->box_lo : nullptr,
                                 f->have_box ? f->box_hi : nullptr, f->seg, f->seg_lo, f->seg_S,
                                 s);
  if (e == hipSuccess)
    e = encode_keys_seg(t->geo, f->xyz, n, f->seg, f->seg_lo, f->seg_S, t->st.key, t->st.id, s);
  uint64_t *ktmp = nullptr;
  int32_t *itmp = nullptr;
  if (e == hipSuccess && n > 1) e = dev_alloc_n(&ktmp, n, s);
  if (e == hipSuccess && n > 1) e = dev_alloc_n(&itmp, n, s);
  if (e == hipSuccess)
    e = radix_sort_pairs(t->st.key, t->st.id, ktmp, itmp, n, t->dim * t->geo.B, s, f->tiles,
                         f->ntiles);
  dev_release(ktmp, s);
  dev_release(itmp, s);
  if (e == hipSuccess)
    e = gather_points(t->dim, f->xyz, n, t->st.id, n, t->st.X, t->st.Y, t->st.Z, t->slot_of, s);
  if (e == hipSuccess) e = relink(t, f->seg, f->seg_leaf, f->max_leaf);
  return e;
}

}  // namespace

extern "C" {

zd_status zd_forest_build(const zd_params *params, const double *xyz, int64_t n,
                          const int64_t *offsets, int32_t n_clouds, const int32_t *leaf_sizes,
                          void *stream, zd_forest *out) {
  zd_forest f = nullptr;
  zd_status st = forest_setup(params, xyz, n, offsets, n_clouds, leaf_sizes, (hipStream_t)stream,
                              &f);
  if (st != ZD_OK) return st;
  hipError_t e = forest_build_pass(f, (hipStream_t)stream);
  if (e != hipSuccess) {
    forest_destroy(f);
    return to_status(e);
  }
  f->built = true;
  *out = f;
  return ZD_OK;
}

zd_status zd_forest_knn(zd_forest f, int32_t k, int32_t *out_ids, double *out_d2, void *stream) {
  if (!f || k < 1) return ZD_EINVAL;
  if (!f->built) return ZD_EINVAL;  // a plan's trees exist after its first run
  if (k > ZD_KMAX) return ZD_EKMAX;
  if (f->t->broken) return ZD_EDEVICE;
  if (f->t->st.n > 0 && (!out_ids || !out_d2)) return ZD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = bind_stream(f->t, s);
  if (e == hipSuccess)
    e = knn_all_points(f->t->dim, f->t->view(), k, out_ids, out_d2, s, f->t->qwaves, f->groups,
                       f->ngroups);
  return to_status(e);
}

zd_status zd_forest_plan(const zd_params *params, const double *xyz, int64_t n,
                         const int64_t *offsets, int32_t n_clouds, const int32_t *leaf_sizes,
                         int32_t k, int32_t *out_ids, double *out_d2, void *stream,
                         zd_forest *out) {
  if (k < 1) return ZD_EINVAL;
  if (k > ZD_KMAX) return ZD_EKMAX;
  if (n > 0 && (!out_ids || !out_d2)) return ZD_EINVAL;
  zd_forest f = nullptr;
  hipStream_t s = (hipStream_t)stream;
  zd_status st = forest_setup(params, xyz, n, offsets, n_clouds, leaf_sizes, s, &f);
  if (st != ZD_OK) return st;
  // scratch for one build + query: sort buffers, digit counts, scan sums,
  // split flags, with room to spare
  f->arena.size = (size_t)n * 24 + ((size_t)64 << 20);
  hipError_t e = hipMalloc(&f->arena.base, f->arena.size);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&f->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipStreamBeginCapture(f->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    arena_activate(&f->arena);
    hipError_t e1 = forest_build_pass(f, f->cap);
    if (e1 == hipSuccess)
      e1 = knn_all_points(f->t->dim, f->t->view(), k, out_ids, out_d2, f->cap, f->t->qwaves,
                          f->groups, f->ngroups);
    arena_activate(nullptr);
    hipError_t e2 = hipStreamEndCapture(f->cap, &f->graph);
    e = e1 != hipSuccess ? e1 : e2;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&f->exec, f->graph, nullptr, nullptr, 0);
  f->t->stream = s;
  if (e != hipSuccess) {
    forest_destroy(f);
    return to_status(e);
  }
  *out = f;
  return ZD_OK;
}

// The wall-clock ticks of `seconds` on the current device.
static int64_t wall_ticks(int seconds) {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    khz = 100000;
  return (int64_t)khz * 1000 * seconds;
}

zd_status zd_forest_plan_persistent(const zd_params *params, const double *xyz, int64_t n,
                                    const int64_t *offsets, int32_t n_clouds,
                                    const int32_t *leaf_sizes, int32_t k, int32_t *out_ids,
                                    double *out_d2, void *stream, zd_forest *out) {
  if (k < 1) return ZD_EINVAL;
  if (k > ZD_KMAX) return ZD_EKMAX;
  if (n > 0 && (!out_ids || !out_d2)) return ZD_EINVAL;
  zd_forest f = nullptr;
  hipStream_t s = (hipStream_t)stream;
  zd_status st = forest_setup(params, xyz, n, offsets, n_clouds, leaf_sizes, s, &f);
  if (st != ZD_OK) return st;
  zd_tree t = f->t;
  const int32_t C = n_clouds;
  f->persistent = true;
  // Builds take clouds by decreasing size.  Query groups go in the order
  // the clouds are predicted to be built: a list schedule of the builds on
  // the launch's workgroups (about four per CU), each cloud costing its
  // size plus a fixed overhead, so that wavefronts rarely wait for a build.
  std::vector<int32_t> order(C);
  for (int32_t c = 0; c < C; ++c) order[c] = c;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return offsets[a + 1] - offsets[a] > offsets[b + 1] - offsets[b];
  });
  int cus = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  std::vector<double> done(C);
  {
    std::priority_queue<double, std::vector<double>, std::greater<double>> slots;
    for (int i = 0; i < 4 * cus; ++i) slots.push(0.0);
    for (int32_t c : order) {
      const double t0 = slots.top();
      slots.pop();
      done[c] = t0 + 4096.0 + (double)(offsets[c + 1] - offsets[c]);
      slots.push(done[c]);
    }
  }
  std::vector<int32_t> qorder(order);
  std::stable_sort(qorder.begin(), qorder.end(),
                   [&](int32_t a, int32_t b) { return done[a] < done[b]; });
  std::vector<int4> qg;
  for (int32_t c : qorder)
    for (int64_t g = offsets[c]; g < offsets[c + 1]; g += 64)
      qg.push_back(make_int4((int)g, (int)std::min<int64_t>(g + 63, offsets[c + 1] - 1), c, 0));
  f->p_ngroups = (int64_t)qg.size();
  hipError_t e = dev_alloc_n(&f->p_order, C, s);
  if (e == hipSuccess) e = dev_alloc_n(&f->p_groups, f->p_ngroups, s);
  if (e == hipSuccess) e = dev_alloc_n(&f->p_ready, C, s);
  if (e == hipSuccess) e = dev_alloc_n(&f->p_ctl, 2, s);
  if (e == hipSuccess) e = dev_alloc_n(&f->p_key2, n, s);
  if (e == hipSuccess) e = dev_alloc_n(&f->p_id2, n, s);
  if (e == hipSuccess) e = dev_alloc_n(&f->p_sb, n, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess)
    e = hipMemcpy(f->p_order, order.data(), sizeof(int32_t) * C, hipMemcpyHostToDevice);
  if (e == hipSuccess && !qg.empty())
    e = hipMemcpy(f->p_groups, qg.data(), sizeof(int4) * qg.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&f->cap, hipStreamNonBlocking);
  PersistArgs a{};
  a.xyz = xyz;
  a.n = n;
  a.offsets = f->offsets;
  a.order = f->p_order;
  a.C = C;
  a.leaf_size = f->seg_leaf;
  a.L = t->L;
  a.g = t->geo;
  a.have_box = f->have_box ? 1 : 0;
  for (int c = 0; c < 3; ++c) {
    a.box.lo[c] = f->box_lo[c];
    a.box.hi[c] = f->box_hi[c];
  }
  a.key2 = f->p_key2;
  a.id2 = f->p_id2;
  a.sb = f->p_sb;
  a.slot_of = t->slot_of;
  a.ctl = f->p_ctl;
  a.ready = f->p_ready;
  a.qgroups = f->p_groups;
  a.ngroups = f->p_ngroups;
  a.out_ids = out_ids;
  a.out_d2 = out_d2;
  a.k = k;
  a.wait_ticks = wall_ticks(10);
  const PersistTree pt{t->st.key, t->st.id, t->st.X, t->st.Y, t->st.Z, t->st.leaf_of,
                       t->st.leaf_begin, t->st.leaf_parent, t->st.inode, t->meta};
  // the graph: clear the counters and flags (fill kernels), then the launch
  if (e == hipSuccess) e = hipStreamBeginCapture(f->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t e1 = fill_i32(f->p_ctl, 0, 2, f->cap);
    if (e1 == hipSuccess) e1 = fill_i32(f->p_ready, 0, C, f->cap);
    if (e1 == hipSuccess && n > 0)
      e1 = t->dim == 3 ? forest_persistent_d3(a, pt, t->view(), f->cap)
                       : forest_persistent_d2(a, pt, t->view(), f->cap);
    hipError_t e2 = hipStreamEndCapture(f->cap, &f->graph);
    e = e1 != hipSuccess ? e1 : e2;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&f->exec, f->graph, nullptr, nullptr, 0);
  t->stream = s;
  if (e != hipSuccess) {
    forest_destroy(f);
    return to_status(e);
  }
  *out = f;
  return ZD_OK;
}

zd_status zd_forest_run(zd_forest f, void *stream) {
  if (!f || !f->exec) return ZD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = bind_stream(f->t, s);
  if (e == hipSuccess) e = hipGraphLaunch(f->exec, s);
  if (e == hipSuccess) f->built = true;
  return to_status(e);
}

zd_status zd_forest_check(zd_forest f) {
  if (!f) return ZD_EINVAL;
  return zd_check(f->t);
}

zd_status zd_forest_free(zd_forest f) {
  forest_destroy(f);
  return ZD_OK;
}

}  // extern "C"
