/*
 * zd.h -- C ABI of libzd, an MI355X (gfx950) implementation of the zd-tree
 * for exact k-nearest neighbours in 2 and 3 dimensions.
 *
 * Method: G. E. Blelloch and M. Dobson, "Parallel Nearest Neighbors in Low
 * Dimensions with Batch Updates" (arXiv 2111.04182).  The tree is a kd-tree
 * whose splits follow the bits of the Morton order of the randomly shifted,
 * integer-rounded points (Section 2, "Data structure" and "Construction");
 * k-NN searches climb from a leaf and descend into sibling subtrees with box
 * pruning (Algorithms 2 and 3); batches of points are inserted and deleted
 * (Algorithm 4 and Section 2, "Batch-dynamic updates").
 *
 * Conventions shared by every call:
 *   - Pointers marked (device) are HIP device pointers; (host) are host
 *     pointers.  Coordinates are structure-of-arrays FP64 in one buffer:
 *     x[0..n), y[0..n), then z[0..n) in 3D.
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *     Calls are stream-ordered: inputs may be reused once the stream has
 *     passed the call.
 *   - The caller owns every input and output buffer.  The library keeps its
 *     own copies of what it needs (the Morton-ordered points, the nodes, the
 *     id map) and releases them in zd_free.  Released device blocks stay in
 *     the library's cache and are reused by later calls on the same stream;
 *     the cache holds at most 32 GiB per device, and is handed back to the
 *     runtime when an allocation fails (and at process exit).
 *   - Errors are returned before anything is enqueued; out-parameters are
 *     untouched on error.  No C++ exception crosses this interface.
 *   - Self-checks: the build counts any inconsistency of its bottom-up climb,
 *     and a search that stops before it has finished (a corrupted tree, or
 *     the step limit of zd_set_walk_limit) counts itself; both counts live
 *     on the device.  Every call that synchronises the tree's stream
 *     (zd_info, zd_export, zd_check, the updates) reads them, and if either
 *     is non-zero returns ZD_EDEVICE and marks the tree broken: its rows
 *     since the last check cannot be trusted, and only zd_free remains
 *     valid.
 *   - Squared distances d2(a,b) = ((dx*dx + dy*dy) + dz*dz), dx = a.x - b.x,
 *     binary64 with no fused multiply-add.  Neighbours are ordered by
 *     (d2, id) ascending; equal d2 goes to the lower id.  Results are exact:
 *     they equal brute force over the live points bit for bit.
 */
#ifndef ZD_H
#define ZD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ZD_API __attribute__((visibility("default")))

typedef struct zd_tree_s *zd_tree;
typedef struct zd_forest_s *zd_forest;

typedef enum {
  ZD_OK = 0,
  ZD_EINVAL = 1,  /* invalid argument */
  ZD_EBOUNDS = 2, /* an inserted point lies outside the declared box */
  ZD_EID = 3,     /* a deleted id is out of range, dead, or repeated */
  ZD_ENOMEM = 4,  /* device allocation failed */
  ZD_EDEVICE = 5, /* a HIP call failed; only zd_free remains valid */
  ZD_EKMAX = 6,   /* k exceeds ZD_KMAX */
  ZD_ELIMIT = 7   /* beyond the fixed scratch of zd_knn_noalloc */
} zd_status;

/* largest supported k */
#define ZD_KMAX 100

/* Build parameters.
 *   dim:        2 or 3.
 *   leaf_size:  L >= 1, the most points a leaf holds (a leaf whose points all
 *               share one Morton key may hold more: Algorithm 1's "no bits
 *               left" case).  The paper calls L + 1 its sizeCutoff.
 *   shift_seed: seed of the random shift (Section 2, "Construction"): shift
 *               c = splitmix64 output number c+1 from the seed, reduced mod
 *               2^(B-1), B = 64/dim bits per coordinate.  Results do not
 *               depend on it, only the tree shape does.
 *   shift:      (host) [dim] explicit shift values in [0, 2^(B-1)), or NULL
 *               to draw them from shift_seed.
 *   box_lo/hi:  (host) [dim] the box that every point, including later
 *               inserts, must lie in (Section 2: the box is declared before
 *               the first build), or both NULL to use the bounding cube of
 *               the build points (lo = per-coordinate minimum, common side =
 *               the largest extent, 1 if all points coincide).  Rounding to
 *               integers (Section 3.1) maps [lo, hi] onto 2^(B-1) cells per
 *               coordinate: cell = clamp(floor((x - lo) * S), 0, 2^(B-1)-1),
 *               S = 2^(B-1) / (hi - lo).
 *   query_waves: launch shape of this tree's k-NN queries: wavefronts per
 *               workgroup, 1, 2 or 4 (0 means 1).  Each wavefront answers 64
 *               queries whatever the value; it changes only how wavefronts are
 *               packed into workgroups, never the rows.  For k > 32 (per-lane
 *               candidate sets partly in LDS) the value is lowered, if needed, until
 *               the workgroup's LDS fits in one CU.  Not in the paper: a tuning
 *               knob of this implementation. */
typedef struct {
  int32_t dim;
  int32_t leaf_size;
  uint64_t shift_seed;
  const uint64_t *shift;
  const double *box_lo;
  const double *box_hi;
  int32_t query_waves;
} zd_params;

/* Build a zd-tree over n points (Section 2, "Construction", Algorithm 1).
 *   xyz: (device) SoA [dim][n] FP64 coordinates.  Point i gets id i.
 *   out: (host) receives the new tree handle.
 * Asynchronous on `stream` when a box is given; with box_lo == NULL the call
 * synchronises `stream` once to read the data's bounding cube.
 * Errors: ZD_EINVAL for a NULL params/out, dim not 2 or 3, leaf_size < 1,
 * n < 0, n > 2^30 - 1 (node links are (node << 1) | side in int32, and a
 * tree of n points has up to n - 1 internal nodes), a NULL xyz with n > 0, n == 0 without a box, only one
 * of box_lo / box_hi given, hi <= lo, a non-finite box, a shift value out
 * of range, or query_waves not 0, 1, 2 or 4; ZD_ENOMEM; ZD_EDEVICE. */
ZD_API zd_status zd_build(const zd_params *params, const double *xyz, int64_t n,
                   void *stream, zd_tree *out);

/* Exact k-NN queries (Algorithms 2 and 3).
 *   q_xyz == NULL: the k-nearest-neighbour graph of the live points
 *     (Section 1.1; the paper's leaf-based search, Section 2): one row per
 *     id in [0, id_capacity); row p holds the k nearest live points q != p.
 *     m must equal the id capacity (zd_info).  Rows of deleted ids are
 *     filled with (-1, +inf).
 *   q_xyz != NULL: (device) SoA [dim][m] dynamic query points (Section 1.1;
 *     the bit-based search of Section 2: descend by the query's Morton bits,
 *     then climb).  Row r answers query r; nothing is excluded.  Queries
 *     outside the box are allowed (their integer coordinates are clamped).
 *   out_ids: (device) [m][k] int32 neighbour ids, out_d2: (device) [m][k]
 *     FP64 squared distances; each row ascending by (d2, id); a row with
 *     fewer than k candidates is padded with (-1, +inf).
 * Asynchronous.  A query only reads the tree: concurrent zd_knn calls on one
 * tree, from several host threads and on several streams, are safe.  A
 * query on a stream other than the tree's own is ordered after the tree's
 * pending work, and the tree's later work (updates, zd_free) after the
 * query, by events; the tree itself is not changed.
 * Errors: ZD_EINVAL (NULL tree or outputs, m < 0, k < 1, m mismatch,
 * m > 2^30 - 1 external queries), ZD_EKMAX (k > ZD_KMAX), ZD_ENOMEM,
 * ZD_EDEVICE (a broken tree, or a HIP failure). */
ZD_API zd_status zd_knn(zd_tree tree, const double *q_xyz, int64_t m, int32_t k,
                 int32_t *out_ids, double *out_d2, void *stream);

/* Root-based exact k-NN (Section 2): Algorithm 2 from the root with an
 * empty candidate set, no climb.  Same arguments, rows, ordering and errors
 * as zd_knn (q_xyz == NULL: all-points rows by id, self excluded; else
 * external queries); only the start of the search differs from zd_knn's
 * leaf-based (all-points) and bit-based (external) searches, which the paper
 * finds more robust on skewed data.  Asynchronous; concurrent with other
 * queries like zd_knn. */
ZD_API zd_status zd_knn_root(zd_tree tree, const double *q_xyz, int64_t m, int32_t k,
                             int32_t *out_ids, double *out_d2, void *stream);

/* zd_knn without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, rows and errors as zd_knn; the call
 * makes no allocation of any kind (no hipMalloc, no library cache, no event).
 *   - External queries (q_xyz != NULL) take their scratch (query keys,
 *     order and sort buffers, about 24 bytes per query) from one fixed
 *     32 MiB device array per GPU, held until the process ends; at most
 *     2^20 = 1,048,576 queries per call, otherwise ZD_ELIMIT before anything
 *     is enqueued.  All-points rows (q_xyz == NULL) need no scratch and take
 *     any size zd_knn takes, except that points placed by small inserts
 *     not yet merged (see zd_insert_batch) answer through the same scratch:
 *     at most 2^20 of them, otherwise ZD_ELIMIT.
 *   - Every call on one GPU shares that GPU's array: calls that overlap in
 *     time on one GPU (two host threads, or two streams not ordered by the
 *     caller) race on it and may return wrong rows.  Order them.
 *   - Nothing orders the call against the tree's own stream: issue it on
 *     that stream, or order it after the tree's last build or update (and
 *     the tree's next update after it) yourself.
 * Errors: as zd_knn, plus ZD_ELIMIT. */
ZD_API zd_status zd_knn_noalloc(zd_tree tree, const double *q_xyz, int64_t m, int32_t k,
                                int32_t *out_ids, double *out_d2, void *stream);

/* Batch insertion (Algorithm 4).  The m new points get ids id_capacity,
 * id_capacity + 1, ...; the id capacity grows by m.
 * A small batch (m <= max(64, n/64)) is applied in place when it can be, as
 * Algorithm 4 does it: each point descends by its key bits to its leaf, is
 * appended to that leaf (up to 8 such points per leaf, kept beside the
 * Morton-ordered array), and the boxes on its path are expanded; no array
 * of the tree is rewritten.  The tree then departs from its canonical shape
 * only where the paper's would split a leaf or an edge; queries stay exact.
 * The canonical shape (a fresh build of the live points) returns with the
 * next batch that does not fit in place, zd_info or zd_export.
 *   xyz: (device) SoA [dim][m].  out_new_ids: (device) [m] or NULL.
 * The batch is all-or-nothing: if any point lies outside the declared box
 * the call returns ZD_EBOUNDS and the tree is unchanged.  The rows of every
 * query afterwards are those of a fresh build of the live points (same box
 * and shift).
 * Synchronises `stream` (to validate the batch).  Updates need exclusive
 * access to the tree.
 * Errors: ZD_EINVAL (also when the live points would exceed 2^30 - 1 or the
 * id capacity 2^31 - 2), ZD_EBOUNDS, ZD_ENOMEM, ZD_EDEVICE. */
ZD_API zd_status zd_insert_batch(zd_tree tree, const double *xyz, int64_t m,
                          int32_t *out_new_ids, void *stream);

/* Batch deletion (Section 2, "Batch-dynamic updates").
 *   ids: (device) [m] int32 ids to delete.
 * A small batch (m <= max(16, n/16), or any batch while small batches are
 * pending) leaves each deleted point's slot in place, marked dead, so no
 * array is rewritten; past that bound on dead slots, or on zd_info or
 * zd_export, the tree is rebuilt from the live points.
 * All-or-nothing: an id out of range, already deleted, or repeated in the
 * batch gives ZD_EID with the tree unchanged.  Afterwards the tree equals a
 * fresh build of the live points (immediately for a large batch, else at
 * the next canonicalisation).  Synchronises `stream`.
 * Errors: ZD_EINVAL, ZD_EID, ZD_ENOMEM, ZD_EDEVICE. */
ZD_API zd_status zd_delete_batch(zd_tree tree, const int32_t *ids, int64_t m,
                          void *stream);

/* Release a tree.  The release is ordered on the stream of the tree's last
 * call; the caller must not have work using the tree on other streams.
 * zd_free(NULL) is a no-op. */
ZD_API zd_status zd_free(zd_tree tree);

/* Sizes of a tree: live points, id capacity (rows of an all-points query),
 * leaves, internal nodes, and depth (the most edges from the root to a leaf;
 * Theorem 1 bounds it by O(log n) on data of bounded aspect ratio; computed
 * on the device only when `depth` is non-NULL).  Any pointer may be NULL.
 * Synchronises the tree's stream and runs the self-checks.
 * Errors: ZD_EINVAL (NULL tree), ZD_EDEVICE (a self-check failed, or HIP). */
ZD_API zd_status zd_info(zd_tree tree, int64_t *n_live, int64_t *id_capacity,
                  int64_t *n_leaves, int64_t *n_internal, int32_t *depth);

/* Small batches applied in place and not yet folded into the canonical
 * shape: points placed beside the sorted arrays by small inserts since the
 * last rebuild (some may since have been deleted), and deleted points that
 * still hold their slot.  Host-side counters: no synchronisation.  Either
 * pointer may be NULL.  Errors: ZD_EINVAL (NULL tree). */
ZD_API zd_status zd_pending(zd_tree tree, int64_t *in_place_points, int64_t *dead_slots);

/* Synchronise the tree's stream and run the self-checks: ZD_OK, or
 * ZD_EDEVICE when the build or a search since the last check found the tree
 * inconsistent (the tree is then broken).  ZD_EINVAL for a NULL tree. */
ZD_API zd_status zd_check(zd_tree tree);

/* Test hook: bound every later search of this tree to `steps` walk steps
 * (node and climb steps; 0 restores the default of 4n + 256, which a valid
 * tree never reaches).  A search that reaches the bound stops early, its row
 * is not exact, and the next zd_check (or other synchronising call) reports
 * ZD_EDEVICE.  Errors: ZD_EINVAL (NULL tree, steps < 0). */
ZD_API zd_status zd_set_walk_limit(zd_tree tree, int64_t steps);

/* Copy the tree to caller-owned host arrays in its canonical in-order form
 * (for tests): the live (key, id) pairs in Morton order, every leaf's size
 * and tight box, and every internal node's split bit and tight box, in
 * order (leaf 0, internal 0, leaf 1, ..., leaf n_leaves-1).  Sizes come from
 * zd_info; boxes are [count][dim].  The box lo/scale/shift used for the keys
 * go to params_out = {lo[dim], hi[dim], S[dim]} and shift_out[dim].  Any
 * pointer may be NULL.  Synchronises the tree's stream. */
ZD_API zd_status zd_export(zd_tree tree, uint64_t *keys, int32_t *ids,
                    int64_t *leaf_count, double *leaf_lo, double *leaf_hi,
                    int32_t *int_bit, double *int_lo, double *int_hi,
                    double *params_out, uint64_t *shift_out);

/* Backward of the k-NN squared distances for a fixed neighbour table.
 * For L = sum over rows r and slots j of grad_d2[r][j] * d2(p_r, p_q),
 * q = ids[r][j] (entries with q < 0 are skipped):
 *   dL/dp_r += 2 (p_r - p_q) g,   dL/dp_q -= 2 (p_r - p_q) g.
 *   xyz:  (device) SoA [dim][stride] points by id (row r is id r).
 *   ids, grad_d2: (device) [rows][k].   grad_xyz: (device) SoA [dim][stride],
 *   overwritten.  Accumulation uses FP64 atomics, so the summation order
 *   (not the set of terms) varies between runs.
 * Asynchronous.  Errors: ZD_EINVAL, ZD_EDEVICE. */
ZD_API zd_status zd_knn_backward(int32_t dim, const double *xyz, int64_t stride,
                          int64_t rows, int32_t k, const int32_t *ids,
                          const double *grad_d2, double *grad_xyz,
                          void *stream);

/* zd_knn_backward without atomics: the edges are sorted by neighbour once
 * (a radix sort of rows * k keys), and one thread per point sums its own
 * terms and then the terms of the rows that chose it, in a fixed order, so
 * every run returns the same bits.  Same arguments and errors as
 * zd_knn_backward, plus ZD_EINVAL when stride or rows * k exceeds 2^31 - 2.
 * Scratch: about 24 bytes per edge, from the library's device cache. */
ZD_API zd_status zd_knn_backward_det(int32_t dim, const double *xyz, int64_t stride,
                                     int64_t rows, int32_t k, const int32_t *ids,
                                     const double *grad_d2, double *grad_xyz, void *stream);

/* zd_knn_backward for the tree's own all-points rows, taken in the tree's
 * Morton order: the terms between points of one 1,024-point Morton tile
 * are summed in LDS and only the others by atomics, into a buffer in
 * sorted order, so most atomics stay on chip and near each other.  The
 * points are the tree's current ones (xyz by id, as given to zd_build and
 * the inserts); ids/grad_d2: (device) [cap][k], the rows of zd_knn(t,
 * NULL, cap, k, ...) on this tree, unchanged since; grad_xyz: (device)
 * [dim][cap], overwritten (zero for dead ids).  Points that small inserts
 * placed in place (pending batches) take their rows in a second pass, in
 * the order of their side pool.  Results equal zd_knn_backward's up to the
 * order of the floating-point additions.  Read-only on the tree (may run
 * beside queries, as zd_knn).  Errors: ZD_EINVAL, ZD_EKMAX, ZD_EDEVICE. */
ZD_API zd_status zd_knn_backward_tree(zd_tree tree, int32_t k, const int32_t *ids,
                                      const double *grad_d2, double *grad_xyz, void *stream);

/* Batched forest: C independent point clouds answered in one pass (an
 * addition beyond the paper, which builds one tree).  Cloud c is points
 * [offsets[c], offsets[c+1]) of xyz; point i keeps id i.  Every cloud gets
 * the tree a separate zd_build would give it (its own bounding cube unless
 * params->box_lo/hi declare one box for all, the params' shift, and leaf
 * size leaf_sizes[c], or params->leaf_size when leaf_sizes is NULL); the
 * clouds share one device tree whose top levels separate them, and
 * neighbours only ever come from the query's own cloud.
 *   xyz: (device) SoA [dim][n].  offsets: (host) [n_clouds + 1], offsets[0]
 *   = 0, non-decreasing, offsets[n_clouds] = n.  leaf_sizes: (host)
 *   [n_clouds] or NULL.
 * zd_forest_build runs build passes on `stream` and returns; it synchronises
 * once to upload its tile and group tables.  Errors: ZD_EINVAL (as zd_build,
 * plus bad offsets or leaf sizes), ZD_ENOMEM, ZD_EDEVICE. */
ZD_API zd_status zd_forest_build(const zd_params *params, const double *xyz, int64_t n,
                                 const int64_t *offsets, int32_t n_clouds,
                                 const int32_t *leaf_sizes, void *stream, zd_forest *out);

/* All-points k-NN rows of every cloud: row i (i < n) holds the k nearest
 * points of point i's cloud other than i, as zd_knn.  out_ids/out_d2:
 * (device) [n][k].  Asynchronous.  On a plan (zd_forest_plan*), the trees
 * of its last zd_forest_run, ordered on the stream of that run.  Errors:
 * ZD_EINVAL (also for a plan that has not run yet), ZD_EKMAX, ZD_EDEVICE. */
ZD_API zd_status zd_forest_knn(zd_forest forest, int32_t k, int32_t *out_ids, double *out_d2,
                               void *stream);

/* A forest whose whole build + all-points query is captured once into a
 * HIP graph: zd_forest_run then rebuilds every tree from the current
 * contents of xyz and writes the rows to out_ids/out_d2 with one graph
 * launch, with no allocation and no host synchronisation.  The pointers
 * xyz, out_ids and out_d2 are bound at plan time and must stay valid.
 * zd_forest_plan synchronises `stream` (allocation, table upload, capture).
 * Errors: as zd_forest_build and zd_forest_knn. */
ZD_API zd_status zd_forest_plan(const zd_params *params, const double *xyz, int64_t n,
                                const int64_t *offsets, int32_t n_clouds,
                                const int32_t *leaf_sizes, int32_t k, int32_t *out_ids,
                                double *out_d2, void *stream, zd_forest *out);
ZD_API zd_status zd_forest_run(zd_forest forest, void *stream);

/* zd_forest_plan with the whole build + query as ONE persistent kernel
 * launch (after two fill kernels that clear its counters), captured in the
 * plan's graph and replayed by zd_forest_run.  Inside the launch, each
 * workgroup takes clouds largest first and builds each one alone with
 * workgroup barriers only (its keys, sort, leaf test, node numbering, boxes
 * and links, numbered inside the cloud's own range of the shared arrays);
 * then every wavefront takes 64-point query groups, in the same cloud
 * order, waiting for its group's cloud to be built.  Rows, trees and
 * errors are those of zd_forest_plan; zd_forest_knn and zd_forest_check
 * work on the trees of the last run.  A wait inside the launch that runs
 * out (10 s) skips its group and makes zd_forest_check report ZD_EDEVICE.
 * Scratch: about 13 bytes per point, and the plan's tables. */
ZD_API zd_status zd_forest_plan_persistent(const zd_params *params, const double *xyz,
                                           int64_t n, const int64_t *offsets, int32_t n_clouds,
                                           const int32_t *leaf_sizes, int32_t k,
                                           int32_t *out_ids, double *out_d2, void *stream,
                                           zd_forest *out);

/* Synchronise the forest's stream and run the self-checks of its build and
 * searches (as zd_check).  Errors: ZD_EINVAL (NULL), ZD_EDEVICE. */
ZD_API zd_status zd_forest_check(zd_forest forest);

/* Release a forest (after its work on the last stream used; a plan's graph
 * and scratch are released after synchronising that stream). */
ZD_API zd_status zd_forest_free(zd_forest forest);

/* A short English description of a status code (static storage). */
ZD_API const char *zd_status_str(zd_status status);

#ifdef __cplusplus
}
#endif

#endif /* ZD_H */
