/*
 * zd_oracle.c -- serial CPU oracle for the zd-tree exact k-NN hot path.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load this library.  The GPU
 * library shares no code, header, table or helper with it.
 *
 * Source: G. E. Blelloch and M. Dobson, "Parallel Nearest Neighbors in Low
 * Dimensions with Batch Updates" (ALENEX 2022, arXiv 2111.04182).
 *
 * Two layers:
 *   (1) The definition of the result (brute force).  Section 1.1 defines the
 *       k-nearest-neighbor graph of P (every point's k nearest other points)
 *       and dynamic queries (points not in P).  zo_brute_* computes exactly
 *       that: for every query, the k smallest (d2, id) pairs, ascending.
 *   (2) The zd-tree itself, step by step in the paper's order:
 *       random shift (Section 2, "Construction"), rounding to integers
 *       (Section 3.1, "Numerical details"), Morton interleave (Section 1.1,
 *       "Morton ordering"), Morton sort, buildTree (Algorithm 1) with empty
 *       cuts pruned (Section 2.1, before Theorem 3), searchDown (Algorithm 2),
 *       searchUp (Algorithm 3), leaf-based and bit-based queries (Section 2,
 *       "Upward search algorithm"), batchInsert (Algorithm 4) and deletion
 *       (Section 2, "Batch-dynamic updates").
 *
 * Readings where the paper is silent or ambiguous (all are listed with their
 * reasons in the design notes of the repository):
 *   - d2(a,b) = ((dx*dx + dy*dy) + dz*dz), dx = a.x - b.x, binary64, no FMA
 *     (the file must be compiled with -ffp-contract=off).  Squared distances
 *     everywhere, as Section 3.1 recommends.
 *   - Candidates are totally ordered by (d2, id); ties go to the lower id.
 *     A candidate enters N iff |N| < k or (d2,id) < (d2,id) of N's worst.
 *   - "q != p" in Algorithms 2 and 3 compares identities (ids), and the
 *     element inserted is the candidate q.
 *   - Leaf iff count <= L (sizeCutoff = L+1) or no bits are left (all keys
 *     equal); empty cuts are skipped, never forked.
 *   - Integer rounding: B = floor(64/d) bits per coordinate; the data box
 *     maps onto the low 2^(B-1) cells: q = clamp(floor((x-lo)*S), 0,
 *     2^(B-1)-1), S = 2^(B-1)/(hi-lo); then the random shift in [0, 2^(B-1))
 *     is added, so the shifted box is at most twice the data box (Section 2.1).
 *   - Morton bit order: bit j of coordinate c lands at key bit d*j + (d-1-c),
 *     so x is the most significant coordinate of each d-bit group.
 *   - Shift values: splitmix64 (Steele, Lea, Flood 2014) evaluated at
 *     counter c+1 from the user seed, reduced mod 2^(B-1).
 *   - Node boxes are the tight FP64 min/max boxes of the node's points.
 *   - searchDown visits a node iff its box distance bd2 <= kth; searchUp stops
 *     climbing iff |N| = k and p lies inside C's box with every face strictly
 *     farther than kth.
 *   - Child order in searchDown: the child whose box centre is nearer first;
 *     on a tie, the right child (the "else" branch of Algorithm 2).
 *   - batchInsert sends bit-0 points to the left child (as Algorithm 1 does);
 *     points leaving a node's key prefix create a new internal node at the
 *     highest differing bit; an overflowing leaf is rebuilt with Algorithm 1.
 *   - Deletion removes points, recomputes tight boxes, turns nodes with
 *     count <= L into leaves and splices out nodes with an empty side, so
 *     the tree after any update sequence equals buildTree of the live set.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ZO_API __attribute__((visibility("default")))

/* status codes (same numbering as the product library's public header, which
 * this file does not include) */
enum { ZO_OK = 0, ZO_EINVAL = 1, ZO_EBOUNDS = 2, ZO_EID = 3, ZO_ENOMEM = 4 };

/* ------------------------------------------------------------------------- */
/* squared distance and the candidate order                                  */
/* ------------------------------------------------------------------------- */

/* d2 between two points given coordinate-by-coordinate (Section 3.1 uses
 * squared distances); the sum is left-to-right with no fused operations. */
static double sq_dist(int dim, const double *a, const double *b) {
  double dx = a[0] - b[0];
  double dy = a[1] - b[1];
  double s = dx * dx + dy * dy;
  if (dim == 3) {
    double dz = a[2] - b[2];
    s = s + dz * dz;
  }
  return s;
}

/* (d, i) < (e, j) in the lexicographic order on (d2, id) */
static int cand_less(double d, int64_t i, double e, int64_t j) {
  return d < e || (d == e && i < j);
}

/* ------------------------------------------------------------------------- */
/* N: the bounded candidate set of Algorithms 2 and 3                        */
/* ------------------------------------------------------------------------- */

typedef struct {
  int k, size;
  double *d2;   /* ascending by (d2, id) */
  int64_t *id;
} nset;

/* distance(p, N, k): +inf while |N| < k, else the worst d2 in N */
static double nset_radius(const nset *N) {
  return N->size < N->k ? INFINITY : N->d2[N->k - 1];
}

/* insert(N, q, k): keep only the k smallest by (d2, id) */
static void nset_insert(nset *N, double d, int64_t id) {
  if (N->size == N->k) {
    if (!cand_less(d, id, N->d2[N->k - 1], N->id[N->k - 1])) return;
    N->size--; /* drop the worst */
  }
  int j = N->size;
  while (j > 0 && cand_less(d, id, N->d2[j - 1], N->id[j - 1])) {
    N->d2[j] = N->d2[j - 1];
    N->id[j] = N->id[j - 1];
    j--;
  }
  N->d2[j] = d;
  N->id[j] = id;
  N->size++;
}

static void nset_emit(const nset *N, int32_t *out_ids, double *out_d2) {
  for (int j = 0; j < N->k; ++j) {
    if (j < N->size) {
      out_ids[j] = (int32_t)N->id[j];
      out_d2[j] = N->d2[j];
    } else {
      out_ids[j] = -1;
      out_d2[j] = INFINITY;
    }
  }
}

/* ------------------------------------------------------------------------- */
/* (1) brute force: the definition                                           */
/* ------------------------------------------------------------------------- */

/* Rows of the k-NN result by brute force over the live points.
 *   pts:   SoA coordinates by id, coordinate c of id i at pts[c*stride + i]
 *   live:  live[i] != 0 iff id i belongs to P (NULL: all ids live)
 *   cap:   number of ids
 *   q:     SoA query coordinates (stride m) or NULL for all-points rows
 *   qids:  for all-points rows, the ids whose rows to compute (NULL: all ids)
 *   m:     number of rows
 * All-points rows exclude the query's own id; dead query ids give a padded
 * row.  Rows are written row-major [m][k]. */
ZO_API int zo_brute_knn(int dim, const double *pts, int64_t stride,
                        const uint8_t *live, int64_t cap, const double *q,
                        const int64_t *qids, int64_t m, int k,
                        int32_t *out_ids, double *out_d2) {
  if ((dim != 2 && dim != 3) || k < 1 || m < 0 || cap < 0) return ZO_EINVAL;
  nset N;
  N.k = k;
  N.d2 = (double *)malloc(sizeof(double) * (size_t)k);
  N.id = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
  if (!N.d2 || !N.id) { free(N.d2); free(N.id); return ZO_ENOMEM; }
  for (int64_t r = 0; r < m; ++r) {
    double p[3] = {0, 0, 0};
    int64_t self = -1;
    N.size = 0;
    if (q) {
      for (int c = 0; c < dim; ++c) p[c] = q[c * m + r];
    } else {
      self = qids ? qids[r] : r;
      if (self < 0 || self >= cap || (live && !live[self])) {
        nset_emit(&N, out_ids + r * k, out_d2 + r * k);
        continue;
      }
      for (int c = 0; c < dim; ++c) p[c] = pts[c * stride + self];
    }
    for (int64_t i = 0; i < cap; ++i) {
      if (i == self || (live && !live[i])) continue;
      double x[3] = {0, 0, 0};
      for (int c = 0; c < dim; ++c) x[c] = pts[c * stride + i];
      double d = sq_dist(dim, p, x);
      if (N.size < k || cand_less(d, i, N.d2[k - 1], N.id[k - 1]))
        nset_insert(&N, d, i);
    }
    nset_emit(&N, out_ids + r * k, out_d2 + r * k);
  }
  free(N.d2);
  free(N.id);
  return ZO_OK;
}

/* ------------------------------------------------------------------------- */
/* (2) the zd-tree: keys                                                      */
/* ------------------------------------------------------------------------- */

/* splitmix64 at counter i (i >= 1) from seed: the published mixing function
 * of Steele, Lea and Flood applied to seed + i * golden-gamma. */
ZO_API uint64_t zo_splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + i * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static int bits_per_dim(int dim) { return 64 / dim; } /* 32 in 2D, 21 in 3D */

/* Quantise one coordinate (Section 3.1: doubles rounded to integers):
 * u = (x - lo) * S, floor, clamp into the low 2^(B-1) cells. */
static uint64_t quantise(double x, double lo, double S, int B) {
  uint64_t top = ((uint64_t)1 << (B - 1)) - 1;
  double u = (x - lo) * S;
  if (!(u >= 0.0)) return 0; /* negative (or NaN) clamps to cell 0 */
  double f = floor(u);
  if (f >= (double)top) return top;
  return (uint64_t)f;
}

/* Morton interleave (Section 1.1): coordinate c's bit j goes to key bit
 * d*j + (d-1-c). */
static uint64_t interleave(int dim, const uint64_t *qc, int B) {
  uint64_t key = 0;
  for (int j = 0; j < B; ++j)
    for (int c = 0; c < dim; ++c)
      key |= ((qc[c] >> j) & 1ULL) << (dim * j + (dim - 1 - c));
  return key;
}

/* Key of one point: quantise, add the random shift (Section 2), interleave. */
static uint64_t point_key(int dim, const double *x, const double *lo,
                          const double *S, const uint64_t *shift) {
  int B = bits_per_dim(dim);
  uint64_t qc[3] = {0, 0, 0};
  for (int c = 0; c < dim; ++c) qc[c] = quantise(x[c], lo[c], S[c], B) + shift[c];
  return interleave(dim, qc, B);
}

/* Keys of n points given box lo, scale S and shift (exposed for tests). */
ZO_API void zo_keys(int dim, const double *lo, const double *S,
                    const uint64_t *shift, const double *xyz, int64_t n,
                    uint64_t *out) {
  for (int64_t i = 0; i < n; ++i) {
    double x[3] = {0, 0, 0};
    for (int c = 0; c < dim; ++c) x[c] = xyz[c * n + i];
    out[i] = point_key(dim, x, lo, S, shift);
  }
}

/* The per-coordinate shift for a seed (exposed for tests). */
ZO_API void zo_shift(int dim, uint64_t seed, uint64_t *out) {
  int B = bits_per_dim(dim);
  uint64_t mask = ((uint64_t)1 << (B - 1)) - 1;
  for (int c = 0; c < dim; ++c) out[c] = zo_splitmix64(seed, (uint64_t)c + 1) & mask;
}

/* ------------------------------------------------------------------------- */
/* the tree                                                                  */
/* ------------------------------------------------------------------------- */

typedef struct entry { uint64_t key; int64_t id; } entry;

static int entry_cmp(const void *a, const void *b) {
  const entry *x = (const entry *)a, *y = (const entry *)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->id != y->id) return x->id < y->id ? -1 : 1;
  return 0;
}

typedef struct node {
  int leaf;
  int bit;                     /* internal: the Morton bit the node splits on */
  struct node *left, *right, *parent;
  double lo[3], hi[3];         /* tight box of the node's points */
  int64_t count;               /* points in the subtree */
  entry *pts;                  /* leaf: its bucket, ascending (key, id) */
} node;

typedef struct {
  int dim, L, B;
  double lo[3], hi[3], S[3];
  uint64_t shift[3];
  int64_t cap, alloc;          /* ids in use / allocated */
  double *x[3];                /* coordinates by id */
  uint8_t *live;
  int64_t n_live;
  node *root;
  /* work counters of the last query call */
} ztree;

static node *node_new(void) {
  node *t = (node *)calloc(1, sizeof(node));
  return t;
}

static void node_free(node *t) {
  if (!t) return;
  node_free(t->left);
  node_free(t->right);
  free(t->pts);
  free(t);
}

static void box_of_points(const ztree *T, node *t, const entry *P, int64_t n) {
  for (int c = 0; c < 3; ++c) { t->lo[c] = INFINITY; t->hi[c] = -INFINITY; }
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < T->dim; ++c) {
      double v = T->x[c][P[i].id];
      if (v < t->lo[c]) t->lo[c] = v;
      if (v > t->hi[c]) t->hi[c] = v;
    }
}

static void box_of_children(const ztree *T, node *t) {
  for (int c = 0; c < T->dim; ++c) {
    t->lo[c] = fmin(t->left->lo[c], t->right->lo[c]);
    t->hi[c] = fmax(t->left->hi[c], t->right->hi[c]);
  }
}

static node *make_leaf(const ztree *T, const entry *P, int64_t n) {
  node *t = node_new();
  if (!t) return NULL;
  t->leaf = 1;
  t->bit = -1;
  t->count = n;
  t->pts = (entry *)malloc(sizeof(entry) * (size_t)(n > 0 ? n : 1));
  if (!t->pts) { free(t); return NULL; }
  memcpy(t->pts, P, sizeof(entry) * (size_t)n);
  box_of_points(T, t, P, n);
  return t;
}

/* splitUsingBit (Section 2, "Construction"): P is sorted by key and all its
 * keys agree above bit b, so the keys with bit b set form a suffix; binary
 * search for its first index. */
static int64_t split_using_bit(const entry *P, int64_t n, int b) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if ((P[mid].key >> b) & 1ULL) hi = mid; else lo = mid + 1;
  }
  return lo;
}

/* buildTree(P, b) -- Algorithm 1.  b counts the bits still available; the bit
 * examined is b-1.  A leaf when no bit is left or size(P) < sizeCutoff
 * (= L + 1).  An empty cut is not forked: the same P continues with the next
 * bit (the pruned tree of Section 2.1). */
static node *build_tree(const ztree *T, const entry *P, int64_t n, int b) {
  while (1) {
    if (b == 0 || n < T->L + 1) return make_leaf(T, P, n);
    int64_t i = split_using_bit(P, n, b - 1);
    if (i == 0 || i == n) { b--; continue; } /* empty cut */
    node *t = node_new();
    if (!t) return NULL;
    t->bit = b - 1;
    t->count = n;
    t->left = build_tree(T, P, i, b - 1);
    t->right = build_tree(T, P + i, n - i, b - 1);
    if (!t->left || !t->right) { node_free(t); return NULL; }
    t->left->parent = t;
    t->right->parent = t;
    box_of_children(T, t);
    return t;
  }
}

static int key_bits(int dim) { return dim * bits_per_dim(dim); } /* 64 or 63 */

/* Work counters of the last query call made by this thread (candidates
 * scored, boxes tested, rows answered).  Thread-local: independent queries
 * on one tree may run on several threads (the search itself only reads the
 * tree). */
typedef struct {
  int64_t cand, box, rows;
} work_count;
static _Thread_local work_count wk;

/* ------------------------------------------------------------------------- */
/* searchDown / searchUp                                                     */
/* ------------------------------------------------------------------------- */

/* squared distance from p to a box (0 inside): the withinBox test of
 * Algorithm 2 is box_dist2 <= distance(p, N, k) */
static double box_dist2(int dim, const double *p, const double *lo, const double *hi) {
  double t[3] = {0, 0, 0};
  for (int c = 0; c < dim; ++c) {
    if (p[c] < lo[c]) t[c] = lo[c] - p[c];
    else if (p[c] > hi[c]) t[c] = p[c] - hi[c];
    else t[c] = 0.0;
  }
  double s = t[0] * t[0] + t[1] * t[1];
  if (dim == 3) s = s + t[2] * t[2];
  return s;
}

/* squared distance from p to a box's centre */
static double centre_dist2(int dim, const double *p, const double *lo, const double *hi) {
  double m[3] = {0, 0, 0};
  for (int c = 0; c < dim; ++c) m[c] = (lo[c] + hi[c]) * 0.5;
  return sq_dist(dim, p, m);
}

static void scan_leaf(ztree *T, const node *C, const double *p, int64_t self, nset *N) {
  for (int64_t i = 0; i < C->count; ++i) {
    int64_t q = C->pts[i].id;
    if (q == self) continue;
    double x[3] = {0, 0, 0};
    for (int c = 0; c < T->dim; ++c) x[c] = T->x[c][q];
    double d = sq_dist(T->dim, p, x);
    wk.cand++;
    if (N->size < N->k || cand_less(d, q, N->d2[N->k - 1], N->id[N->k - 1]))
      nset_insert(N, d, q);
  }
}

/* searchDown(T, p, N) -- Algorithm 2 */
static void search_down(ztree *T, const node *t, const double *p, int64_t self, nset *N) {
  wk.box++;
  if (box_dist2(T->dim, p, t->lo, t->hi) > nset_radius(N)) return;
  if (t->leaf) { scan_leaf(T, t, p, self, N); return; }
  double dl = centre_dist2(T->dim, p, t->left->lo, t->left->hi);
  double dr = centre_dist2(T->dim, p, t->right->lo, t->right->hi);
  if (dl < dr) {
    search_down(T, t->left, p, self, N);
    search_down(T, t->right, p, self, N);
  } else {
    search_down(T, t->right, p, self, N);
    search_down(T, t->left, p, self, N);
  }
}

/* withinBox(C, p, -r) of Algorithm 3 in squared form: N is full, p lies in
 * C's box, and every face of the box is strictly farther than the worst d2. */
static int ball_inside(int dim, const double *p, const node *C, const nset *N) {
  if (N->size < N->k) return 0;
  double r = N->d2[N->k - 1];
  for (int c = 0; c < dim; ++c) {
    if (p[c] < C->lo[c] || p[c] > C->hi[c]) return 0;
    double a = p[c] - C->lo[c], b = C->hi[c] - p[c];
    if (!(a * a > r) || !(b * b > r)) return 0;
  }
  return 1;
}

/* searchUp(C, p) -- Algorithm 3 */
static void search_up(ztree *T, const node *C, const double *p, int64_t self, nset *N) {
  scan_leaf(T, C, p, self, N);
  const node *P = C->parent;
  while (P && !ball_inside(T->dim, p, C, N)) {
    if (P->left == C) search_down(T, P->right, p, self, N);
    else search_down(T, P->left, p, self, N);
    C = P;
    P = C->parent;
  }
}

/* ------------------------------------------------------------------------- */
/* tree construction entry points                                            */
/* ------------------------------------------------------------------------- */

static int ensure_cap(ztree *T, int64_t need) {
  if (need <= T->alloc) return ZO_OK;
  int64_t na = T->alloc ? T->alloc : 16;
  while (na < need) na *= 2;
  for (int c = 0; c < 3; ++c) {
    double *nx = (double *)realloc(T->x[c], sizeof(double) * (size_t)na);
    if (!nx) return ZO_ENOMEM;
    T->x[c] = nx;
  }
  uint8_t *nl = (uint8_t *)realloc(T->live, (size_t)na);
  if (!nl) return ZO_ENOMEM;
  memset(nl + T->alloc, 0, (size_t)(na - T->alloc));
  T->live = nl;
  T->alloc = na;
  return ZO_OK;
}

/* Build: copy points, fix the box (given, or the bounding cube of the data),
 * take the shift (given, or drawn from the seed), key, sort (Section 2,
 * "Construction"), run Algorithm 1. */
ZO_API void zo_free(void *h);

ZO_API void *zo_build(int dim, int leaf_size, const double *box_lo,
                      const double *box_hi, uint64_t seed, const uint64_t *shift,
                      const double *xyz, int64_t n, int *status) {
  *status = ZO_EINVAL;
  if ((dim != 2 && dim != 3) || leaf_size < 1 || n < 0) return NULL;
  if ((box_lo == NULL) != (box_hi == NULL)) return NULL;
  if (n == 0 && !box_lo) return NULL;
  ztree *T = (ztree *)calloc(1, sizeof(ztree));
  if (!T) { *status = ZO_ENOMEM; return NULL; }
  T->dim = dim;
  T->L = leaf_size;
  T->B = bits_per_dim(dim);
  if (ensure_cap(T, n) != ZO_OK) { *status = ZO_ENOMEM; zo_free(T); return NULL; }
  for (int c = 0; c < dim; ++c)
    for (int64_t i = 0; i < n; ++i) T->x[c][i] = xyz[c * n + i];
  for (int64_t i = 0; i < n; ++i) T->live[i] = 1;
  T->cap = n;
  T->n_live = n;
  if (box_lo) {
    for (int c = 0; c < dim; ++c) {
      if (!(box_hi[c] > box_lo[c])) { zo_free(T); *status = ZO_EINVAL; return NULL; }
      T->lo[c] = box_lo[c];
      T->hi[c] = box_hi[c];
    }
    for (int c = 0; c < dim; ++c)
      T->S[c] = ldexp(1.0, T->B - 1) / (T->hi[c] - T->lo[c]);
  } else {
    /* the bounding cube: per-coordinate minimum, common side = the largest
     * extent (1 if every point coincides) */
    double side = 0.0;
    double mn[3], mx[3];
    for (int c = 0; c < dim; ++c) {
      mn[c] = INFINITY; mx[c] = -INFINITY;
      for (int64_t i = 0; i < n; ++i) {
        if (T->x[c][i] < mn[c]) mn[c] = T->x[c][i];
        if (T->x[c][i] > mx[c]) mx[c] = T->x[c][i];
      }
      if (mx[c] - mn[c] > side) side = mx[c] - mn[c];
    }
    if (!(side > 0.0)) side = 1.0;
    for (int c = 0; c < dim; ++c) {
      T->lo[c] = mn[c];
      T->hi[c] = mn[c] + side;
      T->S[c] = ldexp(1.0, T->B - 1) / side;
    }
  }
  if (shift) {
    for (int c = 0; c < dim; ++c) {
      if (shift[c] >> (T->B - 1)) { zo_free(T); *status = ZO_EINVAL; return NULL; }
      T->shift[c] = shift[c];
    }
  } else {
    zo_shift(dim, seed, T->shift);
  }
  if (n > 0) {
    entry *P = (entry *)malloc(sizeof(entry) * (size_t)n);
    if (!P) { *status = ZO_ENOMEM; zo_free(T); return NULL; }
    for (int64_t i = 0; i < n; ++i) {
      double x[3] = {0, 0, 0};
      for (int c = 0; c < dim; ++c) x[c] = T->x[c][i];
      P[i].key = point_key(dim, x, T->lo, T->S, T->shift);
      P[i].id = i;
    }
    qsort(P, (size_t)n, sizeof(entry), entry_cmp);
    T->root = build_tree(T, P, n, key_bits(dim));
    free(P);
    if (!T->root) { *status = ZO_ENOMEM; zo_free(T); return NULL; }
  }
  *status = ZO_OK;
  return T;
}

ZO_API void zo_free(void *h) {
  ztree *T = (ztree *)h;
  if (!T) return;
  node_free(T->root);
  for (int c = 0; c < 3; ++c) free(T->x[c]);
  free(T->live);
  free(T);
}

/* box lo, scale S and shift of a tree (for key parity tests) */
ZO_API void zo_params(void *h, double *lo, double *hi, double *S, uint64_t *shift) {
  ztree *T = (ztree *)h;
  for (int c = 0; c < T->dim; ++c) {
    lo[c] = T->lo[c];
    hi[c] = T->hi[c];
    S[c] = T->S[c];
    shift[c] = T->shift[c];
  }
}

ZO_API void zo_info(void *h, int64_t *n_live, int64_t *cap, int64_t *n_leaves,
                    int64_t *n_internal, int32_t *depth);

/* ------------------------------------------------------------------------- */
/* queries                                                                   */
/* ------------------------------------------------------------------------- */

/* the leaf holding id: descend by the key bits of its own entry */
static const node *leaf_of_key(const node *t, uint64_t key) {
  while (t && !t->leaf) t = ((key >> t->bit) & 1ULL) ? t->right : t->left;
  return t;
}

static uint64_t key_of_id(const ztree *T, int64_t id) {
  double x[3] = {0, 0, 0};
  for (int c = 0; c < T->dim; ++c) x[c] = T->x[c][id];
  return point_key(T->dim, x, T->lo, T->S, T->shift);
}

/* Per-row work of the searches below: when row_cand / row_box are given,
 * row r receives the candidates scored and the boxes tested for its query
 * (test and measurement instrumentation; the search itself is unchanged). */
static void note_work(const ztree *T, int64_t r, int64_t c0, int64_t b0, int64_t *row_cand,
                      int64_t *row_box) {
  if (row_cand) row_cand[r] = wk.cand - c0;
  if (row_box) row_box[r] = wk.box - b0;
}

/* Leaf-based all-points rows (Section 2, "Upward search algorithm"): for
 * every id in qids (NULL: every id < cap) run searchUp from its own leaf.
 * Rows of dead ids are padded. */
ZO_API int zo_knn_rows_work(void *h, const int64_t *qids, int64_t m, int k,
                            int32_t *out_ids, double *out_d2, int64_t *row_cand,
                            int64_t *row_box) {
  ztree *T = (ztree *)h;
  if (k < 1 || m < 0) return ZO_EINVAL;
  nset N;
  N.k = k;
  N.d2 = (double *)malloc(sizeof(double) * (size_t)k);
  N.id = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
  if (!N.d2 || !N.id) { free(N.d2); free(N.id); return ZO_ENOMEM; }
  wk.cand = wk.box = wk.rows = 0;
  for (int64_t r = 0; r < m; ++r) {
    int64_t id = qids ? qids[r] : r;
    const int64_t c0 = wk.cand, b0 = wk.box;
    N.size = 0;
    if (id >= 0 && id < T->cap && T->live[id] && T->root) {
      double p[3] = {0, 0, 0};
      for (int c = 0; c < T->dim; ++c) p[c] = T->x[c][id];
      const node *C = leaf_of_key(T->root, key_of_id(T, id));
      search_up(T, C, p, id, &N);
      wk.rows++;
    }
    note_work(T, r, c0, b0, row_cand, row_box);
    nset_emit(&N, out_ids + r * k, out_d2 + r * k);
  }
  free(N.d2);
  free(N.id);
  return ZO_OK;
}

ZO_API int zo_knn_rows(void *h, const int64_t *qids, int64_t m, int k,
                       int32_t *out_ids, double *out_d2) {
  return zo_knn_rows_work(h, qids, m, k, out_ids, out_d2, NULL, NULL);
}

/* Bit-based dynamic queries (Section 2): key the query with the tree's box
 * and shift (clamped), descend by the node bits to a leaf, run searchUp with
 * nothing excluded. */
ZO_API int zo_knn_ext_work(void *h, const double *q, int64_t m, int k,
                           int32_t *out_ids, double *out_d2, int64_t *row_cand,
                           int64_t *row_box) {
  ztree *T = (ztree *)h;
  if (k < 1 || m < 0) return ZO_EINVAL;
  nset N;
  N.k = k;
  N.d2 = (double *)malloc(sizeof(double) * (size_t)k);
  N.id = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
  if (!N.d2 || !N.id) { free(N.d2); free(N.id); return ZO_ENOMEM; }
  wk.cand = wk.box = wk.rows = 0;
  for (int64_t r = 0; r < m; ++r) {
    double p[3] = {0, 0, 0};
    for (int c = 0; c < T->dim; ++c) p[c] = q[c * m + r];
    const int64_t c0 = wk.cand, b0 = wk.box;
    N.size = 0;
    if (T->root) {
      const node *C = leaf_of_key(T->root, point_key(T->dim, p, T->lo, T->S, T->shift));
      search_up(T, C, p, -1, &N);
    }
    wk.rows++;
    note_work(T, r, c0, b0, row_cand, row_box);
    nset_emit(&N, out_ids + r * k, out_d2 + r * k);
  }
  free(N.d2);
  free(N.id);
  return ZO_OK;
}

ZO_API int zo_knn_ext(void *h, const double *q, int64_t m, int k,
                      int32_t *out_ids, double *out_d2) {
  return zo_knn_ext_work(h, q, m, k, out_ids, out_d2, NULL, NULL);
}

/* Root-based rows (Section 2): searchDown from the root with empty N. */
ZO_API int zo_knn_root_work(void *h, const int64_t *qids, int64_t m, int k,
                            int32_t *out_ids, double *out_d2, int64_t *row_cand,
                            int64_t *row_box) {
  ztree *T = (ztree *)h;
  if (k < 1 || m < 0) return ZO_EINVAL;
  nset N;
  N.k = k;
  N.d2 = (double *)malloc(sizeof(double) * (size_t)k);
  N.id = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
  if (!N.d2 || !N.id) { free(N.d2); free(N.id); return ZO_ENOMEM; }
  wk.cand = wk.box = wk.rows = 0;
  for (int64_t r = 0; r < m; ++r) {
    int64_t id = qids ? qids[r] : r;
    const int64_t c0 = wk.cand, b0 = wk.box;
    N.size = 0;
    if (id >= 0 && id < T->cap && T->live[id] && T->root) {
      double p[3] = {0, 0, 0};
      for (int c = 0; c < T->dim; ++c) p[c] = T->x[c][id];
      search_down(T, T->root, p, id, &N);
      wk.rows++;
    }
    note_work(T, r, c0, b0, row_cand, row_box);
    nset_emit(&N, out_ids + r * k, out_d2 + r * k);
  }
  free(N.d2);
  free(N.id);
  return ZO_OK;
}

ZO_API int zo_knn_root(void *h, const int64_t *qids, int64_t m, int k,
                       int32_t *out_ids, double *out_d2) {
  return zo_knn_root_work(h, qids, m, k, out_ids, out_d2, NULL, NULL);
}

/* candidates evaluated, box tests and rows of the last query call */
ZO_API void zo_counters(void *h, int64_t *cand, int64_t *box, int64_t *rows) {
  (void)h;
  *cand = wk.cand;
  *box = wk.box;
  *rows = wk.rows;
}

/* ------------------------------------------------------------------------- */
/* batch updates                                                             */
/* ------------------------------------------------------------------------- */

static int64_t collect(const node *t, entry *out) {
  if (!t) return 0;
  if (t->leaf) {
    memcpy(out, t->pts, sizeof(entry) * (size_t)t->count);
    return t->count;
  }
  int64_t a = collect(t->left, out);
  return a + collect(t->right, out + a);
}

static uint64_t min_key(const node *t) {
  while (!t->leaf) t = t->left;
  return t->pts[0].key;
}

static uint64_t max_key(const node *t) {
  while (!t->leaf) t = t->right;
  return t->pts[t->count - 1].key;
}

static int high_bit(uint64_t v) { return 63 - __builtin_clzll(v); }

/* merge two ascending entry lists */
static void merge_entries(const entry *a, int64_t na, const entry *b, int64_t nb, entry *out) {
  int64_t i = 0, j = 0, o = 0;
  while (i < na && j < nb) out[o++] = (entry_cmp(&a[i], &b[j]) < 0) ? a[i++] : b[j++];
  while (i < na) out[o++] = a[i++];
  while (j < nb) out[o++] = b[j++];
}

/* batchInsert(T, P) -- Algorithm 4, returning the (possibly new) subtree.
 * P is ascending by (key, id) and non-empty. */
static node *batch_insert(const ztree *T, node *t, const entry *P, int64_t m, int *err) {
  if (m == 0) return t;
  if (!t) return build_tree(T, P, m, key_bits(T->dim));
  /* highest bit on which the merged key set differs */
  uint64_t lo = min_key(t) < P[0].key ? min_key(t) : P[0].key;
  uint64_t hi = max_key(t) > P[m - 1].key ? max_key(t) : P[m - 1].key;
  int g = lo == hi ? -1 : high_bit(lo ^ hi);
  if (t->leaf) {
    entry *merged = (entry *)malloc(sizeof(entry) * (size_t)(t->count + m));
    if (!merged) { *err = ZO_ENOMEM; return t; }
    merge_entries(t->pts, t->count, P, m, merged);
    node *r;
    if (t->count + m < T->L + 1) {
      /* room in the leaf: insert the points into it */
      r = make_leaf(T, merged, t->count + m);
    } else {
      /* split the leaf: rebuild its points with Algorithm 1 */
      r = build_tree(T, merged, t->count + m, key_bits(T->dim));
    }
    free(merged);
    if (!r) { *err = ZO_ENOMEM; return t; }
    r->parent = t->parent;
    node_free(t);
    return r;
  }
  if (g > t->bit) {
    /* some new keys leave the node's prefix: a new internal node on bit g,
     * with the old subtree (all on one side of g) and the new points */
    node *nn = node_new();
    if (!nn) { *err = ZO_ENOMEM; return t; }
    int side = (int)((min_key(t) >> g) & 1ULL);
    int64_t i = split_using_bit(P, m, g);
    node *parent = t->parent;
    nn->bit = g;
    nn->count = t->count + m;
    if (side == 0) {
      nn->left = batch_insert(T, t, P, i, err);
      nn->right = build_tree(T, P + i, m - i, key_bits(T->dim));
    } else {
      nn->left = build_tree(T, P, i, key_bits(T->dim));
      nn->right = batch_insert(T, t, P + i, m - i, err);
    }
    if (!nn->left || !nn->right) { *err = ZO_ENOMEM; return nn; }
    nn->left->parent = nn;
    nn->right->parent = nn;
    nn->parent = parent;
    box_of_children(T, nn);
    return nn;
  }
  /* b = T->bit; i = splitUsingBit(P, b); bit-0 points go left */
  int64_t i = split_using_bit(P, m, t->bit);
  t->left = batch_insert(T, t->left, P, i, err);
  t->right = batch_insert(T, t->right, P + i, m - i, err);
  t->left->parent = t;
  t->right->parent = t;
  t->count += m;
  box_of_children(T, t);
  return t;
}

/* Insert a batch of m points (SoA, stride m); they get ids cap, cap+1, ...
 * The whole batch is rejected (tree unchanged) if a point leaves the
 * declared box. */
ZO_API int zo_insert(void *h, const double *xyz, int64_t m, int32_t *out_new_ids) {
  ztree *T = (ztree *)h;
  if (m < 0) return ZO_EINVAL;
  if (m == 0) return ZO_OK;
  for (int64_t i = 0; i < m; ++i)
    for (int c = 0; c < T->dim; ++c) {
      double v = xyz[c * m + i];
      if (!(v >= T->lo[c] && v <= T->hi[c])) return ZO_EBOUNDS;
    }
  if (ensure_cap(T, T->cap + m) != ZO_OK) return ZO_ENOMEM;
  entry *P = (entry *)malloc(sizeof(entry) * (size_t)m);
  if (!P) return ZO_ENOMEM;
  for (int64_t i = 0; i < m; ++i) {
    int64_t id = T->cap + i;
    for (int c = 0; c < T->dim; ++c) T->x[c][id] = xyz[c * m + i];
    T->live[id] = 1;
    P[i].key = key_of_id(T, id);
    P[i].id = id;
    if (out_new_ids) out_new_ids[i] = (int32_t)id;
  }
  qsort(P, (size_t)m, sizeof(entry), entry_cmp);
  int err = ZO_OK;
  T->root = batch_insert(T, T->root, P, m, &err);
  if (T->root) T->root->parent = NULL;
  free(P);
  T->cap += m;
  T->n_live += m;
  return err;
}

/* Delete D (ascending by (key, id)) from subtree t; returns the new subtree
 * (NULL when emptied).  Tight boxes are recomputed; a node left with at most
 * L points becomes a leaf; a node with an empty side is replaced by the
 * other side. */
static node *batch_delete(const ztree *T, node *t, const entry *D, int64_t m, int *err) {
  if (m == 0 || !t) return t;
  if (t->leaf) {
    int64_t o = 0, j = 0;
    for (int64_t i = 0; i < t->count; ++i) {
      while (j < m && entry_cmp(&D[j], &t->pts[i]) < 0) j++;
      if (j < m && entry_cmp(&D[j], &t->pts[i]) == 0) continue;
      t->pts[o++] = t->pts[i];
    }
    t->count = o;
    if (o == 0) { node_free(t); return NULL; }
    box_of_points(T, t, t->pts, o);
    return t;
  }
  int64_t i = split_using_bit(D, m, t->bit);
  node *parent = t->parent;
  t->left = batch_delete(T, t->left, D, i, err);
  t->right = batch_delete(T, t->right, D + i, m - i, err);
  if (!t->left || !t->right) {
    node *rest = t->left ? t->left : t->right;
    t->left = t->right = NULL;
    node_free(t);
    if (rest) rest->parent = parent;
    return rest;
  }
  t->count = t->left->count + t->right->count;
  if (t->count < T->L + 1) {
    entry *all = (entry *)malloc(sizeof(entry) * (size_t)t->count);
    if (!all) { *err = ZO_ENOMEM; return t; }
    int64_t c = collect(t, all);
    node *leaf = make_leaf(T, all, c);
    free(all);
    if (!leaf) { *err = ZO_ENOMEM; return t; }
    leaf->parent = parent;
    node_free(t);
    return leaf;
  }
  t->left->parent = t;
  t->right->parent = t;
  box_of_children(T, t);
  return t;
}

/* Delete a batch of ids.  The whole batch is rejected (tree unchanged) if an
 * id is out of range, dead, or repeated. */
ZO_API int zo_delete(void *h, const int32_t *ids, int64_t m) {
  ztree *T = (ztree *)h;
  if (m < 0) return ZO_EINVAL;
  if (m == 0) return ZO_OK;
  uint8_t *seen = (uint8_t *)calloc((size_t)(T->cap > 0 ? T->cap : 1), 1);
  if (!seen) return ZO_ENOMEM;
  for (int64_t i = 0; i < m; ++i) {
    int64_t id = ids[i];
    if (id < 0 || id >= T->cap || !T->live[id] || seen[id]) { free(seen); return ZO_EID; }
    seen[id] = 1;
  }
  free(seen);
  entry *D = (entry *)malloc(sizeof(entry) * (size_t)m);
  if (!D) return ZO_ENOMEM;
  for (int64_t i = 0; i < m; ++i) {
    D[i].id = ids[i];
    D[i].key = key_of_id(T, ids[i]);
  }
  qsort(D, (size_t)m, sizeof(entry), entry_cmp);
  int err = ZO_OK;
  T->root = batch_delete(T, T->root, D, m, &err);
  if (T->root) T->root->parent = NULL;
  for (int64_t i = 0; i < m; ++i) T->live[ids[i]] = 0;
  T->n_live -= m;
  free(D);
  return err;
}

/* ------------------------------------------------------------------------- */
/* export (in-order), info                                                   */
/* ------------------------------------------------------------------------- */

static void count_nodes(const node *t, int64_t *nl, int64_t *ni, int d, int32_t *depth) {
  if (!t) return;
  if (d > *depth) *depth = d;
  if (t->leaf) { (*nl)++; return; }
  (*ni)++;
  count_nodes(t->left, nl, ni, d + 1, depth);
  count_nodes(t->right, nl, ni, d + 1, depth);
}

ZO_API void zo_info(void *h, int64_t *n_live, int64_t *cap, int64_t *n_leaves,
                    int64_t *n_internal, int32_t *depth) {
  ztree *T = (ztree *)h;
  *n_live = T->n_live;
  *cap = T->cap;
  *n_leaves = 0;
  *n_internal = 0;
  *depth = 0;
  count_nodes(T->root, n_leaves, n_internal, 0, depth);
}

typedef struct {
  uint64_t *keys; int32_t *ids;               /* [n_live] in-order */
  int64_t *leaf_count;                        /* [n_leaves] */
  double *leaf_lo, *leaf_hi;                  /* [n_leaves][dim] */
  int32_t *int_bit;                           /* [n_internal] in-order */
  double *int_lo, *int_hi;                    /* [n_internal][dim] */
  int64_t np, nl, ni;
  int dim;
} xout;

static void export_rec(const node *t, xout *o) {
  if (t->leaf) {
    for (int64_t i = 0; i < t->count; ++i) {
      o->keys[o->np] = t->pts[i].key;
      o->ids[o->np] = (int32_t)t->pts[i].id;
      o->np++;
    }
    o->leaf_count[o->nl] = t->count;
    for (int c = 0; c < o->dim; ++c) {
      o->leaf_lo[o->nl * o->dim + c] = t->lo[c];
      o->leaf_hi[o->nl * o->dim + c] = t->hi[c];
    }
    o->nl++;
    return;
  }
  export_rec(t->left, o);
  o->int_bit[o->ni] = t->bit;
  for (int c = 0; c < o->dim; ++c) {
    o->int_lo[o->ni * o->dim + c] = t->lo[c];
    o->int_hi[o->ni * o->dim + c] = t->hi[c];
  }
  o->ni++;
  export_rec(t->right, o);
}

/* In-order export: the sorted (key, id) sequence, leaf sizes and boxes, and
 * internal split bits and boxes.  In a full binary tree the in-order sequence
 * alternates leaf, internal, leaf, ..., leaf, and the split bits determine the
 * shape, so this is a canonical representation.  Arrays are sized by
 * zo_info. */
ZO_API void zo_export(void *h, uint64_t *keys, int32_t *ids, int64_t *leaf_count,
                      double *leaf_lo, double *leaf_hi, int32_t *int_bit,
                      double *int_lo, double *int_hi) {
  ztree *T = (ztree *)h;
  xout o = {keys, ids, leaf_count, leaf_lo, leaf_hi, int_bit, int_lo, int_hi, 0, 0, 0, T->dim};
  if (T->root) export_rec(T->root, &o);
}

/* ------------------------------------------------------------------------- */
/* gradient of L = sum over rows and neighbours of g * d2 (closed form)      */
/* ------------------------------------------------------------------------- */

/* For the fixed neighbour table ids[rows][k] (row r = point id r, -1 = none)
 * and upstream weights g[rows][k], d2(p,q) = sum_c (p_c - q_c)^2 gives
 *   dL/dp_c += 2 (p_c - q_c) g,   dL/dq_c -= 2 (p_c - q_c) g.
 * pts and grad are SoA by id with the given stride.  Accumulated in row
 * order, then neighbour order. */
ZO_API void zo_knn_grad(int dim, const double *pts, int64_t stride, int64_t rows,
                        int k, const int32_t *ids, const double *g, double *grad) {
  for (int c = 0; c < dim; ++c)
    for (int64_t i = 0; i < stride; ++i) grad[c * stride + i] = 0.0;
  for (int64_t r = 0; r < rows; ++r)
    for (int j = 0; j < k; ++j) {
      int64_t q = ids[r * k + j];
      if (q < 0) continue;
      double w = g[r * k + j];
      for (int c = 0; c < dim; ++c) {
        double t = 2.0 * (pts[c * stride + r] - pts[c * stride + q]) * w;
        grad[c * stride + r] += t;
        grad[c * stride + q] -= t;
      }
    }
}
