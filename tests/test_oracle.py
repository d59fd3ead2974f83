"""Pins for the CPU oracle: each checks it against something other than itself.

* published generator outputs and hand-worked Morton keys / trees (golden/),
* the rectangle property of the Morton order (paper Section 1.1),
* closed forms (1-D lattices), an independent library (scipy's cKDTree),
* structural invariants of the zd-tree (Section 2 and Algorithm 1),
* agreement of the tree search (Algorithms 2-3, leaf-, root- and bit-based)
  with the brute-force definition on adversarial inputs,
* history independence of batch updates (Algorithm 4 and deletion),
* central finite differences for the gradient.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from tests.treecheck import check_tree, tree_depth

pytestmark = pytest.mark.filterwarnings("ignore")


# ---------------------------------------------------------------- keys ----

def test_splitmix64_published_vector(golden_dir):
    rows = [l.split() for l in open(os.path.join(golden_dir, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    for ctr, hexval in rows:
        assert oracle.splitmix64(0, int(ctr)) == int(hexval, 16)


def test_shift_is_reduced_generator_output():
    # shift_c = splitmix64(seed, c+1) mod 2^(B-1); B = 32 (2D), 21 (3D)
    for dim, B in ((2, 32), (3, 21)):
        s = oracle.shift(dim, 1234)
        assert s.shape == (dim,)
        assert (s < np.uint64(1 << (B - 1))).all()


def test_morton_hand_examples(golden_dir):
    rows = [l.split() for l in open(os.path.join(golden_dir, "morton_hand.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) >= 10
    for r in rows:
        dim = int(r[0])
        x = np.array([[float(v) for v in r[1:1 + dim]]])
        sh = np.array([int(v) for v in r[1 + dim:1 + 2 * dim]], dtype=np.uint64)
        want = int(r[1 + 2 * dim])
        # scale 1 and lo 0 make the rounded coordinate the integer itself
        got = oracle.keys(dim, np.zeros(dim), np.ones(dim), sh, x)[0]
        assert int(got) == want, (r, int(got))


@pytest.mark.parametrize("dim", [2, 3])
def test_morton_rectangle_property(dim):
    # Section 1.1: every point in the box spanned by p and q lies between them
    # in Morton order.  Componentwise p <= r <= q  =>  key(p) <= key(r) <= key(q).
    rng = np.random.default_rng(7)
    B = 64 // dim
    top = 1 << (B - 1)
    sh = oracle.shift(dim, 99)
    for _ in range(20):
        a = rng.integers(0, top, (500, dim)).astype(np.float64)
        b = rng.integers(0, top, (500, dim)).astype(np.float64)
        p, q = np.minimum(a, b), np.maximum(a, b)
        t = rng.random((500, dim))
        r = np.floor(p + t * (q - p))
        kp, kr, kq = (oracle.keys(dim, np.zeros(dim), np.ones(dim), sh, z) for z in (p, r, q))
        assert (kp <= kr).all() and (kr <= kq).all()


@pytest.mark.parametrize("dim", [2, 3])
def test_rounding_fixed_points(dim):
    # box [0,1]: 0 -> cell 0, 0.5 -> cell 2^(B-2), 1 -> last cell 2^(B-1)-1;
    # outside the box clamps; rounding is monotone.
    B = 64 // dim
    lo, hi = np.zeros(dim), np.ones(dim)
    S = np.full(dim, 2.0 ** (B - 1))
    sh = np.zeros(dim, dtype=np.uint64)
    xs = np.array([0.0, 0.5, 1.0, -0.25, 1.75, 0.75])
    pts = np.zeros((len(xs), dim))
    pts[:, 0] = xs
    k = oracle.keys(dim, lo, S, sh, pts)
    # x occupies key bits d*j + d-1: recover coordinate bits from the key
    def xcoord(key):
        v = 0
        for j in range(B):
            v |= ((int(key) >> (dim * j + dim - 1)) & 1) << j
        return v
    got = [xcoord(v) for v in k]
    assert got == [0, 1 << (B - 2), (1 << (B - 1)) - 1, 0, (1 << (B - 1)) - 1, 3 << (B - 3)]
    rng = np.random.default_rng(3)
    x = np.sort(rng.uniform(-0.5, 1.5, 4000))
    p = np.zeros((4000, dim))
    p[:, 0] = x
    kk = oracle.keys(dim, lo, S, sh, p)
    assert (np.diff(kk.astype(object)) >= 0).all()


# ------------------------------------------------------------ the tree ----

def _parse_cases(path):
    cases, cur = [], None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0] == "case":
            cur = dict(name=tok[1], pts={})
        elif tok[0] == "dim":
            cur["dim"] = int(tok[1])
        elif tok[0] == "leaf":
            cur["L"] = int(tok[1])
        elif tok[0] == "point":
            cur["pts"][int(tok[1])] = [float(v) for v in tok[2:]]
        elif tok[0] == "leaves":
            cur["leaves"] = [[int(v) for v in g.split()] for g in line[len("leaves"):].split("|")]
        elif tok[0] == "bits":
            cur["bits"] = [int(v) for v in tok[1:]]
        elif tok[0] == "end":
            cases.append(cur)
    return cases


def test_hand_derived_trees(golden_dir):
    cases = _parse_cases(os.path.join(golden_dir, "tiny_trees.txt"))
    assert len(cases) == 4
    for c in cases:
        d = c["dim"]
        P = np.array([c["pts"][i] for i in range(len(c["pts"]))])
        t = oracle.Tree(P, c["L"], box=(np.zeros(d), np.ones(d)), shift=np.zeros(d, np.uint64))
        ex = t.export()
        starts = np.concatenate([[0], np.cumsum(ex["leaf_count"])])
        leaves = [list(ex["ids"][starts[j]:starts[j + 1]]) for j in range(len(ex["leaf_count"]))]
        assert leaves == c["leaves"], c["name"]
        assert list(ex["int_bit"]) == c["bits"], c["name"]
        check_tree(ex, P, c["L"])


def _datasets():
    yield "uniform2d", W.uniform(3000, 2, 1)
    yield "uniform3d", W.uniform(3000, 3, 2)
    yield "grid2d", W.grid_points((40, 40), 4, 3)
    yield "grid3d", W.grid_points((12, 12, 12), 3, 4)
    yield "dups3d", W.with_duplicates(1500, 3, 200, 5)
    yield "dups2d", W.with_duplicates(1500, 2, 30, 6)
    yield "collinear3d", W.collinear(1500, 3, 7)
    yield "clustered3d", W.clustered_small(2500, 3, 8)
    yield "allequal3d", np.full((40, 3), 0.25)


@pytest.mark.parametrize("L", [1, 4, 16])
def test_tree_invariants(L):
    for name, P in _datasets():
        d = P.shape[1]
        t = oracle.Tree(P, L, seed=11)
        ex = t.export()
        check_tree(ex, P, L)
        inf = t.info()
        assert inf["n_leaves"] == inf["n_internal"] + 1
        assert inf["depth"] == tree_depth(ex["int_bit"])
        assert inf["depth"] <= 64, name


def test_uniform_depth_is_logarithmic():
    # Theorem 1 / Section 4: uniform data gives depth about log2(n / L) + O(1)
    P = W.uniform(20000, 3, 12)
    t = oracle.Tree(P, 16, box=W.UNIT3)
    dep = t.info()["depth"]
    assert np.log2(20000 / 16) <= dep <= np.log2(20000 / 16) + 12


def test_shift_changes_structure_not_results():
    P = W.uniform(2000, 3, 13)
    a = oracle.Tree(P, 8, box=W.UNIT3, seed=1)
    b = oracle.Tree(P, 8, box=W.UNIT3, seed=2)
    assert not np.array_equal(a.export()["ids"], b.export()["ids"])
    ra, rb = a.knn_all(6), b.knn_all(6)
    assert np.array_equal(ra[0], rb[0]) and np.array_equal(ra[1], rb[1])


# ---------------------------------------------------- brute-force pins ----

@pytest.mark.parametrize("dim", [2, 3])
def test_brute_lattice_closed_form(dim):
    # points i*h on a line: the neighbours of i are i-1, i+1, i-2, i+2, ...
    # (at equal distance the lower id first), cut at the ends; d2 = (t*h)^2.
    n, k, h = 37, 9, 0.125
    P = W.lattice_1d(n, dim, 3)
    ids, d2 = oracle.brute_knn(P, k)
    for i in range(n):
        want = []
        for t in range(1, n):
            for j in (i - t, i + t):
                if 0 <= j < n:
                    want.append((j, (t * h) ** 2))
        want = want[:k]
        assert list(ids[i]) == [w[0] for w in want]
        assert list(d2[i]) == [w[1] for w in want]


@pytest.mark.parametrize("dim", [2, 3])
def test_brute_against_scipy_kdtree(dim):
    from scipy.spatial import cKDTree
    P = W.uniform(4000, dim, 21)
    Q = W.uniform(500, dim, 22)
    k = 12
    ids, d2 = oracle.brute_knn(P, k)
    dist, nb = cKDTree(P).query(P, k + 1)
    assert (nb[:, 0] == np.arange(len(P))).all()
    assert np.array_equal(ids, nb[:, 1:])
    assert np.allclose(d2, dist[:, 1:] ** 2, rtol=1e-12, atol=0)
    ids, d2 = oracle.brute_knn(P, k, queries=Q)
    dist, nb = cKDTree(P).query(Q, k)
    assert np.array_equal(ids, nb)
    assert np.allclose(d2, dist ** 2, rtol=1e-12, atol=0)


def test_brute_padding_and_dead_rows():
    P = W.uniform(5, 3, 23)
    ids, d2 = oracle.brute_knn(P, 8)
    assert (ids[:, 4:] == -1).all() and np.isinf(d2[:, 4:]).all()
    assert (ids[:, :4] >= 0).all()
    live = np.array([1, 0, 1, 1, 0], dtype=bool)
    ids, d2 = oracle.brute_knn(P, 3, live=live)
    assert (ids[1] == -1).all() and (ids[4] == -1).all()
    assert set(ids[0][:2]) == {2, 3} and ids[0][2] == -1


def test_brute_row_invariants():
    P = W.grid_points((9, 9, 9), 2, 24)
    k = 20
    ids, d2 = oracle.brute_knn(P, k)
    n = len(P)
    assert (ids != np.arange(n)[:, None]).all()
    for r in range(0, n, 37):
        row = list(zip(d2[r], ids[r]))
        assert row == sorted(row)
        assert len(set(ids[r])) == k
        for j in range(k):
            diff = P[r] - P[ids[r, j]]
            assert d2[r, j] == float(np.sum(diff * diff))  # exact on the grid


# --------------------------------------- tree search == brute force -------

@pytest.mark.parametrize("k", [1, 5, 16])
@pytest.mark.parametrize("L", [1, 8, 16])
def test_leaf_based_search_matches_brute_force(k, L):
    for name, P in _datasets():
        t = oracle.Tree(P, L, seed=31)
        a = t.knn_all(k)
        b = oracle.brute_knn(P, k)
        assert np.array_equal(a[0], b[0]), name
        assert np.array_equal(a[1], b[1]), name


@pytest.mark.parametrize("k", [3, 10])
def test_root_and_bit_based_search_match_brute_force(k):
    for name, P in _datasets():
        d = P.shape[1]
        t = oracle.Tree(P, 8, seed=41)
        a = t.knn_root(k)
        b = oracle.brute_knn(P, k)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), name
        # external queries: some inside, some outside the data, some exact copies
        Q = np.concatenate([W.uniform(200, d, 42) * 1.4 - 0.2, P[:50]])
        a = t.knn(Q, k)
        b = oracle.brute_knn(P, k, queries=Q)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), name


def test_search_work_is_bounded():
    # Lemma 1 / Theorem 2: O(k) candidates per query, independent of n
    per = []
    for n in (4000, 32000):
        P = W.uniform(n, 3, 51)
        t = oracle.Tree(P, 16, box=W.UNIT3)
        t.knn_all(10, qids=np.arange(0, n, 7))
        c = t.counters()
        per.append(c["candidates"] / c["rows"])
    assert per[1] < 1.5 * per[0] and per[1] < 400


def test_uniform2d_10k_full_matches_brute_force():
    P = W.uniform2d_10k()
    t = oracle.Tree(P, 16, box=W.UNIT2)
    a = t.knn_all(10)
    b = oracle.brute_knn(P, 10)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# -------------------------------------------------------------- updates ---

def _canon(ex, id_map=None):
    ids = ex["ids"] if id_map is None else id_map[ex["ids"]]
    return (ex["keys"].tolist(), list(ids), ex["leaf_count"].tolist(), ex["leaf_lo"].tolist(),
            ex["leaf_hi"].tolist(), ex["int_bit"].tolist(), ex["int_lo"].tolist(),
            ex["int_hi"].tolist())


def _fresh(allpts, live, L, seed, dim):
    live_ids = np.flatnonzero(live)
    t = oracle.Tree(allpts[live_ids], L, box=(np.zeros(dim), np.ones(dim)), seed=seed)
    return _canon(t.export(), live_ids)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("L", [1, 4, 16])
def test_updates_are_history_independent(dim, L):
    rng = np.random.default_rng(60 + dim + L)
    P = W.clustered_small(1200, dim, 61).clip(0, 1)
    box = (np.zeros(dim), np.ones(dim))
    t = oracle.Tree(P, L, box=box, seed=5)
    allpts = P.copy()
    live = np.ones(len(P), dtype=bool)
    for rnd in range(6):
        Q = np.concatenate([rng.random((150, dim)), W.with_duplicates(30, dim, 3, rnd).clip(0, 1)])
        new = t.insert(Q)
        assert list(new) == list(range(len(allpts), len(allpts) + len(Q)))
        allpts = np.concatenate([allpts, Q])
        live = np.concatenate([live, np.ones(len(Q), dtype=bool)])
        assert _canon(t.export()) == _fresh(allpts, live, L, 5, dim)
        D = rng.choice(np.flatnonzero(live), 170, replace=False).astype(np.int32)
        t.delete(D)
        live[D] = False
        ex = t.export()
        check_tree(ex, allpts, L, np.flatnonzero(live))
        assert _canon(ex) == _fresh(allpts, live, L, 5, dim)
        a = t.knn_all(7)
        b = oracle.brute_knn(allpts, 7, live=live)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_insert_then_delete_is_identity():
    P = W.uniform(2000, 3, 70)
    t = oracle.Tree(P, 16, box=W.UNIT3, seed=3)
    before = _canon(t.export())
    new = t.insert(W.uniform(700, 3, 71))
    t.delete(new)
    assert _canon(t.export()) == before


def test_delete_everything_then_insert():
    P = W.uniform(300, 2, 72)
    t = oracle.Tree(P, 4, box=W.UNIT2, seed=3)
    t.delete(np.arange(300, dtype=np.int32))
    assert t.info()["n_live"] == 0 and t.export()["leaf_count"].size == 0
    ids, d2 = t.knn_all(3)
    assert (ids == -1).all()
    t.insert(P[:10])
    ids, d2 = t.knn(P[:3], 2)
    assert (ids[:, 0] == np.arange(300, 303)).all()


def test_update_errors_leave_tree_unchanged():
    P = W.uniform(500, 3, 73)
    t = oracle.Tree(P, 8, box=W.UNIT3, seed=3)
    before = _canon(t.export())
    bad = W.uniform(10, 3, 74)
    bad[7, 1] = 1.0000001
    with pytest.raises(oracle.OracleError) as e:
        t.insert(bad)
    assert e.value.code == oracle.EBOUNDS
    for ids in ([1, 2, 2], [3, 500], [-1], [4, 5, 10**6]):
        with pytest.raises(oracle.OracleError) as e:
            t.delete(ids)
        assert e.value.code == oracle.EID
    t.delete([9])
    with pytest.raises(oracle.OracleError) as e:
        t.delete([9])
    assert e.value.code == oracle.EID
    t.insert(P[9:10])  # re-add the same location under a new id
    assert t.info()["n_live"] == 500
    assert before[0] == _canon(t.export())[0]  # same keys


# ------------------------------------------------------------- gradient ---

def test_gradient_central_differences():
    # L = sum_r sum_j g[r,j] d2(p_r, p_ids[r,j]) with the neighbour table held
    # fixed is quadratic in each coordinate, so a central difference is exact
    # up to rounding.  Only the terms touching the perturbed point change.
    P = W.uniform(400, 3, 80)
    k = 6
    ids, _ = oracle.brute_knn(P, k)
    g = np.random.default_rng(81).uniform(0.5, 2.0, ids.shape)
    grad = oracle.knn_grad(P, ids, g)
    rng = np.random.default_rng(82)
    rows = np.arange(len(P))
    for _ in range(150):
        i, c = int(rng.integers(0, len(P))), int(rng.integers(0, 3))
        touch = (rows == i)[:, None] | (ids == i)

        def local(Pm):
            rr, jj = np.nonzero(touch)
            diff = Pm[rr] - Pm[ids[rr, jj]]
            return float(np.sum(g[rr, jj] * np.sum(diff * diff, axis=1)))

        h = 1e-6
        Pp, Pm = P.copy(), P.copy()
        Pp[i, c] += h
        Pm[i, c] -= h
        heff = Pp[i, c] - Pm[i, c]
        fd = (local(Pp) - local(Pm)) / heff
        assert abs(fd - grad[i, c]) <= 1e-6 * max(1.0, abs(grad[i, c]))


def test_gradient_translation_invariance():
    P = W.uniform(1000, 2, 83)
    ids, _ = oracle.brute_knn(P, 5)
    g = np.random.default_rng(84).random(ids.shape)
    grad = oracle.knn_grad(P, ids, g)
    assert np.abs(grad.sum(axis=0)).max() < 1e-12


def _parse_counter_trees(path):
    trees, cur = [], None
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            w = line.split()
            if w[0] == "tree":
                cur = dict(name=w[1], L=int(w[2]), pts=[], rows=[])
            elif w[0] == "end":
                trees.append(cur)
                cur = None
            elif w[0] in ("all", "root", "ext"):
                cur["rows"].append((w[0], w[1], int(w[2]), int(w[3]), int(w[4])))
            else:
                cur["pts"].append([float(v) for v in w])
    return trees


def test_work_counters_hand_counted(golden_dir):
    """Candidates scored and boxes tested per query, counted by hand from
    Algorithms 2 and 3 on two tiny trees (tests/golden/tiny_counters.txt)."""
    trees = _parse_counter_trees(os.path.join(golden_dir, "tiny_counters.txt"))
    assert len(trees) == 2
    n_rows = 0
    for tr in trees:
        P = np.array(tr["pts"])
        t = oracle.Tree(P, tr["L"], box=(np.zeros(2), np.full(2, 8.0)),
                        shift=np.zeros(2, dtype=np.uint64))
        for mode, q, k, cand, box in tr["rows"]:
            if mode == "ext":
                Q = np.array([[float(v) for v in q.split(",")]])
                _, _, c, b = t.knn(Q, k, work=True)
            elif mode == "root":
                _, _, c, b = t.knn_root(k, qids=[int(q)], work=True)
            else:
                _, _, c, b = t.knn_all(k, qids=[int(q)], work=True)
            assert (int(c[0]), int(b[0])) == (cand, box), (tr["name"], mode, q, k)
            n_rows += 1
        # the per-call totals are the sums of the per-row counts
        _, _, c, b = t.knn_all(1, work=True)
        tot = t.counters()
        assert (tot["candidates"], tot["box_tests"]) == (int(c.sum()), int(b.sum()))
        t.close()
    assert n_rows == 14
