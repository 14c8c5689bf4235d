"""Pins of the CPU oracle against facts fixed by mathematics and by the paper, independent
of the oracle's own code: closed forms (complete and Turan graphs), the trace formula for
triangles, brute force over all k-subsets, identities, a hand-derived orientation, and the
orientation's theorems (Sec. 3.1: out-degree bound, round bound)."""
import json
import math
import os

import numpy as np
import pytest

from paper_2002_10047_amd import graphgen as gg

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def esym(sizes, k):
    """Elementary symmetric polynomial e_k of the part sizes (k-cliques of a complete
    multipartite graph pick k distinct parts, one vertex from each)."""
    e = [1] + [0] * k
    for s in sizes:
        for j in range(k, 0, -1):
            e[j] += e[j - 1] * s
    return e[k]


@pytest.mark.parametrize("n", [1, 2, 3, 5, 9, 14, 20])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8])
def test_complete_graph_closed_form(orc, n, k):
    g = gg.complete(n)
    t, pv = orc.count(g, k, per_vertex=True)
    assert t == math.comb(n, k)
    assert np.all(pv == math.comb(n - 1, k - 1))


@pytest.mark.parametrize("n,r", [(10, 2), (12, 3), (17, 4), (23, 5), (30, 7), (9, 9)])
@pytest.mark.parametrize("k", [2, 3, 4, 5, 6])
def test_turan_closed_form(orc, n, r, k):
    g = gg.turan(n, r)
    sizes = [len(range(i, n, r)) for i in range(r)]
    t, pv = orc.count(g, k, per_vertex=True)
    assert t == esym(sizes, k)
    for v in range(n):
        p = v % r
        assert int(pv[v]) == esym(sizes[:p] + sizes[p + 1:], k - 1)


@pytest.mark.parametrize("seed,n,p", [(11, 60, 0.2), (12, 200, 0.08), (13, 300, 0.3)])
def test_triangles_trace(orc, seed, n, p):
    g = gg.gnp(n, p, seed)
    A = np.zeros((n, n))
    u, v = g.edges()
    A[u, v] = 1
    A[v, u] = 1
    A3 = A @ A @ A                     # exact in float64 below 2^53
    t, pv = orc.count(g, 3, per_vertex=True)
    assert t == int(round(np.trace(A3))) // 6
    assert np.array_equal(pv.astype(np.int64), np.rint(np.diag(A3)).astype(np.int64) // 2)


def test_triangles_trace_c1(orc):
    g = gg.config_graph("c1")
    A = np.zeros((g.n, g.n))
    u, v = g.edges()
    A[u, v] = 1
    A[v, u] = 1
    d = np.einsum("ij,ji->i", A @ A, A)
    t, pv = orc.count(g, 3, per_vertex=True)
    assert t == int(round(d.sum())) // 6
    assert np.array_equal(pv.astype(np.int64), np.rint(d).astype(np.int64) // 2)


def test_brute_force_closed_forms(orc):
    for n in [6, 10, 13]:
        for k in range(1, n + 1):
            t, pv = orc.brute(gg.complete(n), k)
            assert t == math.comb(n, k)
            assert np.all(pv == math.comb(n - 1, k - 1))
    assert orc.brute(gg.empty(12), 3)[0] == 0
    assert orc.brute(gg.turan(12, 3), 4)[0] == 0
    assert orc.brute(gg.turan(12, 3), 3)[0] == 64


@pytest.mark.parametrize("seed", range(8))
def test_count_matches_brute_force(orc, seed):
    r = gg.rng(100 + seed)
    n = int(r.integers(8, 31))
    p = float(r.uniform(0.25, 0.8))
    g = gg.gnp(n, p, 200 + seed)
    for k in range(1, 9):
        tb, pvb = orc.brute(g, k)
        t, pv = orc.count(g, k, per_vertex=True)
        assert t == tb, (n, p, k)
        assert np.array_equal(pv, pvb)


def test_planted_clique_brute_40(orc):
    # 40 vertices: G(40, 0.3) plus a planted K12
    g0 = gg.gnp(40, 0.3, 7)
    u, v = g0.edges()
    mem = np.arange(5, 17)
    ia, ib = np.triu_indices(12, 1)
    g = gg.csr_from_pairs(40, np.concatenate([u, mem[ia]]), np.concatenate([v, mem[ib]]))
    for k in [4, 6, 8]:
        tb, pvb = orc.brute(g, k)
        t, pv = orc.count(g, k, per_vertex=True)
        assert t == tb and np.array_equal(pv, pvb)
        assert t >= math.comb(12, k)


def test_identities(orc):
    g = gg.gnp(300, 0.1, 5)
    assert orc.count(g, 1) == g.n
    assert orc.count(g, 2) == g.m
    t2, pv2 = orc.count(g, 2, per_vertex=True)
    assert np.array_equal(pv2.astype(np.int64), g.degrees())
    for k in [3, 4, 5]:
        t, pv = orc.count(g, k, per_vertex=True)
        assert int(pv.sum()) == k * t
    for n in [4, 7, 50]:
        assert orc.count(gg.cycle(n), 3) == 0
        assert orc.count(gg.star(n), 3) == 0
    assert orc.count(gg.cycle(3), 3) == 1
    assert orc.count(gg.empty(0), 3) == 0
    assert orc.count(gg.empty(10), 2) == 0


def test_disjoint_union_additive(orc):
    gs = [gg.gnp(40, 0.4, 1), gg.complete(9), gg.turan(20, 4), gg.cycle(12)]
    u, vo = gg.disjoint_union(gs)
    for k in [3, 4, 5]:
        t, pv = orc.count(u, k, per_vertex=True)
        parts = [orc.count(g, k, per_vertex=True) for g in gs]
        assert t == sum(p[0] for p in parts)
        assert np.array_equal(pv, np.concatenate([p[1] for p in parts]))


def test_threads_and_root_sampling(orc):
    g = gg.config_graph("c1")
    for k in [3, 4, 5]:
        t1, pv1 = orc.count(g, k, per_vertex=True, nthreads=1)
        t4, pv4 = orc.count(g, k, per_vertex=True, nthreads=4)
        assert t1 == t4 and np.array_equal(pv1, pv4)
        assert sum(orc.count(g, k, stride=7, phase=ph) for ph in range(7)) == t1


def test_relabel_invariance(orc):
    g = gg.gnp(120, 0.2, 9)
    perm = gg.rng(3).permutation(g.n)
    h = gg.relabel(g, perm)
    for k in [3, 4, 5, 6]:
        t, pv = orc.count(g, k, per_vertex=True)
        th, pvh = orc.count(h, k, per_vertex=True)
        assert t == th
        assert np.array_equal(pvh[perm], pv)


def test_c1_sanity(orc):
    g = gg.config_graph("c1")
    t, pv = orc.count(g, 4, per_vertex=True)
    assert t >= math.comb(30, 4)
    assert np.all(pv[g.planted] >= math.comb(29, 3))


def test_validate(orc):
    g = gg.gnp(50, 0.2, 1)
    assert orc.validate(g) == 0
    bad = gg.Graph(g.n, g.offsets.copy(), g.indices.copy())
    bad.indices[0] = bad.indices[1]          # duplicate / unsorted
    assert orc.validate(bad) == 4
    u, v = g.edges()
    one = gg.csr_from_pairs(g.n, u[:1], v[:1])
    asym = gg.Graph(one.n, one.offsets.copy(), one.indices.copy())
    row = int(np.nonzero(np.diff(asym.offsets))[0][1])
    asym.indices = asym.indices.copy()
    asym.indices[asym.offsets[row]] = (asym.indices[asym.offsets[row]] + 1) % g.n
    assert orc.validate(asym) != 0
    selfl = gg.Graph(3, np.array([0, 1, 2, 2]), np.array([0, 2, 1], np.int32))
    assert orc.validate(selfl) == 3


# ---------------------------------------------------------------- orientation

def test_orient_hand_example(orc):
    with open(os.path.join(GOLD, "orient_example.json")) as f:
        gold = json.load(f)
    e = np.array(gold["edges"])
    g = gg.csr_from_pairs(gold["n"], e[:, 0], e[:, 1])
    o = orc.orient(g, gold["eps"])
    assert list(o["thresholds"]) == gold["thresholds"]
    assert list(o["round"]) == gold["round"]
    assert list(o["deg_at_peel"]) == gold["deg_at_peel"]
    assert list(o["rank"]) == gold["rank"]
    for r, row in gold["out_rows_rank_space"].items():
        r = int(r)
        assert list(o["oidx"][o["ooff"][r]:o["ooff"][r + 1]]) == row


def orientation_properties(g, o, eps, degen):
    n = g.n
    rank, rnd, dap = o["rank"], o["round"], o["deg_at_peel"]
    ooff, oidx = o["ooff"], o["oidx"]
    assert np.array_equal(np.sort(rank), np.arange(n))
    # round bound: fewer than c_r/(2+eps) vertices survive a round
    bound = max(1, math.ceil(math.log(n) / math.log(2 + eps) - 1e-12)) if n > 1 else 1
    assert o["rounds"] <= bound
    # each undirected edge once, arcs ascend, rows ascending
    assert ooff[-1] == g.m
    rows = np.repeat(np.arange(n), np.diff(ooff))
    assert np.all(oidx > rows)
    assert np.all((np.diff(oidx) > 0) | (np.diff(rows) > 0))
    inv = np.empty(n, np.int64)
    inv[rank] = np.arange(n)
    a = inv[rows]
    b = inv[oidx]
    u, v = g.edges()
    assert np.array_equal(np.sort(np.minimum(a, b) * n + np.maximum(a, b)), np.sort(u * n + v))
    # out-degree at most the threshold of the vertex's round, and at most its
    # degree when it was removed
    dplus = np.diff(ooff)[rank]
    thr = o["thresholds"][rnd]
    assert np.all(dplus <= thr)
    assert np.all(dplus <= dap)
    # average degree of any subgraph is at most 2 x degeneracy
    if n:
        assert dplus.max() <= 2 * (2 + eps) * degen


@pytest.mark.parametrize("eps", [0.0, 0.5, 1.0, 2.0])
def test_orient_properties(orc, eps):
    for g in [gg.gnp(500, 0.02, 3), gg.config_graph("c1"), gg.rmat(12, 40000, seed=5),
              gg.complete(30), gg.empty(5), gg.star(40), gg.turan(40, 5)]:
        o = orc.orient(g, eps)
        orientation_properties(g, o, eps, orc.degeneracy(g))


def test_degeneracy_pins(orc):
    assert orc.degeneracy(gg.complete(12)) == 11
    assert orc.degeneracy(gg.cycle(10)) == 2
    assert orc.degeneracy(gg.star(10)) == 1
    assert orc.degeneracy(gg.empty(4)) == 0
    assert orc.degeneracy(gg.turan(12, 3)) == 8


def test_orient_threshold_rounding(orc):
    # threshold 3 * S / c with S = 2m: star with 7 leaves, eps = 1: S = 14, c = 8,
    # T_0 = floor(42 / 8) = 5: the centre (degree 7) survives round 0
    o = orc.orient(gg.star(8), 1.0)
    assert list(o["thresholds"]) == [5, 0]
    assert o["round"][0] == 1 and np.all(o["round"][1:] == 0)


# ---------------------------------------------------------------- local cliques

def test_local_cliques_complete(orc):
    n = 11
    g = gg.complete(n)
    o = orc.orient(g, 1.0)
    c = orc.local_cliques(n, o["ooff"], o["oidx"], 5)
    for r in range(n):
        for j in range(1, 6):
            assert c[r, j - 1] == math.comb(n - 1 - r, j)


def test_local_cliques_sum_is_total(orc):
    for g in [gg.gnp(200, 0.15, 4), gg.config_graph("c1")]:
        o = orc.orient(g, 1.0)
        c = orc.local_cliques(g.n, o["ooff"], o["oidx"], 6)
        for k in range(2, 8):
            assert int(c[:, k - 2].sum()) == orc.count(g, k)


def test_features_definition(orc):
    # directed path 0->1->2 plus 0->2 (a triangle in rank space)
    ooff = np.array([0, 2, 3, 3])
    oidx = np.array([1, 2, 2], np.int32)
    f = orc.features(3, ooff, oidx, np.array([0, 0, 1]))
    assert f.tolist() == [[2, 1, 0], [1, 0, 0], [0, 0, 1]]


def test_local_cliques_roots_agree_with_all_roots(orc):
    # the sampled variant (parallel over listed roots) against the all-roots routine,
    # itself pinned above by closed forms and by summing to the brute-force-pinned total
    g = gg.rmat(12, 40000, seed=5)
    o = orc.orient(g, 1.0)
    full = orc.local_cliques(g.n, o["ooff"], o["oidx"], 5)
    roots = np.random.default_rng(3).choice(g.n, 300, replace=False)
    roots = np.concatenate([roots, np.argsort(-np.diff(o["ooff"]))[:20]])
    for nt in (1, 4):
        part = orc.local_cliques_roots(g.n, o["ooff"], o["oidx"], 5, roots, nthreads=nt)
        assert np.array_equal(part, full[roots])
    assert orc.local_cliques_roots(g.n, o["ooff"], o["oidx"], 5, np.zeros(0, np.int64)).shape == (0, 5)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_vertex_cliques_closed_forms(orc, k):
    # K_n: every vertex is in C(n-1, k-1) k-cliques; Turan T(12,4), part sizes 3: a vertex
    # is in e_{k-1} of the other three parts' sizes
    g = gg.complete(13)
    assert orc.vertex_cliques(g, k, np.arange(13)).tolist() == [math.comb(12, k - 1)] * 13
    t = gg.turan(12, 4)
    e = [1, 9, 27, 27][k - 1] if k <= 4 else 0
    assert orc.vertex_cliques(t, k, np.arange(12)).tolist() == [e] * 12


def test_vertex_cliques_agree_with_per_vertex_count(orc):
    for g in [gg.gnp(120, 0.3, 7), gg.config_graph("c1"), gg.rmat(11, 20000, seed=8)]:
        verts = np.random.default_rng(1).choice(g.n, min(g.n, 150), replace=False)
        for k in (3, 4, 5):
            _, pv = orc.count(g, k, per_vertex=True, nthreads=4)
            assert np.array_equal(orc.vertex_cliques(g, k, verts, nthreads=4), pv[verts]), (g.name, k)


def _induced(g, verts):
    """Subgraph of g induced by verts (relabelled 0..len-1), built with numpy."""
    verts = np.sort(np.asarray(verts))
    pos = -np.ones(g.n, np.int64)
    pos[verts] = np.arange(verts.size)
    u = np.repeat(np.arange(g.n), np.diff(g.offsets))
    v = g.indices.astype(np.int64)
    keep = (pos[u] >= 0) & (pos[v] >= 0) & (u < v)
    return gg.csr_from_pairs(verts.size, pos[u[keep]], pos[v[keep]])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_sparsify_keeps_the_monochromatic_cliques(orc, seed):
    # the sparsified graph is the disjoint union of the colour classes' induced subgraphs,
    # so its k-cliques are the monochromatic k-cliques of G
    g = gg.gnp(300, 0.12, seed)
    for c in (1, 2, 3, 5):
        col = gg.colors(g.n, c, 100 + seed)
        h = orc.sparsify(g, col)
        assert orc.validate(h) == 0
        for k in (2, 3, 4):
            want = sum(orc.count(_induced(g, np.nonzero(col == x)[0]), k) for x in range(c))
            assert orc.count(h, k) == want, (c, k)
    assert orc.sparsify(g, np.zeros(g.n, np.int32)).m == g.m


def _clique_pairs(g, k):
    """All k-cliques (brute force) and s_z = ordered pairs of distinct k-cliques sharing
    z vertices."""
    import itertools
    adj = [set(g.indices[g.offsets[v]:g.offsets[v + 1]].tolist()) for v in range(g.n)]
    cl = [set(c) for c in itertools.combinations(range(g.n), k)
          if all(b in adj[a] for a, b in itertools.combinations(c, 2))]
    s = [0] * (k + 1)
    for i, a in enumerate(cl):
        for j, b in enumerate(cl):
            if i != j:
                s[len(a & b)] += 1
    return len(cl), s


def test_colorful_estimator_mean_and_variance(orc):
    # the appendix's sampling theorem: E[Y] = X and
    # Var[Y] = p^-2(k-1) (X (p^(k-1) - p^2(k-1)) + sum_{z=2}^{k-1} s_z (p^(2(k-1)-z+1) - p^2(k-1)))
    g = gg.gnp(16, 0.55, 5)
    k, c, T = 3, 2, 4000
    p = 1.0 / c
    X, s = _clique_pairs(g, k)
    assert X == orc.count(g, k)
    var = p ** (-2 * (k - 1)) * (X * (p ** (k - 1) - p ** (2 * (k - 1))) +
                                 sum(s[z] * (p ** (2 * (k - 1) - z + 1) - p ** (2 * (k - 1))) for z in range(2, k)))
    ys = np.array([orc.colorful_estimate(orc.count(orc.sparsify(g, gg.colors(g.n, c, 9000 + t)), k), c, k)
                   for t in range(T)])
    assert abs(ys.mean() - X) <= 5.0 * np.sqrt(var / T), (ys.mean(), X, var)
    # sample variance of T draws: within 15% of the theorem's value (its own relative
    # standard error is about sqrt(2/T) times a kurtosis factor, a few percent here)
    assert abs(ys.var(ddof=1) / var - 1.0) < 0.15, (ys.var(ddof=1), var)


def test_orderings_hand_examples(orc):
    # path 0-1-2-3-4, Goodrich-Pszona with eps = 1 (worked by hand from Alg. 3):
    # round 0: c = 5, ceil(5/3) = 2 lowest (degree, id) -> 0, 4; round 1: c = 3, one
    # vertex -> 1 (degree 1); round 2: c = 2 -> 2 (degree 1, id 2 < 3); round 3 -> 3
    p = gg.csr_from_pairs(5, np.array([0, 1, 2, 3]), np.array([1, 2, 3, 4]))
    r = orc.orient(p, 1.0, method=orc.ORIENT_GOODRICH_PSZONA)
    assert r["round"].tolist() == [0, 1, 2, 3, 0]
    assert r["rank"].tolist() == [0, 2, 3, 4, 1]
    # degree ordering of a star: leaves (degree 1) first by id, the centre last
    s = gg.star(6)
    d = orc.orient(s, 1.0, method=orc.ORIENT_DEGREE)
    deg = np.diff(s.offsets)
    centre = int(np.argmax(deg))
    assert d["rank"][centre] == s.n - 1
    assert np.diff(d["ooff"])[s.n - 1] == 0 and np.all(np.diff(d["ooff"])[: s.n - 1] == 1)
    # k-core ordering of the path: thresholds 1, 1, ... (every round removes degree <= 1)
    k = orc.orient(p, 1.0, method=orc.ORIENT_KCORE)
    assert k["round"].tolist() == [0, 1, 2, 1, 0] and k["thresholds"].tolist() == [1, 1, 1]


@pytest.mark.parametrize("method", [1, 2, 3])
def test_orderings_bounds_and_invariance(orc, method):
    import math
    eps = 1.0
    for g in [gg.gnp(300, 0.1, 2), gg.config_graph("c1"), gg.rmat(12, 40000, seed=3), gg.turan(40, 5),
              gg.complete(15), gg.cycle(9)]:
        r = orc.orient(g, eps, method=method)
        dplus = np.diff(r["ooff"])
        dg = orc.degeneracy(g)
        if method == orc.ORIENT_KCORE:
            assert dplus.max(initial=0) <= dg            # a degeneracy ordering
        if method == orc.ORIENT_GOODRICH_PSZONA:
            # c shrinks by a factor <= 2/(2+eps) per round; removed degrees < (2+eps) alpha
            assert r["rounds"] <= math.ceil(math.log(max(g.n, 1)) / math.log((2 + eps) / 2)) + 1
            assert dplus.max(initial=0) <= (2 + eps) * dg
        if method == orc.ORIENT_DEGREE:
            deg = np.diff(g.offsets)
            order = np.lexsort((np.arange(g.n), deg))
            assert np.array_equal(r["rank"][order], np.arange(g.n))
        # every ordering counts the same cliques
        lc = orc.local_cliques(g.n, r["ooff"], r["oidx"], 5)
        for k in range(2, 7):
            assert int(lc[:, k - 2].sum()) == orc.count(g, k), (g.name, method, k)


def _densest_brute(g, k):
    """max over nonempty vertex subsets S of (k-cliques inside S) / |S|, n <= 14."""
    import itertools
    adj = [set(g.indices[g.offsets[v]:g.offsets[v + 1]].tolist()) for v in range(g.n)]
    cl = [c for c in itertools.combinations(range(g.n), k)
          if all(b in adj[a] for a, b in itertools.combinations(c, 2))]
    best = 0.0
    for mask in range(1, 1 << g.n):
        size = bin(mask).count("1")
        inside = sum(1 for c in cl if all(mask >> v & 1 for v in c))
        best = max(best, inside / size)
    return best


def test_approx_peel_closed_form_and_guarantee(orc):
    # K_n: every vertex has C(n-1,k-1) = k * density cliques, so one round removes all
    for n, k in ((10, 3), (9, 4), (7, 2)):
        d, r, mask = orc.approx_peel(gg.complete(n), k, 0.5)
        assert d == math.comb(n, k) / n and r == 1 and mask.all()
    # the 1/(k(1+eps)) guarantee against the exact k-clique densest subgraph (brute force)
    for seed in (1, 2, 3):
        g = gg.gnp(13, 0.45, seed)
        for k, eps in ((2, 0.5), (3, 0.25), (3, 1.0), (4, 0.5)):
            opt = _densest_brute(g, k)
            d, r, mask = orc.approx_peel(g, k, eps)
            assert opt / (k * (1 + eps)) - 1e-12 <= d <= opt + 1e-12, (seed, k, eps, d, opt)
            # the reported set has that density
            if mask.any():
                h = orc._induced(g, mask)
                assert orc.count(h, k) / mask.sum() == d


def k4_with_isolated(z):
    """K_4 on vertices 0..3 plus z isolated vertices."""
    u = [a for a in range(4) for b in range(a + 1, 4)]
    v = [b for a in range(4) for b in range(a + 1, 4)]
    return gg.csr_from_pairs(4 + z, np.array(u), np.array(v))


def test_approx_peel_threshold_tie(orc):
    # Sec. 4.2 removes the vertices with AT MOST k(1+eps) times the density cliques.  K_4
    # plus 4 isolated vertices at k = 3, eps = 1: density 4/8, threshold 3 * 2 * 4 / 8 = 3,
    # exactly the count of every K_4 vertex.  "At most" removes all 8 in one round (best
    # density 1/2); a strict "<" would keep the K_4 for a second round at density 1.
    d, r, mask = orc.approx_peel(k4_with_isolated(4), 3, 1.0)
    assert (d, r) == (0.5, 1) and mask.all()
    # one isolated vertex fewer: threshold 24/7 > 3, the same single round either way
    d, r, mask = orc.approx_peel(k4_with_isolated(3), 3, 1.0)
    assert (d, r) == (4 / 7, 1)
    # five more: threshold 24/9 < 3 keeps the K_4 (density 1 in round 2)
    d, r, mask = orc.approx_peel(k4_with_isolated(5), 3, 1.0)
    assert (d, r) == (1.0, 2) and mask.tolist() == [True] * 4 + [False] * 5


def test_peel_closed_forms_and_guarantee(orc):
    # K_n: all counts equal, one round, density C(n,k)/n
    for n, k in ((10, 3), (8, 4)):
        d, r, rnd = orc.peel(gg.complete(n), k)
        assert r == 1 and d == math.comb(n, k) / n and np.all(rnd == 0)
    # K_6 plus a pendant path 5-6-7: round 0 removes 6, 7 (no triangles), round 1 the
    # clique; best density = C(6,3)/6 after round 0
    u = [a for a in range(6) for b in range(a + 1, 6)] + [5, 6]
    v = [b for a in range(6) for b in range(a + 1, 6)] + [6, 7]
    g = gg.csr_from_pairs(8, np.array(u), np.array(v))
    d, r, rnd = orc.peel(g, 3)
    assert rnd.tolist() == [1] * 6 + [0, 0] and r == 2 and d == 20 / 6
    # the 1/k guarantee against the exact densest subgraph (brute force)
    for seed in (1, 2, 3):
        g = gg.gnp(13, 0.5, seed)
        for k in (3, 4):
            opt = _densest_brute(g, k)
            d, r, rnd = orc.peel(g, k)
            assert opt / k - 1e-12 <= d <= opt + 1e-12, (seed, k, d, opt)
