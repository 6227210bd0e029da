"""GHD planning on the host (sections 2.3 and 3.2): widths against closed
forms and an independent LP solver, the chosen decomposition against a
brute-force search over every decomposition of small hypergraphs, and the
selection push-down rule.  No GPU is used."""
import itertools
import random

import numpy as np
import pytest
from scipy.optimize import linprog

from paper_1708_07859_amd import lh


def E(*attr_lists, sel=(), root=()):
    return [{"attrs": list(a), "sel": i in sel, "root": i in root} for i, a in enumerate(attr_lists)]


# ---------------------------------------------------------------- widths ---

@pytest.mark.parametrize("name,n_attrs,edges,want", [
    ("one edge", 2, [[0, 1]], 1.0),
    ("triangle", 3, [[0, 1], [1, 2], [0, 2]], 1.5),
    ("4-cycle", 4, [[0, 1], [1, 2], [2, 3], [3, 0]], 2.0),
    ("5-cycle", 5, [[i, (i + 1) % 5] for i in range(5)], 2.5),
    ("K4", 4, [[a, b] for a in range(4) for b in range(a + 1, 4)], 2.0),
    ("Loomis-Whitney 4", 4, [[x for x in range(4) if x != i] for i in range(4)], 4.0 / 3.0),
    ("path of 4 edges", 5, [[i, i + 1] for i in range(4)], 3.0),
    ("star of 3 edges", 4, [[0, 1], [0, 2], [0, 3]], 3.0),
])
def test_fhw_closed_forms(name, n_attrs, edges, want):
    # rho*: K_n has n/2, the odd cycle C_n has n/2, LW_n has n/(n-1); a
    # path or star needs one edge per leaf attribute
    got = lh.ghd_fhw(n_attrs, E(*edges), (1 << len(edges)) - 1)
    assert got == pytest.approx(want, abs=1e-9), name


def lp_cover(edge_masks, bag):
    """Fractional edge cover by scipy's LP solver (an independent method)."""
    es = [edge_masks[e] for e in range(len(edge_masks)) if bag >> e & 1]
    chi = 0
    for m in es:
        chi |= m
    vs = [v for v in range(32) if chi >> v & 1]
    A = np.array([[-(1.0 if m >> v & 1 else 0.0) for m in es] for v in vs])
    r = linprog(np.ones(len(es)), A_ub=A, b_ub=-np.ones(len(vs)), bounds=[(0, None)] * len(es), method="highs")
    assert r.status == 0
    return r.fun


def random_hypergraph(rng, n_edges, n_attrs, max_arity=3):
    """n_edges edges over exactly n_attrs attributes: each attribute goes to a
    random edge, then edges are topped up to a random arity."""
    n_attrs = min(n_attrs, n_edges * max_arity)
    while True:
        edges = [set() for _ in range(n_edges)]
        for v in range(n_attrs):
            edges[rng.randrange(n_edges)].add(v)
        if all(len(e) <= max_arity for e in edges):
            break
    for e in edges:
        want = rng.randint(max(1, len(e)), max_arity)
        while len(e) < min(want, n_attrs):
            e.add(rng.randrange(n_attrs))
    return [sorted(e) for e in edges]


def masks_of(edges):
    return [sum(1 << v for v in e) for e in edges]


@pytest.mark.parametrize("seed", range(40))
def test_fhw_matches_lp_solver(seed):
    rng = random.Random(seed)
    n_edges = rng.randint(1, 8)
    edges = random_hypergraph(rng, n_edges, rng.randint(2, 10), 4)
    n_attrs = 1 + max(v for e in edges for v in e)
    m = masks_of(edges)
    for bag in rng.sample(range(1, 1 << n_edges), min(20, (1 << n_edges) - 1)):
        assert lh.ghd_fhw(n_attrs, E(*edges), bag) == pytest.approx(lp_cover(m, bag), abs=1e-7)


# ------------------------------------------------- brute-force decompositions

def set_partitions(items):
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for part in set_partitions(rest):
        for i in range(len(part)):
            yield part[:i] + [[first] + part[i]] + part[i + 1:]
        yield [[first]] + part


def rooted_trees(k):
    """Every rooted labelled tree on k nodes as a parent list (root: -1)."""
    if k == 1:
        yield [-1]
        return
    for code in itertools.product(range(k), repeat=k - 2):
        # Pruefer decoding to an edge list
        degree = [1] * k
        for x in code:
            degree[x] += 1
        edges = []
        seq = list(code)
        for x in seq:
            leaf = min(i for i in range(k) if degree[i] == 1)
            edges.append((leaf, x))
            degree[leaf] -= 1
            degree[x] -= 1
        u, v = [i for i in range(k) if degree[i] == 1]
        edges.append((u, v))
        adj = {i: [] for i in range(k)}
        for a, b in edges:
            adj[a].append(b)
            adj[b].append(a)
        for root in range(k):
            parent = [None] * k
            parent[root] = -1
            stack = [root]
            while stack:
                a = stack.pop()
                for b in adj[a]:
                    if parent[b] is None:
                        parent[b] = a
                        stack.append(b)
            yield parent


def brute_best(edges, sel, root_edges, out_mask):
    """Lexicographically best (width, nodes, depth, shared, -selection depth,
    sum of width x depth) over every GHD assigning each edge to exactly one
    node."""
    m = masks_of(edges)
    cover = {}
    best = None
    for part in set_partitions(list(range(len(edges)))):
        bags = [sum(1 << e for e in p) for p in part]
        chis = [0] * len(bags)
        for i, p in enumerate(part):
            for e in p:
                chis[i] |= m[e]
        for b in bags:
            if b not in cover:
                cover[b] = lp_cover(m, b)
        k = len(bags)
        for parent in rooted_trees(k):
            root = parent.index(-1)
            if (bags[root] & root_edges) != root_edges or (chis[root] & out_mask) != out_mask:
                continue
            if any(parent[t] >= 0 and not (chis[t] & chis[parent[t]]) for t in range(k)):
                continue
            ok = True
            for v in range(32):
                holders = [t for t in range(k) if chis[t] >> v & 1]
                tops = [t for t in holders if parent[t] < 0 or not (chis[parent[t]] >> v & 1)]
                if holders and len(tops) != 1:
                    ok = False
                    break
            if not ok:
                continue
            depth = [0] * k

            def d(t):
                return 0 if parent[t] < 0 else 1 + d(parent[t])
            depth = [d(t) for t in range(k)]
            width = max(cover[b] for b in bags)
            shared = sum(bin(chis[t] & chis[parent[t]]).count("1") for t in range(k) if parent[t] >= 0)
            seld = sum(depth[t] * bin(bags[t] & sel).count("1") for t in range(k))
            wdepth = sum(cover[bags[t]] * depth[t] for t in range(k))
            key = (round(width, 9), k, max(depth), shared, -seld, round(wdepth, 9))
            if best is None or key < best:
                best = key
    return best


@pytest.mark.parametrize("seed", range(80))
def test_choice_is_the_brute_force_optimum(seed):
    rng = random.Random(1000 + seed)
    n_edges = rng.randint(2, 5)
    edges = random_hypergraph(rng, n_edges, rng.randint(3, 6))
    n_attrs = 1 + max(v for e in edges for v in e)
    sel = [i for i in range(n_edges) if rng.random() < 0.4]
    out = sorted(rng.sample(range(n_attrs), rng.randint(0, 2)))
    sel_mask = sum(1 << i for i in sel)
    out_mask = sum(1 << v for v in out)
    g = lh.ghd_choose(n_attrs, E(*edges, sel=sel), out=out)
    want = brute_best(edges, sel_mask, 0, out_mask)
    ordinary = [t for t in range(g["n_nodes"]) if not g["pushed"][t]]
    if want[0] <= 1.0 + 1e-9:
        # width 1 is run as one generic-join node
        assert ordinary == [0]
        assert g["edges"][0] == (1 << n_edges) - 1
    else:
        dep = [0] * g["n_nodes"]
        for t in range(1, g["n_nodes"]):
            dep[t] = dep[g["parent"][t]] + 1
        wdepth = sum(g["node_fhw"][t] * dep[t] for t in ordinary)
        got = (round(g["fhw"], 9), len(ordinary), g["depth"], g["shared"], -g["sel_depth"], round(wdepth, 9))
        assert got == want
    check_structure(g, edges, sel_mask, out_mask)


def check_structure(g, edges, sel_mask, out_mask, root_edges=0):
    m = masks_of(edges)
    n = g["n_nodes"]
    assert g["parent"][0] == -1 and not g["pushed"][0]
    seen = 0
    for t in range(n):
        chi = 0
        for e in range(len(edges)):
            if g["edges"][t] >> e & 1:
                chi |= m[e]
        assert g["attrs"][t] == chi
        if t:
            assert 0 <= g["parent"][t] < t
        if g["pushed"][t]:
            # one filtered edge of a parent holding two or more edges
            p = g["parent"][t]
            assert bin(g["edges"][t]).count("1") == 1 and g["edges"][t] & sel_mask
            assert g["edges"][p] & g["edges"][t] and bin(g["edges"][p]).count("1") >= 2
        else:
            assert not (seen & g["edges"][t])
            seen |= g["edges"][t]
    assert seen == (1 << len(edges)) - 1
    assert (g["attrs"][0] & out_mask) == out_mask
    assert (g["edges"][0] & root_edges) == root_edges
    # every filtered edge sharing a node with another edge was pushed down
    for t in range(n):
        if g["pushed"][t] or bin(g["edges"][t]).count("1") < 2:
            continue
        for e in range(len(edges)):
            if (g["edges"][t] >> e & 1) and (sel_mask >> e & 1):
                assert any(g["pushed"][u] and g["parent"][u] == t and g["edges"][u] == 1 << e for u in range(n))


# ------------------------------------------------------------ named shapes

def test_triangle_is_one_node():
    g = lh.ghd_choose(3, E([0, 1], [1, 2], [0, 2]))
    assert g["n_nodes"] == 1 and g["fhw"] == pytest.approx(1.5)


def test_acyclic_query_is_compressed_to_one_node():
    # a path has width 1 under a decomposition; it is run as one node
    g = lh.ghd_choose(5, E([0, 1], [1, 2], [2, 3], [3, 4]), out=[0])
    assert g["n_nodes"] == 1 and g["edges"][0] == 0b1111


def test_five_cycle_has_width_two():
    # the cycle's fractional cover is 5/2, a two-node decomposition has 2
    g = lh.ghd_choose(5, E(*[[i, (i + 1) % 5] for i in range(5)]))
    assert g["fhw"] == pytest.approx(2.0) and g["n_nodes"] == 2


def q5_edges():
    # c=0, o=1, s=2, n=3, r=4: customer(c,n) orders(o,c) lineitem(o,s)
    # supplier(s,n) nation(n,r) region(r); selections on orders and region
    return E([0, 3], [1, 0], [1, 2], [2, 3], [3, 4], [4], sel=(1, 5))


def test_q5_shape_two_nodes_and_pushed_selections():
    g = lh.ghd_choose(5, q5_edges(), out=[3])
    # both two-node trees tie on the four rules; the cycle (width 2) is the
    # root so that the tail's result restricts it
    assert g["edges"][0] == 0b001111
    ordinary = [t for t in range(g["n_nodes"]) if not g["pushed"][t]]
    bags = sorted(g["edges"][t] for t in ordinary)
    # the 4-cycle of customer, orders, lineitem, supplier (width 2) and the
    # nation/region tail (width 1); one node over everything has width 3
    assert bags == sorted([0b001111, 0b110000])
    assert g["fhw"] == pytest.approx(2.0) and g["depth"] == 1 and g["shared"] == 1
    assert lh.ghd_fhw(5, q5_edges(), 0b111111) == pytest.approx(3.0)
    pushed = sorted(g["edges"][t] for t in range(g["n_nodes"]) if g["pushed"][t])
    assert pushed == [0b000010, 0b100000]
    check_structure(g, [e["attrs"] for e in q5_edges()], 0b100010, 1 << 3)


def test_tie_break_prefers_fewer_nodes_then_less_depth():
    # Q5's tail may hang as one node {nation, region} or as a chain
    # nation -> region: same width, the chain has more nodes and depth
    g = lh.ghd_choose(5, q5_edges(), out=[3])
    assert sum(1 for t in range(g["n_nodes"]) if not g["pushed"][t]) == 2
    # a bag-of-stars: two triangles sharing attribute 0; one node has width
    # 3, two nodes 1.5 each with one shared vertex
    two = E([0, 1], [1, 2], [0, 2], [0, 3], [3, 4], [0, 4])
    g = lh.ghd_choose(5, two)
    assert g["fhw"] == pytest.approx(1.5) and g["n_nodes"] == 2 and g["shared"] == 1


def test_selection_depth_tie_break():
    # two triangles sharing attribute 0, a selection on an edge of the second
    # one: both roots give width 1.5, two nodes, depth 1, one shared vertex;
    # the deeper selection puts the unfiltered triangle at the root
    edges = E([0, 1], [1, 2], [0, 2], [0, 3], [3, 4], [0, 4], sel=(4,))
    g = lh.ghd_choose(5, edges)
    assert g["sel_depth"] == 1
    assert g["edges"][0] == 0b000111


def test_root_must_hold_outputs_and_group_relations():
    two = E([0, 1], [1, 2], [0, 2], [0, 3], [3, 4], [0, 4])
    g = lh.ghd_choose(5, two, out=[4])
    assert g["attrs"][0] >> 4 & 1
    two[1]["root"] = True
    g = lh.ghd_choose(5, two)
    assert g["edges"][0] >> 1 & 1


def test_choose_rejects_bad_input():
    with pytest.raises(lh.LHError):
        lh.ghd_choose(3, [])
    with pytest.raises(lh.LHError):
        lh.ghd_choose(3, E(*[[0, 1]] * 9))
    with pytest.raises(lh.LHError):
        lh.ghd_choose(3, E([0, 5]))
    with pytest.raises(lh.LHError):
        lh.ghd_choose(3, E([0, 1]), out=[7])
