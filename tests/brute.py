"""Brute-force checkers for tiny graphs (pure Python, independent of the oracle).

* ``rooted_string`` -- the DFS bitstring of a rooted tree: '1' away from the
  root, '0' back, children visited in descending lexicographic order of their
  own '1 s 0' words (the encoding of Sec. 3.2 and its example figure).
* ``treelet_counts`` -- c(T_C, v) straight from its definition (Sec. 2.1): every
  subtree of G (edge set forming a tree, not necessarily induced) that is
  colourful, counted once per vertex it may be rooted at.
* ``pair_join_counts`` -- the per-edge pair join of Sec. 3.1: for each edge
  (v, u) and each pair of non-zero counts at v and u with disjoint colour sets
  whose merge is valid, add the product to the merged treelet, then divide by
  beta_T. A second algorithm for the same table.
* ``colourful_graphlets`` -- colourful induced k-vertex connected subgraphs and
  their isomorphism class (via networkx), for the estimator identities.
"""
from __future__ import annotations

import itertools
from collections import defaultdict

import networkx as nx


def _adj(g):
    return [set(int(x) for x in g.neighbors(v)) for v in range(g.n)]


def rooted_string(adj: dict, root) -> str:
    """Canonical DFS bitstring of the tree given by ``adj`` (dict of sets), rooted at ``root``."""

    def rec(v, p):
        words = sorted(("1" + rec(w, v) + "0" for w in adj[v] if w != p), reverse=True)
        return "".join(words)

    return rec(root, None)


def root_children_words(s: str) -> list:
    """Split a rooted string into its top-level '1 x 0' words."""
    out, depth, start = [], 0, 0
    for i, ch in enumerate(s):
        depth += 1 if ch == "1" else -1
        if depth == 0:
            out.append(s[start:i + 1])
            start = i + 1
    return out


def _is_tree(vs, edges):
    if len(edges) != len(vs) - 1:
        return False
    parent = {v: v for v in vs}

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x

    for a, b in edges:
        ra, rb = find(a), find(b)
        if ra == rb:
            return False
        parent[ra] = rb
    return True


def connected_subsets(g, size: int):
    """All connected vertex subsets of the given size (tiny graphs only)."""
    adj = _adj(g)
    found = set()

    def grow(cur, frontier):
        if len(cur) == size:
            found.add(frozenset(cur))
            return
        for w in sorted(frontier):
            if w in cur:
                continue
            nxt = cur | {w}
            key = frozenset(nxt)
            if key in _seen:
                continue
            _seen.add(key)
            grow(nxt, (frontier | adj[w]) - nxt)

    for v in range(g.n):
        _seen = {frozenset([v])}
        grow({v}, adj[v] - {v})
    return sorted(found, key=lambda s: sorted(s))


def subtrees(g, size: int):
    """Every subtree on ``size`` vertices as (vertex set, edge tuple)."""
    adj = _adj(g)
    out = []
    if size == 1:
        return [(frozenset([v]), ()) for v in range(g.n)]
    for vs in connected_subsets(g, size):
        es = [(a, b) for a in vs for b in adj[a] if a < b and b in vs]
        for sub in itertools.combinations(es, size - 1):
            if _is_tree(vs, sub):
                out.append((vs, sub))
    return out


def treelet_counts(g, colors, k: int, hmax: int | None = None):
    """{h: {(v, rooted string, colour mask): count}} from the definition."""
    hmax = k if hmax is None else hmax
    res = {}
    for h in range(1, hmax + 1):
        cnt = defaultdict(int)
        for vs, es in subtrees(g, h):
            cols = {int(colors[v]) for v in vs}
            if len(cols) != h:
                continue
            mask = sum(1 << c for c in cols)
            adj = {v: set() for v in vs}
            for a, b in es:
                adj[a].add(b)
                adj[b].add(a)
            for r in vs:
                cnt[(r, rooted_string(adj, r), mask)] += 1
        res[h] = dict(cnt)
    return res


def count_subtrees(g, size: int) -> int:
    return len(subtrees(g, size))


def rooted_copies(g, size: int):
    """{(v, rooted string): number of uncoloured rooted copies}."""
    cnt = defaultdict(int)
    for vs, es in subtrees(g, size):
        adj = {v: set() for v in vs}
        for a, b in es:
            adj[a].add(b)
            adj[b].add(a)
        for r in vs:
            cnt[(r, rooted_string(adj, r))] += 1
    return dict(cnt)


def pair_join_counts(g, colors, k: int):
    """The table by the pair join of Sec. 3.1 (strings for shapes, masks for colours)."""
    adj = _adj(g)
    levels = {1: {(v, "", 1 << int(colors[v])): 1 for v in range(g.n)}}
    by_vertex = {1: defaultdict(list)}
    for (v, s, m), c in levels[1].items():
        by_vertex[1][v].append((s, m, c))
    for h in range(2, k + 1):
        acc = defaultdict(int)
        for v in range(g.n):
            for hp in range(1, h):
                hpp = h - hp
                for (s1, m1, c1) in by_vertex[hp][v]:
                    kids = root_children_words(s1)
                    for u in adj[v]:
                        for (s2, m2, c2) in by_vertex[hpp][u]:
                            if m1 & m2:
                                continue
                            w = "1" + s2 + "0"
                            # T'' must not be smaller than any root child of T'
                            if any(w < x for x in kids):
                                continue
                            merged = w + s1
                            acc[(v, merged, m1 | m2)] += c1 * c2
        lev = {}
        bv = defaultdict(list)
        for (v, s, m), c in acc.items():
            words = root_children_words(s)
            beta = sum(1 for x in words if x == words[0])
            assert c % beta == 0
            lev[(v, s, m)] = c // beta
            bv[v].append((s, m, c // beta))
        levels[h] = lev
        by_vertex[h] = bv
    return levels


def colourful_graphlets(g, colors, k: int):
    """List of (vertex tuple, networkx graph) of colourful induced connected k-subsets."""
    adj = _adj(g)
    out = []
    for vs in connected_subsets(g, k):
        if len({int(colors[v]) for v in vs}) != k:
            continue
        H = nx.Graph()
        H.add_nodes_from(vs)
        H.add_edges_from((a, b) for a in vs for b in adj[a] if a < b and b in vs)
        out.append((tuple(sorted(vs)), H))
    return out


def aut_rooted(s: str) -> int:
    """Size of the automorphism group of the rooted tree with string s."""
    from math import factorial
    words = root_children_words(s)
    res = 1
    seen = defaultdict(int)
    for w in words:
        seen[w] += 1
        res *= aut_rooted(w[1:-1])
    for c in seen.values():
        res *= factorial(c)
    return res
