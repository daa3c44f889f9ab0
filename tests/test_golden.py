"""Pins of the oracle against worked examples printed in the paper (tests/golden/)."""
from __future__ import annotations

import os
from collections import defaultdict

import oracle as O
import brute

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _fields(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            key, *vals = line.split()
            out[key] = vals
    return out


def test_treelet_encoding_figure():
    # Sec. 3.2, the figure of a coloured rooted treelet and its encoding
    f = _fields("treelet_encoding_fig.txt")
    parents = [int(x) for x in f["parents"]]
    colours = [int(x) for x in f["colours"]]
    s_T, s_C = f["s_T"][0], f["s_C"][0]
    adj = defaultdict(set)
    for i, p in enumerate(parents):
        if p >= 0:
            adj[i].add(p)
            adj[p].add(i)
    h = len(parents)
    # the brute-force canonical encoding of the printed tree is the printed s_T
    assert brute.rooted_string(adj, 0) == s_T
    # the oracle enumerates that shape, under that string, exactly once
    strings = [O.shape_string(h, r) for r in range(O.num_shapes(h))]
    assert strings.count(s_T) == 1
    rank = strings.index(s_T)
    # the colour set's characteristic vector (bit l = colour l) is the printed s_C,
    # and with k = 8 colours the oracle gives the coloured treelet a key
    mask = sum(1 << c for c in colours)
    assert format(mask, "08b") == s_C
    assert 0 <= O.key(8, h, rank, mask) < O.num_keys(8)
    # the order over shapes is the lexicographic order of their strings (Sec. 3.2)
    assert strings == sorted(strings)


def test_star_count_footnote():
    # Sec. 3.2 footnote on 128-bit counts: about 10^22 6-stars at a degree-2^16 node
    import numpy as np

    import graphgen as gg
    f = _fields("star_count_footnote.txt")
    k, d, approx = int(f["k"][0]), int(f["degree"][0]), float(f["approx"][0])
    g = gg.star(d)
    tab = O.Table(g, np.zeros(g.n, np.uint8), k, O.ROOT_BALANCED)
    stars = tab.star_count()
    # the oracle's star count (every k-star centred at the hub; leaves have degree 1)
    assert stars == _binom(d, k - 1)
    assert approx / 2 < stars < approx * 2
    assert stars > 2 ** 64   # beyond 64-bit counts, as the footnote warns


def _binom(n, r):
    out = 1
    for i in range(r):
        out = out * (n - i) // (i + 1)
    return out
