"""The oracle: TEST INFRASTRUCTURE ONLY.

A plain, slow, single-threaded CPU implementation (``oracle.c``) of succinct
colour coding: the build-up dynamic program of Eq. (1), totals, the uniform and
shape-restricted colourful-treelet sampler, graphlet classification, spanning
tree numbers and AGS. Only ``tests/``, the smoke check and the benchmark's
CPU-baseline leg may import this package. It shares no code with the GPU
library and neither imports the other.

Counts are exact unsigned 128-bit integers; they cross into Python as
(lo, hi) uint64 pairs and are returned as Python ints or object arrays where a
plain view is needed.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRC16 = os.path.join(_HERE, "oracle16.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ROOT_ZERO = 0
ROOT_ALL = 1
ROOT_BALANCED = 2   # round skipping: level k-1 skipped, level k at designated balanced rootings

OK, EINVAL, ENOMEM, EOVERFLOW, EEMPTY = 0, -1, -2, -3, -5


class OracleError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"oracle status {status}: {msg}")
        self.status = status


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-shared", "-fPIC",
                               "-ffp-contract=off", _SRC, _SRC16, "-o", _LIB + ".tmp"])
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC), os.path.getmtime(_SRC16)):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i64, i32, u64, u32 = C.c_int64, C.c_int32, C.c_uint64, C.c_uint32
        sig = {
            "orc_last_error": (C.c_char_p, []),
            "orc_num_shapes": (C.c_int, [C.c_int]),
            "orc_shape_string": (C.c_int, [C.c_int, C.c_int, C.c_char_p, C.c_int]),
            "orc_shape_decomp": (C.c_int, [C.c_int, C.c_int, P, P, P, P]),
            "orc_num_unrooted": (C.c_int, [C.c_int]),
            "orc_shape_unrooted": (C.c_int, [C.c_int, C.c_int]),
            "orc_key": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_uint]),
            "orc_num_keys": (C.c_int, [C.c_int]),
            "orc_check_csr": (C.c_int, [i64, P, P]),
            "orc_build": (C.c_int, [i64, P, P, P, C.c_int, C.c_int, C.POINTER(P)]),
            "orc_table_free": (None, [P]),
            "orc_level_nnz": (i64, [P, C.c_int]),
            "orc_export_level": (C.c_int, [P, C.c_int, P, P, P, P]),
            "orc_totals": (None, [P, P, P]),
            "orc_eta": (None, [P, P]),
            "orc_occ": (C.c_int, [P, i64, C.c_int, P]),
            "orc_philox4x64": (None, [P, P, P]),
            "orc_uniform_below": (C.c_int, [u64, u64, u64, u64, u64, u32, P]),
            "orc_color_biased": (C.c_int, [i64, C.c_int, u32, u64, u64, P]),
            "orc_colour_set_prob": (C.c_double, [C.c_int, u32, C.c_int, C.c_int]),
            "orc_sample": (C.c_int, [P, C.c_int, i64, u64, u64, u64, P, P]),
            "orc_canonical_code": (u32, [u32, C.c_int]),
            "orc_num_classes": (C.c_int, [C.c_int]),
            "orc_catalog_codes": (C.c_int, [C.c_int, P]),
            "orc_classify": (C.c_int, [i64, P, P, C.c_int, P, i64, P, P]),
            "orc_spanning_trees": (i64, [u32, C.c_int]),
            "orc_spanning_trees_by_shape": (C.c_int, [u32, C.c_int, P]),
            "orc_ags": (C.c_int, [P, i64, i64, i64, u64, u64, P, P, P, P, P]),
            "orc_estimate": (C.c_int, [P, P, P, i64, C.c_double, P, P]),
            "orc16_last_error": (C.c_char_p, []),
            "orc16_build": (C.c_int, [i64, P, P, P, C.c_int, C.c_int, C.POINTER(P)]),
            "orc16_table_free": (None, [P]),
            "orc16_level_nnz": (i64, [P, C.c_int]),
            "orc16_export_level": (C.c_int, [P, C.c_int, P, P, P]),
            "orc16_total": (None, [P, P]),
            "orc16_u256_ops": (None, [P, P, C.c_uint64, P, P, P, P, P]),
            "orc_balanced_rank": (C.c_int, [C.c_int, C.c_int]),
            "orc_balanced_orbit": (C.c_int, [C.c_int, C.c_int]),
            "orc_star_class": (C.c_int, [C.c_int]),
            "orc_star_count": (C.c_int, [P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _check(st: int):
    if st != OK:
        raise OracleError(st, lib().orc_last_error().decode())


def _u128(lo, hi) -> int:
    return int(lo) | (int(hi) << 64)


# --------------------------------------------------------------------------
# Treelet algebra
# --------------------------------------------------------------------------

def num_shapes(h: int) -> int:
    """Number r_h of rooted treelet shapes on h nodes."""
    return lib().orc_num_shapes(h)


def shape_string(h: int, r: int) -> str:
    """Canonical DFS bitstring of the rank-r rooted shape on h nodes."""
    buf = C.create_string_buffer(64)
    _check(lib().orc_shape_string(h, r, buf, 64))
    return buf.value.decode()


def shape_decomp(h: int, r: int):
    """(|T'|, rank T', rank T'', beta_T) of the canonical decomposition."""
    v = [C.c_int() for _ in range(4)]
    _check(lib().orc_shape_decomp(h, r, *[C.byref(x) for x in v]))
    return tuple(x.value for x in v)


def num_unrooted(h: int) -> int:
    return lib().orc_num_unrooted(h)


def shape_unrooted(h: int, r: int) -> int:
    return lib().orc_shape_unrooted(h, r)


def balanced_rank(h: int, j: int) -> int:
    """Designated (balanced) rooted rank of unrooted h-shape j, -1 for the star."""
    return lib().orc_balanced_rank(h, j)


def balanced_orbit(h: int, j: int) -> int:
    """Nodes of a copy of unrooted shape j at which the designated rooting occurs."""
    return lib().orc_balanced_orbit(h, j)


def star_class(h: int) -> int:
    return lib().orc_star_class(h)


def key(k: int, h: int, rank: int, mask: int) -> int:
    return lib().orc_key(k, h, rank, mask)


def num_keys(k: int) -> int:
    return lib().orc_num_keys(k)


# --------------------------------------------------------------------------
# Table
# --------------------------------------------------------------------------

class Table:
    """The oracle's count table for one graph and colouring."""

    def __init__(self, g, colors: np.ndarray, k: int, rooting: int = ROOT_ZERO):
        self.g = g
        self.k = k
        self.rooting = rooting
        self.colors = np.ascontiguousarray(colors, dtype=np.uint8)
        self._h = C.c_void_p()
        _check(lib().orc_build(g.n, _p(g.row_ptr), _p(g.col_idx), _p(self.colors), k, rooting,
                               C.byref(self._h)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().orc_table_free(h)
            self._h = None

    def level_nnz(self, h: int) -> int:
        return int(lib().orc_level_nnz(self._h, h))

    def export_level(self, h: int):
        """(off int64[n+1], key uint16[nnz], lo uint64[nnz], hi uint64[nnz])."""
        nnz = self.level_nnz(h)
        off = np.zeros(self.g.n + 1, np.int64)
        key = np.zeros(max(nnz, 1), np.uint16)
        lo = np.zeros(max(nnz, 1), np.uint64)
        hi = np.zeros(max(nnz, 1), np.uint64)
        _check(lib().orc_export_level(self._h, h, _p(off), _p(key), _p(lo), _p(hi)))
        return off, key[:nnz], lo[:nnz], hi[:nnz]

    def level_dict(self, h: int) -> dict:
        """{(v, key): count} of level h, counts as Python ints."""
        off, key, lo, hi = self.export_level(h)
        out = {}
        for v in range(self.g.n):
            for q in range(off[v], off[v + 1]):
                out[(v, int(key[q]))] = _u128(lo[q], hi[q])
        return out

    def totals(self):
        """(t, [t_j]) as Python ints."""
        nu = num_unrooted(self.k)
        t = np.zeros(2, np.uint64)
        tj = np.zeros(2 * max(nu, 1), np.uint64)
        lib().orc_totals(self._h, _p(t), _p(tj))
        return _u128(t[0], t[1]), [_u128(tj[2 * j], tj[2 * j + 1]) for j in range(nu)]

    def eta(self) -> list:
        out = np.zeros(2 * max(self.g.n, 1), np.uint64)
        lib().orc_eta(self._h, _p(out))
        return [_u128(out[2 * v], out[2 * v + 1]) for v in range(self.g.n)]

    def occ(self, v: int, key: int = -1) -> int:
        out = np.zeros(2, np.uint64)
        _check(lib().orc_occ(self._h, v, key, _p(out)))
        return _u128(out[0], out[1])

    def star_count(self) -> int:
        """Uncoloured k-stars of the graph: sum over v of binom(d_v, k-1)."""
        out = np.zeros(2, np.uint64)
        _check(lib().orc_star_count(self._h, _p(out)))
        return int(out[0]) | (int(out[1]) << 64)

    def sample(self, n: int, seed: int, stream: int = 0, shape: int = -1, first_index: int = 0):
        """(verts int32[n, k], parent int8[n, k])."""
        verts = np.zeros((max(n, 1), self.k), np.int32)
        par = np.zeros((max(n, 1), self.k), np.int8)
        _check(lib().orc_sample(self._h, shape, n, seed, stream, first_index, _p(verts), _p(par)))
        return verts[:n], par[:n]

    def ags(self, cbar: int, round_size: int, budget: int, seed: int, stream: int = 0):
        """AGS rounds; returns dict with hits, w, n_j, round shapes."""
        s = num_classes(self.k)
        ns = num_unrooted(self.k)
        hits = np.zeros(s, np.int64)
        w = np.zeros(s, np.float64)
        nj = np.zeros(ns, np.int64)
        shapes = np.zeros(max(budget // max(round_size, 1), 1), np.int32)
        nr = C.c_int64()
        _check(lib().orc_ags(self._h, cbar, round_size, budget, seed, stream,
                             _p(hits), _p(w), _p(nj), _p(shapes), C.byref(nr)))
        return {"hits": hits, "w": w, "n_j": nj, "round_shapes": shapes[:nr.value]}


class Table16:
    """The oracle's sparse table for k <= 16 (oracle16.c): keys s_T << 16 | C."""

    def __init__(self, g, colors: np.ndarray, k: int, rooting: int = ROOT_ZERO):
        self.g, self.k, self.rooting = g, k, rooting
        self.colors = np.ascontiguousarray(colors, dtype=np.uint8)
        self._h = C.c_void_p()
        st = lib().orc16_build(g.n, _p(g.row_ptr), _p(g.col_idx), _p(self.colors), k, rooting, C.byref(self._h))
        if st != OK:
            raise OracleError(st, lib().orc16_last_error().decode())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().orc16_table_free(h)
            self._h = None

    def level_nnz(self, h: int) -> int:
        return int(lib().orc16_level_nnz(self._h, h))

    def export_words(self, h: int):
        """(off int64[n+1], key uint64[nnz], words uint64[nnz, 4]): counts as four
        64-bit words, least significant first."""
        nnz = self.level_nnz(h)
        off = np.zeros(self.g.n + 1, np.int64)
        key = np.zeros(max(nnz, 1), np.uint64)
        words = np.zeros((max(nnz, 1), 4), np.uint64)
        st = lib().orc16_export_level(self._h, h, _p(off), _p(key), _p(words))
        if st != OK:
            raise OracleError(st, lib().orc16_last_error().decode())
        return off, key[:nnz], words[:nnz]

    def export_level(self, h: int):
        """(off, key, lo, hi): the low two words of each count (all of it below 2^128)."""
        off, key, words = self.export_words(h)
        return off, key, words[:, 0].copy(), words[:, 1].copy()

    def level_dict(self, h: int) -> dict:
        """{(v, key): count} of level h."""
        off, key, words = self.export_words(h)
        return {(v, int(key[q])): words_int(words[q]) for v in range(self.g.n) for q in range(off[v], off[v + 1])}

    def total(self) -> int:
        t = np.zeros(4, np.uint64)
        lib().orc16_total(self._h, _p(t))
        return words_int(t)


def words_int(w) -> int:
    """An unsigned integer from 64-bit words, least significant first."""
    return sum(int(x) << (64 * i) for i, x in enumerate(w))


def u256_ops(a: int, b: int, d: int):
    """The oracle's 256-bit arithmetic on (a, b, d): (a + b, a * b, a // d, a % d,
    sum overflowed, product overflowed), results mod 2^256."""
    wa = np.array([(a >> (64 * i)) & (2 ** 64 - 1) for i in range(4)], np.uint64)
    wb = np.array([(b >> (64 * i)) & (2 ** 64 - 1) for i in range(4)], np.uint64)
    s, p, q = (np.zeros(4, np.uint64) for _ in range(3))
    rem = C.c_uint64(0)
    flags = C.c_int(0)
    lib().orc16_u256_ops(_p(wa), _p(wb), d, _p(s), _p(p), _p(q), C.byref(rem), C.byref(flags))
    return words_int(s), words_int(p), words_int(q), rem.value, bool(flags.value & 1), bool(flags.value & 2)


def key16(shape_bits: int, mask: int) -> int:
    return (shape_bits << 16) | mask


def estimate(tab: "Table", hits, n: int = 0, w=None, pk: float = 0.0):
    """(colourful-copy estimates c_i, graph-copy estimates g_i = c_i / p_k) per class (Sec. 2.2);
    uniform hits of n samples, or AGS hits with their weights w."""
    s = num_classes(tab.k)
    hits = np.ascontiguousarray(hits, dtype=np.int64)
    wv = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    c = np.zeros(s, np.float64)
    g = np.zeros(s, np.float64)
    _check(lib().orc_estimate(tab._h, _p(hits), _p(wv) if wv is not None else None, n, pk, _p(c), _p(g)))
    return c, g


def check_csr(g) -> int:
    return lib().orc_check_csr(g.n, _p(g.row_ptr), _p(g.col_idx))


# --------------------------------------------------------------------------
# Random numbers
# --------------------------------------------------------------------------

def philox4x64(ctr, key) -> list:
    c = np.array(ctr, np.uint64)
    kk = np.array(key, np.uint64)
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64(_p(c), _p(kk), _p(out))
    return [int(x) for x in out]


def uniform_below(N: int, seed: int, stream: int, idx: int, draw: int) -> int:
    out = np.zeros(2, np.uint64)
    _check(lib().orc_uniform_below(N & (2**64 - 1), N >> 64, seed, stream, idx, draw, _p(out)))
    return _u128(out[0], out[1])


def lambda_units(lam: float) -> int:
    """lambda in units of 2^-32 (the biased colouring's exact parameter)"""
    return int(round(lam * 2 ** 32))


def color_biased(n: int, k: int, L: int, seed: int, stream: int = 0) -> np.ndarray:
    """Biased colouring (Sec. 3.5): colour 0 w.p. 1 - (k-1) L/2^32, others L/2^32 each."""
    out = np.zeros(max(n, 1), np.uint8)
    _check(lib().orc_color_biased(n, k, L, seed, stream, _p(out)))
    return out[:n]


def colour_set_prob(k: int, L: int, j: int, has_zero: bool) -> float:
    return float(lib().orc_colour_set_prob(k, L, j, 1 if has_zero else 0))


# --------------------------------------------------------------------------
# Graphlets
# --------------------------------------------------------------------------

def canonical_code(code: int, k: int) -> int:
    return int(lib().orc_canonical_code(code, k))


def num_classes(k: int) -> int:
    return int(lib().orc_num_classes(k))


def catalog_codes(k: int) -> np.ndarray:
    out = np.zeros(num_classes(k), np.uint32)
    _check(lib().orc_catalog_codes(k, _p(out)))
    return out


def classify(g, k: int, verts: np.ndarray):
    """(code uint32[n], class int32[n]) of each sample's induced k-graphlet."""
    verts = np.ascontiguousarray(verts, dtype=np.int32).reshape(-1, k)
    n = verts.shape[0]
    code = np.zeros(max(n, 1), np.uint32)
    cls = np.zeros(max(n, 1), np.int32)
    _check(lib().orc_classify(g.n, _p(g.row_ptr), _p(g.col_idx), k, _p(verts), n, _p(code), _p(cls)))
    return code[:n], cls[:n]


def spanning_trees(code: int, k: int) -> int:
    return int(lib().orc_spanning_trees(code, k))


def spanning_trees_by_shape(code: int, k: int) -> np.ndarray:
    out = np.zeros(max(num_unrooted(k), 1), np.int64)
    _check(lib().orc_spanning_trees_by_shape(code, k, _p(out)))
    return out[:num_unrooted(k)]


def pair_index(k: int):
    """Row-major numbering of the pairs i < j used by the adjacency code."""
    idx = {}
    q = 0
    for i in range(k):
        for j in range(i + 1, k):
            idx[(i, j)] = q
            q += 1
    return idx
