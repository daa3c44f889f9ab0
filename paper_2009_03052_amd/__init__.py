"""Python binding of libscc (succinct colour coding on one MI355X).

Argument marshalling only: every step runs in the HIP library ``libscc.so``
(built in-tree by ``build.py``). PyTorch provides device memory (through its
caching allocator, handed to the library as allocator hooks) and streams.
Importing this package fails loudly when the library is missing.

The names follow the C ABI in ``include/scc.h``: :class:`Table` wraps
``scc_build_table`` and the queries on a table (``occ``, ``export_level``,
``sample``, ``classify``, ``ags``); :func:`catalog` wraps ``scc_catalog``;
:func:`build_batch` wraps ``scc_build_batch``; :class:`Server` wraps the
``scc_server_*`` calls.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscc.so")

OK, EINVAL, ENOMEM, EOVERFLOW, EDEVICE, EEMPTY, EBUSY, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
ROOT_ZERO, ROOT_ALL, ROOT_BALANCED = 0, 1, 2
GATHER_AUTO, GATHER_GROUPED, GATHER_ROW = 0, 1, 2
WIDTH_AUTO, WIDTH_PER_LANE, WIDTH_PER_WAVE = 0, 1, 2

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2009_03052_amd/build.py "
                      "(there is no fallback path)")

_lib = C.CDLL(LIB_PATH)

_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class _Allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", C.c_void_p)]


class _Csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("on_device", C.c_int)]


class _BuildOpts(C.Structure):
    _fields_ = [("rooting", C.c_int), ("max_bits", C.c_int), ("stream", C.c_void_p),
                ("alloc", C.POINTER(_Allocator)), ("hub_degree", C.c_int), ("no_validate", C.c_int),
                ("gather_mode", C.c_int), ("vlc", C.c_int), ("width_test", C.c_int)]


class _Instance(C.Structure):
    _fields_ = [("g", _Csr), ("colors", C.c_void_p), ("k", C.c_int)]


class _BatchOpts(C.Structure):
    _fields_ = [("tile", C.c_int), ("hub_degree", C.c_int), ("autotune", C.c_int), ("waves", C.c_int),
                ("plain_nnz", C.c_int64)]


class BatchReport(C.Structure):
    _fields_ = [("tile", C.c_int), ("hub_degree", C.c_int), ("waves", C.c_int), ("tuned", C.c_int),
                ("grid", C.c_int), ("items", C.c_int64), ("launch_ms", C.c_double), ("pack_ms", C.c_double),
                ("total_ms", C.c_double), ("setup_ms", C.c_double), ("nprobe", C.c_int),
                ("probe_tile", C.c_int * 16), ("probe_hub", C.c_int * 16), ("probe_waves", C.c_int * 16),
                ("probe_ms", C.c_double * 16), ("plain_instances", C.c_int), ("plain_ms", C.c_double)]

    def as_dict(self):
        return {"tile": self.tile, "hub_degree": self.hub_degree, "waves": self.waves, "tuned": bool(self.tuned),
                "grid": self.grid, "items": self.items, "launch_ms": self.launch_ms, "pack_ms": self.pack_ms,
                "total_ms": self.total_ms, "setup_ms": self.setup_ms, "plain_instances": self.plain_instances,
                "plain_ms": self.plain_ms,
                "probes": [(self.probe_tile[i], self.probe_hub[i], self.probe_waves[i], self.probe_ms[i])
                           for i in range(self.nprobe)]}


class TableInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("k", C.c_int), ("rooting", C.c_int), ("num_unrooted", C.c_int),
                ("nnz", C.c_int64 * 9), ("wide_vertices", C.c_int64 * 9), ("bytes", C.c_int64),
                ("t", C.c_uint64 * 2), ("tj", (C.c_uint64 * 2) * 32), ("level_ms", C.c_double * 9),
                ("gather_ms", C.c_double * 9), ("num_hubs", C.c_int), ("stars", C.c_uint64 * 2),
                ("record_bytes", C.c_int64), ("vlc", C.c_int), ("combine_ms", C.c_double * 9),
                ("totals_ms", C.c_double), ("wide_input_rows", (C.c_int64 * 3) * 9), ("lane_width_test", C.c_int),
                ("sorted_sum_rows", C.c_int), ("grouped_combine", C.c_int)]


class _Build16Opts(C.Structure):
    _fields_ = [("rooting", C.c_int), ("stream", C.c_void_p), ("alloc", C.POINTER(_Allocator)),
                ("no_validate", C.c_int), ("chunk_terms", C.c_int64), ("max_bits", C.c_int)]


class Table16Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("k", C.c_int), ("rooting", C.c_int), ("nnz", C.c_int64 * 17),
                ("terms", C.c_int64 * 17), ("nbr_terms", C.c_int64 * 17), ("sum_nnz", C.c_int64 * 17),
                ("chunks", C.c_int64 * 17), ("bytes", C.c_int64), ("peak_bytes", C.c_int64),
                ("t", C.c_uint64 * 4), ("count_bits", C.c_int), ("level_ms", C.c_double * 17),
                ("sort_ms", C.c_double * 17),
                ("sort_bytes", C.c_double * 17), ("build_ms", C.c_double)]


class _ServerOpts(C.Structure):
    _fields_ = [("tables", C.POINTER(C.c_void_p)), ("n_tables", C.c_int), ("hbm_budget", C.c_int64),
                ("max_pending", C.c_int), ("max_active", C.c_int), ("step_samples", C.c_int64), ("chunk", C.c_int64),
                ("grid", C.c_int), ("fifo", C.c_int), ("ags_weight", C.c_double), ("stream", C.c_void_p),
                ("alloc", C.POINTER(_Allocator)), ("age_tau", C.c_double), ("small_request", C.c_int64),
                ("small_step", C.c_int64)]


class _Request(C.Structure):
    _fields_ = [("kind", C.c_int), ("table", C.c_int), ("shape", C.c_int), ("classify", C.c_int),
                ("session", C.c_int), ("n", C.c_int64), ("seed", C.c_uint64), ("stream_id", C.c_uint64),
                ("first_index", C.c_uint64)]


class _Result(C.Structure):
    _fields_ = [("id", C.c_int64), ("status", C.c_int), ("k", C.c_int), ("shape", C.c_int), ("n", C.c_int64),
                ("first_index", C.c_uint64), ("verts", C.c_void_p), ("parent", C.c_void_p), ("cls", C.c_void_p),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64), ("samples", C.c_int64),
                ("steps", C.c_int64), ("arena_peak", C.c_int64), ("arena_used", C.c_int64), ("busy_s", C.c_double),
                ("span_s", C.c_double), ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double),
                ("max_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_P = C.c_void_p
_i64, _u64, _i32 = C.c_int64, C.c_uint64, C.c_int32
_SIGS = {
    "scc_build_table": (C.c_int, [C.POINTER(_Csr), _P, C.c_int, C.POINTER(_BuildOpts), C.POINTER(_P)]),
    "scc_table_destroy": (None, [_P]),
    "scc_table_info_get": (C.c_int, [_P, C.POINTER(TableInfo)]),
    "scc_gather_bytes": (C.c_int, [_P, _P]),
    "scc_combine_bytes": (C.c_int, [_P, _P, C.POINTER(C.c_double)]),
    "scc_probe_random_reads": (C.c_int, [_P, _u64, C.c_int, _i64, _u64, _P, _P, C.POINTER(C.c_float)]),
    "scc_occ": (C.c_int, [_P, _i64, _i32, _P]),
    "scc_export_level": (C.c_int, [_P, C.c_int, C.POINTER(_i64), _P, _P, _P, _P, _P]),
    "scc_sample": (C.c_int, [_P, _i32, _i64, _u64, _u64, _u64, _P, _P, _P]),
    "scc_sample_noalloc": (C.c_int, [_P, _i32, _i64, _u64, _u64, _u64, _P, _P, _P]),
    "scc_classify": (C.c_int, [_P, _P, _i64, _P, _P, _P]),
    "scc_catalog": (C.c_int, [C.c_int, C.POINTER(_i64), _P, _P, _P, _P]),
    "scc_ags": (C.c_int, [_P, _i64, _i64, _i64, _u64, _u64, _P, _P, _P, _P, C.POINTER(_i64), _P]),
    "scc_estimate": (C.c_int, [_P, _P, _P, _i64, C.c_double, _P, _P]),
    "scc_build_batch": (C.c_int, [C.POINTER(_Instance), C.c_int, C.POINTER(_BuildOpts), C.POINTER(_BatchOpts),
                                  C.POINTER(_P), C.POINTER(BatchReport)]),
    "scc_server_create": (C.c_int, [C.POINTER(_ServerOpts), C.POINTER(_P)]),
    "scc_server_ags_open": (C.c_int, [_P, C.c_int, _i64, _u64, _u64, C.POINTER(C.c_int)]),
    "scc_server_ags_result": (C.c_int, [_P, C.c_int, _P, _P, _P, _P, _i64, C.POINTER(_i64)]),
    "scc_server_submit": (C.c_int, [_P, C.POINTER(_Request), C.POINTER(_i64)]),
    "scc_server_wait": (C.c_int, [_P, _i64, C.c_double, C.POINTER(_Result)]),
    "scc_server_release": (C.c_int, [_P, _i64]),
    "scc_server_get_stats": (C.c_int, [_P, C.POINTER(ServerStats)]),
    "scc_server_destroy": (None, [_P]),
    "scc16_build_table": (C.c_int, [C.POINTER(_Csr), _P, C.c_int, C.POINTER(_Build16Opts), C.POINTER(_P)]),
    "scc16_table_destroy": (None, [_P]),
    "scc16_table_info_get": (C.c_int, [_P, C.POINTER(Table16Info)]),
    "scc16_export_level": (C.c_int, [_P, C.c_int, C.POINTER(_i64), _P, _P, _P, C.c_int, _P]),
    "scc_release_caches": (None, []),
    "scc_num_unrooted": (C.c_int, [C.c_int]),
    "scc_balanced_rooting": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int)]),
    "scc_star_shape": (C.c_int, [C.c_int]),
    "scc_color_biased": (C.c_int, [_i64, C.c_int, C.c_double, _u64, _u64, _P, _P]),
    "scc_colour_set_probability": (C.c_double, [C.c_int, C.c_double, C.c_int, C.c_int]),
    "scc_last_error": (C.c_char_p, []),
    "scc_version": (C.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class SccError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"scc status {status}: {msg}")
        self.status = status


def _check(st: int):
    if st != OK:
        raise SccError(st, _lib.scc_last_error().decode(errors="replace"))


def exported_symbols() -> list:
    return sorted(_SIGS)


def version() -> str:
    return _lib.scc_version().decode()


# PyTorch's caching allocator behind the library's allocator hooks
def _torch_alloc(nbytes, stream, ctx):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                  int(stream) if stream else None)
    except Exception:
        return None


def _torch_free(ptr, stream, ctx):
    torch.cuda.caching_allocator_delete(ptr)


_alloc_cb = _ALLOC_FN(_torch_alloc)
_free_cb = _FREE_FN(_torch_free)
TORCH_ALLOCATOR = _Allocator(_alloc_cb, _free_cb, None)


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _u128(lo, hi) -> int:
    return int(lo) | (int(hi) << 64)


class DeviceGraph:
    """A CSR graph resident on the GPU (int64 row_ptr, int32 col_idx)."""

    def __init__(self, row_ptr, col_idx, device="cuda"):
        self.row_ptr = torch.as_tensor(np.asarray(row_ptr), dtype=torch.int64).to(device).contiguous()
        self.col_idx = torch.as_tensor(np.asarray(col_idx), dtype=torch.int32).to(device).contiguous()
        self.n = int(self.row_ptr.numel() - 1)
        self.nnz = int(self.col_idx.numel())

    @classmethod
    def from_graph(cls, g, device="cuda"):
        return cls(g.row_ptr, g.col_idx, device)


class Table:
    """The count table of one graph and colouring (``scc_build_table``).

    ``graph`` is a :class:`DeviceGraph` (borrowed device arrays, ``on_device = 1``)
    or any object with ``n``, ``row_ptr`` and ``col_idx`` numpy arrays (a host
    graph: the library copies it and the colours, ``on_device = 0``). The input
    is checked on the device unless ``validate=False``.
    """

    def __init__(self, graph, colors, k: int, rooting: int = ROOT_ZERO, max_bits: int = 128,
                 validate: bool = True, stream=None, use_torch_allocator: bool = True, hub_degree: int = 0,
                 gather_mode: int = 0, vlc: bool = False, width_test: int = WIDTH_AUTO):
        self.graph = graph
        self.k = k
        self._stream = stream
        if isinstance(graph, DeviceGraph):
            self.device = graph.row_ptr.device
            self.colors = torch.as_tensor(np.asarray(colors) if not torch.is_tensor(colors) else colors,
                                          dtype=torch.uint8).to(self.device).contiguous()
            csr = _Csr(graph.n, graph.nnz, graph.row_ptr.data_ptr(), graph.col_idx.data_ptr(), 1)
            cptr = _ptr(self.colors)
        else:
            self.device = torch.device("cuda", torch.cuda.current_device())
            rp = np.ascontiguousarray(graph.row_ptr, dtype=np.int64)
            ci = np.ascontiguousarray(graph.col_idx, dtype=np.int32)
            self.colors = np.ascontiguousarray(colors.cpu().numpy() if torch.is_tensor(colors) else colors,
                                               dtype=np.uint8)
            csr = _Csr(int(rp.size - 1), int(ci.size), rp.ctypes.data, ci.ctypes.data, 0)
            cptr = C.c_void_p(self.colors.ctypes.data)
        opts = _BuildOpts(rooting, max_bits, _stream_ptr(stream),
                          C.pointer(TORCH_ALLOCATOR) if use_torch_allocator else None, hub_degree,
                          0 if validate else 1, gather_mode, 1 if vlc else 0, width_test)
        self._h = _P()
        _check(_lib.scc_build_table(C.byref(csr), cptr, k, C.byref(opts), C.byref(self._h)))

    @classmethod
    def _wrap(cls, handle, graph, colors, k):
        t = cls.__new__(cls)
        t.graph, t.colors, t.k, t._stream, t._h = graph, colors, k, None, _P(handle)
        t.device = graph.row_ptr.device
        return t

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.scc_table_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> TableInfo:
        out = TableInfo()
        _check(_lib.scc_table_info_get(self._h, C.byref(out)))
        return out

    def gather_bytes(self) -> list:
        out = (C.c_double * 9)()
        _check(_lib.scc_gather_bytes(self._h, out))
        return list(out)

    def combine_bytes(self):
        """(per-level combine bytes [9], level-k totals bytes) (``scc_combine_bytes``)."""
        out = (C.c_double * 9)()
        tot = C.c_double(0)
        _check(_lib.scc_combine_bytes(self._h, out, C.byref(tot)))
        return list(out), tot.value

    def totals(self):
        """(t, [t_j]) as Python ints."""
        i = self.info()
        return _u128(i.t[0], i.t[1]), [_u128(i.tj[j][0], i.tj[j][1]) for j in range(i.num_unrooted)]

    def star_count(self) -> int:
        """Uncoloured k-stars of the graph (tables built with ROOT_BALANCED; else 0)."""
        i = self.info()
        return _u128(i.stars[0], i.stars[1])

    def occ(self, v: int, key: int = -1) -> int:
        out = (C.c_uint64 * 2)()
        _check(_lib.scc_occ(self._h, v, key, out))
        return _u128(out[0], out[1])

    def export_level(self, h: int, stream=None, to_host: bool = True):
        """(off int64[n+1], key uint16[nnz], lo uint64[nnz], hi uint64[nnz]) as numpy arrays, or
        (to_host=False) as device tensors of the same bits (int64, int16, int64, int64)."""
        nnz = _i64()
        _check(_lib.scc_export_level(self._h, h, C.byref(nnz), None, None, None, None, None))
        dev = self.device
        off = torch.empty(self.info().n + 1, dtype=torch.int64, device=dev)
        key = torch.empty(max(nnz.value, 1), dtype=torch.int16, device=dev)
        lo = torch.empty(max(nnz.value, 1), dtype=torch.int64, device=dev)
        hi = torch.empty(max(nnz.value, 1), dtype=torch.int64, device=dev)
        _check(_lib.scc_export_level(self._h, h, C.byref(nnz), _ptr(off), _ptr(key), _ptr(lo), _ptr(hi),
                                     _stream_ptr(stream)))
        n = nnz.value
        if not to_host:
            return off, key[:n], lo[:n], hi[:n]
        return (off.cpu().numpy(), key[:n].cpu().numpy().view(np.uint16), lo[:n].cpu().numpy().view(np.uint64),
                hi[:n].cpu().numpy().view(np.uint64))

    def sample(self, n: int, seed: int, stream_id: int = 0, shape: int = -1, first_index: int = 0, stream=None,
               out=None):
        """(verts int32[n, k], parent int8[n, k]) device tensors."""
        dev = self.device
        if out is None:
            verts = torch.empty((max(n, 1), self.k), dtype=torch.int32, device=dev)
            par = torch.empty((max(n, 1), self.k), dtype=torch.int8, device=dev)
        else:
            verts, par = out
        _check(_lib.scc_sample(self._h, shape, n, seed, stream_id, first_index, _ptr(verts), _ptr(par),
                               _stream_ptr(stream)))
        return verts[:n], par[:n]

    def sample_noalloc(self, verts: torch.Tensor, par: torch.Tensor, seed: int, stream_id: int = 0, shape: int = -1,
                       first_index: int = 0, stream=None):
        """``scc_sample_noalloc`` into caller-owned device tensors verts int32[n, k], par int8[n, k]."""
        n = int(verts.shape[0])
        _check(_lib.scc_sample_noalloc(self._h, shape, n, seed, stream_id, first_index, _ptr(verts), _ptr(par),
                                       _stream_ptr(stream)))

    def classify(self, verts: torch.Tensor, stream=None, want_code: bool = True, out=None):
        """(code uint32 as int32[n] or None, class uint32 as int32[n]) device tensors."""
        verts = verts.contiguous()
        n = verts.shape[0]
        dev = verts.device
        if out is None:
            cls = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
            code = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if want_code else None
        else:
            code, cls = out
        _check(_lib.scc_classify(self._h, _ptr(verts), n, _ptr(code), _ptr(cls), _stream_ptr(stream)))
        return (code[:n] if code is not None else None), cls[:n]

    def estimate(self, hits, n: int = 0, w=None, p_k: float = 0.0):
        """``scc_estimate``: (colourful-copy estimates, graph-copy estimates) per class."""
        s = num_classes(self.k)
        hits = np.ascontiguousarray(hits, dtype=np.int64)
        wv = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        c = np.zeros(s, np.float64)
        g = np.zeros(s, np.float64)
        _check(_lib.scc_estimate(self._h, hits.ctypes.data_as(_P), wv.ctypes.data_as(_P) if wv is not None else None,
                                 n, p_k, c.ctypes.data_as(_P), g.ctypes.data_as(_P)))
        return c, g

    def ags(self, cbar: int, round_size: int, budget: int, seed: int, stream_id: int = 0, stream=None):
        s = num_classes(self.k)
        nu = self.info().num_unrooted
        hits = np.zeros(s, np.int64)
        w = np.zeros(s, np.float64)
        nj = np.zeros(nu, np.int64)
        shapes = np.zeros(max(budget // max(round_size, 1), 1), np.int32)
        nr = _i64()
        _check(_lib.scc_ags(self._h, cbar, round_size, budget, seed, stream_id,
                            hits.ctypes.data_as(_P), w.ctypes.data_as(_P), nj.ctypes.data_as(_P),
                            shapes.ctypes.data_as(_P), C.byref(nr), _stream_ptr(stream)))
        return {"hits": hits, "w": w, "n_j": nj, "round_shapes": shapes[:nr.value]}



class Table16:
    """The count table for k up to 16 with sparse records (``scc16_build_table``).

    Keys are ``s_T << 16 | C`` (DFS bitstring and colour mask). ``graph`` is a
    :class:`DeviceGraph` or a host graph, as for :class:`Table`.
    """

    def __init__(self, graph, colors, k: int, rooting: int = ROOT_ZERO, validate: bool = True,
                 chunk_terms: int = 0, stream=None, use_torch_allocator: bool = True, max_bits: int = 0):
        self.graph, self.k, self._stream = graph, k, stream
        if isinstance(graph, DeviceGraph):
            self.device = graph.row_ptr.device
            self.colors = torch.as_tensor(np.asarray(colors) if not torch.is_tensor(colors) else colors,
                                          dtype=torch.uint8).to(self.device).contiguous()
            csr = _Csr(graph.n, graph.nnz, graph.row_ptr.data_ptr(), graph.col_idx.data_ptr(), 1)
            cptr = _ptr(self.colors)
        else:
            self.device = torch.device("cuda", torch.cuda.current_device())
            rp = np.ascontiguousarray(graph.row_ptr, dtype=np.int64)
            ci = np.ascontiguousarray(graph.col_idx, dtype=np.int32)
            self.colors = np.ascontiguousarray(colors.cpu().numpy() if torch.is_tensor(colors) else colors,
                                               dtype=np.uint8)
            csr = _Csr(int(rp.size - 1), int(ci.size), rp.ctypes.data, ci.ctypes.data, 0)
            cptr = C.c_void_p(self.colors.ctypes.data)
        opts = _Build16Opts(rooting, _stream_ptr(stream), C.pointer(TORCH_ALLOCATOR) if use_torch_allocator else None,
                            0 if validate else 1, chunk_terms, max_bits)
        self._h = _P()
        _check(_lib.scc16_build_table(C.byref(csr), cptr, k, C.byref(opts), C.byref(self._h)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.scc16_table_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> Table16Info:
        out = Table16Info()
        _check(_lib.scc16_table_info_get(self._h, C.byref(out)))
        return out

    def total(self) -> int:
        i = self.info()
        return sum(int(i.t[q]) << (64 * q) for q in range(4))

    def count_bits(self) -> int:
        return self.info().count_bits

    def export_words(self, h: int, nwords: int = 4, stream=None, to_host: bool = True):
        """(off int64[n+1], key uint64[nnz], words uint64[nnz, nwords]): counts as 64-bit
        words, least significant first (numpy arrays, or device tensors of the same bits)."""
        nnz = _i64()
        _check(_lib.scc16_export_level(self._h, h, C.byref(nnz), None, None, None, nwords, None))
        dev = self.device
        m = max(nnz.value, 1)
        off = torch.empty(self.info().n + 1, dtype=torch.int64, device=dev)
        key = torch.empty(m, dtype=torch.int64, device=dev)
        words = torch.empty((m, nwords), dtype=torch.int64, device=dev)
        _check(_lib.scc16_export_level(self._h, h, C.byref(nnz), _ptr(off), _ptr(key), _ptr(words), nwords,
                                       _stream_ptr(stream)))
        n = nnz.value
        if not to_host:
            return off, key[:n], words[:n]
        return off.cpu().numpy(), key[:n].cpu().numpy().view(np.uint64), words[:n].cpu().numpy().view(np.uint64)

    def export_level(self, h: int, stream=None, to_host: bool = True):
        """(off, key, lo, hi) of a table of 128-bit counts (see export_words)."""
        off, key, words = self.export_words(h, 2, stream, to_host)
        if not to_host:
            return off, key, words[:, 0], words[:, 1]
        return off, key, words[:, 0].copy(), words[:, 1].copy()

def build_batch(instances, rooting: int = ROOT_ZERO, max_bits: int = 128, tile: int = 0, hub_degree: int = 0,
                autotune: bool = False, stream=None, use_torch_allocator: bool = True, waves: int = 0,
                validate: bool = True, plain_nnz: int = 0):
    """``scc_build_batch``: instances is a list of (DeviceGraph, colours, k).
    Instances with at least ``plain_nnz`` CSR entries (0: 2^21; -1: none) are built by
    the level kernels, the others in one persistent launch. Returns ([Table], report dict)."""
    n = len(instances)
    arr = (_Instance * n)()
    keep = []
    for i, (g, colors, k) in enumerate(instances):
        col = torch.as_tensor(np.asarray(colors) if not torch.is_tensor(colors) else colors,
                              dtype=torch.uint8).to(g.row_ptr.device).contiguous()
        keep.append(col)
        arr[i] = _Instance(_Csr(g.n, g.nnz, g.row_ptr.data_ptr(), g.col_idx.data_ptr(), 1), col.data_ptr(), k)
    opts = _BuildOpts(rooting, max_bits, _stream_ptr(stream),
                      C.pointer(TORCH_ALLOCATOR) if use_torch_allocator else None, 0, 0 if validate else 1)
    bo = _BatchOpts(tile, hub_degree, 1 if autotune else 0, waves, plain_nnz)
    outs = (_P * n)()
    rep = BatchReport()
    _check(_lib.scc_build_batch(arr, n, C.byref(opts), C.byref(bo), outs, C.byref(rep)))
    tables = [Table._wrap(outs[i], instances[i][0], keep[i], instances[i][2]) for i in range(n)]
    return tables, rep.as_dict()


REQ_SAMPLE, REQ_AGS_ROUND = 0, 1


class _DeviceArray:
    """A device buffer of the library seen through __cuda_array_interface__ (no copy)."""

    def __init__(self, ptr: int, shape: tuple, typestr: str):
        self.__cuda_array_interface__ = {"shape": shape, "typestr": typestr, "data": (int(ptr), False),
                                         "version": 2, "strides": None}


def _device_view(ptr, shape, typestr):
    if not ptr or 0 in shape:
        return None
    return torch.as_tensor(_DeviceArray(ptr, shape, typestr), device="cuda")


class Server:
    """``scc_server_*``: resident tables, admission by a device-memory budget,
    continuous batching of sample and AGS-round requests."""

    def __init__(self, tables, hbm_budget: int = 1 << 30, max_pending: int = 0, max_active: int = 0,
                 step_samples: int = 0, chunk: int = 0, grid: int = 0, fifo: bool = False, stream=None,
                 use_torch_allocator: bool = True, ags_weight: float = 0.0, age_tau: float = 0.0,
                 small_request: int = 0, small_step: int = 0):
        self.tables = list(tables)
        arr = (C.c_void_p * len(self.tables))(*[t._h.value for t in self.tables])
        self._arr = arr
        opts = _ServerOpts(C.cast(arr, C.POINTER(C.c_void_p)), len(self.tables), int(hbm_budget), max_pending,
                           max_active, step_samples, chunk, grid, 1 if fifo else 0, float(ags_weight),
                           C.c_void_p(stream.cuda_stream) if stream is not None else None,
                           C.pointer(TORCH_ALLOCATOR) if use_torch_allocator else None, float(age_tau),
                           int(small_request), int(small_step))
        h = _P()
        _check(_lib.scc_server_create(C.byref(opts), C.byref(h)))
        self._h = h

    def ags_open(self, table: int, cbar: int, seed: int, stream_id: int = 0) -> int:
        sid = C.c_int()
        _check(_lib.scc_server_ags_open(self._h, table, cbar, seed, stream_id, C.byref(sid)))
        return sid.value

    def ags_result(self, session: int, table: int, cap: int = 1 << 16):
        k = self.tables[table].k
        s = num_classes(k)
        nu = self.tables[table].info().num_unrooted
        hits = np.zeros(s, np.int64)
        w = np.zeros(s, np.float64)
        nj = np.zeros(nu, np.int64)
        shapes = np.zeros(cap, np.int32)
        nr = _i64()
        _check(_lib.scc_server_ags_result(self._h, session, hits.ctypes.data_as(_P), w.ctypes.data_as(_P),
                                          nj.ctypes.data_as(_P), shapes.ctypes.data_as(_P), cap, C.byref(nr)))
        return {"hits": hits, "w": w, "n_j": nj, "round_shapes": shapes[:min(nr.value, cap)]}

    def submit(self, table: int, n: int, seed: int = 0, stream_id: int = 0, first_index: int = 0, shape: int = -1,
               classify: bool = False, session: int = -1) -> int:
        """A sample request, or (session >= 0) the next round of an AGS session."""
        kind = REQ_AGS_ROUND if session >= 0 else REQ_SAMPLE
        q = _Request(kind, table, shape, 1 if classify else 0, max(session, 0), n, seed, stream_id, first_index)
        rid = _i64()
        _check(_lib.scc_server_submit(self._h, C.byref(q), C.byref(rid)))
        return rid.value

    def wait(self, rid: int, timeout: float = 120.0, copy: bool = True):
        r = _Result()
        _check(_lib.scc_server_wait(self._h, rid, float(timeout), C.byref(r)))
        out = {"id": r.id, "status": r.status, "k": r.k, "shape": r.shape, "n": r.n, "first_index": r.first_index,
               "t_submit": r.t_submit, "t_admit": r.t_admit, "t_start": r.t_start, "t_done": r.t_done}
        v = _device_view(r.verts, (r.n, r.k), "<i4")
        p = _device_view(r.parent, (r.n, r.k), "|i1")
        c = _device_view(r.cls, (r.n,), "<u4")
        if copy:
            v = v.clone() if v is not None else None
            p = p.clone() if p is not None else None
            c = c.clone() if c is not None else None
        out.update(verts=v, parent=p, cls=c)
        return out

    def release(self, rid: int):
        _check(_lib.scc_server_release(self._h, rid))

    def stats(self):
        st = ServerStats()
        _check(_lib.scc_server_get_stats(self._h, C.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            _lib.scc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def num_unrooted(k: int) -> int:
    return _lib.scc_num_unrooted(k)


def balanced_rooting(k: int, j: int):
    """(designated rooted rank, orbit) of unrooted k-shape j under round skipping; (-1, 0) for the star."""
    orb = C.c_int(0)
    r = _lib.scc_balanced_rooting(k, j, C.byref(orb))
    return r, orb.value


def star_shape(k: int) -> int:
    return _lib.scc_star_shape(k)


def color_biased(n: int, k: int, lam: float, seed: int, stream_id: int = 0, device="cuda", stream=None,
                 out: torch.Tensor | None = None) -> torch.Tensor:
    """``scc_color_biased``: uint8[n] device colours under the biased law (Sec. 3.5)."""
    col = out if out is not None else torch.empty(max(n, 1), dtype=torch.uint8, device=device)
    _check(_lib.scc_color_biased(n, k, lam, seed, stream_id, _ptr(col), _stream_ptr(stream)))
    return col[:n]


def probe_random_reads(buf: torch.Tensor, record_bytes: int, n_reads: int, salt: int = 0, stream=None) -> float:
    """``scc_probe_random_reads``: device ms of n_reads random record reads from buf (zero-filled, on the GPU)."""
    sink = torch.zeros(1, dtype=torch.int64, device=buf.device)
    ms = C.c_float(0)
    _check(_lib.scc_probe_random_reads(_ptr(buf), buf.numel() * buf.element_size(), record_bytes, n_reads, salt,
                                       _ptr(sink), _stream_ptr(stream), C.byref(ms)))
    return float(ms.value)


def colour_set_probability(k: int, lam: float, j: int, has_zero: bool = True) -> float:
    """Probability that j given vertices get a given j-colour set (lam <= 0: uniform colours)."""
    return float(_lib.scc_colour_set_probability(k, lam, j, 1 if has_zero else 0))


def colorful_probability(k: int, lam: float = 0.0) -> float:
    """p_k: probability that a k-vertex set is colourful (uniform colours when lam <= 0)."""
    return colour_set_probability(k, lam, k, True)


def num_classes(k: int) -> int:
    n = _i64()
    _check(_lib.scc_catalog(k, C.byref(n), None, None, None, _stream_ptr()))
    return n.value


def catalog(k: int, with_sigma: bool = True, with_sigma_ij: bool = False):
    """dict with class codes, sigma_i and (optionally) sigma_ij."""
    s = num_classes(k)
    codes = np.zeros(s, np.uint32)
    sigma = np.zeros(s, np.int64) if with_sigma else None
    nu = _lib.scc_num_unrooted(k)
    sij = np.zeros(s * nu, np.int64) if with_sigma_ij else None
    n = _i64()
    _check(_lib.scc_catalog(k, C.byref(n), codes.ctypes.data_as(_P),
                            sigma.ctypes.data_as(_P) if sigma is not None else None,
                            sij.ctypes.data_as(_P) if sij is not None else None, _stream_ptr()))
    return {"codes": codes, "sigma": sigma, "sigma_ij": sij.reshape(s, nu) if sij is not None else None}


def release_caches():
    _lib.scc_release_caches()
