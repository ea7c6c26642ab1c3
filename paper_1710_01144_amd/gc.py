"""Thin ctypes binding of libgc.so (the C ABI in include/gc.h).

Argument marshalling only: device buffers are torch tensors on the current
HIP device, passed by data pointer together with torch's current stream.
Every computation runs in the library's HIP kernels; if libgc.so is missing
the binding raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libgc.so")
_lib = None

GC_OK = 0
GC_EINVAL = -1
GC_ENOTSYM = -2
GC_EDISCONNECTED = -3
GC_ERANGE = -4
GC_EWORKSPACE = -5
GC_ENOMEM = -6
GC_EDEVICE = -7

GC_VALIDATE = 0x1
GC_DIRECTED = 0x2

ORDER_PLAIN = 0
ORDER_CELF = 1
ORDER_LEARNED = 2
ORDERS = {"plain": ORDER_PLAIN, "celf": ORDER_CELF, "learned": ORDER_LEARNED}

EXPORTED = ["gc_load_csr", "gc_free_graph", "gc_graph_n", "gc_graph_nnz", "gc_workspace_size",
            "gc_workspace_init", "gc_closest_node", "gc_update_dist", "gc_marginal_gains",
            "gc_gain_words", "gc_greedy_group", "gc_strerror", "gc_last_error", "gc_mlp_block_bytes", "gc_mlp_pack",
            "gc_mlp_forward", "gc_mlp_scratch_floats", "gc_mlp_backward", "gc_mlp_adam",
            "gc_node_features", "gc_timing_enable", "gc_timing_last_ms", "gc_greedy_many",
            "gc_topk_closeness", "gc_get_tuning", "gc_set_tuning", "gc_bits_size", "gc_bits_prepare",
            "gc_bits_gains", "gc_marginal_gains_noalloc", "gc_load_csr_weighted", "gc_batch_union_size",
            "gc_greedy_batch"]
TUNING_FIELDS = ("unroll", "unroll_small", "min_edges", "min_edges_small", "level_wgs_per_cu")
MLP_PARAMS = 4801
MLP_IN = 8
MLP_HIDDEN = 64


class GCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("gc error %d: %s" % (code, msg))
        self.code = code


class GcOpts(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("bitset_width", ctypes.c_int32),
                ("block", ctypes.c_int32), ("nprefix", ctypes.c_int32),
                ("h_prefix", ctypes.POINTER(ctypes.c_int32)), ("d_mlp", ctypes.c_void_p),
                ("debug_checks", ctypes.c_int32), ("block_growth", ctypes.c_int32),
                ("log_capacity", ctypes.c_int64),
                ("h_log_round", ctypes.POINTER(ctypes.c_int32)),
                ("h_log_node", ctypes.POINTER(ctypes.c_int32)),
                ("h_log_gain", ctypes.POINTER(ctypes.c_int64)),
                ("h_log_feat", ctypes.POINTER(ctypes.c_float)),
                ("h_log_count", ctypes.POINTER(ctypes.c_int64)),
                ("d_bits", ctypes.c_void_p), ("bits_bytes", ctypes.c_size_t), ("bits_levels", ctypes.c_int32),
                ("early_exit", ctypes.c_int32), ("early_exit_seed", ctypes.c_int32)]


class GcTuning(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in TUNING_FIELDS] + [("reserved", ctypes.c_int32 * 3)]


class GcStats(ctypes.Structure):
    _fields_ = [("evals_total", ctypes.c_int64), ("evals_round1", ctypes.c_int64),
                ("evals_later", ctypes.c_int64), ("edges_alg", ctypes.c_int64),
                ("visited", ctypes.c_int64), ("gain_launches", ctypes.c_int64),
                ("closest_sources", ctypes.c_int64), ("dist_bytes", ctypes.c_int32),
                ("ecc_s1", ctypes.c_int32), ("ms_total", ctypes.c_double),
                ("ms_closest", ctypes.c_double), ("ms_round1", ctypes.c_double),
                ("ms_later", ctypes.c_double), ("ms_update", ctypes.c_double),
                ("ms_mlp", ctypes.c_double),
                ("entries_word", ctypes.c_int64), ("entries_root", ctypes.c_int64),
                ("entries_last", ctypes.c_int64), ("edges_word", ctypes.c_int64),
                ("edges_last", ctypes.c_int64), ("touched_word", ctypes.c_int64),
                ("ms_gain_gpu", ctypes.c_double), ("mlp_launches", ctypes.c_int64),
                ("bits_words", ctypes.c_int64),
                ("h_evals_per_round", ctypes.POINTER(ctypes.c_int64)), ("cut_evals", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "h_evals_per_round"}


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libgc.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError("libgc.so not built: run `python -m paper_1710_01144_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    lib.gc_load_csr.restype = ctypes.c_int
    lib.gc_load_csr.argtypes = [i32, i64, vp, vp, u32, vp, ctypes.POINTER(vp)]
    lib.gc_load_csr_weighted.restype = ctypes.c_int
    lib.gc_load_csr_weighted.argtypes = [i32, i64, vp, vp, vp, u32, vp, ctypes.POINTER(vp)]
    lib.gc_free_graph.restype = None
    lib.gc_free_graph.argtypes = [vp]
    lib.gc_graph_n.restype = i32
    lib.gc_graph_n.argtypes = [vp]
    lib.gc_graph_nnz.restype = i64
    lib.gc_graph_nnz.argtypes = [vp]
    lib.gc_workspace_size.restype = ctypes.c_int
    lib.gc_workspace_size.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.gc_workspace_init.restype = ctypes.c_int
    lib.gc_workspace_init.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.gc_closest_node.restype = ctypes.c_int
    lib.gc_topk_closeness.restype = ctypes.c_int
    lib.gc_topk_closeness.argtypes = [vp, i32, vp, ctypes.c_size_t, vp, ctypes.POINTER(i32),
                                      ctypes.POINTER(ctypes.c_int64)]
    lib.gc_closest_node.argtypes = [vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(i32),
                                    ctypes.POINTER(i64)]
    lib.gc_update_dist.restype = ctypes.c_int
    lib.gc_update_dist.argtypes = [vp, i32, vp, i32, vp, ctypes.c_size_t, vp, vp]
    lib.gc_marginal_gains.restype = ctypes.c_int
    lib.gc_marginal_gains.argtypes = [vp, vp, i32, vp, i32, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.gc_marginal_gains_noalloc.restype = ctypes.c_int
    lib.gc_marginal_gains_noalloc.argtypes = [vp, vp, i32, vp, i32, vp, vp, vp, vp]
    lib.gc_gain_words.restype = ctypes.c_int
    lib.gc_gain_words.argtypes = [vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(i64)]
    lib.gc_greedy_group.restype = ctypes.c_int
    lib.gc_greedy_group.argtypes = [vp, i32, ctypes.POINTER(GcOpts), vp, ctypes.c_size_t, vp,
                                    ctypes.POINTER(i32), ctypes.POINTER(i64),
                                    ctypes.POINTER(GcStats)]
    lib.gc_greedy_many.restype = ctypes.c_int
    lib.gc_greedy_many.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(i32), ctypes.POINTER(GcOpts),
                                   i32, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_size_t),
                                   ctypes.POINTER(vp), ctypes.POINTER(i32), ctypes.POINTER(i64),
                                   ctypes.POINTER(GcStats)]
    lib.gc_batch_union_size.restype = ctypes.c_int
    lib.gc_batch_union_size.argtypes = [i32, ctypes.POINTER(vp), i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.gc_greedy_batch.restype = ctypes.c_int
    lib.gc_greedy_batch.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(i32), ctypes.POINTER(GcOpts),
                                    i32, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_size_t),
                                    ctypes.POINTER(vp), vp, ctypes.c_size_t, ctypes.POINTER(i32),
                                    ctypes.POINTER(i64), ctypes.POINTER(GcStats)]
    lib.gc_mlp_block_bytes.restype = ctypes.c_size_t
    lib.gc_mlp_block_bytes.argtypes = []
    lib.gc_mlp_pack.restype = ctypes.c_int
    lib.gc_mlp_pack.argtypes = [vp, vp, vp]
    lib.gc_mlp_forward.restype = ctypes.c_int
    lib.gc_mlp_forward.argtypes = [vp, vp, i32, vp, vp, vp, vp]
    lib.gc_mlp_scratch_floats.restype = ctypes.c_size_t
    lib.gc_mlp_scratch_floats.argtypes = [i32]
    lib.gc_mlp_backward.restype = ctypes.c_int
    lib.gc_mlp_backward.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp, vp, vp]
    lib.gc_mlp_adam.restype = ctypes.c_int
    lib.gc_mlp_adam.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, vp]
    lib.gc_node_features.restype = ctypes.c_int
    lib.gc_node_features.argtypes = [vp, vp, i32, vp, i32, vp, vp, vp, i32, i32, i32, vp, vp]
    lib.gc_bits_size.restype = ctypes.c_int
    lib.gc_bits_size.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.gc_bits_prepare.restype = ctypes.c_int
    lib.gc_bits_prepare.argtypes = [vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(i32)]
    lib.gc_bits_gains.restype = ctypes.c_int
    lib.gc_bits_gains.argtypes = [vp, vp, ctypes.c_size_t, i32, vp, i32, vp, ctypes.c_int64, vp, vp]
    lib.gc_get_tuning.restype = ctypes.c_int
    lib.gc_get_tuning.argtypes = [vp, ctypes.POINTER(GcTuning)]
    lib.gc_set_tuning.restype = ctypes.c_int
    lib.gc_set_tuning.argtypes = [vp, ctypes.POINTER(GcTuning)]
    lib.gc_timing_enable.restype = ctypes.c_int
    lib.gc_timing_enable.argtypes = [ctypes.c_int]
    lib.gc_timing_last_ms.restype = ctypes.c_double
    lib.gc_timing_last_ms.argtypes = []
    lib.gc_strerror.restype = ctypes.c_char_p
    lib.gc_strerror.argtypes = [ctypes.c_int]
    lib.gc_last_error.restype = ctypes.c_char_p
    lib.gc_last_error.argtypes = []
    _lib = lib
    return lib


def timing_enable(on: bool = True):
    _check(load_library().gc_timing_enable(1 if on else 0))


def timing_last_ms() -> float:
    return float(load_library().gc_timing_last_ms())


def _check(rc: int):
    if rc != GC_OK:
        lib = load_library()
        raise GCError(rc, lib.gc_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class Graph:
    """A device CSR graph plus its library handle and workspace.

    row_ptr, col_idx: int32 tensors on the current HIP device (or numpy arrays,
    which are copied there).  weight: None, or uint8 edge lengths (one per
    CSR entry) for a weighted graph, whose distances are int32
    (dist_bytes = 4).  The tensors are kept alive by this object.
    """

    def __init__(self, row_ptr, col_idx, validate: bool = True, workspace: bool = True,
                 directed: bool = False, weight=None):
        lib = load_library()
        dev = torch.device("cuda", torch.cuda.current_device())
        if isinstance(row_ptr, np.ndarray):
            row_ptr = torch.from_numpy(np.ascontiguousarray(row_ptr, dtype=np.int32))
        if isinstance(col_idx, np.ndarray):
            col_idx = torch.from_numpy(np.ascontiguousarray(col_idx, dtype=np.int32))
        self.row_ptr = row_ptr.to(dev, dtype=torch.int32).contiguous()
        self.col_idx = col_idx.to(dev, dtype=torch.int32).contiguous()
        if self.col_idx.numel() == 0:
            self.col_idx = torch.zeros(1, dtype=torch.int32, device=dev)[:0]
        self.n = int(self.row_ptr.numel() - 1)
        self.nnz = int(self.col_idx.numel())
        h = ctypes.c_void_p()
        self.directed = bool(directed)
        flags = (GC_VALIDATE if validate else 0) | (GC_DIRECTED if directed else 0)
        self.weight = None
        if weight is not None:
            if isinstance(weight, np.ndarray):
                weight = torch.from_numpy(np.ascontiguousarray(weight, dtype=np.uint8))
            if weight.numel() != self.nnz:
                raise ValueError("one length per CSR entry (%d), got %d" % (self.nnz, weight.numel()))
            self.weight = weight.to(dev, dtype=torch.uint8).contiguous()
            _check(lib.gc_load_csr_weighted(self.n, self.nnz, _ptr(self.row_ptr), _ptr(self.col_idx),
                                            _ptr(self.weight), flags, _stream(), ctypes.byref(h)))
        else:
            _check(lib.gc_load_csr(self.n, self.nnz, _ptr(self.row_ptr), _ptr(self.col_idx), flags, _stream(),
                                   ctypes.byref(h)))
        self.handle = h
        self.ws = None
        self.ws_bytes = 0
        if workspace:
            self.alloc_workspace()

    @classmethod
    def from_graphgen(cls, g, **kw):
        kw.setdefault("directed", bool(getattr(g, "directed", False)))
        kw.setdefault("weight", getattr(g, "weight", None))
        return cls(g.row_ptr, g.col_idx, **kw)

    @property
    def weighted(self) -> bool:
        return self.weight is not None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.gc_free_graph(h)
            self.handle = None

    def workspace_size(self, bitset_width: int = 0) -> int:
        sz = ctypes.c_size_t()
        _check(load_library().gc_workspace_size(self.handle, bitset_width, ctypes.byref(sz)))
        return int(sz.value)

    def alloc_workspace(self, bitset_width: int = 0):
        self.ws_bytes = self.workspace_size(bitset_width)
        # 256-byte alignment: torch's caching allocator returns 512-byte aligned blocks
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.row_ptr.device)
        _check(load_library().gc_workspace_init(self.handle, _ptr(self.ws), self.ws_bytes, _stream()))

    def use_workspace(self, buf):
        """Run on a caller-owned uint8 device buffer (at least workspace_size()
        bytes, e.g. one buffer shared by graphs processed one after another);
        it is initialised for this graph."""
        need = self.workspace_size()
        if buf.numel() < need:
            raise ValueError("workspace buffer has %d bytes, graph needs %d" % (buf.numel(), need))
        self.ws = buf
        self.ws_bytes = need
        _check(load_library().gc_workspace_init(self.handle, _ptr(self.ws), self.ws_bytes, _stream()))

    # ------------------------------------------------------------ operations
    def closest_node(self):
        node, far = ctypes.c_int32(), ctypes.c_int64()
        _check(load_library().gc_closest_node(self.handle, _ptr(self.ws), self.ws_bytes, _stream(),
                                              ctypes.byref(node), ctypes.byref(far)))
        return int(node.value), int(far.value)

    def topk_closeness(self, k: int):
        """The k nodes of least F({v}) and their farness, ascending (F, id)."""
        nodes = np.zeros(int(k), dtype=np.int32)
        far = np.zeros(int(k), dtype=np.int64)
        _check(load_library().gc_topk_closeness(
            self.handle, int(k), _ptr(self.ws), self.ws_bytes, _stream(),
            nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            far.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return nodes, far

    def new_dist(self, dist_bytes: int = 1):
        """A d(S,.) buffer for S = {} (all INF), padded to whole 4-byte words
        (dist_bytes 4: int32 with INF = 2^31 - 1, for weighted graphs)."""
        if dist_bytes == 4:
            return torch.full((self.n,), 2**31 - 1, dtype=torch.int32, device=self.row_ptr.device)
        dt = torch.uint8 if dist_bytes == 1 else torch.int16
        nwords = (self.n * dist_bytes + 3) // 4
        buf = torch.full((nwords * 4 // dist_bytes,), -1, dtype=dt, device=self.row_ptr.device)
        return buf

    def update_dist(self, node: int, dist, dist_bytes: int, farness):
        _check(load_library().gc_update_dist(self.handle, int(node), _ptr(dist), dist_bytes,
                                             _ptr(self.ws), self.ws_bytes, _stream(), _ptr(farness)))

    def marginal_gains(self, dist, dist_bytes: int, cand, stats: bool = False):
        cand = cand.to(self.row_ptr.device, dtype=torch.int32).contiguous()
        count = int(cand.numel())
        if count > 0:
            lo, hi = int(cand.min()), int(cand.max())
            if lo < 0 or hi >= self.n:
                raise ValueError("candidate ids must lie in [0, %d) (got %d..%d)" % (self.n, lo, hi))
        gain = torch.empty(max(count, 1), dtype=torch.int64, device=self.row_ptr.device)
        edges = torch.empty_like(gain) if stats else None
        vis = torch.empty(max(count, 1), dtype=torch.int32, device=self.row_ptr.device) if stats else None
        _check(load_library().gc_marginal_gains(self.handle, _ptr(dist), dist_bytes, _ptr(cand), count,
                                                _ptr(gain), _ptr(edges), _ptr(vis), _ptr(self.ws),
                                                self.ws_bytes, _stream()))
        if stats:
            return gain[:count], edges[:count], vis[:count]
        return gain[:count]

    def marginal_gains_noalloc(self, dist, dist_bytes: int, cand, gain, edges=None, visited=None):
        """gc_marginal_gains_noalloc into caller-given output tensors (int64
        gain[count], optional int64 edges and int32 visited): no allocation
        by the library, and none here."""
        count = int(cand.numel())
        _check(load_library().gc_marginal_gains_noalloc(self.handle, _ptr(dist), dist_bytes, _ptr(cand),
                                                        count, _ptr(gain), _ptr(edges), _ptr(visited),
                                                        _stream()))

    def gain_words(self) -> dict:
        """Word-level work of the last marginal_gains call (see gc_gain_words)."""
        out = (ctypes.c_int64 * 6)()
        _check(load_library().gc_gain_words(self.handle, _ptr(self.ws), self.ws_bytes, _stream(), out))
        return dict(zip(("entries", "entries_root", "entries_last", "edges", "edges_last", "touched"),
                        (int(x) for x in out)))

    def node_features(self, dist, dist_bytes, ub, last_eval, dist_at_eval, round_, k, ecc1,
                      cand=None):
        dev = self.row_ptr.device
        count = self.n if cand is None else int(cand.numel())
        feat = torch.empty((max(count, 1), MLP_IN), dtype=torch.float32, device=dev)
        _check(load_library().gc_node_features(self.handle, _ptr(dist), dist_bytes,
                                               _ptr(cand), count, _ptr(ub), _ptr(last_eval),
                                               _ptr(dist_at_eval), int(round_), int(k), int(ecc1),
                                               _ptr(feat), _stream()))
        return feat[:count]

    def bits_prepare(self, levels: int):
        """Bit-vector rows of every level (gc_bits_prepare) in a new device
        buffer that holds `levels` levels; returns the number stored."""
        lib = load_library()
        nb = ctypes.c_size_t()
        _check(lib.gc_bits_size(self.handle, int(levels), ctypes.byref(nb)))
        self.bits, self.bits_levels = None, 0
        buf = torch.empty(nb.value, dtype=torch.uint8, device=self.row_ptr.device)
        lv = ctypes.c_int32()
        _check(lib.gc_bits_prepare(self.handle, _ptr(buf), nb.value, _stream(), ctypes.byref(lv)))
        self.bits, self.bits_levels = buf, int(lv.value)
        return self.bits_levels

    def bits_gains(self, dist, dist_bytes: int, cand) -> torch.Tensor:
        """g(v, S) of the candidates by the bit-vector sum (gc_bits_gains)."""
        cand = cand.to(device=self.row_ptr.device, dtype=torch.int32).contiguous()
        gain = torch.zeros(cand.numel(), dtype=torch.int64, device=self.row_ptr.device)
        _check(load_library().gc_bits_gains(self.handle, _ptr(self.bits), self.bits.numel(), self.bits_levels,
                                            _ptr(dist), dist_bytes, _ptr(cand), cand.numel(), _ptr(gain),
                                            _stream()))
        return gain

    def get_tuning(self) -> dict:
        """The engine's launch shapes for this graph (gc_tuning)."""
        t = GcTuning()
        _check(load_library().gc_get_tuning(self.handle, ctypes.byref(t)))
        return {f: int(getattr(t, f)) for f in TUNING_FIELDS}

    def set_tuning(self, **shape):
        """Change some launch shapes; results do not depend on them."""
        cur = self.get_tuning()
        unknown = set(shape) - set(cur)
        if unknown:
            raise ValueError("unknown tuning fields: %s" % sorted(unknown))
        cur.update({k: int(v) for k, v in shape.items()})
        t = GcTuning(*[cur[f] for f in TUNING_FIELDS])
        _check(load_library().gc_set_tuning(self.handle, ctypes.byref(t)))

    def greedy_group(self, k: int, order: str = "plain", block: int = 0, prefix=None,
                     mlp_params=None, log_capacity: int = 0, debug: bool = False,
                     block_growth: int = 0, bits: bool = False, early_exit: int = 0,
                     early_exit_seed: int = 0):
        """bits=True: bitGreedy++ (gains by the bit-vector sum from the rows
        bits_prepare() stored).  early_exit=1: the early exit of the first gain
        round (see gc_opts.early_exit)."""
        lib = load_library()
        opts = GcOpts()
        if bits:
            if getattr(self, "bits", None) is None:
                raise ValueError("bits=True needs bits_prepare() first")
            opts.d_bits = ctypes.c_void_p(self.bits.data_ptr())
            opts.bits_bytes = self.bits.numel()
            opts.bits_levels = self.bits_levels
        opts.order = ORDERS[order]
        opts.bitset_width = 64
        opts.block = int(block)
        opts.block_growth = int(block_growth)
        opts.debug_checks = 1 if debug else 0
        opts.early_exit = int(early_exit)
        opts.early_exit_seed = int(early_exit_seed)
        keep = []
        if prefix is not None and len(prefix) > 0:
            arr = np.ascontiguousarray(prefix, dtype=np.int32)
            keep.append(arr)
            opts.nprefix = int(arr.shape[0])
            opts.h_prefix = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        if mlp_params is not None:
            opts.d_mlp = ctypes.c_void_p(mlp_params.data_ptr())
        log = None
        if log_capacity > 0:
            log = {"round": np.zeros(log_capacity, np.int32), "node": np.zeros(log_capacity, np.int32),
                   "gain": np.zeros(log_capacity, np.int64),
                   "feat": np.zeros((log_capacity, 8), np.float32), "count": np.zeros(1, np.int64)}
            opts.log_capacity = log_capacity
            opts.h_log_round = log["round"].ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            opts.h_log_node = log["node"].ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            opts.h_log_gain = log["gain"].ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            opts.h_log_feat = log["feat"].ctypes.data_as(ctypes.POINTER(ctypes.c_float))
            opts.h_log_count = log["count"].ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        group = np.zeros(k, dtype=np.int32)
        far = np.zeros(k, dtype=np.int64)
        per_round = np.zeros(k, dtype=np.int64)
        st = GcStats()
        st.h_evals_per_round = per_round.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        _check(lib.gc_greedy_group(self.handle, int(k), ctypes.byref(opts), _ptr(self.ws),
                                   self.ws_bytes, _stream(),
                                   group.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   far.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   ctypes.byref(st)))
        stats = st.as_dict()
        stats["evals_per_round"] = per_round
        if log is not None:
            c = int(min(log["count"][0], log_capacity))
            stats["log"] = {key: v[:c] for key, v in log.items() if key != "count"}
        return group, far, stats


class Many:
    """Runs many independent greedy jobs through gc_greedy_many: `workers`
    host threads, each with its own stream and a workspace sized for the
    largest graph (allocated here once and reused across calls)."""

    def __init__(self, graphs, workers: int = 4):
        self.graphs = list(graphs)
        self.workers = max(1, min(int(workers), 64))
        dev = self.graphs[0].row_ptr.device
        need = max(G.workspace_size() for G in self.graphs)
        self.ws = [torch.empty(need, dtype=torch.uint8, device=dev) for _ in range(self.workers)]
        self.ws_bytes = need
        # default-priority streams, one per worker
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(self.workers)]

    def run(self, ks, order: str = "plain", block: int = 0, block_growth: int = 0,
            mlp_params=None, lockstep: bool = False):
        """(groups, farness, stats): per job, in the order of `graphs`.
        lockstep=True: gc_greedy_batch (first rounds on the workers, every
        later round of every job in shared calls over the union of the
        graphs; plain or CELF order)."""
        lib = load_library()
        cnt = len(self.graphs)
        ks = [int(k) for k in ks]
        assert len(ks) == cnt
        opts = GcOpts()
        opts.order = ORDERS[order]
        opts.bitset_width = 64
        opts.block = int(block)
        opts.block_growth = int(block_growth)
        if mlp_params is not None:
            opts.d_mlp = ctypes.c_void_p(mlp_params.data_ptr())
        handles = (ctypes.c_void_p * cnt)(*[G.handle for G in self.graphs])
        karr = (ctypes.c_int32 * cnt)(*ks)
        ws = (ctypes.c_void_p * self.workers)(*[t.data_ptr() for t in self.ws])
        wsb = (ctypes.c_size_t * self.workers)(*([self.ws_bytes] * self.workers))
        st = (ctypes.c_void_p * self.workers)(*[s.cuda_stream for s in self.streams])
        tot = sum(ks)
        group = np.zeros(tot, dtype=np.int32)
        far = np.zeros(tot, dtype=np.int64)
        stats = (GcStats * cnt)()
        # the jobs must see every earlier write of the caller's stream
        torch.cuda.current_stream().synchronize()
        if lockstep:
            need = ctypes.c_size_t()
            _check(lib.gc_batch_union_size(cnt, handles, int(block), ctypes.byref(need)))
            if getattr(self, "union", None) is None or self.union.numel() < need.value:
                self.union = None
                self.union = torch.empty(need.value, dtype=torch.uint8, device=self.ws[0].device)
            _check(lib.gc_greedy_batch(cnt, handles, karr, ctypes.byref(opts), self.workers, ws, wsb, st,
                                       ctypes.c_void_p(self.union.data_ptr()), need.value,
                                       group.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       far.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), stats))
        else:
            _check(lib.gc_greedy_many(cnt, handles, karr, ctypes.byref(opts), self.workers, ws, wsb, st,
                                      group.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      far.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), stats))
        out_g, out_f, off = [], [], 0
        for k in ks:
            out_g.append(group[off:off + k])
            out_f.append(far[off:off + k])
            off += k
        return out_g, out_f, [stats[i].as_dict() for i in range(cnt)]


class Mlp:
    """Device state of the candidate-ordering MLP: float32 master weights,
    Adam moments and the packed bf16 inference block (all torch tensors)."""

    def __init__(self, master, device=None):
        lib = load_library()
        dev = device or torch.device("cuda", torch.cuda.current_device())
        m = torch.as_tensor(np.asarray(master, dtype=np.float32))
        assert m.numel() == MLP_PARAMS
        self.master = m.to(dev).contiguous()
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.block = torch.zeros(int(lib.gc_mlp_block_bytes()), dtype=torch.uint8, device=dev)
        self.step = 0
        self.pack()

    def pack(self):
        _check(load_library().gc_mlp_pack(_ptr(self.master), _ptr(self.block), _stream()))

    def forward(self, x, activations: bool = False):
        x = x.contiguous()
        count = int(x.shape[0])
        dev = self.master.device
        out = torch.empty(max(count, 1), dtype=torch.float32, device=dev)
        h1 = h2 = None
        if activations:
            h1 = torch.empty((max(count, 1), MLP_HIDDEN), dtype=torch.float32, device=dev)
            h2 = torch.empty_like(h1)
        _check(load_library().gc_mlp_forward(_ptr(self.block), _ptr(x), count, _ptr(out), _ptr(h1),
                                             _ptr(h2), _stream()))
        if activations:
            return out[:count], h1[:count], h2[:count]
        return out[:count]

    def backward(self, x, h1, h2, out, y):
        lib = load_library()
        count = int(x.shape[0])
        dev = self.master.device
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=dev)
        scratch = torch.empty(int(lib.gc_mlp_scratch_floats(count)), dtype=torch.float32, device=dev)
        _check(lib.gc_mlp_backward(_ptr(self.block), _ptr(x.contiguous()), _ptr(h1), _ptr(h2),
                                   _ptr(out), _ptr(y.contiguous()), count, _ptr(grad), _ptr(scratch),
                                   _stream()))
        return grad

    def adam(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        _check(load_library().gc_mlp_adam(_ptr(self.master), _ptr(self.m), _ptr(self.v), _ptr(grad),
                                          self.step, lr, beta1, beta2, eps, _stream()))
        self.pack()

    def train(self, X, Y, steps: int = 2000, batch: int = 1024, lr: float = 3e-3, seed: int = 0):
        """Minibatch Adam on (X, Y) (numpy float32); batches are contiguous
        slices of a host-side permutation redrawn every epoch."""
        dev = self.master.device
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.ascontiguousarray(Y, dtype=np.float32)
        N = X.shape[0]
        batch = min(batch, N)
        rng = np.random.default_rng(seed)
        losses = []
        s = 0
        while s < steps:
            perm = rng.permutation(N)
            Xd = torch.from_numpy(X[perm]).to(dev)
            Yd = torch.from_numpy(Y[perm]).to(dev)
            for lo in range(0, N - batch + 1, batch):
                if s >= steps:
                    break
                xb, yb = Xd[lo:lo + batch], Yd[lo:lo + batch]
                out, h1, h2 = self.forward(xb, activations=True)
                g = self.backward(xb, h1, h2, out, yb)
                self.adam(g, lr=lr)
                if s % 100 == 0 or s == steps - 1:
                    losses.append(float(((out - yb) ** 2).mean().item()))
                s += 1
        return losses
