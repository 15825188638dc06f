"""MI355X (gfx950) level-wise wavelet tree: Python binding of the C ABI in include/wt.h.

The binding only marshals arguments: every step of construction and of the queries runs in
the HIP kernels of ``libwt.so``. PyTorch supplies device memory (input/output tensors) and the
current HIP stream. There is no CPU fallback: importing works without the library, but every
call that needs it raises ``WTLibraryMissing`` until ``python -m paper_2505_03372_amd.buildlib``
has produced it.

    import torch, paper_2505_03372_amd as wt
    t = wt.build(sym_tensor_on_gpu, sigma=256)
    t.access(pos)            # torch.uint32, 0xFFFFFFFF for positions >= n
    t.rank(sym, pos)         # torch.uint64
    t.select(sym, k)         # torch.uint64, n when k > count, 2^64-1 when k == 0
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwt.so")

WT_OK, WT_ERR_ARG, WT_ERR_SYMBOL_RANGE, WT_ERR_OOM, WT_ERR_HIP, WT_ERR_STATE = range(6)
PART_BITS, PART_L1, PART_L2, PART_SAMPLES1, PART_SAMPLES0, PART_NODE_START, PART_NODE_R0, PART_CUM_HIST, \
    PART_ALPHABET, PART_WM_STARTS, PART_HUFF_CODES = range(11)
BUILD_PROFILE = 1
BUILD_MATRIX = 2
BUILD_WIDE = 4
BUILD_HUFFMAN = 8
BUILD_NARROW = 32
BUILD_HOST_TWO_PASS = 16
MAX_LEVELS = 24
MAX_SIGMA = 1 << 24
ACCESS_INVALID = 0xFFFFFFFF
U64_MAX = (1 << 64) - 1

# names declared by include/wt.h
ABI_FUNCTIONS = ("wt_set_allocator", "wt_build", "wt_free", "wt_access", "wt_rank", "wt_select", "wt_info",
                 "wt_export", "wt_build_profile", "wt_last_error", "wt_version", "wt_learn_select",
                 "wt_select_learned", "wt_learned_info", "wt_learned_model", "wt_mlp_loss_grad",
                 "wt_build_forest", "wt_forest_tree", "wt_forest_info", "wt_forest_free", "wt_query_mixed",
                 "wt_autotune", "wt_server_create", "wt_server_run", "wt_server_destroy", "wt_query_profiling",
                 "wt_query_profile", "wt_bv_build", "wt_select_noalloc", "wt_query_host", "wt_query_host_release",
                 "wt_build_host")
OP_ACCESS, OP_RANK, OP_SELECT, OP_SELECT_LEARNED = 0, 1, 2, 3
TUNE_NB, TUNE_SB = 21, 7
MLP_PARAMS = 49


class HostOpts(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_uint64), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class HostStats(ctypes.Structure):
    _fields_ = [("chunks", ctypes.c_uint32), ("pinned", ctypes.c_uint32), ("graph", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("ms", ctypes.c_float), ("reserved2", ctypes.c_uint32)]


HOST_NO_GRAPH = 1


class WTLibraryMissing(RuntimeError):
    pass


class WTError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("wt status %d: %s" % (status, msg))
        self.status = status


class BuildOpts(ctypes.Structure):
    _fields_ = [("l2_bits", ctypes.c_uint32), ("sample_rate", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("sigma", ctypes.c_uint64), ("levels", ctypes.c_uint32),
                ("sym_bytes", ctypes.c_uint32), ("l2_bits", ctypes.c_uint32), ("sample_rate", ctypes.c_uint32),
                ("level_n", ctypes.c_uint64 * MAX_LEVELS), ("level_ones", ctypes.c_uint64 * MAX_LEVELS),
                ("bytes_bits", ctypes.c_uint64), ("bytes_l1", ctypes.c_uint64), ("bytes_l2", ctypes.c_uint64),
                ("bytes_samples", ctypes.c_uint64), ("bytes_nodes", ctypes.c_uint64), ("bytes_total", ctypes.c_uint64),
                ("alphabet_extracted", ctypes.c_uint32), ("matrix", ctypes.c_uint32), ("max_symbol", ctypes.c_uint64),
                ("huffman", ctypes.c_uint32), ("reserved1", ctypes.c_uint32)]


class LearnOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_uint32), ("max_points", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("flags", ctypes.c_uint32)]


class LearnedInfo(ctypes.Structure):
    _fields_ = [("models", ctypes.c_uint32), ("params_per_model", ctypes.c_uint32),
                ("mean_err_blocks", ctypes.c_double), ("max_err_blocks", ctypes.c_double),
                ("mean_err_init_blocks", ctypes.c_double), ("max_err_init_blocks", ctypes.c_double),
                ("final_loss_mean", ctypes.c_double), ("train_ms", ctypes.c_float), ("reserved", ctypes.c_uint32)]


class LearnedModel(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("side", ctypes.c_uint32), ("eps", ctypes.c_int32),
                ("points", ctypes.c_uint32), ("start", ctypes.c_uint64), ("len", ctypes.c_uint64),
                ("count", ctypes.c_uint64), ("rank0", ctypes.c_uint64), ("params", ctypes.c_float * 49),
                ("pieces", ctypes.c_uint32), ("knots", ctypes.c_float * 16), ("slope", ctypes.c_float * 17),
                ("intercept", ctypes.c_float * 17), ("err_mean", ctypes.c_float), ("err_max", ctypes.c_float),
                ("err_init_mean", ctypes.c_float), ("err_init_max", ctypes.c_float), ("loss", ctypes.c_float)]


class SeqDesc(ctypes.Structure):
    _fields_ = [("d_sym", ctypes.c_void_p), ("n", ctypes.c_uint64), ("sigma", ctypes.c_uint64),
                ("l2_bits", ctypes.c_uint32), ("sample_rate", ctypes.c_uint32)]


class TuneTable(ctypes.Structure):
    _fields_ = [("l2_bits", (ctypes.c_uint32 * 7) * 21), ("sample_rate", (ctypes.c_uint32 * 7) * 21)]


class TuneOpts(ctypes.Structure):
    _fields_ = [("max_probe_n", ctypes.c_uint64), ("queries", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("queries_per_symbol", ctypes.c_double), ("space_cap", ctypes.c_double)]


class TuneReport(ctypes.Structure):
    _fields_ = [("buckets", ctypes.c_uint32), ("probes", ctypes.c_uint32), ("total_ms", ctypes.c_float),
                ("reserved", ctypes.c_uint32), ("cost_ns_per_symbol", (ctypes.c_float * 7) * 21)]


class ForestOpts(ctypes.Structure):
    _fields_ = [("tune", ctypes.POINTER(TuneTable)), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ForestInfo(ctypes.Structure):
    _fields_ = [("trees", ctypes.c_uint32), ("levels_max", ctypes.c_uint32), ("symbols", ctypes.c_uint64),
                ("bytes_trees", ctypes.c_uint64), ("bytes_scratch", ctypes.c_uint64),
                ("graph_kernels", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("plan_ms", ctypes.c_float),
                ("capture_ms", ctypes.c_float), ("graph_ms", ctypes.c_float), ("total_ms", ctypes.c_float)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_uint32), ("coalesce_q", ctypes.c_uint32), ("mem_budget", ctypes.c_uint64),
                ("sim_ns_per_query", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("h_tree", ctypes.c_void_p), ("h_op", ctypes.c_void_p), ("h_sym", ctypes.c_void_p),
                ("h_arg", ctypes.c_void_p), ("h_out", ctypes.c_void_p), ("q", ctypes.c_uint64),
                ("arrival_s", ctypes.c_double)]


class Completion(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("slot", ctypes.c_uint32), ("status", ctypes.c_int32)]


class ServeStats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_uint32), ("rejected", ctypes.c_uint32), ("peak_in_flight", ctypes.c_uint32),
                ("batches", ctypes.c_uint32), ("queries", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64),
                ("makespan_s", ctypes.c_double), ("qps", ctypes.c_double), ("lat_p50_s", ctypes.c_double),
                ("lat_p99_s", ctypes.c_double), ("lat_mean_s", ctypes.c_double), ("lat_max_s", ctypes.c_double)]


class BuildHostStats(ctypes.Structure):
    _fields_ = [("chunks", ctypes.c_uint32), ("pinned", ctypes.c_uint32), ("passes", ctypes.c_uint32),
                ("ms_counts", ctypes.c_float), ("ms_build", ctypes.c_float), ("ms_total", ctypes.c_float),
                ("work_bytes", ctypes.c_uint64)]


class ProfEntry(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_char * 32), ("level", ctypes.c_int32), ("ms", ctypes.c_float)]


_lib = None


def lib():
    """The loaded libwt.so; raises WTLibraryMissing when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise WTLibraryMissing("%s is missing: build it with `python -m paper_2505_03372_amd.buildlib`" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    L.wt_build.restype = ctypes.c_int
    L.wt_build.argtypes = [vp, u64, u32, u64, ctypes.POINTER(BuildOpts), vp, ctypes.POINTER(vp)]
    L.wt_build_host.restype = ctypes.c_int
    L.wt_build_host.argtypes = [vp, u64, u32, u64, ctypes.POINTER(BuildOpts), u64, ctypes.POINTER(BuildHostStats), vp,
                                ctypes.POINTER(vp)]
    L.wt_bv_build.restype = ctypes.c_int
    L.wt_bv_build.argtypes = [vp, u64, ctypes.POINTER(BuildOpts), vp, ctypes.POINTER(vp)]
    L.wt_free.restype = ctypes.c_int
    L.wt_free.argtypes = [vp]
    L.wt_access.restype = ctypes.c_int
    L.wt_access.argtypes = [vp, vp, u64, vp, vp]
    L.wt_rank.restype = ctypes.c_int
    L.wt_rank.argtypes = [vp, vp, vp, u64, vp, vp]
    L.wt_select.restype = ctypes.c_int
    L.wt_select.argtypes = [vp, vp, vp, u64, vp, vp]
    L.wt_select_noalloc.restype = ctypes.c_int
    L.wt_select_noalloc.argtypes = [vp, vp, vp, u64, vp, vp]
    L.wt_query_host.restype = ctypes.c_int
    L.wt_query_host.argtypes = [vp, ctypes.c_int, vp, vp, u64, vp, ctypes.POINTER(HostOpts), ctypes.POINTER(HostStats),
                                vp]
    L.wt_query_host_release.restype = ctypes.c_int
    L.wt_query_host_release.argtypes = []
    L.wt_info.restype = ctypes.c_int
    L.wt_info.argtypes = [vp, ctypes.POINTER(Info)]
    L.wt_export.restype = ctypes.c_int
    L.wt_export.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    L.wt_build_profile.restype = ctypes.c_int
    L.wt_build_profile.argtypes = [vp, ctypes.POINTER(ProfEntry), u32, ctypes.POINTER(u32)]
    L.wt_last_error.restype = ctypes.c_char_p
    L.wt_last_error.argtypes = []
    L.wt_version.restype = ctypes.c_char_p
    L.wt_version.argtypes = []
    L.wt_set_allocator.restype = ctypes.c_int
    L.wt_set_allocator.argtypes = [vp, vp, vp]
    L.wt_learn_select.restype = ctypes.c_int
    L.wt_learn_select.argtypes = [vp, ctypes.POINTER(LearnOpts), vp]
    L.wt_select_learned.restype = ctypes.c_int
    L.wt_select_learned.argtypes = [vp, vp, vp, u64, vp, vp]
    L.wt_learned_info.restype = ctypes.c_int
    L.wt_learned_info.argtypes = [vp, ctypes.POINTER(LearnedInfo)]
    L.wt_build_forest.restype = ctypes.c_int
    L.wt_build_forest.argtypes = [ctypes.POINTER(SeqDesc), u32, u32, ctypes.POINTER(ForestOpts), vp,
                                  ctypes.POINTER(vp)]
    L.wt_forest_tree.restype = ctypes.c_int
    L.wt_forest_tree.argtypes = [vp, u32, ctypes.POINTER(vp)]
    L.wt_forest_info.restype = ctypes.c_int
    L.wt_forest_info.argtypes = [vp, ctypes.POINTER(ForestInfo)]
    L.wt_forest_free.restype = ctypes.c_int
    L.wt_forest_free.argtypes = [vp]
    L.wt_query_mixed.restype = ctypes.c_int
    L.wt_query_mixed.argtypes = [vp, vp, vp, vp, vp, u64, vp, vp]
    L.wt_autotune.restype = ctypes.c_int
    L.wt_autotune.argtypes = [ctypes.POINTER(SeqDesc), u32, u32, ctypes.POINTER(TuneOpts), vp,
                              ctypes.POINTER(TuneTable), ctypes.POINTER(TuneReport)]
    L.wt_query_profiling.restype = ctypes.c_int
    L.wt_query_profiling.argtypes = [ctypes.c_int]
    L.wt_query_profile.restype = ctypes.c_int
    L.wt_query_profile.argtypes = [ctypes.POINTER(ProfEntry), u32, ctypes.POINTER(u32)]
    L.wt_server_create.restype = ctypes.c_int
    L.wt_server_create.argtypes = [vp, ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
    L.wt_server_run.restype = ctypes.c_int
    L.wt_server_run.argtypes = [vp, ctypes.POINTER(Request), u32, ctypes.POINTER(Completion),
                                ctypes.POINTER(ServeStats)]
    L.wt_server_destroy.restype = ctypes.c_int
    L.wt_server_destroy.argtypes = [vp]
    L.wt_learned_model.restype = ctypes.c_int
    L.wt_learned_model.argtypes = [vp, u32, ctypes.POINTER(LearnedModel)]
    L.wt_mlp_loss_grad.restype = ctypes.c_int
    L.wt_mlp_loss_grad.argtypes = [vp, vp, vp, u32, vp, vp]
    _lib = L
    return L


def _check(status: int):
    if status != WT_OK:
        raise WTError(status, lib().wt_last_error().decode())


def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> int:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _dev_ptr(t, dtype, name):
    torch = _torch()
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0)


_SYM_DTYPES = None


def _sym_dtypes():
    global _SYM_DTYPES
    if _SYM_DTYPES is None:
        torch = _torch()
        _SYM_DTYPES = {torch.uint8: 1, torch.uint16: 2, torch.uint32: 4}
    return _SYM_DTYPES


class Tree:
    """A wavelet tree resident in HBM (owned by libwt)."""

    def __init__(self, handle: int, keepalive=None, borrowed: bool = False):
        self._h = ctypes.c_void_p(handle)
        self._keep = keepalive
        self._borrowed = borrowed
        self._inf = None

    @property
    def info(self) -> dict:
        """Sizes and layout of the tree (read from the library on first use)."""
        if self._inf is None:
            self._inf = self._info()
        return self._inf

    @property
    def handle(self):
        return self._h

    def _info(self) -> dict:
        inf = Info()
        _check(lib().wt_info(self._h, ctypes.byref(inf)))
        L = inf.levels
        return dict(n=inf.n, sigma=inf.sigma, levels=L, sym_bytes=inf.sym_bytes, l2_bits=inf.l2_bits,
                    sample_rate=inf.sample_rate, level_n=list(inf.level_n[:L]), level_ones=list(inf.level_ones[:L]),
                    bytes_bits=inf.bytes_bits, bytes_l1=inf.bytes_l1, bytes_l2=inf.bytes_l2,
                    bytes_samples=inf.bytes_samples, bytes_nodes=inf.bytes_nodes, bytes_total=inf.bytes_total,
                    alphabet_extracted=bool(inf.alphabet_extracted), matrix=bool(inf.matrix), max_symbol=inf.max_symbol,
                    huffman=bool(inf.huffman))

    @property
    def n(self) -> int:
        return self.info["n"]

    @property
    def sigma(self) -> int:
        return self.info["sigma"]

    def access(self, pos, out=None, stream=None):
        torch = _torch()
        q = pos.numel()
        if out is None:
            out = torch.empty(q, dtype=torch.uint32, device=pos.device)
        _check(lib().wt_access(self._h, _dev_ptr(pos, torch.uint64, "pos"), q, _dev_ptr(out, torch.uint32, "out"),
                               ctypes.c_void_p(_stream_handle(stream))))
        return out

    def rank(self, sym, pos, out=None, stream=None):
        torch = _torch()
        q = pos.numel()
        if sym.numel() != q:
            raise ValueError("sym and pos must have the same length")
        if out is None:
            out = torch.empty(q, dtype=torch.uint64, device=pos.device)
        _check(lib().wt_rank(self._h, _dev_ptr(sym, torch.uint32, "sym"), _dev_ptr(pos, torch.uint64, "pos"), q,
                             _dev_ptr(out, torch.uint64, "out"), ctypes.c_void_p(_stream_handle(stream))))
        return out

    def select(self, sym, k, out=None, stream=None):
        torch = _torch()
        q = k.numel()
        if sym.numel() != q:
            raise ValueError("sym and k must have the same length")
        if out is None:
            out = torch.empty(q, dtype=torch.uint64, device=k.device)
        _check(lib().wt_select(self._h, _dev_ptr(sym, torch.uint32, "sym"), _dev_ptr(k, torch.uint64, "k"), q,
                               _dev_ptr(out, torch.uint64, "out"), ctypes.c_void_p(_stream_handle(stream))))
        return out

    def select_noalloc(self, sym, k, out, stream=None):
        """select through wt_select_noalloc (no device allocation; out must be given, q <= 2^20)."""
        torch = _torch()
        q = k.numel()
        if sym.numel() != q or out.numel() != q:
            raise ValueError("sym, k and out must have the same length")
        _check(lib().wt_select_noalloc(self._h, _dev_ptr(sym, torch.uint32, "sym"), _dev_ptr(k, torch.uint64, "k"),
                                       q, _dev_ptr(out, torch.uint64, "out"),
                                       ctypes.c_void_p(_stream_handle(stream))))
        return out

    def query_host(self, op: int, arg, sym=None, out=None, chunk: int = 0, graph: bool = True, stream=None):
        """wt_query_host: op OP_ACCESS / OP_RANK / OP_SELECT over host arrays (numpy or CPU tensors, pinned
        or pageable); returns (answers, stats)."""
        q = int(arg.shape[0])
        if out is None:
            out = np.empty(q, dtype=np.uint32 if op == OP_ACCESS else np.uint64)
        if sym is not None and int(sym.shape[0]) != q:
            raise ValueError("sym and arg must have the same length")
        opts = HostOpts(chunk, 0 if graph else HOST_NO_GRAPH, 0)
        st = HostStats()
        _check(lib().wt_query_host(self._h, op, ctypes.c_void_p(_host_ptr(sym) if sym is not None else 0),
                                   ctypes.c_void_p(_host_ptr(arg)), q, ctypes.c_void_p(_host_ptr(out)),
                                   ctypes.byref(opts), ctypes.byref(st), ctypes.c_void_p(_stream_handle(stream))))
        return out, {f: getattr(st, f) for f, _ in HostStats._fields_ if not f.startswith("reserved")}

    def learn_select(self, epochs: int = 0, max_points: int = 0, lr: float = 0.0, stream=None) -> dict:
        """Train the learned select index of this tree on the GPU; returns its statistics."""
        opts = LearnOpts(epochs, max_points, lr, 0)
        _check(lib().wt_learn_select(self._h, ctypes.byref(opts), ctypes.c_void_p(_stream_handle(stream))))
        return self.learned_info()

    def learned_info(self) -> dict:
        inf = LearnedInfo()
        _check(lib().wt_learned_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in LearnedInfo._fields_ if f != "reserved"}

    def learned_model(self, slot: int) -> dict:
        """One model of the learned index (training record and its compiled piecewise-linear form)."""
        m = LearnedModel()
        _check(lib().wt_learned_model(self._h, slot, ctypes.byref(m)))
        d = {}
        for f, _ in LearnedModel._fields_:
            v = getattr(m, f)
            d[f] = np.array(v[:], dtype=np.float32) if isinstance(v, ctypes.Array) else v
        return d

    def select_learned(self, sym, k, out=None, stream=None):
        torch = _torch()
        q = k.numel()
        if sym.numel() != q:
            raise ValueError("sym and k must have the same length")
        if out is None:
            out = torch.empty(q, dtype=torch.uint64, device=k.device)
        _check(lib().wt_select_learned(self._h, _dev_ptr(sym, torch.uint32, "sym"), _dev_ptr(k, torch.uint64, "k"), q,
                                       _dev_ptr(out, torch.uint64, "out"), ctypes.c_void_p(_stream_handle(stream))))
        return out

    def export(self, part: int, level: int = 0) -> np.ndarray:
        need = ctypes.c_size_t(0)
        _check(lib().wt_export(self._h, level, part, None, 0, ctypes.byref(need)))
        dt = np.uint16 if part == PART_L2 else np.uint32 if part == PART_ALPHABET else np.uint64
        buf = np.zeros(max(need.value // np.dtype(dt).itemsize, 1), dtype=dt)
        _check(lib().wt_export(self._h, level, part, ctypes.c_void_p(buf.ctypes.data), buf.nbytes,
                               ctypes.byref(need)))
        return buf[: need.value // np.dtype(dt).itemsize]

    def profile(self) -> list:
        cnt = ctypes.c_uint32(0)
        _check(lib().wt_build_profile(self._h, None, 0, ctypes.byref(cnt)))
        arr = (ProfEntry * max(cnt.value, 1))()
        _check(lib().wt_build_profile(self._h, arr, cnt.value, ctypes.byref(cnt)))
        return [dict(kernel=arr[i].kernel.decode(), level=arr[i].level, ms=arr[i].ms) for i in range(cnt.value)]

    def free(self):
        if self._h is not None and self._h.value:
            if not self._borrowed:
                _check(lib().wt_free(self._h))
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_bitvector(words, n_bits: int, l2_bits: int = 512, sample_rate: int = 4096, stream=None) -> Tree:
    """Rank/select support of a plain bit array: `words` is a device tensor of uint64 words (bit j at bit
    j mod 64 of word j / 64); the result is a tree over the binary alphabet (sigma = 2, one level):
    access(i) is bit i, rank(b, i) is rank_b(i), select(b, k) the position of the k-th bit b."""
    torch = _torch()
    if n_bits and (words.dtype != torch.uint64 or not words.is_cuda or not words.is_contiguous()
                   or words.numel() * 64 < n_bits):
        raise ValueError("words must be a contiguous device tensor of uint64 holding n_bits bits")
    opts = BuildOpts(l2_bits, sample_rate, 0, 0)
    h = ctypes.c_void_p(0)
    _check(lib().wt_bv_build(ctypes.c_void_p(words.data_ptr() if n_bits else 0), n_bits, ctypes.byref(opts),
                             ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(h)))
    return Tree(h.value)


def build_host(sym: np.ndarray, sigma: int, chunk: int = 0, l2_bits: int = 512, sample_rate: int = 4096,
               wide: bool = False, two_pass: bool = False, narrow: bool = False, stream=None):
    """Build the tree of a host array (numpy uint8/uint16/uint32, page-locked or pageable) in chunks of
    `chunk` symbols (0: 2^27); the same tree as build() of a device copy. two_pass: copy the array twice
    and keep only a few chunks on the device. Returns (tree, stats)."""
    widths = {np.dtype(np.uint8): 1, np.dtype(np.uint16): 2, np.dtype(np.uint32): 4}
    if sym.dtype not in widths or not sym.flags["C_CONTIGUOUS"]:
        raise TypeError("symbols must be a contiguous uint8, uint16 or uint32 array")
    opts = BuildOpts(l2_bits, sample_rate, (BUILD_WIDE if wide else 0) | (BUILD_HOST_TWO_PASS if two_pass else 0)
                     | (BUILD_NARROW if narrow else 0), 0)
    st = BuildHostStats()
    h = ctypes.c_void_p(0)
    _check(lib().wt_build_host(ctypes.c_void_p(sym.ctypes.data if sym.size else 0), sym.size, widths[sym.dtype], sigma,
                               ctypes.byref(opts), chunk, ctypes.byref(st), ctypes.c_void_p(_stream_handle(stream)),
                               ctypes.byref(h)))
    return Tree(h.value), {f: getattr(st, f) for f, _ in BuildHostStats._fields_}


def build(sym, sigma: int, l2_bits: int = 512, sample_rate: int = 4096, profile: bool = False, stream=None,
          matrix: bool = False, wide: bool = False, huffman: bool = False, narrow: bool = False) -> Tree:
    """Build the wavelet tree of a contiguous device tensor of uint8/uint16/uint32 symbols. sigma: declared
    alphabet size (symbols in [0, sigma)), or 0 to extract the alphabet (the distinct values). matrix: build
    the wavelet matrix instead (same queries). wide / narrow: keep full-width codes at every level, or
    narrow them at any size (default: narrow from 2^24 symbols on; the same tree either way).
    huffman: Huffman-shaped tree (codes of an optimal length-limited prefix code of the counts)."""
    dts = _sym_dtypes()
    if sym.dtype not in dts:
        raise TypeError("symbols must be uint8, uint16 or uint32 (got %s)" % sym.dtype)
    if not sym.is_cuda or not sym.is_contiguous():
        raise ValueError("symbols must be a contiguous device tensor")
    opts = BuildOpts(l2_bits, sample_rate, (BUILD_PROFILE if profile else 0) | (BUILD_MATRIX if matrix else 0)
                     | (BUILD_WIDE if wide else 0) | (BUILD_HUFFMAN if huffman else 0)
                     | (BUILD_NARROW if narrow else 0), 0)
    h = ctypes.c_void_p(0)
    _check(lib().wt_build(ctypes.c_void_p(sym.data_ptr() if sym.numel() else 0), sym.numel(), dts[sym.dtype], sigma,
                          ctypes.byref(opts), ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(h)))
    return Tree(h.value)


class Forest:
    """Trees built together by wt_build_forest (owned by libwt; trees are borrowed handles)."""

    def __init__(self, handle: int, keepalive=None):
        self._h = ctypes.c_void_p(handle)
        self._keep = keepalive
        inf = ForestInfo()
        _check(lib().wt_forest_info(self._h, ctypes.byref(inf)))
        self.info = {f: getattr(inf, f) for f, _ in ForestInfo._fields_ if f != "reserved"}
        self.trees = []
        for j in range(inf.trees):
            t = ctypes.c_void_p(0)
            _check(lib().wt_forest_tree(self._h, j, ctypes.byref(t)))
            self.trees.append(Tree(t.value, keepalive=self, borrowed=True))

    def __len__(self):
        return len(self.trees)

    def __getitem__(self, j) -> Tree:
        return self.trees[j]

    def query_mixed(self, tree, op, sym, arg, out=None, stream=None):
        """Mixed access/rank/select: tree (uint32), op (uint8: OP_ACCESS/OP_RANK/OP_SELECT), sym (uint32),
        arg (uint64: position or k); returns uint64 results in query order."""
        torch = _torch()
        q = arg.numel()
        if tree.numel() != q or op.numel() != q or sym.numel() != q:
            raise ValueError("tree, op, sym and arg must have the same length")
        if out is None:
            out = torch.empty(q, dtype=torch.uint64, device=arg.device)
        _check(lib().wt_query_mixed(self._h, _dev_ptr(tree, torch.uint32, "tree"), _dev_ptr(op, torch.uint8, "op"),
                                    _dev_ptr(sym, torch.uint32, "sym"), _dev_ptr(arg, torch.uint64, "arg"), q,
                                    _dev_ptr(out, torch.uint64, "out"), ctypes.c_void_p(_stream_handle(stream))))
        return out

    def free(self):
        if self._h is not None and self._h.value:
            for t in self.trees:
                t._h = ctypes.c_void_p(0)
            _check(lib().wt_forest_free(self._h))
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def make_tune_table(entries: dict) -> TuneTable:
    """{(n_bucket, sigma_bucket): (l2_bits, sample_rate)} -> TuneTable."""
    tt = TuneTable()
    for (nb, sb), (l2, s) in entries.items():
        tt.l2_bits[nb][sb] = l2
        tt.sample_rate[nb][sb] = s
    return tt


def tune_bucket(n: int, sigma: int):
    """Shape bucket of the tuning table: (floor(log2 n) // 2, floor(log2 sigma) // 4), clamped."""
    nb = min((max(n, 1).bit_length() - 1) // 2, TUNE_NB - 1)
    sb = min((max(sigma, 1).bit_length() - 1) // 4, TUNE_SB - 1)
    return nb, sb


_SEQ_DESC_NP = np.dtype([("d_sym", "<u8"), ("n", "<u8"), ("sigma", "<u8"), ("l2_bits", "<u4"),
                         ("sample_rate", "<u4")])


def _descs(seqs, sigmas, l2_bits=None, sample_rates=None):
    if len(seqs) == 0 or len(seqs) != len(sigmas):
        raise ValueError("need one sigma per sequence")
    dts = _sym_dtypes()
    dt = seqs[0].dtype
    if dt not in dts:
        raise TypeError("symbols must be uint8, uint16 or uint32 (got %s)" % dt)
    # one pass per property (a single pass reading several properties of each view is much slower)
    bad = [j for j, d in enumerate([x.dtype for x in seqs]) if d != dt]
    bad += [j for j, c in enumerate([x.is_cuda for x in seqs]) if not c]
    bad += [j for j, c in enumerate([x.is_contiguous() for x in seqs]) if not c]
    if bad:
        raise ValueError("sequence %d: contiguous device tensor of %s expected" % (min(bad), dt))
    ns = np.array([x.numel() for x in seqs], dtype=np.uint64)
    ptrs = np.array([x.data_ptr() for x in seqs], dtype=np.uint64)
    descs = (SeqDesc * len(seqs))()
    assert ctypes.sizeof(SeqDesc) == _SEQ_DESC_NP.itemsize
    arr = np.frombuffer(descs, dtype=_SEQ_DESC_NP)
    arr["d_sym"] = np.where(ns > 0, ptrs, 0)
    arr["n"] = ns
    arr["sigma"] = np.asarray(sigmas, dtype=np.uint64)
    arr["l2_bits"] = np.asarray(l2_bits, dtype=np.uint32) if l2_bits is not None else 0
    arr["sample_rate"] = np.asarray(sample_rates, dtype=np.uint32) if sample_rates is not None else 0
    return descs, dts[dt]


def autotune(seqs, sigmas, max_probe_n: int = 0, queries: int = 0, queries_per_symbol: float = 0.0,
             space_cap: float = 0.0, stream=None):
    """Pick |L2| and s per shape bucket by timing probe builds and queries on the device.
    Returns (TuneTable, report dict)."""
    descs, w = _descs(seqs, sigmas)
    opts = TuneOpts(max_probe_n, queries, 0, queries_per_symbol, space_cap)
    tt, rep = TuneTable(), TuneReport()
    _check(lib().wt_autotune(descs, len(seqs), w, ctypes.byref(opts), ctypes.c_void_p(_stream_handle(stream)),
                             ctypes.byref(tt), ctypes.byref(rep)))
    report = dict(buckets=rep.buckets, probes=rep.probes, total_ms=rep.total_ms,
                  choice={(nb, sb): (tt.l2_bits[nb][sb], tt.sample_rate[nb][sb])
                          for nb in range(TUNE_NB) for sb in range(TUNE_SB) if tt.l2_bits[nb][sb]},
                  cost_ns_per_symbol={(nb, sb): rep.cost_ns_per_symbol[nb][sb]
                                      for nb in range(TUNE_NB) for sb in range(TUNE_SB) if tt.l2_bits[nb][sb]})
    return tt, report


def save_tune(tt: TuneTable, path: str):
    """Tuning table as JSON: {"n_bucket,sigma_bucket": [l2_bits, sample_rate]} (tuned buckets only)."""
    import json
    d = {"%d,%d" % (nb, sb): [tt.l2_bits[nb][sb], tt.sample_rate[nb][sb]]
         for nb in range(TUNE_NB) for sb in range(TUNE_SB) if tt.l2_bits[nb][sb]}
    with open(path, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)


def load_tune(path: str) -> TuneTable:
    import json
    with open(path) as fh:
        d = json.load(fh)
    return make_tune_table({tuple(int(x) for x in k.split(",")): tuple(v) for k, v in d.items()})


def build_forest(seqs, sigmas, l2_bits=None, sample_rates=None, tune: TuneTable = None, stream=None,
                 wide: bool = False) -> Forest:
    """Build one tree per device tensor of `seqs` (all uint8, all uint16 or all uint32; views of one buffer
    are fine) in one captured graph launch. l2_bits / sample_rates: per-sequence lists (0 = tuned/default);
    wide: carry full-width codes through every level (same trees)."""
    descs, w = _descs(seqs, sigmas, l2_bits, sample_rates)
    opts = ForestOpts(ctypes.pointer(tune) if tune is not None else None, BUILD_WIDE if wide else 0, 0)
    h = ctypes.c_void_p(0)
    _check(lib().wt_build_forest(descs, len(seqs), w, ctypes.byref(opts), ctypes.c_void_p(_stream_handle(stream)),
                                 ctypes.byref(h)))
    return Forest(h.value)


def _host_ptr(a) -> int:
    """Address of a host array: numpy array or CPU torch tensor (page-locked ones copy asynchronously)."""
    if a is None:
        return 0
    if isinstance(a, np.ndarray):
        if not a.flags.c_contiguous:
            raise ValueError("host arrays must be contiguous")
        return a.ctypes.data
    if getattr(a, "is_cuda", False):
        raise ValueError("server requests take host arrays")
    return a.data_ptr()


class Server:
    """Continuous-batching server over a resident forest (or a simulated executor when sim_ns_per_query > 0)."""

    def __init__(self, forest=None, slots: int = 0, mem_budget: int = 0, sim_ns_per_query: float = 0.0,
                 coalesce: int = 0):
        """slots: batches in flight (0: 8); coalesce: largest total of coalesced requests (0: 16384, 1: none)."""
        opts = ServerOpts(slots, coalesce, mem_budget, sim_ns_per_query)
        h = ctypes.c_void_p(0)
        _check(lib().wt_server_create(forest._h if forest is not None else None, ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self._forest = forest

    def run(self, requests):
        """requests: sorted by arrival, each a dict with tree, op, sym, arg, out (host arrays of q entries: u32, u8,
        u32, u64, u64) and arrival_s; or, for a simulated server, just q and arrival_s.
        Returns (list of completion dicts, stats dict)."""
        R = (Request * max(len(requests), 1))()
        for i, r in enumerate(requests):
            q = int(r["q"]) if "q" in r else len(r["arg"])
            R[i] = Request(_host_ptr(r.get("tree")), _host_ptr(r.get("op")), _host_ptr(r.get("sym")),
                           _host_ptr(r.get("arg")), _host_ptr(r.get("out")), q, float(r["arrival_s"]))
        C = (Completion * max(len(requests), 1))()
        st = ServeStats()
        _check(lib().wt_server_run(self._h, R, len(requests), C, ctypes.byref(st)))
        comps = [dict(arrival_s=C[i].arrival_s, admit_s=C[i].admit_s, done_s=C[i].done_s, slot=C[i].slot,
                      status=C[i].status) for i in range(len(requests))]
        stats = {f: getattr(st, f) for f, _ in ServeStats._fields_ if f != "reserved"}
        return comps, stats

    def close(self):
        if self._h is not None and self._h.value:
            _check(lib().wt_server_destroy(self._h))
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def query_profiling(on: bool = True):
    """Record per-kernel durations of this thread's query calls (read with query_profile)."""
    _check(lib().wt_query_profiling(1 if on else 0))


def query_profile() -> list:
    """Durations of the kernels of this thread's query calls since the last read (waits for them)."""
    cnt = ctypes.c_uint32(0)
    arr = (ProfEntry * 4096)()
    _check(lib().wt_query_profile(arr, 4096, ctypes.byref(cnt)))
    return [dict(kernel=arr[i].kernel.decode(), ms=arr[i].ms) for i in range(min(cnt.value, 4096))]


def mlp_loss_grad(params, u, v, stream=None):
    """Loss and gradient of the learned-select network on the device (the training kernel's code):
    returns a float32 tensor [loss, d loss / d param_0 .. param_48]."""
    torch = _torch()
    P = u.numel()
    out = torch.empty(1 + MLP_PARAMS, dtype=torch.float32, device=u.device)
    _check(lib().wt_mlp_loss_grad(_dev_ptr(params, torch.float32, "params"), _dev_ptr(u, torch.float32, "u"),
                                  _dev_ptr(v, torch.float32, "v"), P, _dev_ptr(out, torch.float32, "out"),
                                  ctypes.c_void_p(_stream_handle(stream))))
    return out


def version() -> str:
    return lib().wt_version().decode()
