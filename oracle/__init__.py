"""Plain CPU oracle for the level-wise wavelet tree — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The product path (``paper_2505_03372_amd``)
never imports it and fails loudly when its HIP library is missing.

The arithmetic lives in ``wt_oracle.c`` (plain C, definitions written out; see the
header of that file for the passages of the thesis each function follows). This
module only marshals numpy arrays and adds the pure-Python brute-force answers
(``brute_*``) used on tiny inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wt_oracle.c")
_SRC_PAR = os.path.join(_HERE, "wt_oracle_par.c")
_LIB = os.path.join(_HERE, "libwtoracle.so")

ACCESS_INVALID = 0xFFFFFFFF
U64_MAX = (1 << 64) - 1

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u16p = ctypes.POINTER(ctypes.c_uint16)


def build_lib(force: bool = False) -> str:
    """Compile wt_oracle.c and its all-core form wt_oracle_par.c (OpenMP) into libwtoracle.so with gcc."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_PAR))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", tmp, _SRC, _SRC_PAR])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build_lib())
        L.oracle_num_levels.restype = ctypes.c_int
        L.oracle_num_levels.argtypes = [ctypes.c_uint64]
        L.oracle_codes.argtypes = [ctypes.c_uint64, _u64p, _u32p]
        L.oracle_hist.restype = ctypes.c_int
        L.oracle_hist.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, _u64p]
        L.oracle_level_bits.restype = ctypes.c_int
        L.oracle_level_bits.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64,
                                        ctypes.c_uint64, _u64p, _u64p]
        L.oracle_level_bits_codes.restype = ctypes.c_int
        L.oracle_level_bits_codes.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64,
                                              ctypes.c_int, _u64p, _u32p, ctypes.c_uint64, _u64p, _u64p]
        L.oracle_nodes_codes.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64,
                                         ctypes.c_int, _u64p, _u32p, ctypes.c_int, _u64p, _u64p, _u64p]
        L.oracle_huffman_lengths.restype = ctypes.c_int
        L.oracle_huffman_lengths.argtypes = [_u64p, ctypes.c_uint64, ctypes.c_int, _u32p]
        L.oracle_huffman_codes.restype = ctypes.c_int
        L.oracle_huffman_codes.argtypes = [_u32p, ctypes.c_uint64, _u64p, _u32p]
        L.oracle_directory.argtypes = [_u64p, ctypes.c_uint64, ctypes.c_uint64, _u64p, _u16p]
        L.oracle_samples.argtypes = [_u64p, ctypes.c_uint64, ctypes.c_uint64, _u64p, _u64p, _u64p, _u64p]
        L.oracle_nodes.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, ctypes.c_int,
                                   _u64p, _u64p, _u64p]
        L.oracle_access.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, _u64p, ctypes.c_uint64, _u32p]
        L.oracle_rank.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, _u32p, _u64p,
                                  ctypes.c_uint64, _u64p]
        L.oracle_select.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, _u32p, _u64p,
                                    ctypes.c_uint64, _u64p]
        _f64p = ctypes.POINTER(ctypes.c_double)
        L.oracle_mlp_forward.restype = ctypes.c_double
        L.oracle_mlp_forward.argtypes = [_f64p, ctypes.c_double]
        L.oracle_mlp_loss_grad.restype = ctypes.c_double
        L.oracle_mlp_loss_grad.argtypes = [_f64p, _f64p, _f64p, ctypes.c_int, _f64p]
        L.oracle_wm_level_bits.restype = ctypes.c_int
        L.oracle_wm_level_bits.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64,
                                           ctypes.c_uint64, _u64p, _u64p]
        L.oracle_wm_starts.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, _u64p]
        L.oracle_alphabet.restype = ctypes.c_uint64
        L.oracle_alphabet.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, _u64p]
        L.oracle_par_threads.restype = ctypes.c_int
        L.oracle_par_threads.argtypes = [ctypes.c_int]
        L.oracle_par_access.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, _u64p, ctypes.c_uint64, _u32p,
                                        ctypes.c_int]
        L.oracle_par_rank.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, _u32p, _u64p,
                                      ctypes.c_uint64, _u64p, ctypes.c_int]
        L.oracle_par_select.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, _u32p,
                                        _u64p, ctypes.c_uint64, _u64p, ctypes.c_int]
        L.oracle_par_tree.restype = ctypes.c_int
        L.oracle_par_tree.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64,
                                      ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, _u64p, _u64p,
                                      ctypes.c_uint64, _u64p, ctypes.c_uint64, _u16p, ctypes.c_uint64, _u64p, _u64p,
                                      _u64p, _u64p, ctypes.c_int]
        _lib = L
    return _lib


def _seq(S: np.ndarray) -> np.ndarray:
    S = np.ascontiguousarray(S)
    assert S.dtype in (np.uint8, np.uint16, np.uint32, np.uint64), S.dtype
    return S


def _p(a, t):
    return a.ctypes.data_as(t)


def num_levels(sigma: int) -> int:
    return int(lib().oracle_num_levels(sigma))


def codes(sigma: int):
    """Reduced-tree codes (left-aligned to L bits) and code lengths of all symbols."""
    code = np.zeros(max(sigma, 1), dtype=np.uint64)
    ln = np.zeros(max(sigma, 1), dtype=np.uint32)
    lib().oracle_codes(sigma, _p(code, _u64p), _p(ln, _u32p))
    return code[:sigma], ln[:sigma]


def huffman_limit(m: int) -> int:
    """Longest code a Huffman-shaped tree of m >= 2 occurring symbols may use: ceil(lg m) + 8, at most
    24 (the most levels a tree has)."""
    return min(24, max(1, (m - 1).bit_length()) + 8)


def huffman_lengths(h: np.ndarray, limit: int | None = None) -> np.ndarray:
    """Optimal code lengths, none above `limit`, for the counts h (package-merge; wt_oracle.c)."""
    h = np.ascontiguousarray(h, dtype=np.uint64)
    m = int(np.count_nonzero(h))
    if limit is None:
        limit = huffman_limit(max(m, 2))
    ln = np.zeros(max(h.size, 1), dtype=np.uint32)
    rc = lib().oracle_huffman_lengths(_p(h, _u64p), h.size, limit, _p(ln, _u32p))
    if rc < 0:
        raise ValueError("2^limit is below the number of symbols")
    return ln[: h.size]


def huffman_codes(lens: np.ndarray):
    """Canonical codes for the lengths: (left-aligned codes, ranks in code order, L)."""
    lens = np.ascontiguousarray(lens, dtype=np.uint32)
    code = np.zeros(max(lens.size, 1), dtype=np.uint64)
    rk = np.zeros(max(lens.size, 1), dtype=np.uint32)
    L = lib().oracle_huffman_codes(_p(lens, _u32p), lens.size, _p(code, _u64p), _p(rk, _u32p))
    return code[: lens.size], rk[: lens.size], int(L)


def hist(S: np.ndarray, sigma: int) -> np.ndarray:
    S = _seq(S)
    h = np.zeros(max(sigma, 1), dtype=np.uint64)
    bad = lib().oracle_hist(ctypes.c_void_p(S.ctypes.data), S.size, S.dtype.itemsize, sigma, _p(h, _u64p))
    if bad:
        raise ValueError("symbol out of range")
    return h[:sigma]


def alphabet(S: np.ndarray) -> np.ndarray:
    """The minimal alphabet: the distinct values of S in increasing order (wt_oracle.c)."""
    S = _seq(S)
    vals = np.zeros(max(S.size, 1), dtype=np.uint64)
    d = lib().oracle_alphabet(ctypes.c_void_p(S.ctypes.data), S.size, S.dtype.itemsize, _p(vals, _u64p))
    return vals[:d].copy()


class OracleTree:
    """Every part of the tree, computed from its definition (see wt_oracle.c)."""

    def __init__(self, S: np.ndarray, sigma: int, l2_bits: int = 512, sample_rate: int = 4096,
                 with_nodes: bool = True, huffman: bool = False):
        S = _seq(S)
        self.n = int(S.size)
        self.sigma = int(sigma)
        self.l2_bits = l2_bits
        self.sample_rate = sample_rate
        self.huffman = huffman
        self.hist = hist(S, sigma)
        self.cum_hist = np.zeros(sigma + 1, dtype=np.uint64)
        self.cum_hist[1:] = np.cumsum(self.hist, dtype=np.uint64)
        if huffman:
            # Huffman-shaped: canonical codes of the optimal length-limited code for these counts
            self.lens = huffman_lengths(self.hist)
            self.codes, self.rank, self.L = huffman_codes(self.lens)
        else:
            self.codes, self.lens = codes(sigma)
            self.L = num_levels(sigma)
        L = self.L
        stride = max(1, (self.n + 63) // 64)
        bits = np.zeros((max(L, 1), stride), dtype=np.uint64)
        level_n = np.zeros(max(L, 1), dtype=np.uint64)
        if huffman:
            rc = lib().oracle_level_bits_codes(ctypes.c_void_p(S.ctypes.data), self.n, S.dtype.itemsize, sigma, L,
                                               _p(self.codes, _u64p), _p(self.lens, _u32p), stride,
                                               _p(bits, _u64p), _p(level_n, _u64p))
        else:
            rc = lib().oracle_level_bits(ctypes.c_void_p(S.ctypes.data), self.n, S.dtype.itemsize, sigma, stride,
                                         _p(bits, _u64p), _p(level_n, _u64p))
        if rc != 0:
            raise ValueError("symbol out of range")
        self.level_n = [int(x) for x in level_n[:L]]
        self.bits, self.L1, self.L2, self.samples1, self.samples0, self.ones = [], [], [], [], [], []
        self.node_start, self.node_r0 = [], []
        for l in range(L):
            nl = self.level_n[l]
            row = np.ascontiguousarray(bits[l, : (nl + 63) // 64])
            self.bits.append(row)
            rowp = np.ascontiguousarray(bits[l])
            L1 = np.zeros((nl + 65535) // 65536 + 1, dtype=np.uint64)
            L2 = np.zeros((nl + l2_bits - 1) // l2_bits + 1, dtype=np.uint16)
            lib().oracle_directory(_p(rowp, _u64p), nl, l2_bits, _p(L1, _u64p), _p(L2, _u16p))
            self.L1.append(L1)
            self.L2.append(L2)
            cap = nl // sample_rate + 1
            s1 = np.zeros(cap, dtype=np.uint64)
            s0 = np.zeros(cap, dtype=np.uint64)
            n1 = ctypes.c_uint64(0)
            n0 = ctypes.c_uint64(0)
            lib().oracle_samples(_p(rowp, _u64p), nl, sample_rate, _p(s1, _u64p), ctypes.byref(n1),
                                 _p(s0, _u64p), ctypes.byref(n0))
            self.samples1.append(s1[: n1.value].copy())
            self.samples0.append(s0[: n0.value].copy())
            self.ones.append(int(L1[-1]))
            if with_nodes:
                st = np.zeros(1 << l, dtype=np.uint64)
                r0 = np.zeros(1 << l, dtype=np.uint64)
                if huffman:
                    lib().oracle_nodes_codes(ctypes.c_void_p(S.ctypes.data), self.n, S.dtype.itemsize, sigma, L,
                                             _p(self.codes, _u64p), _p(self.lens, _u32p), l, _p(rowp, _u64p),
                                             _p(st, _u64p), _p(r0, _u64p))
                else:
                    lib().oracle_nodes(ctypes.c_void_p(S.ctypes.data), self.n, S.dtype.itemsize, sigma, l,
                                       _p(rowp, _u64p), _p(st, _u64p), _p(r0, _u64p))
                self.node_start.append(st)
                self.node_r0.append(r0)

    def bit(self, l: int, j: int) -> int:
        return int((int(self.bits[l][j // 64]) >> (j % 64)) & 1)

    def bit_string(self, l: int) -> str:
        return "".join(str(self.bit(l, j)) for j in range(self.level_n[l]))


class OracleMatrix:
    """Every part of the wavelet matrix of S (all n elements at every level; see wt_oracle.c), with the
    same rank directory and select samples per level as the tree."""

    def __init__(self, S: np.ndarray, sigma: int, l2_bits: int = 512, sample_rate: int = 4096):
        S = _seq(S)
        self.n = int(S.size)
        self.sigma = int(sigma)
        self.L = num_levels(sigma)
        L, n = self.L, self.n
        stride = max(1, (n + 63) // 64)
        bits = np.zeros((max(L, 1), stride), dtype=np.uint64)
        zeros = np.zeros(max(L, 1), dtype=np.uint64)
        rc = lib().oracle_wm_level_bits(ctypes.c_void_p(S.ctypes.data), n, S.dtype.itemsize, sigma, stride,
                                        _p(bits, _u64p), _p(zeros, _u64p))
        if rc != 0:
            raise ValueError("symbol out of range")
        self.zeros = [int(z) for z in zeros[:L]]
        self.starts = np.zeros(max(sigma, 1), dtype=np.uint64)
        lib().oracle_wm_starts(ctypes.c_void_p(S.ctypes.data), n, S.dtype.itemsize, sigma, _p(self.starts, _u64p))
        self.starts = self.starts[:sigma]
        self.bits, self.L1, self.L2, self.samples1, self.samples0, self.ones = [], [], [], [], [], []
        for l in range(L):
            row = np.ascontiguousarray(bits[l, : (n + 63) // 64])
            self.bits.append(row)
            rowp = np.ascontiguousarray(bits[l])
            L1 = np.zeros((n + 65535) // 65536 + 1, dtype=np.uint64)
            L2 = np.zeros((n + l2_bits - 1) // l2_bits + 1, dtype=np.uint16)
            lib().oracle_directory(_p(rowp, _u64p), n, l2_bits, _p(L1, _u64p), _p(L2, _u16p))
            self.L1.append(L1)
            self.L2.append(L2)
            cap = n // sample_rate + 1
            s1 = np.zeros(cap, dtype=np.uint64)
            s0 = np.zeros(cap, dtype=np.uint64)
            n1 = ctypes.c_uint64(0)
            n0 = ctypes.c_uint64(0)
            lib().oracle_samples(_p(rowp, _u64p), n, sample_rate, _p(s1, _u64p), ctypes.byref(n1),
                                 _p(s0, _u64p), ctypes.byref(n0))
            self.samples1.append(s1[: n1.value].copy())
            self.samples0.append(s0[: n0.value].copy())
            self.ones.append(int(L1[-1]))

    def bit(self, l: int, j: int) -> int:
        return int((int(self.bits[l][j // 64]) >> (j % 64)) & 1)

    def bit_string(self, l: int) -> str:
        return "".join(str(self.bit(l, j)) for j in range(self.n))


def access(S: np.ndarray, pos: np.ndarray) -> np.ndarray:
    S = _seq(S)
    pos = np.ascontiguousarray(pos, dtype=np.uint64)
    out = np.empty(pos.size, dtype=np.uint32)
    lib().oracle_access(ctypes.c_void_p(S.ctypes.data), S.size, S.dtype.itemsize, _p(pos, _u64p), pos.size,
                        _p(out, _u32p))
    return out


def rank(S: np.ndarray, sigma: int, c: np.ndarray, i: np.ndarray) -> np.ndarray:
    S = _seq(S)
    c = np.ascontiguousarray(c, dtype=np.uint32)
    i = np.ascontiguousarray(i, dtype=np.uint64)
    out = np.empty(c.size, dtype=np.uint64)
    lib().oracle_rank(ctypes.c_void_p(S.ctypes.data), S.size, S.dtype.itemsize, sigma, _p(c, _u32p),
                      _p(i, _u64p), c.size, _p(out, _u64p))
    return out


def select(S: np.ndarray, sigma: int, c: np.ndarray, k: np.ndarray) -> np.ndarray:
    S = _seq(S)
    c = np.ascontiguousarray(c, dtype=np.uint32)
    k = np.ascontiguousarray(k, dtype=np.uint64)
    out = np.empty(c.size, dtype=np.uint64)
    lib().oracle_select(ctypes.c_void_p(S.ctypes.data), S.size, S.dtype.itemsize, sigma, _p(c, _u32p),
                        _p(k, _u64p), c.size, _p(out, _u64p))
    return out


# ---- all-core form (OpenMP; wt_oracle_par.c): same answers, work spread over host threads ----


def par_threads(nthreads: int = 0) -> int:
    """Threads the all-core functions use (0: OpenMP's default, i.e. OMP_NUM_THREADS or the cores)."""
    return int(lib().oracle_par_threads(nthreads))


def par_access(S: np.ndarray, pos: np.ndarray, nthreads: int = 0) -> np.ndarray:
    S = _seq(S)
    pos = np.ascontiguousarray(pos, dtype=np.uint64)
    out = np.empty(pos.size, dtype=np.uint32)
    lib().oracle_par_access(ctypes.c_void_p(S.ctypes.data), S.size, S.dtype.itemsize, _p(pos, _u64p), pos.size,
                            _p(out, _u32p), nthreads)
    return out


def par_rank(S: np.ndarray, sigma: int, c: np.ndarray, i: np.ndarray, nthreads: int = 0) -> np.ndarray:
    assert sigma >= 1
    S = _seq(S)
    c = np.ascontiguousarray(c, dtype=np.uint32)
    i = np.ascontiguousarray(i, dtype=np.uint64)
    out = np.empty(c.size, dtype=np.uint64)
    lib().oracle_par_rank(ctypes.c_void_p(S.ctypes.data), S.size, S.dtype.itemsize, sigma, _p(c, _u32p),
                          _p(i, _u64p), c.size, _p(out, _u64p), nthreads)
    return out


def par_select(S: np.ndarray, sigma: int, c: np.ndarray, k: np.ndarray, nthreads: int = 0) -> np.ndarray:
    assert sigma >= 1
    S = _seq(S)
    c = np.ascontiguousarray(c, dtype=np.uint32)
    k = np.ascontiguousarray(k, dtype=np.uint64)
    out = np.empty(c.size, dtype=np.uint64)
    lib().oracle_par_select(ctypes.c_void_p(S.ctypes.data), S.size, S.dtype.itemsize, sigma, _p(c, _u32p),
                            _p(k, _u64p), c.size, _p(out, _u64p), nthreads)
    return out


def par_tree(S: np.ndarray, sigma: int, l2_bits: int = 512, sample_rate: int = 4096, nthreads: int = 0) -> dict:
    """Every level's bits, directory and samples, one level per thread (wt_oracle_par.c)."""
    S = _seq(S)
    n = int(S.size)
    L = num_levels(sigma)
    Lr = max(L, 1)
    stride = max(1, (n + 63) // 64)
    l1s = (n + 65535) // 65536 + 1
    l2s = (n + l2_bits - 1) // l2_bits + 1
    ss = n // sample_rate + 1
    bits = np.zeros((Lr, stride), dtype=np.uint64)
    level_n = np.zeros(Lr, dtype=np.uint64)
    L1 = np.zeros((Lr, l1s), dtype=np.uint64)
    L2 = np.zeros((Lr, l2s), dtype=np.uint16)
    s1 = np.zeros((Lr, ss), dtype=np.uint64)
    s0 = np.zeros((Lr, ss), dtype=np.uint64)
    n1 = np.zeros(Lr, dtype=np.uint64)
    n0 = np.zeros(Lr, dtype=np.uint64)
    rc = lib().oracle_par_tree(ctypes.c_void_p(S.ctypes.data), n, S.dtype.itemsize, sigma, l2_bits, sample_rate,
                               stride, _p(bits, _u64p), _p(level_n, _u64p), l1s, _p(L1, _u64p), l2s, _p(L2, _u16p),
                               ss, _p(s1, _u64p), _p(n1, _u64p), _p(s0, _u64p), _p(n0, _u64p), nthreads)
    if rc != 0:
        raise ValueError("symbol out of range")
    out = {"L": L, "level_n": [int(x) for x in level_n[:L]], "bits": [], "L1": [], "L2": [], "samples1": [],
           "samples0": []}
    for l in range(L):
        nl = out["level_n"][l]
        out["bits"].append(bits[l, : (nl + 63) // 64])
        out["L1"].append(L1[l, : (nl + 65535) // 65536 + 1])
        out["L2"].append(L2[l, : (nl + l2_bits - 1) // l2_bits + 1])
        out["samples1"].append(s1[l, : int(n1[l])])
        out["samples0"].append(s0[l, : int(n0[l])])
    return out


# ---- learned select predictor (FP64 reference of the 1 -> 16 -> 1 ReLU network) ----

MLP_PARAMS = 49


def mlp_init() -> np.ndarray:
    """The starting point of training: y = relu(u) = u on [0, 1] (w1 = 1, b1_k = -k/16, w2 = e_0, b2 = 0)."""
    th = np.zeros(MLP_PARAMS, dtype=np.float64)
    th[0:16] = 1.0
    th[16:32] = -np.arange(16) / 16.0
    th[32] = 1.0
    return th


def mlp_forward(theta, u) -> np.ndarray:
    th = np.ascontiguousarray(theta, dtype=np.float64)
    p = th.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return np.array([lib().oracle_mlp_forward(p, float(x)) for x in np.atleast_1d(u)])


def mlp_loss_grad(theta, u, v):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    g = np.zeros(MLP_PARAMS, dtype=np.float64)
    f = ctypes.POINTER(ctypes.c_double)
    loss = lib().oracle_mlp_loss_grad(th.ctypes.data_as(f), u.ctypes.data_as(f), v.ctypes.data_as(f), u.size,
                                      g.ctypes.data_as(f))
    return loss, g


# ---- pure-Python brute force (tiny inputs only) ----

def brute_access(S, i):
    return int(S[i]) if 0 <= i < len(S) else ACCESS_INVALID


def brute_rank(S, sigma, c, i):
    n = len(S)
    if i > n:
        return U64_MAX
    if c >= sigma:
        return 0
    return sum(1 for j in range(i) if int(S[j]) == c)


def brute_select(S, sigma, c, k):
    n = len(S)
    if k == 0:
        return U64_MAX
    if c >= sigma:
        return n
    seen = 0
    for j in range(n):
        if int(S[j]) == c:
            seen += 1
            if seen == k:
                return j
    return n
