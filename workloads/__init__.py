"""Seeded synthetic workloads (inputs only) for the wavelet-tree hot path.

Shared by the CPU oracle tests, the GPU parity tests and ``bench.py``. The module
holds no wavelet-tree arithmetic: it draws symbol sequences and query arguments
from counter-based SplitMix64 streams (``gen.c``) with the shapes and value
distributions of the thesis's workloads:

* ``plain_small``  : n = 2^20 u8, alphabet 256, i.i.d. uniform; 2^16 queries of each kind.
* ``text_zipf``    : n = 2^30 u8, alphabet 256, Zipf(s=1.0) frequencies over a seeded
                     permutation of the symbols (a stand-in for the CommonCrawl text of the
                     thesis's evaluation, whose order-0 entropy is about 6.2 bits); 2^26 queries each.
* ``large_alpha``  : n = 2^28 u32, alphabet 2^20 (20 levels); first half uniform, second half
                     Zipf(s=1.2) over a seeded permutation; 2^24 rank and select queries.

Query recipe: access positions uniform in [0, n); rank symbols drawn from S (S[uniform(n)])
with positions uniform in [0, n); select symbols drawn from S with k uniform in [1, count].
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libwtgen.so")

TAG_TEXT, TAG_PERM, TAG_ACC, TAG_RANK_C, TAG_RANK_I, TAG_SEL_C, TAG_SEL_K, TAG_TEXT2 = range(1, 9)
TAG_TREE_N, TAG_TREE_SIGMA, TAG_MIX_TREE, TAG_MIX_OP, TAG_MIX_U1, TAG_MIX_U2 = range(9, 15)
TAG_TREE_BASE = 0x1000  # sub-seed of tree j: subseed(base, TAG_TREE_BASE + j)

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_f64p = ctypes.POINTER(ctypes.c_double)


def build_lib(force: bool = False) -> str:
    """Compile gen.c into libwtgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build_lib())
        L.gen_mix64.restype = ctypes.c_uint64
        L.gen_mix64.argtypes = [ctypes.c_uint64]
        L.gen_subseed.restype = ctypes.c_uint64
        L.gen_subseed.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.gen_raw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, _u64p]
        L.gen_fill_uniform.argtypes = [ctypes.c_uint64] * 5 + [ctypes.c_int, ctypes.c_void_p]
        L.gen_permutation.argtypes = [ctypes.c_uint64, ctypes.c_uint64, _u32p]
        L.gen_zipf_cdf.argtypes = [ctypes.c_uint64, ctypes.c_double, _f64p]
        L.gen_fill_zipf.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, _f64p,
                                    ctypes.c_uint64, _u32p, ctypes.c_int, ctypes.c_void_p]
        L.gen_fill_loguniform.argtypes = [ctypes.c_uint64] * 5 + [_u64p]
        L.gen_draw_from_seq.argtypes = [ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                        ctypes.c_uint64, _u32p]
        L.gen_draw_rank_in_count.argtypes = [ctypes.c_uint64, _u32p, _u64p, ctypes.c_uint64, _u64p]
        L.gen_bits.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                               _u64p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray, t=None):
    return a.ctypes.data_as(t) if t is not None else ctypes.c_void_p(a.ctypes.data)


def dtype_for(width: int):
    return {1: np.uint8, 2: np.uint16, 4: np.uint32}[width]


def subseed(base: int, tag: int) -> int:
    return int(lib().gen_subseed(base, tag))


def raw(seed: int, a: int, b: int) -> np.ndarray:
    out = np.empty(b - a, dtype=np.uint64)
    lib().gen_raw(seed, a, b, _ptr(out, _u64p))
    return out


def mix64(x: int) -> int:
    return int(lib().gen_mix64(x))


def uniform(seed: int, n: int, m: int, width: int = 8, lo: int = 0, out: np.ndarray | None = None,
            a: int = 0) -> np.ndarray:
    """Elements [a, a+n) of the stream mapped to uniform integers in [lo, lo+m)."""
    if out is None:
        out = np.empty(n, dtype=np.uint64 if width == 8 else dtype_for(width))
    assert out.dtype.itemsize == width and out.flags.c_contiguous
    # gen_fill_uniform indexes its output by the absolute stream index, so pass a shifted base pointer.
    base = out.ctypes.data - a * width
    lib().gen_fill_uniform(seed, a, a + n, lo, m, width, ctypes.c_void_p(base))
    return out


def permutation(seed: int, K: int) -> np.ndarray:
    perm = np.empty(K, dtype=np.uint32)
    lib().gen_permutation(seed, K, _ptr(perm, _u32p))
    return perm


def zipf(seed: int, n: int, K: int, s: float, width: int, perm: np.ndarray | None,
         out: np.ndarray | None = None, a: int = 0) -> np.ndarray:
    """Elements [a, a+n) of the stream mapped to perm[Zipf(s) rank - 1] over K ranks."""
    cdf = np.empty(K, dtype=np.float64)
    lib().gen_zipf_cdf(K, s, _ptr(cdf, _f64p))
    if out is None:
        out = np.empty(n, dtype=dtype_for(width))
    assert out.dtype.itemsize == width and out.flags.c_contiguous
    base = out.ctypes.data - a * width
    lib().gen_fill_zipf(seed, a, a + n, _ptr(cdf, _f64p), K,
                        _ptr(perm, _u32p) if perm is not None else None, width, ctypes.c_void_p(base))
    return out


def loguniform(seed: int, n: int, lo: int, hi: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    lib().gen_fill_loguniform(seed, 0, n, lo, hi, _ptr(out, _u64p))
    return out


def draw_from_seq(seed: int, S: np.ndarray, q: int) -> np.ndarray:
    out = np.empty(q, dtype=np.uint32)
    if S.size == 0:
        out[:] = 0
        return out
    lib().gen_draw_from_seq(seed, _ptr(S), S.size, S.dtype.itemsize, q, _ptr(out, _u32p))
    return out


def draw_k(seed: int, c: np.ndarray, counts: np.ndarray, q: int) -> np.ndarray:
    out = np.empty(q, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.uint32)
    counts = np.ascontiguousarray(counts, dtype=np.uint64)
    lib().gen_draw_rank_in_count(seed, _ptr(c, _u32p), _ptr(counts, _u64p), q, _ptr(out, _u64p))
    return out


@dataclass
class Workload:
    name: str
    S: np.ndarray
    sigma: int
    acc_pos: np.ndarray | None = None
    rank_c: np.ndarray | None = None
    rank_i: np.ndarray | None = None
    sel_c: np.ndarray | None = None
    sel_k: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.S.size)


CONFIGS = {
    # name: (config index, n, width, sigma, queries per kind)
    "plain_small": (0, 1 << 20, 1, 256, 1 << 16),
    "text_zipf": (1, 1 << 30, 1, 256, 1 << 26),
    "large_alpha": (2, 1 << 28, 4, 1 << 20, 1 << 24),
}


def base_seed(index: int) -> int:
    return 0x5EED0000 + index


def make_text(name: str, n: int | None = None) -> tuple[np.ndarray, int]:
    idx, n0, width, sigma, _ = CONFIGS[name]
    n = n0 if n is None else n
    base = base_seed(idx)
    if name == "plain_small":
        S = uniform(subseed(base, TAG_TEXT), n, sigma, width)
    elif name == "text_zipf":
        perm = permutation(subseed(base, TAG_PERM), sigma)
        S = zipf(subseed(base, TAG_TEXT), n, sigma, 1.0, width, perm)
    elif name == "large_alpha":
        S = np.empty(n, dtype=dtype_for(width))
        h = n // 2
        uniform(subseed(base, TAG_TEXT), h, sigma, width, out=S[:h])
        perm = permutation(subseed(base, TAG_PERM), sigma)
        zipf(subseed(base, TAG_TEXT2), n - h, sigma, 1.2, width, perm, out=S[h:], a=h)
    else:
        raise KeyError(name)
    return S, sigma


def make_queries(name: str, S: np.ndarray, sigma: int, q: int | None = None, kinds=("access", "rank", "select")):
    idx, _, _, _, q0 = CONFIGS[name]
    q = q0 if q is None else q
    base = base_seed(idx)
    n = S.size
    out = {}
    if "access" in kinds:
        out["acc_pos"] = uniform(subseed(base, TAG_ACC), q, max(n, 1))
    if "rank" in kinds:
        out["rank_c"] = draw_from_seq(subseed(base, TAG_RANK_C), S, q)
        out["rank_i"] = uniform(subseed(base, TAG_RANK_I), q, max(n, 1))
    if "select" in kinds:
        c = draw_from_seq(subseed(base, TAG_SEL_C), S, q)
        counts = np.bincount(S, minlength=sigma).astype(np.uint64) if n else np.zeros(sigma, np.uint64)
        out["sel_c"] = c
        out["sel_k"] = draw_k(subseed(base, TAG_SEL_K), c, counts, q)
    return out


def make(name: str, n: int | None = None, q: int | None = None, kinds=("access", "rank", "select")) -> Workload:
    S, sigma = make_text(name, n)
    qs = make_queries(name, S, sigma, q, kinds)
    return Workload(name=name, S=S, sigma=sigma, **qs)


# ---- bit arrays of the rank/select benchmark (thesis Section 6.1, after Kurpicz's experiments) ----

BITVEC = dict(index=5, n_bits=1 << 32, fills=(0.1, 0.5, 0.9), queries=100_000_000, l2_bits=512, sample_rate=16384)


def bit_words(seed: int, n_bits: int, fill: float, adversarial: bool) -> np.ndarray:
    """u64 words of a bit array whose fraction `fill` of bits are ones (in expectation). Uniform: every bit
    is one with probability fill. Adversarial: 99 % of the ones in the last fraction `fill` of the array
    and 1 % in the first 1 - fill, i.e. densities 0.99 there and 0.01 fill / (1 - fill) before."""
    words = np.zeros(max((n_bits + 63) // 64, 1), dtype=np.uint64)
    if adversarial:
        split = int(round((1.0 - fill) * n_bits))
        p_lo = 0.01 * fill / (1.0 - fill) if fill < 1.0 else 0.0
        p_hi = 0.99
    else:
        split, p_lo, p_hi = 0, fill, fill
    lib().gen_bits(seed, n_bits, split, p_lo, p_hi, _ptr(words, _u64p))
    return words[: (n_bits + 63) // 64]


def unpack_bits(words: np.ndarray, n_bits: int) -> np.ndarray:
    """Bits as a u8 array of 0/1 (bit j of the array at index j)."""
    return np.unpackbits(words.view(np.uint8), bitorder="little")[:n_bits]


def make_bitvec_queries(seed: int, n_bits: int, ones: int, q: int) -> dict:
    """access and rank positions uniform in [0, n) and [0, n]; select k uniform in [1, count_b]."""
    zeros = n_bits - ones
    out = {"pos": uniform(subseed(seed, 1), q, max(n_bits, 1)), "rank_i": uniform(subseed(seed, 2), q, n_bits + 1)}
    out["k1"] = 1 + uniform(subseed(seed, 3), q, max(ones, 1)) if ones else np.zeros(q, np.uint64)
    out["k0"] = 1 + uniform(subseed(seed, 4), q, max(zeros, 1)) if zeros else np.zeros(q, np.uint64)
    return out


# ---- batched forest: many sequences of uneven length and alphabet ----

FOREST = dict(index=3, trees=1024, width=2, n_range=(1 << 10, 1 << 24), sigma_range=(4, 1 << 16), zipf_s=1.0,
              queries=1 << 24)


@dataclass
class ForestWorkload:
    S: np.ndarray          # every sequence, concatenated
    offsets: np.ndarray    # u64[trees + 1]: sequence j is S[offsets[j]:offsets[j + 1]]
    sigmas: np.ndarray     # u64[trees]
    tree: np.ndarray | None = None  # mixed queries: u32 tree, u8 op, u32 symbol, u64 argument
    op: np.ndarray | None = None
    sym: np.ndarray | None = None
    arg: np.ndarray | None = None

    @property
    def trees(self) -> int:
        return int(self.sigmas.size)

    def seq(self, j: int) -> np.ndarray:
        return self.S[int(self.offsets[j]):int(self.offsets[j + 1])]


def _unit(seed: int, n: int) -> np.ndarray:
    """Elements [0, n) of the stream as doubles in [0, 1): (out >> 11) * 2^-53."""
    return (raw(seed, 0, n) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def _scaled(u: np.ndarray, m: np.ndarray) -> np.ndarray:
    """floor(u * m) clamped to [0, m - 1] (m >= 1), per element."""
    m = m.astype(np.float64)
    return np.minimum(np.floor(u * m), np.maximum(m - 1, 0)).astype(np.uint64)


def make_forest(trees: int | None = None, n_range=None, sigma_range=None, queries: int | None = None,
                width: int | None = None, zipf_s: float | None = None, index: int | None = None) -> ForestWorkload:
    """Sequence j: length log-uniform in n_range, alphabet log-uniform in sigma_range, Zipf(s) symbol
    frequencies over a per-tree seeded permutation. Mixed queries: tree uniform, op uniform over
    {access, rank, select}, position uniform in the tree, symbol drawn from the tree's sequence, k
    uniform in [1, count]."""
    cfg = dict(FOREST)
    for k, v in dict(trees=trees, n_range=n_range, sigma_range=sigma_range, queries=queries, width=width,
                     zipf_s=zipf_s, index=index).items():
        if v is not None:
            cfg[k] = v
    base = base_seed(cfg["index"])
    T = cfg["trees"]
    ns = loguniform(subseed(base, TAG_TREE_N), T, *cfg["n_range"])
    sig = loguniform(subseed(base, TAG_TREE_SIGMA), T, *cfg["sigma_range"])
    offsets = np.zeros(T + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(ns, dtype=np.uint64)
    S = np.empty(int(offsets[-1]), dtype=dtype_for(cfg["width"]))
    for j in range(T):
        tj = subseed(base, TAG_TREE_BASE + j)
        perm = permutation(subseed(tj, TAG_PERM), int(sig[j]))
        zipf(subseed(tj, TAG_TEXT), int(ns[j]), int(sig[j]), cfg["zipf_s"], cfg["width"], perm,
             out=S[int(offsets[j]):int(offsets[j + 1])])
    fw = ForestWorkload(S=S, offsets=offsets, sigmas=sig)
    q = cfg["queries"]
    if q:
        tree = uniform(subseed(base, TAG_MIX_TREE), q, T, 4).astype(np.uint32)
        op = uniform(subseed(base, TAG_MIX_OP), q, 3, 1).astype(np.uint8)
        u1 = _unit(subseed(base, TAG_MIX_U1), q)
        u2 = _unit(subseed(base, TAG_MIX_U2), q)
        n_t = ns[tree]
        pos = _scaled(u1, n_t)                       # access / rank position, index of the drawn symbol
        sym = np.zeros(q, dtype=np.uint32)
        arg = np.zeros(q, dtype=np.uint64)
        has = n_t > 0
        sym[has] = S[(offsets[tree[has]] + pos[has]).astype(np.int64)]
        arg[op == 0] = pos[op == 0]
        rk = op == 1
        arg[rk] = _scaled(u2[rk], n_t[rk])
        sel = np.nonzero(op == 2)[0]
        if sel.size:
            order = sel[np.argsort(tree[sel], kind="stable")]
            tt = tree[order]
            bounds = np.searchsorted(tt, np.arange(T + 1))
            for j in range(T):
                a, b = bounds[j], bounds[j + 1]
                if a == b:
                    continue
                idx = order[a:b]
                cnt = np.bincount(fw.seq(j), minlength=int(sig[j])).astype(np.uint64)
                arg[idx] = 1 + _scaled(u2[idx], np.maximum(cnt[sym[idx]], 1))
        fw.tree, fw.op, fw.sym, fw.arg = tree, op, sym, arg
    return fw
