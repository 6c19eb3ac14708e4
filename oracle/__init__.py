"""CPU oracle for the learned integer compressor (arXiv 2412.10770).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path
(``paper_2412_10770_amd``) never does, and the two share no code.

Two layers:

* plain definitions (Def. 1): ``decompress`` is the key list itself,
  ``decompress_range(b, e)`` is ``K[b:e]``, ``access(i)`` is ``K[i]``, and
  ``lower_bound(q)`` is the first index with ``K[i] >= q`` (the textbook
  lower bound, ``numpy.searchsorted(K, q, 'left')``);
* the encoding (Def. 2, Eq. 1, Sec. II-A): ``compress`` fits the anchored
  fixed-point eps-PLA per block -- greedily, or with the fewest segments of
  the same class (``fit="min"``) -- or the optimal fit over lines with a free
  fixed-point intercept (``fit="opt"``), and writes blob v1; ``decode``
  is an independent blob decoder.  Both live in ``lcref.c`` (plain C,
  ``unsigned __int128`` cone arithmetic, bit-by-bit packing).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lcref.c")
_LIB = os.path.join(_HERE, "liblcref.so")

REF_OK = 0
REF_EINVAL = -1
REF_ENOSPC = -2
REF_EFORMAT = -3
REF_EUNSORTED = -5

HEADER_FIELDS = ("key_bytes", "log2_block", "frac_bits", "width", "eps", "max_nseg", "max_seg_bytes", "n",
                 "nblocks", "nseg_total", "off_first", "off_dir", "off_res", "res_stride",
                 "off_seg", "blob_bytes", "flags")


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile lcref.c with gcc (-O2, no intrinsics) into a shared library."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-Wextra", "-o", tmp, src])
        os.replace(tmp, out)
    return out


def _bind(path: str):
    L = ctypes.CDLL(path)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    L.lcref_width.argtypes = [ctypes.c_uint32]
    L.lcref_width.restype = ctypes.c_int
    L.lcref_fit_block.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p]
    L.lcref_fit_block.restype = ctypes.c_uint32
    L.lcref_fit_block_min.argtypes = L.lcref_fit_block.argtypes
    L.lcref_fit_block_min.restype = ctypes.c_uint32
    L.lcref_fit_block_opt.argtypes = L.lcref_fit_block.argtypes + [ctypes.c_void_p]
    L.lcref_fit_block_opt.restype = ctypes.c_uint32
    L.lcref_compress.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, u8p, ctypes.c_uint64,
                                 ctypes.POINTER(ctypes.c_uint64)]
    L.lcref_compress.restype = ctypes.c_int
    L.lcref_decode.argtypes = [u8p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint64]
    L.lcref_decode.restype = ctypes.c_int
    L.lcref_header.argtypes = [u8p, ctypes.c_uint64, ctypes.c_void_p]
    L.lcref_header.restype = ctypes.c_int
    return L


FITS = ("greedy", "min", "opt")


def _fit_code(fit: str) -> int:
    if fit not in FITS:
        raise ValueError(f"fit must be one of {FITS}, not {fit!r}")
    return FITS.index(fit)


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def _keys_array(keys) -> np.ndarray:
    a = np.ascontiguousarray(keys)
    if a.dtype in (np.uint32, np.int32):
        return a.view(np.uint32)
    if a.dtype in (np.uint64, np.int64):
        return a.view(np.uint64)
    raise TypeError(f"keys must be 4- or 8-byte integers, got {a.dtype}")


def _u8p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


class Ref:
    """The encoder/decoder of one build of lcref.c (the default build, or a
    variant compiled from a modified copy by the oracle's own tests)."""

    def __init__(self, path: str):
        self.L = _bind(path)

    def width(self, eps: int) -> int:
        """Residual width ceil(log2(2 eps + 1)) as the oracle computes it."""
        return int(self.L.lcref_width(eps))

    def fit_block(self, keys, eps: int, frac_bits: int = 0, fit: str = "greedy"):
        """Fit of one block.  fit: "greedy" (each anchored segment as long as
        it goes) or "min" (fewest segments of the same anchored class) return
        (start, anchor, A) arrays; "opt" (free fixed-point intercept C,
        fewest segments) returns (start, floor(C / 2^F) mod 2^64, A,
        C mod 2^F)."""
        k = np.ascontiguousarray(_keys_array(keys), dtype=np.uint64)
        nb = len(k)
        st = np.zeros(max(nb, 1), np.uint32)
        an = np.zeros(max(nb, 1), np.uint64)
        sl = np.zeros(max(nb, 1), np.uint64)
        fc = _fit_code(fit)
        if fc == 2:
            fr = np.zeros(max(nb, 1), np.uint64)
            m = self.L.lcref_fit_block_opt(k.ctypes.data, nb, eps, frac_bits, st.ctypes.data, an.ctypes.data,
                                           sl.ctypes.data, fr.ctypes.data)
            return st[:m].copy(), an[:m].copy(), sl[:m].copy(), fr[:m].copy()
        fn = self.L.lcref_fit_block_min if fc else self.L.lcref_fit_block
        m = fn(k.ctypes.data, nb, eps, frac_bits, st.ctypes.data, an.ctypes.data, sl.ctypes.data)
        return st[:m].copy(), an[:m].copy(), sl[:m].copy()

    def compress(self, keys, eps: int, log2_block: int = 10, frac_bits: int = 0,
                 fit: str = "greedy") -> np.ndarray:
        """Encode sorted keys into a blob v1 (uint8 array)."""
        k = _keys_array(keys)
        kb = k.dtype.itemsize
        need = ctypes.c_uint64(0)
        ptr = k.ctypes.data if len(k) else None
        fc = _fit_code(fit)
        rc = self.L.lcref_compress(ptr, len(k), kb, log2_block, eps, frac_bits, fc, None, 0,
                                   ctypes.byref(need))
        if rc not in (REF_OK, REF_ENOSPC):
            raise OracleError(rc, "compress")
        out = np.zeros(need.value, np.uint8)
        rc = self.L.lcref_compress(ptr, len(k), kb, log2_block, eps, frac_bits, fc, _u8p(out),
                                   len(out), ctypes.byref(need))
        if rc != REF_OK:
            raise OracleError(rc, "compress")
        return out

    def header(self, blob) -> dict:
        b = np.ascontiguousarray(blob, dtype=np.uint8)
        f = np.zeros(len(HEADER_FIELDS), np.uint64)
        rc = self.L.lcref_header(_u8p(b), len(b), f.ctypes.data)
        if rc != REF_OK:
            raise OracleError(rc, "header")
        return {k: int(v) for k, v in zip(HEADER_FIELDS, f)}

    def decode(self, blob) -> np.ndarray:
        """Decode a blob v1 into its key list."""
        b = np.ascontiguousarray(blob, dtype=np.uint8)
        h = self.header(b)
        out = np.zeros(max(h["n"], 1), np.uint32 if h["key_bytes"] == 4 else np.uint64)
        rc = self.L.lcref_decode(_u8p(b), len(b), out.ctypes.data, h["n"])
        if rc != REF_OK:
            raise OracleError(rc, "decode")
        return out[:h["n"]]


_default = None


def default() -> Ref:
    global _default
    if _default is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _default = Ref(_LIB)
    return _default


def width(eps: int) -> int:
    return default().width(eps)


def fit_block(keys, eps: int, frac_bits: int = 0, fit: str = "greedy"):
    return default().fit_block(keys, eps, frac_bits, fit)


def compress(keys, eps: int, log2_block: int = 10, frac_bits: int = 0,
             fit: str = "greedy") -> np.ndarray:
    return default().compress(keys, eps, log2_block, frac_bits, fit)


def header(blob) -> dict:
    return default().header(blob)


def decode(blob) -> np.ndarray:
    return default().decode(blob)


# --- plain definitions (Def. 1): no compressed format involved -----------------

def decompress(keys) -> np.ndarray:
    return _keys_array(keys).copy()


def decompress_range(keys, begin: int, end: int) -> np.ndarray:
    return _keys_array(keys)[begin:end].copy()


def access(keys, idx) -> np.ndarray:
    return _keys_array(keys)[np.asarray(idx, dtype=np.int64)]


def lower_bound(keys, q) -> np.ndarray:
    k = _keys_array(keys)
    return np.searchsorted(k, np.asarray(q, dtype=k.dtype), side="left").astype(np.uint64)


# --- query operators (Sec. III-A list AND / OR, Sec. III-C quantile and AQP) --

def intersect(a, b) -> np.ndarray:
    """AND of two sorted lists (Sec. III-A): the sorted set of keys in both."""
    return np.intersect1d(_keys_array(a), _keys_array(b))


def union(a, b) -> np.ndarray:
    """OR of two sorted lists (Sec. III-A): the sorted set of keys in either."""
    return np.union1d(_keys_array(a), _keys_array(b))


def quantile(keys, k, q: int) -> np.ndarray:
    """k-th q-quantile (Sec. III-C), 0-based: K[min(floor(N * k / q), N - 1)]
    (Python integers for N * k)."""
    kk = _keys_array(keys)
    n = len(kk)
    idx = [min((n * int(x)) // int(q), n - 1) for x in np.asarray(k).ravel()]
    return kk[np.asarray(idx, dtype=np.int64)]


def predict(keys, eps: int, log2_block: int = 10, frac_bits: int = 0,
            fit: str = "greedy") -> np.ndarray:
    """The fitted eps-PLA without residuals (Def. 2; the AQP reading of
    Sec. III-C): per block, segment t starting at s_t with anchor a_t, slope
    A_t and intercept fraction c_t (0 but for fit="opt") predicts
    f(i) = a_t + floor((A_t (i - s_t) + c_t) / 2^F) for the keys up to the
    next start; |K[i] - f(i)| <= eps.  Python integers, reduced modulo
    2^(8 key_bytes); the segments come from this oracle's own fit."""
    kk = _keys_array(keys)
    mask = (1 << (8 * kk.dtype.itemsize)) - 1
    out = np.zeros_like(kk)
    B = 1 << log2_block
    for b0 in range(0, len(kk), B):
        blk = kk[b0:b0 + B]
        seg = fit_block(blk, eps, frac_bits, fit)
        st, an, sl = seg[:3]
        fr = seg[3].tolist() if fit == "opt" else [0] * len(st)
        ends = list(st[1:]) + [len(blk)]
        for s, e, a, A, c in zip(st.tolist(), ends, an.tolist(), sl.tolist(), fr):
            for j in range(int(s), int(e)):
                out[b0 + j] = (int(a) + ((int(A) * (j - int(s)) + int(c)) >> frac_bits)) & mask
    return out
