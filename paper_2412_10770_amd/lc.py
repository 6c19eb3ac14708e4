"""Python binding of the C ABI in include/lc.h (ctypes; marshalling only).

PyTorch provides device memory and the stream; every step of encoding,
decoding and querying runs in the HIP kernels of ``liblc.so``.  There is no
fallback: if the library is not built, importing this module raises.

Keys travel as 1-D contiguous device tensors holding the unsigned bit
patterns: ``torch.int32``/``torch.uint32`` for 4-byte keys and
``torch.int64``/``torch.uint64`` for 8-byte keys.  Decoded keys come back as
``torch.int32`` / ``torch.int64`` bit patterns.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime liblc.so binds to)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblc.so")

LC_OK = 0
LC_EINVAL = -1
LC_ENOSPC = -2
LC_EFORMAT = -3
LC_EDEVICE = -4
LC_ETOOBIG = -5
NOALLOC_SCRATCH_BYTES = 64 << 20  # LC_NOALLOC_SCRATCH_BYTES: workspace limit of lc_compress_noalloc
LC_FLAG_UNSORTED = 1
LC_FLAG_RANGE = 2
LC_FLAG_INTERNAL = 4
LC_FLAG_BADLIST = 8
SETOP_INTERSECT = 1
SETOP_UNION = 2
BATCH_MAX_CANDIDATES = 8
HEADER_BYTES = 128
DEFAULT_LOG2_BLOCK = 10
DEFAULT_FRAC_BITS = 0

EXPORTED = ("lc_compress_bound", "lc_compress", "lc_compress_noalloc", "lc_info", "lc_decompress", "lc_decompress_range",
            "lc_access", "lc_lower_bound", "lc_quantile", "lc_decompress_approx", "lc_setop_bound", "lc_setop",
            "lc_batch_plan", "lc_batch_compress", "lc_batch_sizes",
            "lc_batch_pick_eps", "lc_batch_decompress", "lc_batch_and_plan", "lc_batch_and", "lc_server_create", "lc_server_run",
            "lc_server_destroy", "lc_strerror")


class lc_params(ctypes.Structure):
    _fields_ = [("key_bytes", ctypes.c_uint8), ("log2_block", ctypes.c_uint8),
                ("frac_bits", ctypes.c_uint8), ("fit", ctypes.c_uint8), ("eps", ctypes.c_uint32)]


class lc_blob_info(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint32) for f in
                ("key_bytes", "log2_block", "frac_bits", "width", "eps", "max_nseg", "max_seg_bytes",
                 "flags")] + \
               [(f, ctypes.c_uint64) for f in
                ("n", "nblocks", "nseg_total", "off_first", "off_dir", "off_res", "res_stride",
                 "off_seg", "blob_bytes")]


class lc_batch_params(ctypes.Structure):
    _fields_ = [("key_bytes", ctypes.c_uint8), ("log2_block", ctypes.c_uint8), ("frac_bits", ctypes.c_uint8),
                ("tiling", ctypes.c_uint8), ("nlists", ctypes.c_uint32), ("max_eps", ctypes.c_uint32),
                ("fit", ctypes.c_uint32)] + \
               [(f, ctypes.c_uint64) for f in ("total_blocks", "total_groups", "blob_bytes", "ws_bytes")]


# struct lc_batch_list, one 64-byte record per list
BATCH_LIST_DTYPE = np.dtype([("key_off", "<u8"), ("n", "<u8"), ("blob_off", "<u8"), ("blob_cap", "<u8"),
                             ("block_off", "<u8"), ("group_off", "<u8"), ("eps", "<u4"), ("reserved", "<u4", (3,))])
assert BATCH_LIST_DTYPE.itemsize == 64
# struct lc_list_pair
PAIR_DTYPE = np.dtype([("a", "<u4"), ("b", "<u4"), ("probe", "<u4"), ("target", "<u4"), ("key_off", "<u8"),
                       ("block_off", "<u8"), ("n", "<u8")])
assert PAIR_DTYPE.itemsize == 40


class lc_serve_config(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32)]


class lc_serve_stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("launches", "max_batch_seen", "peak_arena_bytes", "arena_waits")]


# struct lc_request / lc_request_result
REQUEST_DTYPE = np.dtype([("op", "<u4"), ("reserved", "<u4"), ("a", "<u8"), ("b", "<u8"), ("arrival_ns", "<u8"),
                          ("d_dest", "<u8")])
RESULT_DTYPE = np.dtype([("admit_ns", "<i8"), ("launch_ns", "<i8"), ("complete_ns", "<i8"), ("status", "<i4"),
                         ("launch", "<u4")])
assert REQUEST_DTYPE.itemsize == 40 and RESULT_DTYPE.itemsize == 32
OP_RANGE, OP_ACCESS, OP_LOWER_BOUND = 1, 2, 3


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    P, I = ctypes.POINTER(lc_params), ctypes.POINTER(lc_blob_info)
    sig = {
        "lc_compress_bound": [u64, P, ctypes.POINTER(u64), ctypes.POINTER(u64)],
        "lc_compress": [vp, u64, P, vp, u64, vp, u64, vp, vp, vp],
        "lc_compress_noalloc": [vp, u64, P, vp, u64, vp, vp, vp],
        "lc_info": [vp, u64, I],
        "lc_decompress": [vp, I, vp, vp],
        "lc_decompress_range": [vp, I, u64, u64, vp, vp],
        "lc_access": [vp, I, vp, u64, vp, vp, vp],
        "lc_lower_bound": [vp, I, vp, u64, vp, vp],
        "lc_quantile": [vp, I, vp, u64, u64, u32, vp, vp],
        "lc_decompress_approx": [vp, I, u64, u64, vp, vp],
        "lc_setop_bound": [I, I, u32, ctypes.POINTER(u64), ctypes.POINTER(u64)],
        "lc_setop": [u32, vp, I, vp, I, vp, u64, vp, u64, vp, vp],
        "lc_batch_plan": [ctypes.POINTER(lc_batch_params), vp],
        "lc_batch_compress": [vp, u64, vp, ctypes.POINTER(lc_batch_params), vp, u64, vp, u64, vp, vp, vp],
        "lc_batch_sizes": [vp, u64, vp, ctypes.POINTER(lc_batch_params), vp, u32, vp, u64, vp, vp, vp],
        "lc_batch_pick_eps": [vp, ctypes.POINTER(lc_batch_params), vp, vp, u32, vp],
        "lc_batch_decompress": [vp, u64, vp, ctypes.POINTER(lc_batch_params), u32, vp, u64, vp, vp],
        "lc_batch_and_plan": [ctypes.POINTER(lc_batch_params), vp, vp, u32, ctypes.POINTER(u64), ctypes.POINTER(u64),
                              ctypes.POINTER(u64)],
        "lc_batch_and": [vp, u64, vp, ctypes.POINTER(lc_batch_params), vp, u32, u64, u64, u32, vp, u64, vp, vp, vp, vp],
        "lc_server_create": [vp, I, vp, u64, ctypes.POINTER(lc_serve_config), ctypes.POINTER(vp)],
        "lc_server_run": [vp, vp, u64, vp, ctypes.POINTER(lc_serve_stats)],
        "lc_server_destroy": [vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32
    L.lc_strerror.argtypes = [ctypes.c_int32]
    L.lc_strerror.restype = ctypes.c_char_p
    return L


lib = _load()


class LcError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


def strerror(code: int) -> str:
    return lib.lc_strerror(code).decode()


def _check(rc: int, what: str):
    if rc != LC_OK:
        raise LcError(rc, what)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _key_bytes(t: torch.Tensor) -> int:
    if t.dtype in (torch.int32, torch.uint32):
        return 4
    if t.dtype in (torch.int64, torch.uint64):
        return 8
    raise TypeError(f"keys must be 4- or 8-byte integers, got {t.dtype}")


def _dev(t: torch.Tensor, what: str):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous device tensor")


def key_dtype(key_bytes: int) -> torch.dtype:
    return torch.int32 if key_bytes == 4 else torch.int64


FITS = {"greedy": 0, "min": 1, "opt": 2}   # LC_FIT_GREEDY, LC_FIT_MIN, LC_FIT_OPT


def _fit(fit) -> int:
    if fit in FITS:
        return FITS[fit]
    if fit in FITS.values():
        return int(fit)
    raise ValueError(f"fit must be one of {sorted(FITS)}, not {fit!r}")


def params(key_bytes: int, eps: int, log2_block: int = DEFAULT_LOG2_BLOCK,
           frac_bits: int = DEFAULT_FRAC_BITS, fit="greedy") -> lc_params:
    return lc_params(key_bytes, log2_block, frac_bits, _fit(fit), eps)


def compress_bound(n: int, key_bytes: int, eps: int, log2_block: int = DEFAULT_LOG2_BLOCK,
                   frac_bits: int = DEFAULT_FRAC_BITS, fit="greedy"):
    """(blob_max, ws_bytes): worst-case blob size and workspace size (the
    optimal fit needs room for its intercept fractions)."""
    blob_max, ws = ctypes.c_uint64(), ctypes.c_uint64()
    p = params(key_bytes, eps, log2_block, frac_bits, fit)
    _check(lib.lc_compress_bound(n, ctypes.byref(p), ctypes.byref(blob_max), ctypes.byref(ws)),
           "lc_compress_bound")
    return blob_max.value, ws.value


def info(header) -> lc_blob_info:
    """Parse a blob header (host bytes / numpy / CPU tensor, >= 128 bytes)."""
    if isinstance(header, torch.Tensor):
        header = header.detach().cpu().contiguous().numpy()
    buf = bytes(memoryview(header).cast("B")[:HEADER_BYTES]) if not isinstance(header, bytes) else header
    out = lc_blob_info()
    raw = ctypes.create_string_buffer(buf, len(buf))
    _check(lib.lc_info(ctypes.cast(raw, ctypes.c_void_p), len(buf), ctypes.byref(out)), "lc_info")
    return out


@dataclass
class Blob:
    """A compressed key list resident in device memory."""
    data: torch.Tensor   # uint8, exactly info.blob_bytes long
    info: lc_blob_info

    @property
    def n(self) -> int:
        return self.info.n

    @property
    def key_bytes(self) -> int:
        return self.info.key_bytes

    @property
    def nbytes(self) -> int:
        return self.info.blob_bytes

    @property
    def ratio(self) -> float:
        """size(K^c) / size(K) (Def. 1), counting every blob byte."""
        return self.nbytes / max(1, self.n * self.key_bytes)

    @property
    def bits_per_key(self) -> float:
        return 8.0 * self.nbytes / max(1, self.n)

    @classmethod
    def from_device(cls, data: torch.Tensor) -> "Blob":
        inf = info(data[:HEADER_BYTES].cpu())
        return cls(data[:inf.blob_bytes], inf)


def compress_async(keys: torch.Tensor, eps: int, blob: torch.Tensor, workspace: torch.Tensor,
                   blob_bytes: torch.Tensor, flags: torch.Tensor, log2_block: int = DEFAULT_LOG2_BLOCK,
                   frac_bits: int = DEFAULT_FRAC_BITS, stream=None, fit="greedy"):
    """Enqueue lc_compress into caller-provided buffers; no synchronisation.
    fit: "greedy", "min" (fewest anchored segments) or "opt" (free
    fixed-point intercept, fewest segments of that class; the blob carries
    the intercept fractions)."""
    _dev(keys, "keys")
    kb = _key_bytes(keys)
    p = params(kb, eps, log2_block, frac_bits, fit)
    _check(lib.lc_compress(ctypes.c_void_p(keys.data_ptr()), keys.numel(), ctypes.byref(p),
                           ctypes.c_void_p(blob.data_ptr()), blob.numel(),
                           ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                           ctypes.c_void_p(blob_bytes.data_ptr()), ctypes.c_void_p(flags.data_ptr()),
                           _stream(stream)), "lc_compress")


def compress_noalloc_async(keys: torch.Tensor, eps: int, blob: torch.Tensor, blob_bytes: torch.Tensor,
                           flags: torch.Tensor, log2_block: int = DEFAULT_LOG2_BLOCK,
                           frac_bits: int = DEFAULT_FRAC_BITS, stream=None, fit="greedy"):
    """Enqueue lc_compress_noalloc (the library's static scratch as the
    workspace; nothing allocated); no synchronisation.  Raises LcError with
    LC_ETOOBIG when the workspace would exceed NOALLOC_SCRATCH_BYTES."""
    _dev(keys, "keys")
    kb = _key_bytes(keys)
    p = params(kb, eps, log2_block, frac_bits, fit)
    _check(lib.lc_compress_noalloc(ctypes.c_void_p(keys.data_ptr()), keys.numel(), ctypes.byref(p),
                                   ctypes.c_void_p(blob.data_ptr()), blob.numel(),
                                   ctypes.c_void_p(blob_bytes.data_ptr()), ctypes.c_void_p(flags.data_ptr()),
                                   _stream(stream)), "lc_compress_noalloc")


def compress(keys: torch.Tensor, eps: int, log2_block: int = DEFAULT_LOG2_BLOCK,
             frac_bits: int = DEFAULT_FRAC_BITS, stream=None, fit="greedy") -> Blob:
    """Enc of Def. 1 on the GPU; synchronises to learn the blob size.
    fit: "greedy", "min" or "opt" (as compress_async)."""
    _dev(keys, "keys")
    kb = _key_bytes(keys)
    blob_max, ws_bytes = compress_bound(keys.numel(), kb, eps, log2_block, frac_bits, fit)
    dev = keys.device
    blob = torch.empty(blob_max, dtype=torch.uint8, device=dev)
    ws = torch.empty(max(ws_bytes, 16), dtype=torch.uint8, device=dev)
    nbytes = torch.zeros(1, dtype=torch.int64, device=dev)
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    compress_async(keys, eps, blob, ws, nbytes, flags, log2_block, frac_bits, stream, fit)
    fl = int(flags.item())
    if fl & LC_FLAG_UNSORTED:
        raise LcError(LC_EINVAL, "lc_compress: keys are not sorted (LC_FLAG_UNSORTED)")
    if fl & LC_FLAG_INTERNAL:
        raise LcError(LC_EDEVICE, "lc_compress: internal step limit hit (LC_FLAG_INTERNAL)")
    size = int(nbytes.item())
    del ws
    data = blob[:size].clone()
    return Blob(data, info(data[:HEADER_BYTES].cpu()))


def decompress(blob: Blob, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Dec of Def. 1: all n keys."""
    if out is None:
        out = torch.empty(blob.n, dtype=key_dtype(blob.key_bytes), device=blob.data.device)
    _check(lib.lc_decompress(ctypes.c_void_p(blob.data.data_ptr()), ctypes.byref(blob.info),
                             ctypes.c_void_p(out.data_ptr()), _stream(stream)), "lc_decompress")
    return out


def decompress_range(blob: Blob, begin: int, end: int, out: torch.Tensor | None = None,
                     stream=None) -> torch.Tensor:
    """Keys [begin, end)."""
    if out is None:
        out = torch.empty(max(0, end - begin), dtype=key_dtype(blob.key_bytes), device=blob.data.device)
    _check(lib.lc_decompress_range(ctypes.c_void_p(blob.data.data_ptr()), ctypes.byref(blob.info),
                                   begin, end, ctypes.c_void_p(out.data_ptr()), _stream(stream)),
           "lc_decompress_range")
    return out


def access(blob: Blob, idx: torch.Tensor, out: torch.Tensor | None = None,
           flags: torch.Tensor | None = None, stream=None, check: bool = True) -> torch.Tensor:
    """K[idx[q]] for every q.  With check=True, synchronises and raises on an index >= n."""
    _dev(idx, "idx")
    if idx.dtype not in (torch.int64, torch.uint64):
        raise TypeError("idx must be a 64-bit integer tensor")
    if out is None:
        out = torch.empty(idx.numel(), dtype=key_dtype(blob.key_bytes), device=idx.device)
    own_flags = flags is None
    if own_flags:
        flags = torch.zeros(1, dtype=torch.int32, device=idx.device)
    _check(lib.lc_access(ctypes.c_void_p(blob.data.data_ptr()), ctypes.byref(blob.info),
                         ctypes.c_void_p(idx.data_ptr()), idx.numel(), ctypes.c_void_p(out.data_ptr()),
                         ctypes.c_void_p(flags.data_ptr()), _stream(stream)), "lc_access")
    if check and own_flags and int(flags.item()) & LC_FLAG_RANGE:
        raise LcError(LC_EINVAL, "lc_access: an index is >= n (LC_FLAG_RANGE)")
    return out


def lower_bound(blob: Blob, q: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """First i with K[i] >= q (n if none), as int64."""
    _dev(q, "q")
    if _key_bytes(q) != blob.key_bytes:
        raise TypeError("queries must have the blob's key width")
    if out is None:
        out = torch.empty(q.numel(), dtype=torch.int64, device=q.device)
    _check(lib.lc_lower_bound(ctypes.c_void_p(blob.data.data_ptr()), ctypes.byref(blob.info),
                              ctypes.c_void_p(q.data_ptr()), q.numel(), ctypes.c_void_p(out.data_ptr()),
                              _stream(stream)), "lc_lower_bound")
    return out


# ---------------------------------------------------------------------------
# Queries on the compressed form: quantile, approximate decode, list AND / OR
# ---------------------------------------------------------------------------

def quantile(blob: Blob, k: torch.Tensor, q: int, approx: bool = False, out: torch.Tensor | None = None,
             stream=None) -> torch.Tensor:
    """k-th q-quantiles K[min(floor(n k / q), n - 1)] for every k (int64
    tensor); approx: the model's prediction of that key (within eps)."""
    _dev(k, "k")
    if k.dtype not in (torch.int64, torch.uint64):
        raise TypeError("k must be a 64-bit integer tensor")
    if out is None:
        out = torch.empty(k.numel(), dtype=key_dtype(blob.key_bytes), device=k.device)
    _check(lib.lc_quantile(_ptr(blob.data), ctypes.byref(blob.info), _ptr(k), q, k.numel(), int(approx), _ptr(out),
                           _stream(stream)), "lc_quantile")
    return out


def decompress_approx(blob: Blob, begin: int = 0, end: int | None = None, out: torch.Tensor | None = None,
                      stream=None) -> torch.Tensor:
    """Keys [begin, end) from the model alone (no residuals): each within eps."""
    end = blob.n if end is None else end
    if out is None:
        out = torch.empty(max(0, end - begin), dtype=key_dtype(blob.key_bytes), device=blob.data.device)
    _check(lib.lc_decompress_approx(_ptr(blob.data), ctypes.byref(blob.info), begin, end, _ptr(out),
                                    _stream(stream)), "lc_decompress_approx")
    return out


def setop_bound(a: Blob, b: Blob, op: int):
    """(out_max keys, workspace bytes) of lc_setop."""
    out_max, ws = ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib.lc_setop_bound(ctypes.byref(a.info), ctypes.byref(b.info), op, ctypes.byref(out_max),
                              ctypes.byref(ws)), "lc_setop_bound")
    return out_max.value, ws.value


def setop_async(op: int, a: Blob, b: Blob, ws: torch.Tensor, out: torch.Tensor, count: torch.Tensor, stream=None):
    """Enqueue lc_setop into caller-provided buffers (count: device int64[1])."""
    _check(lib.lc_setop(op, _ptr(a.data), ctypes.byref(a.info), _ptr(b.data), ctypes.byref(b.info), _ptr(ws),
                        ws.numel(), _ptr(out), out.numel(), _ptr(count), _stream(stream)), "lc_setop")


def _setop(op: int, a: Blob, b: Blob, stream=None) -> torch.Tensor:
    if a.key_bytes != b.key_bytes:
        raise TypeError("both lists must have the same key width")
    out_max, ws_bytes = setop_bound(a, b, op)
    dev = a.data.device
    ws = torch.empty(max(ws_bytes, 16), dtype=torch.uint8, device=dev)
    out = torch.empty(max(out_max, 1), dtype=key_dtype(a.key_bytes), device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    setop_async(op, a, b, ws, out, count, stream)
    return out[:int(count.item())]


def intersect(a: Blob, b: Blob, stream=None) -> torch.Tensor:
    """AND of two compressed lists (sorted, each key once)."""
    return _setop(SETOP_INTERSECT, a, b, stream)


def union(a: Blob, b: Blob, stream=None) -> torch.Tensor:
    """OR of two compressed lists (sorted, each key once)."""
    return _setop(SETOP_UNION, a, b, stream)


# ---------------------------------------------------------------------------
# Batches of lists
# ---------------------------------------------------------------------------

def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


TILINGS = {"auto": 0, "rows": 1, "lanes": 2}  # LC_TILING_*


def _tiling(tiling) -> int:
    if tiling in TILINGS:
        return TILINGS[tiling]
    if tiling in TILINGS.values():
        return int(tiling)
    raise ValueError(f"tiling must be one of {sorted(TILINGS)}, not {tiling!r}")


def batch_plan(lengths, eps, key_bytes: int, max_eps: int | None = None, log2_block: int = DEFAULT_LOG2_BLOCK,
               frac_bits: int = DEFAULT_FRAC_BITS, key_offsets=None, tiling="auto", fit="greedy"):
    """lc_batch_plan: (lc_batch_params, host table) for lists of the given
    lengths, stored one after another in the key array unless key_offsets is
    given.  eps: one value or one per list; max_eps sizes the blob slots;
    tiling: the greedy fit's wave tiling ("auto", "rows" or "lanes"; same
    blobs); fit: "greedy", "min" or "opt" for every list (as compress)."""
    lengths = np.asarray(lengths, dtype=np.uint64).ravel()
    nl = lengths.size
    table = np.zeros(nl, dtype=BATCH_LIST_DTYPE)
    table["n"] = lengths
    if key_offsets is None:
        key_offsets = np.concatenate([[0], np.cumsum(lengths, dtype=np.uint64)[:-1]]) if nl else lengths
    table["key_off"] = np.asarray(key_offsets, dtype=np.uint64)
    table["eps"] = np.broadcast_to(np.asarray(eps, dtype=np.uint32), (nl,))
    if max_eps is None:
        max_eps = int(table["eps"].max()) if nl else 0
    p = lc_batch_params(key_bytes, log2_block, frac_bits, _tiling(tiling), nl, max_eps, _fit(fit), 0, 0, 0, 0)
    _check(lib.lc_batch_plan(ctypes.byref(p), table.ctypes.data_as(ctypes.c_void_p)), "lc_batch_plan")
    return p, table


def batch_sizes_async(keys, lists, p, cands, ws, sizes, stats, stream=None):
    """Enqueue lc_batch_sizes: sizes[c * nlists + l] for every candidate eps."""
    cand = (ctypes.c_uint32 * len(cands))(*cands)
    _check(lib.lc_batch_sizes(_ptr(keys), keys.numel(), _ptr(lists), ctypes.byref(p), cand, len(cands),
                              _ptr(ws), ws.numel(), _ptr(sizes), _ptr(stats), _stream(stream)), "lc_batch_sizes")


def batch_pick_eps_async(lists, p, sizes, cands, stream=None):
    """Enqueue lc_batch_pick_eps: every list's eps := its argmin-size candidate."""
    cand = (ctypes.c_uint32 * len(cands))(*cands)
    _check(lib.lc_batch_pick_eps(_ptr(lists), ctypes.byref(p), _ptr(sizes), cand, len(cands), _stream(stream)),
           "lc_batch_pick_eps")


def batch_compress_async(keys, lists, p, blob, ws, sizes, stats, stream=None):
    """Enqueue lc_batch_compress into caller-provided buffers."""
    _check(lib.lc_batch_compress(_ptr(keys), keys.numel(), _ptr(lists), ctypes.byref(p), _ptr(blob), blob.numel(),
                                 _ptr(ws), ws.numel(), _ptr(sizes), _ptr(stats), _stream(stream)),
           "lc_batch_compress")


def batch_decompress_async(blob, lists, p, max_seg_bytes: int, out, stats, stream=None):
    """Enqueue lc_batch_decompress into out (all lists, at their key offsets)."""
    _check(lib.lc_batch_decompress(_ptr(blob), blob.numel(), _ptr(lists), ctypes.byref(p), max_seg_bytes,
                                   _ptr(out), out.numel(), _ptr(stats), _stream(stream)), "lc_batch_decompress")


@dataclass
class Batch:
    """A batch of compressed lists: one blob v1 per list, in slots of one buffer."""
    params: lc_batch_params
    table: np.ndarray       # host copy of the list table (eps as compressed)
    lists: torch.Tensor     # device copy (uint8, 64 bytes per list)
    data: torch.Tensor      # the batch buffer (uint8)
    sizes: np.ndarray       # blob bytes per list
    max_seg_bytes: int
    nkeys: int              # keys in the concatenated array

    @property
    def key_bytes(self) -> int:
        return self.params.key_bytes

    @property
    def nbytes(self) -> int:
        """Bytes of all list blobs (the slots' unused tails not counted)."""
        return int(self.sizes.sum())

    @property
    def eps(self) -> np.ndarray:
        return self.table["eps"].copy()

    def blob(self, l: int) -> Blob:
        off, size = int(self.table["blob_off"][l]), int(self.sizes[l])
        data = self.data[off:off + size]
        return Blob(data, info(data[:HEADER_BYTES].cpu()))


def _raise_flags(fl: int, what: str):
    if fl & LC_FLAG_UNSORTED:
        raise LcError(LC_EINVAL, f"{what}: a list is not sorted (LC_FLAG_UNSORTED)")
    if fl & LC_FLAG_BADLIST:
        raise LcError(LC_EINVAL, f"{what}: a list does not fit the buffers (LC_FLAG_BADLIST)")
    if fl & LC_FLAG_INTERNAL:
        raise LcError(LC_EDEVICE, f"{what}: internal step limit hit (LC_FLAG_INTERNAL)")


def batch_compress(keys: torch.Tensor, lengths, eps=None, candidates=None, log2_block: int = DEFAULT_LOG2_BLOCK,
                   frac_bits: int = DEFAULT_FRAC_BITS, stream=None, check: bool = True, tiling="auto",
                   fit="greedy") -> Batch:
    """Compress the lists stored one after another in keys.  Either eps (one
    value or one per list) or candidates (the autotuner picks each list's eps
    among them by exact blob size, ties to the smaller).  tiling: the greedy
    fit's wave tiling (same blobs either way); fit: "greedy", "min" or "opt"
    for every list of the batch."""
    _dev(keys, "keys")
    kb = _key_bytes(keys)
    if (eps is None) == (candidates is None):
        raise ValueError("give exactly one of eps and candidates")
    cands = sorted(set(int(c) for c in candidates)) if candidates is not None else None
    p, table = batch_plan(lengths, cands[0] if cands else eps, kb, max(cands) if cands else None, log2_block,
                          frac_bits, tiling=tiling, fit=fit)
    dev = keys.device
    nl = p.nlists
    lists = torch.from_numpy(table.view(np.uint8).copy()).to(dev)
    ws = torch.empty(max(p.ws_bytes, 16), dtype=torch.uint8, device=dev)
    stats = torch.zeros(2, dtype=torch.int32, device=dev)
    if cands:
        csizes = torch.empty(len(cands) * nl, dtype=torch.int64, device=dev)
        batch_sizes_async(keys, lists, p, cands, ws, csizes, stats, stream)
        batch_pick_eps_async(lists, p, csizes, cands, stream)
    blob = torch.empty(max(p.blob_bytes, 16), dtype=torch.uint8, device=dev)
    sizes = torch.empty(nl, dtype=torch.int64, device=dev)
    batch_compress_async(keys, lists, p, blob, ws, sizes, stats, stream)
    st = stats.cpu().numpy()
    if check:
        _raise_flags(int(st[0]), "lc_batch_compress")
    del ws
    final = lists.cpu().numpy().view(BATCH_LIST_DTYPE).copy()
    return Batch(p, final, lists, blob, sizes.cpu().numpy().astype(np.uint64), int(st[1]) & 0xFFFFFFFF,
                 keys.numel())


def batch_decompress(batch: Batch, out: torch.Tensor | None = None, stream=None, check: bool = True) -> torch.Tensor:
    """All lists of the batch, at their key offsets (the layout compressed)."""
    if out is None:
        out = torch.empty(batch.nkeys, dtype=key_dtype(batch.key_bytes), device=batch.data.device)
    stats = torch.zeros(1, dtype=torch.int32, device=out.device)
    batch_decompress_async(batch.data, batch.lists, batch.params, batch.max_seg_bytes, out, stats, stream)
    if check:
        _raise_flags(int(stats.item()), "lc_batch_decompress")
    return out


def batch_and_plan(batch: Batch, pairs):
    """lc_batch_and_plan for pairs (sequence of (a, b) list indices): the
    planned pair table and (total_keys, total_blocks, ws_bytes)."""
    pr = np.asarray(pairs, dtype=np.uint32).reshape(-1, 2)
    t = np.zeros(len(pr), dtype=PAIR_DTYPE)
    t["a"], t["b"] = pr[:, 0], pr[:, 1]
    tk, tb, ws = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib.lc_batch_and_plan(ctypes.byref(batch.params), batch.table.ctypes.data_as(ctypes.c_void_p),
                                 t.ctypes.data_as(ctypes.c_void_p), len(t), ctypes.byref(tk), ctypes.byref(tb),
                                 ctypes.byref(ws)), "lc_batch_and_plan")
    return t, (tk.value, tb.value, ws.value)


def batch_and_async(batch: Batch, d_pairs, npairs: int, totals, ws, out, counts, stats, stream=None):
    """Enqueue lc_batch_and with a planned device pair table."""
    tk, tb, _ = totals
    _check(lib.lc_batch_and(_ptr(batch.data), batch.data.numel(), _ptr(batch.lists), ctypes.byref(batch.params),
                            _ptr(d_pairs), npairs, tk, tb, batch.max_seg_bytes, _ptr(ws), ws.numel(), _ptr(out),
                            _ptr(counts), _ptr(stats), _stream(stream)), "lc_batch_and")


def batch_intersect(batch: Batch, pairs, stream=None):
    """AND of every pair (a, b) of lists of the batch, in one pass: returns a
    list of device tensors, the sorted keys in both lists of each pair."""
    table, totals = batch_and_plan(batch, pairs)
    dev = batch.data.device
    d_pairs = torch.from_numpy(table.view(np.uint8).copy()).to(dev)
    ws = torch.empty(max(totals[2], 16), dtype=torch.uint8, device=dev)
    out = torch.empty(max(totals[0], 1), dtype=key_dtype(batch.key_bytes), device=dev)
    counts = torch.zeros(len(table), dtype=torch.int64, device=dev)
    stats = torch.zeros(1, dtype=torch.int32, device=dev)
    batch_and_async(batch, d_pairs, len(table), totals, ws, out, counts, stats, stream)
    _raise_flags(int(stats.item()), "lc_batch_and")
    c = counts.cpu().numpy()
    return [out[int(o):int(o) + int(k)] for o, k in zip(table["key_off"], c)]


# ---------------------------------------------------------------------------
# Request server
# ---------------------------------------------------------------------------

class Server:
    """Continuous-batching request loop over one device-resident blob (the
    loop itself runs in liblc.so).  The arena is the HBM budget for results."""

    def __init__(self, blob: Blob, arena_bytes: int = 2 << 30, max_batch: int = 1024, max_inflight: int = 4):
        self.blob = blob
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=blob.data.device)
        cfg = lc_serve_config(max_batch, max_inflight)
        h = ctypes.c_void_p()
        torch.cuda.synchronize(blob.data.device)  # blob and arena complete before other streams read them
        _check(lib.lc_server_create(_ptr(blob.data), ctypes.byref(blob.info), _ptr(self.arena), arena_bytes,
                                    ctypes.byref(cfg), ctypes.byref(h)), "lc_server_create")
        self._h = h

    def run(self, requests: np.ndarray):
        """Serve a structured array of REQUEST_DTYPE; returns (results of
        RESULT_DTYPE, stats dict).  Blocks until every request completed."""
        req = np.ascontiguousarray(requests, dtype=REQUEST_DTYPE)
        res = np.zeros(len(req), dtype=RESULT_DTYPE)
        st = lc_serve_stats()
        torch.cuda.synchronize(self.blob.data.device)  # d_dest buffers ready
        rc = lib.lc_server_run(self._h, req.ctypes.data_as(ctypes.c_void_p), len(req),
                               res.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st))
        _check(rc, "lc_server_run")
        return res, {f: getattr(st, f) for f, _ in lc_serve_stats._fields_}

    def close(self):
        if self._h:
            lib.lc_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def requests(ops, a, b=None, arrival_ns=None, d_dest=None) -> np.ndarray:
    """Build a REQUEST_DTYPE array."""
    ops = np.asarray(ops, dtype=np.uint32)
    r = np.zeros(len(ops), dtype=REQUEST_DTYPE)
    r["op"] = ops
    r["a"] = np.asarray(a, dtype=np.uint64)
    if b is not None:
        r["b"] = np.asarray(b, dtype=np.uint64)
    if arrival_ns is not None:
        r["arrival_ns"] = np.asarray(arrival_ns, dtype=np.uint64)
    if d_dest is not None:
        r["d_dest"] = np.asarray(d_dest, dtype=np.uint64)
    return r


# ---------------------------------------------------------------------------
# Batch autotuner
# ---------------------------------------------------------------------------

def time_batch_fit(keys: torch.Tensor, lengths, eps_candidates=(7, 31, 127), log2_block: int = DEFAULT_LOG2_BLOCK,
                   tilings=("rows", "lanes"), reps: int = 3, frac_bits: int = DEFAULT_FRAC_BITS):
    """Mean time (ms, HIP events, after one warm-up) of the batch's whole
    compress -- size pass over eps_candidates, on-device pick, compress --
    for each wave tiling of the fit.  The blobs are identical; only the time
    differs.  Returns {tiling: ms}."""
    kb = _key_bytes(keys)
    cands = sorted(set(int(c) for c in eps_candidates))
    out = {}
    for tl in tilings:
        p, table = batch_plan(lengths, cands[0], kb, max(cands), log2_block, frac_bits, tiling=tl)
        dev = keys.device
        lists = torch.from_numpy(table.view(np.uint8).copy()).to(dev)
        ws = torch.empty(max(p.ws_bytes, 16), dtype=torch.uint8, device=dev)
        blob = torch.empty(max(p.blob_bytes, 16), dtype=torch.uint8, device=dev)
        csizes = torch.empty(len(cands) * p.nlists, dtype=torch.int64, device=dev)
        sizes = torch.empty(p.nlists, dtype=torch.int64, device=dev)
        stats = torch.zeros(2, dtype=torch.int32, device=dev)

        def run():
            batch_sizes_async(keys, lists, p, cands, ws, csizes, stats)
            batch_pick_eps_async(lists, p, csizes, cands)
            batch_compress_async(keys, lists, p, blob, ws, sizes, stats)

        run()
        torch.cuda.synchronize()
        _raise_flags(int(stats[0].item()), "lc_batch_compress")
        marks = []
        for _ in range(max(1, reps)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            run()
            e1.record()
            marks.append((e0, e1))
        torch.cuda.synchronize()
        out[tl] = float(sum(a.elapsed_time(b) for a, b in marks) / len(marks))
        del ws, blob
    return out


def _pick(report, objective):
    fastest = min(r["decode_ms"] for r in report)
    if objective == "speed":
        return min(report, key=lambda r: (r["decode_ms"], r["bytes"]))
    if objective == "balanced":
        return min((r for r in report if r["decode_ms"] <= 1.1 * fastest), key=lambda r: (r["bytes"], r["decode_ms"]))
    return min(report, key=lambda r: (r["bytes"], r["decode_ms"]))


def autotune_batch(keys: torch.Tensor, lengths, eps_candidates=(7, 31, 127), block_candidates=(8, 9, 10, 11, 12),
                   objective: str = "size", time_reps: int = 3, frac_bits: int = DEFAULT_FRAC_BITS, stream=None,
                   tilings=("rows", "lanes"), fit_candidates=None):
    """Pick the batch's block size (and, per list, eps among eps_candidates)
    by measurement.  For every log2 block size the whole batch is compressed
    with the on-device eps autotune (greedy fit, frac_bits); its exact total
    bytes and its batch decode time (HIP events, mean of time_reps runs) are
    recorded.  objective "size": fewest bytes (ties: faster decode); "speed":
    fastest decode; "balanced": fewest bytes among the candidates whose
    decode is within 10% of the fastest.  Then, at the chosen block size,
    every (fit, F) of fit_candidates (e.g. (("greedy", 0), ("opt", 0)),
    greedy at frac_bits always included) is measured the same way and the
    objective picks among them too; last, the greedy fit's wave tiling is
    picked by timing the whole compress under each of tilings (same bytes,
    so only speed decides).  Returns (chosen Batch, report list): one entry
    per block size (greedy, frac_bits) and one per further (fit, F) at the
    chosen block size; the chosen entry has "chosen" set and, for the greedy
    fit, the tiling times and the tiling picked."""
    if objective not in ("size", "speed", "balanced"):
        raise ValueError("objective is 'size', 'speed' or 'balanced'")
    report, batches = [], {}
    out = torch.empty(keys.numel(), dtype=key_dtype(_key_bytes(keys)), device=keys.device)

    def measure(lb, fit, F):
        b = batch_compress(keys, lengths, candidates=eps_candidates, log2_block=lb, frac_bits=F, stream=stream,
                           fit=fit)
        batch_decompress(b, out=out, stream=stream)  # warm, and checks the flags
        t = []
        for _ in range(max(1, time_reps)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            batch_decompress(b, out=out, stream=stream, check=False)
            e1.record()
            torch.cuda.synchronize()
            t.append(e0.elapsed_time(e1))
        r = {"log2_block": lb, "fit": fit, "frac_bits": F, "bytes": b.nbytes, "decode_ms": float(sum(t) / len(t))}
        report.append(r)
        batches[id(r)] = b
        return r

    for lb in block_candidates:
        measure(lb, "greedy", frac_bits)
    best = _pick(report, objective)
    for fit, F in (fit_candidates or ()):
        if (fit, F) != ("greedy", frac_bits):
            measure(best["log2_block"], fit, F)
    best = _pick([r for r in report if r["log2_block"] == best["log2_block"]], objective)
    for r in report:
        r["chosen"] = r is best
    if tilings and best["fit"] == "greedy":
        t = time_batch_fit(keys, lengths, eps_candidates, best["log2_block"], tilings, time_reps, best["frac_bits"])
        best["compress_ms_by_tiling"] = t
        best["tiling"] = min(t, key=t.get)
    chosen = batches[id(best)]
    batches.clear()
    return chosen, report
