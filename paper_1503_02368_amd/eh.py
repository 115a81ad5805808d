"""ctypes binding of the C ABI declared in include/eh.h.

Argument marshalling only: every counting step runs in the HIP library.
PyTorch supplies device memory (its caching allocator, through the ABI's
allocator hooks) and the stream work is launched on.  Importing this module
does not touch the GPU; :func:`load` raises if the library was not built.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; EH_LIBRARY names another build of the same ABI (for
# comparing builds side by side)
LIB_PATH = os.environ.get("EH_LIBRARY") or os.path.join(_HERE, "_lib", "libeh.so")

# status codes and enums (eh.h)
EH_OK, EH_PENDING = 0, 1
EH_EINVAL, EH_ENOMEM, EH_EHIP, EH_EBUSY, EH_ENOTFOUND, EH_EOVERFLOW, EH_ESTATE = -1, -2, -3, -4, -5, -6, -7
TRIANGLE, CLIQUE4 = 3, 4
LAYOUT_UINT, LAYOUT_HYBRID, LAYOUT_BITSET_ALL = 0, 1, 2
ORDER_DEGREE, ORDER_REV_DEGREE, ORDER_INPUT, ORDER_BFS, ORDER_HYBRID, ORDER_STRONG_RUNS = 0, 1, 2, 3, 4, 5
ORDERS = {"degree": ORDER_DEGREE, "rev_degree": ORDER_REV_DEGREE, "input": ORDER_INPUT,
          "bfs": ORDER_BFS, "hybrid": ORDER_HYBRID, "strong_runs": ORDER_STRONG_RUNS}
KERNEL_AUTO, KERNEL_STAGED, KERNEL_PAIRWISE = 0, 1, 2
STAGE_AUTO, STAGE_SOURCE, STAGE_TARGET = 0, 1, 2
ALGO_AUTO, ALGO_MERGE, ALGO_SEARCH = 0, 1, 2
SETS_UINT, SETS_SET, SETS_BITSET, SETS_COMPOSITE = 0, 1, 2, 3
SET_LAYOUTS = {"uint": SETS_UINT, "set": SETS_SET, "bitset": SETS_BITSET, "composite": SETS_COMPOSITE}

# every symbol include/eh.h declares
SYMBOLS = [
    "eh_ctx_create", "eh_ctx_destroy", "eh_last_error", "eh_status_str", "eh_abi_version",
    "eh_ctx_set_tuning", "eh_ctx_get_tuning", "eh_build_trie", "eh_build_batch",
    "eh_trie_info_get", "eh_trie_free", "eh_count_triangles", "eh_count_4cliques",
    "eh_count_async", "eh_count_add_async", "eh_count_rooted", "eh_count_batch", "eh_count_batch_async",
    "eh_server_create", "eh_submit", "eh_poll", "eh_wait", "eh_server_drain", "eh_server_destroy",
    "eh_host_trie_build", "eh_host_trie_info", "eh_host_trie_arrays", "eh_host_trie_free",
    "eh_build_trie_device", "eh_trie_host_arrays", "eh_trie_device_arrays", "eh_count_lollipop",
    "eh_build_batch_device", "eh_sets_build", "eh_sets_info_get", "eh_sets_free",
    "eh_intersect_pairs", "eh_intersect_pairs_async", "eh_host_sets_build", "eh_host_sets_info",
    "eh_host_sets_arrays", "eh_host_sets_free", "eh_stream_read", "eh_count_add_noalloc",
]


class EHError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)),
                ("free", ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)),
                ("self", ctypes.c_void_p)]


# struct layouts below are those of this ABI version of include/eh.h
ABI_VERSION = 11000


class _Tuning(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_uint32), ("staging", ctypes.c_uint32), ("algo", ctypes.c_uint32),
                ("gamma", ctypes.c_float), ("chunk_work", ctypes.c_uint32),
                ("waves_per_cu", ctypes.c_uint32), ("group_lanes", ctypes.c_uint32),
                ("use_bitsets", ctypes.c_uint32), ("dynamic", ctypes.c_uint32),
                ("stage_words", ctypes.c_uint32), ("xcds", ctypes.c_uint32),
                ("unroll", ctypes.c_uint32), ("grab", ctypes.c_uint32),
                ("search_below", ctypes.c_uint32), ("group", ctypes.c_uint32),
                ("reverse", ctypes.c_uint32), ("k4_local", ctypes.c_uint32)]


class _BuildOpts(ctypes.Structure):
    _fields_ = [("layout", ctypes.c_uint32), ("tau", ctypes.c_float), ("s_min", ctypes.c_uint32),
                ("order", ctypes.c_uint32), ("symmetric", ctypes.c_uint32)]


class _TrieInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("n_graphs", ctypes.c_uint32), ("m_plus", ctypes.c_uint64),
                ("n_bitset_sets", ctypes.c_uint64), ("bitset_words", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("b_merge", ctypes.c_uint64),
                ("max_out_degree", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("b_target", ctypes.c_uint64)]


class _SetOpts(ctypes.Structure):
    _fields_ = [("layout", ctypes.c_uint32), ("block_log", ctypes.c_uint32),
                ("block_min", ctypes.c_uint32), ("tau", ctypes.c_float), ("s_min", ctypes.c_uint32)]


class _SetsInfo(ctypes.Structure):
    _fields_ = [("n_sets", ctypes.c_uint32), ("block_log", ctypes.c_uint32),
                ("n_members", ctypes.c_uint64), ("n_segments", ctypes.c_uint64),
                ("n_bitset_segments", ctypes.c_uint64), ("uint_members", ctypes.c_uint64),
                ("bitset_blocks", ctypes.c_uint64), ("bitset_words", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64)]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_active", ctypes.c_uint32),
                ("max_queued", ctypes.c_uint32), ("step_items", ctypes.c_uint32),
                ("policy", ctypes.c_uint32)]


class _ReqStats(ctypes.Structure):
    _fields_ = [("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64), ("items", ctypes.c_uint64)]


_lib = None
_lock = threading.Lock()
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_vp = ctypes.c_void_p


def load():
    """Loads the built library; raises FileNotFoundError if it is missing."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1503_02368_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        S = ctypes.c_int32
        sig = {
            "eh_ctx_create": [ctypes.c_int, _vp, ctypes.POINTER(_Allocator), ctypes.POINTER(_vp)],
            "eh_ctx_destroy": [_vp],
            "eh_ctx_set_tuning": [_vp, ctypes.POINTER(_Tuning)],
            "eh_ctx_get_tuning": [_vp, ctypes.POINTER(_Tuning)],
            "eh_build_trie": [_vp, _u32p, _u32p, ctypes.c_uint64, ctypes.c_uint32,
                              ctypes.POINTER(_BuildOpts), ctypes.POINTER(_vp)],
            "eh_build_batch": [_vp, ctypes.c_uint32, _u32p, _u64p, _u32p, _u32p,
                               ctypes.POINTER(_BuildOpts), ctypes.POINTER(_vp)],
            "eh_trie_info_get": [_vp, ctypes.POINTER(_TrieInfo)],
            "eh_trie_free": [_vp],
            "eh_count_triangles": [_vp, _vp, _u64p, _vp],
            "eh_count_4cliques": [_vp, _vp, _u64p],
            "eh_count_async": [_vp, _vp, ctypes.c_int, _vp],
            "eh_count_add_async": [_vp, _vp, ctypes.c_int, _vp],
            "eh_count_rooted": [_vp, _vp, ctypes.c_int, _u32p, ctypes.c_uint32, _u64p],
            "eh_count_batch": [_vp, _vp, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, _u64p],
            "eh_count_batch_async": [_vp, _vp, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, _vp],
            "eh_server_create": [_vp, _vp, ctypes.POINTER(_ServerOpts), ctypes.POINTER(_vp)],
            "eh_submit": [_vp, ctypes.c_int, _u32p, ctypes.c_uint32, _u64p],
            "eh_poll": [_vp, ctypes.c_uint64, _u64p, ctypes.POINTER(_ReqStats)],
            "eh_wait": [_vp, ctypes.c_uint64, ctypes.c_uint32, _u64p, ctypes.POINTER(_ReqStats)],
            "eh_server_drain": [_vp, ctypes.c_uint32, ctypes.c_uint32, _u64p, _u64p,
                                ctypes.POINTER(_ReqStats), ctypes.POINTER(ctypes.c_uint32)],
            "eh_server_destroy": [_vp],
            "eh_host_trie_build": [_u32p, _u32p, ctypes.c_uint64, ctypes.c_uint32,
                                   ctypes.POINTER(_BuildOpts), ctypes.POINTER(_vp)],
            "eh_host_trie_info": [_vp, ctypes.POINTER(_TrieInfo)],
            "eh_host_trie_arrays": [_vp, _u32p, _u32p, _u32p, _u32p, _u32p, _u32p, _u32p],
            "eh_host_trie_free": [_vp],
            "eh_build_trie_device": [_vp, _vp, _vp, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.POINTER(_BuildOpts), ctypes.POINTER(_vp)],
            "eh_trie_host_arrays": [_vp, _u32p, _u32p, _u32p, _u32p, _u32p, _u32p, _u32p],
            "eh_trie_device_arrays": [_vp, _vp, _u32p, _u32p, _u32p, _u32p],
            "eh_count_lollipop": [_vp, _vp, _u64p],
            "eh_build_batch_device": [_vp, ctypes.c_uint32, _u32p, _u64p, _vp, _vp,
                                      ctypes.POINTER(_BuildOpts), ctypes.POINTER(_vp)],
            "eh_sets_build": [_vp, ctypes.c_uint32, _u64p, _u32p, ctypes.POINTER(_SetOpts),
                              ctypes.POINTER(_vp)],
            "eh_sets_info_get": [_vp, ctypes.POINTER(_SetsInfo)],
            "eh_sets_free": [_vp],
            "eh_intersect_pairs": [_vp, _vp, ctypes.c_uint64, _vp, _vp, ctypes.c_uint32, _u64p],
            "eh_intersect_pairs_async": [_vp, _vp, ctypes.c_uint64, _vp, _vp, ctypes.c_uint32, _vp],
            "eh_stream_read": [_vp, _vp, ctypes.c_uint64, ctypes.c_uint32, _vp],
            "eh_count_add_noalloc": [_vp, _vp, ctypes.c_int, _vp],
            "eh_host_sets_build": [ctypes.c_uint32, _u64p, _u32p, ctypes.POINTER(_SetOpts),
                                   ctypes.POINTER(_vp)],
            "eh_host_sets_info": [_vp, ctypes.POINTER(_SetsInfo)],
            "eh_host_sets_arrays": [_vp, _u32p, _u32p, _u32p, _u32p],
            "eh_host_sets_free": [_vp],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = S
        lib.eh_last_error.argtypes = [_vp]
        lib.eh_last_error.restype = ctypes.c_char_p
        lib.eh_status_str.argtypes = [S]
        lib.eh_status_str.restype = ctypes.c_char_p
        lib.eh_abi_version.argtypes = []
        lib.eh_abi_version.restype = S
        if lib.eh_abi_version() != ABI_VERSION:
            raise RuntimeError(f"libeh ABI {lib.eh_abi_version()} != binding ABI {ABI_VERSION}: rebuild")
        _lib = lib
        return lib


def _p32(a):
    return a.ctypes.data_as(_u32p)


def _p64(a):
    return a.ctypes.data_as(_u64p)


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def _opts(layout, tau, s_min, order, symmetric=0):
    return _BuildOpts(int(layout), float(tau), int(s_min), int(order), int(bool(symmetric)))


def _info_dict(info: _TrieInfo) -> dict:
    return {k: int(getattr(info, k)) for k, _ in _TrieInfo._fields_ if k != "reserved"}


def host_trie(n, src, dst, layout=LAYOUT_HYBRID, tau=32.0, s_min=1, order=ORDER_DEGREE,
              symmetric=False) -> dict:
    """Runs only the host half of the trie build (no GPU) and returns its arrays."""
    lib = load()
    src, dst = _u32(src), _u32(dst)
    h = _vp()
    o = _opts(layout, tau, s_min, order, symmetric)
    st = lib.eh_host_trie_build(_p32(src), _p32(dst), src.size, int(n), ctypes.byref(o), ctypes.byref(h))
    if st != EH_OK:
        raise EHError(st, lib.eh_last_error(None).decode() or lib.eh_status_str(st).decode())
    try:
        info = _TrieInfo()
        lib.eh_host_trie_info(h, ctypes.byref(info))
        d = _info_dict(info)
        nn, m, w = d["n"], d["m_plus"], d["bitset_words"]
        arr = {k: np.zeros(sz, np.uint32) for k, sz in
               (("rank", nn), ("row", nn + 1), ("col", m), ("bs_off", nn), ("bs_base", nn),
                ("bs_nw", nn), ("bs_words", w))}
        lib.eh_host_trie_arrays(h, *(_p32(arr[k]) for k in
                                     ("rank", "row", "col", "bs_off", "bs_base", "bs_nw", "bs_words")))
        d.update(arr)
        return d
    finally:
        lib.eh_host_trie_free(h)


def _set_opts(layout, block_log, block_min, tau, s_min):
    return _SetOpts(int(layout), int(block_log), int(block_min), float(tau), int(s_min))


def _sets_input(off, members):
    off = np.ascontiguousarray(off, dtype=np.uint64)
    members = np.ascontiguousarray(members, dtype=np.uint32)
    if off.ndim != 1 or off.size < 1:
        raise ValueError("off needs n_sets + 1 entries")
    if int(off[-1]) != members.size:
        raise ValueError("off[-1] must equal the number of members")
    return off, members


def host_sets(off, members, layout=SETS_COMPOSITE, block_log=8, block_min=0, tau=32.0,
              s_min=1) -> dict:
    """Runs only the host encoding of a set store (no GPU) and returns its arrays:
    seg_off[n_sets+1], seg[n_segments, 4] = {first block, last block, start, members |
    2^31 for a bitset run}, vals, words, plus the sizes of eh_sets_info."""
    lib = load()
    off, members = _sets_input(off, members)
    h = _vp()
    o = _set_opts(layout, block_log, block_min, tau, s_min)
    st = lib.eh_host_sets_build(off.size - 1, _p64(off), _p32(members), ctypes.byref(o),
                                ctypes.byref(h))
    if st != EH_OK:
        raise EHError(st, lib.eh_last_error(None).decode() or lib.eh_status_str(st).decode())
    try:
        info = _SetsInfo()
        lib.eh_host_sets_info(h, ctypes.byref(info))
        d = {k: int(getattr(info, k)) for k, _ in _SetsInfo._fields_}
        arr = {"seg_off": np.zeros(d["n_sets"] + 1, np.uint32),
               "seg": np.zeros(4 * d["n_segments"], np.uint32),
               "vals": np.zeros(d["uint_members"], np.uint32),
               "words": np.zeros(d["bitset_words"], np.uint32)}
        lib.eh_host_sets_arrays(h, *(_p32(arr[k]) for k in ("seg_off", "seg", "vals", "words")))
        arr["seg"] = arr["seg"].reshape(-1, 4)
        d.update(arr)
        return d
    finally:
        lib.eh_host_sets_free(h)


class Context:
    """An eh_ctx on one device, launching on torch's current stream by default."""

    def __init__(self, device: int = 0, stream=None, torch_allocator: bool = True,
                 allocator=None):
        """allocator: an object with alloc(nbytes, stream) -> device pointer (int) or
        None, and free(ptr, stream), that the library calls for all its device memory
        (in place of torch's caching allocator)."""
        import torch
        self._lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the engine has no CPU path")
        self.device = device
        torch.cuda.set_device(device)
        if stream is None:
            # a stream of our own (default priority): handle 0 would be read as
            # "no stream given" by eh_ctx_create
            stream = torch.cuda.Stream(device)
        if not stream.cuda_stream:
            raise ValueError("pass a non-default stream: the ABI reads a null handle as 'none given'")
        self.stream = stream
        handle = _vp(stream.cuda_stream)
        self._alloc = None
        alloc_p = None
        if allocator is not None:
            @ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
            def _ua(_self, nbytes, s):
                try:
                    return allocator.alloc(int(nbytes), s or 0)
                except Exception:
                    return None

            @ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
            def _uf(_self, ptr, s):
                try:
                    allocator.free(ptr, s or 0)
                except Exception:
                    pass

            self._alloc = _Allocator(_ua, _uf, None)
            alloc_p = ctypes.byref(self._alloc)
        elif torch_allocator:
            dev = device

            @ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
            def _a(_self, nbytes, s):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, s or 0)
                except Exception:
                    return None

            @ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
            def _f(_self, ptr, _s):
                try:
                    torch.cuda.caching_allocator_delete(ptr)
                except Exception:
                    pass  # interpreter shutdown: torch is already gone, so is the memory

            self._alloc = _Allocator(_a, _f, None)
            alloc_p = ctypes.byref(self._alloc)
        h = _vp()
        st = self._lib.eh_ctx_create(int(device), handle, alloc_p, ctypes.byref(h))
        if st != EH_OK:
            raise EHError(st, "eh_ctx_create: " + self._lib.eh_last_error(None).decode())
        self._h = h
        self._tries = []
        self._sets = []

    def _check(self, st, what):
        if st != EH_OK:
            raise EHError(st, f"{what}: {self._lib.eh_last_error(self._h).decode()}")

    def close(self):
        if getattr(self, "_h", None):
            for t in list(self._tries):
                t.free()
            for t in list(self._sets):
                t.free()
            self._lib.eh_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tuning ----------------------------------------------------------
    def get_tuning(self) -> dict:
        t = _Tuning()
        self._check(self._lib.eh_ctx_get_tuning(self._h, ctypes.byref(t)), "get_tuning")
        return {k: (float(getattr(t, k)) if k == "gamma" else int(getattr(t, k))) for k, _ in _Tuning._fields_}

    def set_tuning(self, **kw) -> dict:
        cur = self.get_tuning()
        unknown = set(kw) - set(cur)
        if unknown:
            raise KeyError(f"unknown tuning keys {sorted(unknown)}")
        cur.update(kw)
        t = _Tuning(**{k: (float(v) if k == "gamma" else int(v)) for k, v in cur.items()})
        self._check(self._lib.eh_ctx_set_tuning(self._h, ctypes.byref(t)), "set_tuning")
        return self.get_tuning()

    # -- tries -------------------------------------------------------------
    def build_trie(self, n, src, dst, layout=LAYOUT_HYBRID, tau=32.0, s_min=1,
                   order=ORDER_DEGREE, symmetric=False) -> "Trie":
        src, dst = _u32(src), _u32(dst)
        if src.shape != dst.shape:
            raise ValueError("src and dst differ in length")
        h = _vp()
        o = _opts(layout, tau, s_min, order, symmetric)
        self._check(self._lib.eh_build_trie(self._h, _p32(src), _p32(dst), src.size, int(n),
                                            ctypes.byref(o), ctypes.byref(h)), "build_trie")
        return Trie(self, h)

    def build_trie_device(self, n, d_src, d_dst, layout=LAYOUT_HYBRID, tau=32.0, s_min=1,
                          order=ORDER_DEGREE, symmetric=False) -> "Trie":
        """The same trie, built on the GPU from device tensors of raw pairs (4-byte
        elements, e.g. torch.int32 holding ids below 2^31)."""
        if d_src.numel() != d_dst.numel():
            raise ValueError("src and dst differ in length")
        for t in (d_src, d_dst):
            if not t.is_cuda or t.element_size() != 4 or not t.is_contiguous():
                raise ValueError("pairs must be contiguous 4-byte device tensors")
        import torch
        # the pairs were written on torch's current stream; the build reads them on ours
        self.stream.wait_stream(torch.cuda.current_stream())
        h = _vp()
        o = _opts(layout, tau, s_min, order, symmetric)
        self._check(self._lib.eh_build_trie_device(self._h, _vp(d_src.data_ptr()),
                                                   _vp(d_dst.data_ptr()), d_src.numel(), int(n),
                                                   ctypes.byref(o), ctypes.byref(h)),
                    "build_trie_device")
        return Trie(self, h)

    def build_batch_device(self, batch, d_src, d_dst, layout=LAYOUT_HYBRID, tau=32.0, s_min=1,
                           order=ORDER_DEGREE, symmetric=False) -> "Trie":
        """The batch trie built on the GPU: sizes and offsets from `batch` (host),
        local-id pairs from device tensors of 4-byte elements."""
        import torch
        for t in (d_src, d_dst):
            if not t.is_cuda or t.element_size() != 4 or not t.is_contiguous():
                raise ValueError("pairs must be contiguous 4-byte device tensors")
        nv = _u32(batch.n_vertices)
        off = np.ascontiguousarray(batch.edge_off, dtype=np.uint64)
        if d_src.numel() < int(off[-1]) or d_dst.numel() < int(off[-1]):
            raise ValueError("fewer pairs than edge_off names")
        self.stream.wait_stream(torch.cuda.current_stream())
        h = _vp()
        o = _opts(layout, tau, s_min, order, symmetric)
        self._check(self._lib.eh_build_batch_device(self._h, nv.size, _p32(nv), _p64(off),
                                                    _vp(d_src.data_ptr()), _vp(d_dst.data_ptr()),
                                                    ctypes.byref(o), ctypes.byref(h)),
                    "build_batch_device")
        return Trie(self, h)

    def device_arrays(self, trie) -> dict:
        """The device arrays the counting kernels read, copied to host memory."""
        i = trie.info
        n, m, w = i["n"], i["m_plus"], i["bitset_words"]
        arr = {"vdesc": np.zeros(2 * n, np.uint32), "col": np.zeros(m + w, np.uint32),
               "bsdesc": np.zeros(4 * n if i["n_bitset_sets"] else 0, np.uint32),
               "vert": np.zeros(n, np.uint32)}
        self._check(self._lib.eh_trie_device_arrays(self._h, trie._h, *(_p32(arr[k]) for k in
                                                                       ("vdesc", "col", "bsdesc",
                                                                        "vert"))),
                    "trie_device_arrays")
        return arr

    def build_edgelist(self, el, **kw) -> "Trie":
        return self.build_trie(el.n, el.src, el.dst, **kw)

    def build_batch(self, batch, layout=LAYOUT_HYBRID, tau=32.0, s_min=1,
                    order=ORDER_DEGREE, symmetric=False) -> "Trie":
        nv = _u32(batch.n_vertices)
        off = np.ascontiguousarray(batch.edge_off, dtype=np.uint64)
        src, dst = _u32(batch.src), _u32(batch.dst)
        h = _vp()
        o = _opts(layout, tau, s_min, order, symmetric)
        self._check(self._lib.eh_build_batch(self._h, nv.size, _p32(nv), _p64(off), _p32(src), _p32(dst),
                                             ctypes.byref(o), ctypes.byref(h)), "build_batch")
        return Trie(self, h)

    # -- counting ----------------------------------------------------------
    def count_triangles(self, trie, per_root: bool = False):
        out = ctypes.c_uint64(0)
        roots = None
        if per_root:
            import torch
            roots = torch.empty(trie.info["n"], dtype=torch.int64, device=f"cuda:{self.device}")
        self._check(self._lib.eh_count_triangles(self._h, trie._h, ctypes.byref(out),
                                                 _vp(roots.data_ptr()) if roots is not None else None),
                    "count_triangles")
        if per_root:
            return int(out.value), roots.cpu().numpy().view(np.uint64)
        return int(out.value)

    def count_lollipop(self, trie) -> int:
        """COUNT(*) of Lollipop(x,y,z,w) :- R(x,y),S(y,z),T(x,z),U(x,w) on a symmetric trie."""
        out = ctypes.c_uint64(0)
        self._check(self._lib.eh_count_lollipop(self._h, trie._h, ctypes.byref(out)), "count_lollipop")
        return int(out.value)

    def count_4cliques(self, trie) -> int:
        out = ctypes.c_uint64(0)
        self._check(self._lib.eh_count_4cliques(self._h, trie._h, ctypes.byref(out)), "count_4cliques")
        return int(out.value)

    def count(self, trie, pattern: int) -> int:
        return self.count_triangles(trie) if pattern == TRIANGLE else self.count_4cliques(trie)

    def count_async(self, trie, pattern: int, d_total) -> None:
        """Enqueues a count whose result lands in d_total (a 1-element int64 CUDA tensor)."""
        self._check(self._lib.eh_count_async(self._h, trie._h, int(pattern), _vp(d_total.data_ptr())),
                    "count_async")

    def count_add_async(self, trie, pattern: int, d_total) -> None:
        """Enqueues one counting launch that adds its count into d_total."""
        self._check(self._lib.eh_count_add_async(self._h, trie._h, int(pattern), _vp(d_total.data_ptr())),
                    "count_add_async")

    def count_add_noalloc(self, trie, pattern: int, d_total) -> None:
        """As count_add_async, allocating nothing (static scratch; needs the
        plan cached by an earlier count with the same tuning)."""
        self._check(self._lib.eh_count_add_noalloc(self._h, trie._h, int(pattern),
                                                   _vp(d_total.data_ptr())), "count_add_noalloc")

    def stream_read_async(self, d_buf, d_sink, blocks_per_cu: int = 0) -> None:
        """Enqueues the streaming-read probe over the tensor d_buf (every byte
        read once), folding what it read into the uint64 tensor d_sink."""
        nbytes = d_buf.numel() * d_buf.element_size()
        self._check(self._lib.eh_stream_read(self._h, _vp(d_buf.data_ptr()), nbytes,
                                             int(blocks_per_cu), _vp(d_sink.data_ptr())),
                    "stream_read")

    def count_rooted(self, trie, pattern: int, roots) -> int:
        r = _u32(roots)
        out = ctypes.c_uint64(0)
        self._check(self._lib.eh_count_rooted(self._h, trie._h, int(pattern), _p32(r), r.size,
                                              ctypes.byref(out)), "count_rooted")
        return int(out.value)

    def count_batch(self, trie, pattern: int, first: int = 0, count: int | None = None) -> np.ndarray:
        if count is None:
            count = trie.info["n_graphs"] - first
        out = np.zeros(count, np.uint64)
        self._check(self._lib.eh_count_batch(self._h, trie._h, int(pattern), int(first), int(count),
                                             _p64(out)), "count_batch")
        return out

    def count_batch_async(self, trie, pattern: int, first: int, count: int, d_out) -> None:
        self._check(self._lib.eh_count_batch_async(self._h, trie._h, int(pattern), int(first), int(count),
                                                   _vp(d_out.data_ptr())), "count_batch_async")

    # -- set stores ---------------------------------------------------------
    def build_sets(self, off, members, layout=SETS_COMPOSITE, block_log=8, block_min=0, tau=32.0,
                   s_min=1) -> "Sets":
        """Encodes sets members[off[i]:off[i+1]] (each strictly ascending) and uploads them."""
        off, members = _sets_input(off, members)
        h = _vp()
        o = _set_opts(layout, block_log, block_min, tau, s_min)
        self._check(self._lib.eh_sets_build(self._h, off.size - 1, _p64(off), _p32(members),
                                            ctypes.byref(o), ctypes.byref(h)), "sets_build")
        return Sets(self, h)

    def intersect_pairs(self, sets, d_pairs, d_counts=None, lanes: int = 0) -> int:
        """Sum of |A & B| over the pairs of d_pairs (an int32 CUDA tensor of shape
        [n, 2] of set indices); d_counts (int32 CUDA tensor of n) receives each pair's count."""
        n = int(d_pairs.numel()) // 2
        out = ctypes.c_uint64(0)
        self._check(self._lib.eh_intersect_pairs(
            self._h, sets._h, n, _vp(d_pairs.data_ptr()) if n else None,
            _vp(d_counts.data_ptr()) if d_counts is not None else None, int(lanes),
            ctypes.byref(out)), "intersect_pairs")
        return int(out.value)

    def intersect_pairs_async(self, sets, d_pairs, d_total, d_counts=None, lanes: int = 0) -> None:
        """Enqueues the intersections; adds their sum into d_total (a 1-element int64 CUDA tensor)."""
        n = int(d_pairs.numel()) // 2
        self._check(self._lib.eh_intersect_pairs_async(
            self._h, sets._h, n, _vp(d_pairs.data_ptr()) if n else None,
            _vp(d_counts.data_ptr()) if d_counts is not None else None, int(lanes),
            _vp(d_total.data_ptr())), "intersect_pairs_async")

    def server(self, trie, hbm_budget_bytes=0, max_active=0, max_queued=0, step_items=0,
               policy=0) -> "Server":
        return Server(self, trie, hbm_budget_bytes, max_active, max_queued, step_items, policy)


class Trie:
    def __init__(self, ctx: Context, h):
        self.ctx = ctx
        self._h = h
        ctx._tries.append(self)
        info = _TrieInfo()
        ctx._check(ctx._lib.eh_trie_info_get(h, ctypes.byref(info)), "trie_info")
        self.info = _info_dict(info)

    def refresh_info(self) -> dict:
        info = _TrieInfo()
        self.ctx._check(self.ctx._lib.eh_trie_info_get(self._h, ctypes.byref(info)), "trie_info")
        self.info = _info_dict(info)
        return self.info

    def host_arrays(self) -> dict:
        """The trie's host copy, in the layout of host_trie()."""
        i = self.info
        n, m, w = i["n"], i["m_plus"], i["bitset_words"]
        arr = {k: np.zeros(sz, np.uint32) for k, sz in
               (("rank", n), ("row", n + 1), ("col", m), ("bs_off", n), ("bs_base", n),
                ("bs_nw", n), ("bs_words", w))}
        self.ctx._check(self.ctx._lib.eh_trie_host_arrays(
            self._h, *(_p32(arr[k]) for k in ("rank", "row", "col", "bs_off", "bs_base", "bs_nw",
                                              "bs_words"))), "trie_host_arrays")
        return arr

    def free(self):
        if self._h:
            self.ctx._lib.eh_trie_free(self._h)
            self._h = None
            if self in self.ctx._tries:
                self.ctx._tries.remove(self)


class Sets:
    def __init__(self, ctx: Context, h):
        self.ctx = ctx
        self._h = h
        ctx._sets.append(self)
        info = _SetsInfo()
        ctx._check(ctx._lib.eh_sets_info_get(h, ctypes.byref(info)), "sets_info")
        self.info = {k: int(getattr(info, k)) for k, _ in _SetsInfo._fields_}

    def free(self):
        if self._h:
            self.ctx._lib.eh_sets_free(self._h)
            self._h = None
            if self in self.ctx._sets:
                self.ctx._sets.remove(self)


@dataclass
class ReqResult:
    count: int
    t_submit_ns: int
    t_admit_ns: int
    t_done_ns: int
    items: int


class Server:
    def __init__(self, ctx: Context, trie: Trie, budget, max_active, max_queued, step_items,
                 policy=0):
        self.ctx = ctx
        self._lib = ctx._lib
        o = _ServerOpts(int(budget), int(max_active), int(max_queued), int(step_items), int(policy))
        h = _vp()
        ctx._check(self._lib.eh_server_create(ctx._h, trie._h, ctypes.byref(o), ctypes.byref(h)),
                   "server_create")
        self._h = h

    def submit(self, pattern: int, roots) -> int:
        r = _u32(roots)
        t = ctypes.c_uint64(0)
        st = self._lib.eh_submit(self._h, int(pattern), _p32(r), r.size, ctypes.byref(t))
        if st != EH_OK:
            raise EHError(st, "submit: " + self._lib.eh_status_str(st).decode())
        return int(t.value)

    def _result(self, st, c, s):
        if st == EH_PENDING:
            return None
        if st != EH_OK:
            raise EHError(st, "poll: " + self._lib.eh_status_str(st).decode())
        return ReqResult(int(c.value), int(s.t_submit_ns), int(s.t_admit_ns), int(s.t_done_ns), int(s.items))

    def poll(self, ticket: int):
        c = ctypes.c_uint64(0)
        s = _ReqStats()
        return self._result(self._lib.eh_poll(self._h, int(ticket), ctypes.byref(c), ctypes.byref(s)), c, s)

    def wait(self, ticket: int, timeout_ms: int = 60000):
        c = ctypes.c_uint64(0)
        s = _ReqStats()
        return self._result(self._lib.eh_wait(self._h, int(ticket), int(timeout_ms), ctypes.byref(c),
                                              ctypes.byref(s)), c, s)

    def drain(self, cap: int = 1024, timeout_ms: int = 10):
        """Finished requests in completion order: a list of (ticket, ReqResult)."""
        t = np.zeros(cap, np.uint64)
        c = np.zeros(cap, np.uint64)
        s = (_ReqStats * cap)()
        n = ctypes.c_uint32(0)
        st = self._lib.eh_server_drain(self._h, int(cap), int(timeout_ms), _p64(t), _p64(c), s,
                                       ctypes.byref(n))
        if st != EH_OK:
            raise EHError(st, "drain: " + self._lib.eh_status_str(st).decode())
        return [(int(t[i]), ReqResult(int(c[i]), int(s[i].t_submit_ns), int(s[i].t_admit_ns),
                                      int(s[i].t_done_ns), int(s[i].items)))
                for i in range(n.value)]

    def close(self):
        if self._h:
            self._lib.eh_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
