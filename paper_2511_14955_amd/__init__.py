"""Python binding of libintergrams.so (the Intergrams per-pass scan on MI355X).

Argument marshalling only: every step of a pass, of featurize and of serving
runs in the library's HIP kernels.  There is no CPU fallback: if the shared
library is missing or fails to load, importing the binding's entry points
raises.

PyTorch is optional here; when given, torch CUDA tensors are passed as device
pointers and torch's current stream can be handed to the library.
"""
import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# IG_LIBRARY may name another build of the library (the host-sanitized libintergrams_san.so)
LIB_PATH = os.environ.get("IG_LIBRARY") or os.path.join(_HERE, "libintergrams.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "ig.h")

IG_OK, IG_EINVAL, IG_ESTATE, IG_ENOMEM, IG_ETRUNC, IG_EOVERFLOW, IG_EDEVICE, IG_EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
FREQ_DOC, FREQ_OCC = 0, 1
FLAG_NO_GRAPH, FLAG_PER_FILE = 1, 2
NOALLOC_SCRATCH_BYTES = 64 << 20   # IG_NOALLOC_SCRATCH_BYTES
REQ_FEATURIZE, REQ_COUNT = 0, 1

_ERRNAMES = {IG_EINVAL: "IG_EINVAL", IG_ESTATE: "IG_ESTATE", IG_ENOMEM: "IG_ENOMEM", IG_ETRUNC: "IG_ETRUNC",
             IG_EOVERFLOW: "IG_EOVERFLOW", IG_EDEVICE: "IG_EDEVICE", IG_EBUSY: "IG_EBUSY"}


class IGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_ERRNAMES.get(code, "?"), code, msg))
        self.code = code


class ig_key(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]


# optional device allocator hooks of ig_config
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class ig_config(ctypes.Structure):
    _fields_ = [("symbol_bits", ctypes.c_uint32), ("freq", ctypes.c_int), ("count_bits", ctypes.c_uint32),
                ("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("hbm_budget", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_user", ctypes.c_void_p)]


class ig_pass_stats(ctypes.Structure):
    _fields_ = [("pass_ms", ctypes.c_double), ("scan_ms", ctypes.c_double), ("select_ms", ctypes.c_double),
                ("windows", ctypes.c_uint64), ("distinct", ctypes.c_uint64), ("input_bytes", ctypes.c_uint64),
                ("replays", ctypes.c_uint32), ("chunk_syms", ctypes.c_uint32), ("block", ctypes.c_uint32),
                ("grid", ctypes.c_uint32), ("records", ctypes.c_uint64), ("dedup_ms", ctypes.c_double),
                ("set_cap", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class _tune_cand(ctypes.Structure):
    _fields_ = [("chunk_syms", ctypes.c_uint32), ("block", ctypes.c_uint32), ("set_cap", ctypes.c_uint32),
                ("wg_per_cu", ctypes.c_uint32), ("map_slots_log2", ctypes.c_uint32),
                ("filter_max_words", ctypes.c_uint32), ("pass_ms", ctypes.c_double)]


class ig_table_shape(ctypes.Structure):
    _fields_ = [("map_slots_log2", ctypes.c_uint32), ("filter_bits_per_key", ctypes.c_uint32),
                ("filter_max_words", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("sparse_slots", ctypes.c_uint64), ("record_capacity", ctypes.c_uint64)]


IG_TUNE_MAX = 32


class ig_tune_report(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_uint32), ("cand", _tune_cand * IG_TUNE_MAX), ("best", ctypes.c_uint32),
                ("identical", ctypes.c_int), ("from_cache", ctypes.c_int)]


class ig_serve_config(ctypes.Structure):
    _fields_ = [("max_inflight_bytes", ctypes.c_uint64), ("n_streams", ctypes.c_uint32),
                ("max_batch", ctypes.c_uint32), ("queue_capacity", ctypes.c_uint64)]


class ig_result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("kind", ctypes.c_int), ("status", ctypes.c_int),
                ("t_arrival", ctypes.c_double), ("t_done", ctypes.c_double), ("n", ctypes.c_uint64)]


class ig_serve_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("peak_inflight_bytes", ctypes.c_uint64), ("bytes_in", ctypes.c_uint64),
                ("peak_running", ctypes.c_uint64)]


_lib = None


def header_functions():
    """Names of the functions that include/ig.h declares."""
    with open(HEADER) as fh:
        text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
    return sorted(set(re.findall(r"\b(ig_[a-z_]+)\s*\(", text)))


def load_library(path=LIB_PATH):
    """Load libintergrams.so (raises if it is not built)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libintergrams.so is not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    vp, u64, u32, i32, dbl = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double
    P = ctypes.POINTER
    lib.ig_config_default.argtypes = [P(ig_config)]
    lib.ig_config_default.restype = None
    lib.ig_create.argtypes = [P(ig_config), P(vp)]
    lib.ig_destroy.argtypes = [vp]
    lib.ig_destroy.restype = None
    lib.ig_load_batch.argtypes = [vp, vp, u64, P(u64), u64, i32]
    lib.ig_pass.argtypes = [vp, u32, u64]
    lib.ig_rewind.argtypes = [vp]
    lib.ig_intergrams.argtypes = [vp, u32, u64, dbl]
    lib.ig_measure_read_bw.argtypes = [vp, u64, u32, P(dbl)]
    lib.ig_topk.argtypes = [vp, u64, vp, vp, P(u64)]
    lib.ig_table_info.argtypes = [vp, P(u32), P(u64)]
    lib.ig_featurize.argtypes = [vp, vp, u64, P(u64), u64, P(u64), vp, u64, P(u64)]
    lib.ig_featurize_loaded.argtypes = [vp, P(u64), vp, u64, P(u64)]
    lib.ig_featurize_noalloc.argtypes = [vp, vp, u64, P(u64), u64, P(u64), vp, u64, P(u64)]
    lib.ig_last_pass_stats.argtypes = [vp, P(ig_pass_stats)]
    lib.ig_last_error.argtypes = [vp]
    lib.ig_last_error.restype = ctypes.c_char_p
    lib.ig_autotune.argtypes = [vp, u32, u64, P(ig_tune_report)]
    lib.ig_get_launch.argtypes = [vp, P(u32), P(u32), P(u32), P(u32)]
    lib.ig_set_launch.argtypes = [vp, u32, u32, u32, u32]
    lib.ig_get_tables.argtypes = [vp, P(ig_table_shape)]
    lib.ig_set_tables.argtypes = [vp, P(ig_table_shape)]
    lib.ig_serve_start.argtypes = [vp, P(ig_serve_config)]
    lib.ig_submit.argtypes = [vp, i32, vp, u64, P(u64), u64, u64, dbl]
    lib.ig_poll.argtypes = [vp, P(ig_result), u64, vp, vp, u64, vp, P(u64)]
    lib.ig_serve_now.argtypes = []
    lib.ig_serve_now.restype = dbl
    lib.ig_serve_stop.argtypes = [vp]
    lib.ig_serve_get_stats.argtypes = [vp, P(ig_serve_stats)]
    if path == LIB_PATH:
        _lib = lib
    return lib


def _u64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _as_host(corpus_or_data, offsets=None):
    if offsets is None:
        data, offsets = corpus_or_data.data, corpus_or_data.offsets
    else:
        data = corpus_or_data
    return data, np.ascontiguousarray(offsets, np.uint64)


class Intergrams:
    """One library context on one GPU."""

    def __init__(self, symbol_bits=8, freq=FREQ_DOC, count_bits=64, device=0, stream=None, hbm_budget=0, flags=0,
                 allocator=None):
        """allocator: optional (alloc(bytes, stream) -> device pointer int or 0, free(pointer, stream))
        pair of Python callables that then hold every device buffer of the context."""
        self._lib = load_library()
        cfg = ig_config()
        self._lib.ig_config_default(ctypes.byref(cfg))
        cfg.symbol_bits, cfg.freq, cfg.count_bits, cfg.device = symbol_bits, freq, count_bits, device
        cfg.stream = stream if stream is None or isinstance(stream, int) else int(stream.cuda_stream)
        cfg.hbm_budget, cfg.flags = hbm_budget, flags
        self._hooks = None
        if allocator is not None:
            fa, ff = allocator
            self._hooks = (ALLOC_FN(lambda n, st, u: fa(n, st) or None), FREE_FN(lambda p, st, u: ff(p, st)))
            cfg.alloc, cfg.free = self._hooks
        h = ctypes.c_void_p()
        rc = self._lib.ig_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc:
            raise IGError(rc, "ig_create failed")
        self._h = h
        self._m = 0
        self.symbol_bits = symbol_bits

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ig_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc):
        if rc:
            raise IGError(rc, self._lib.ig_last_error(self._h).decode(errors="replace"))
        return rc

    def load(self, corpus_or_data, offsets=None):
        """Load a gen.Corpus, or (data, offsets); data may be a numpy array or a torch CUDA tensor."""
        data, offs = _as_host(corpus_or_data, offsets)
        if hasattr(data, "is_cuda") and data.is_cuda:
            ptr, nbytes, on_dev = data.data_ptr(), data.numel() * data.element_size(), 1
        else:
            data = np.ascontiguousarray(data, np.uint8)
            ptr, nbytes, on_dev = data.ctypes.data, data.nbytes, 0
        self._check(self._lib.ig_load_batch(self._h, ptr, nbytes, _u64p(offs), len(offs) - 1, on_dev))
        self._m = len(offs) - 1

    def pass_(self, n, k_keep):
        return self._check(self._lib.ig_pass(self._h, n, k_keep))

    def intergrams(self, n, k, z=1.0):
        """Algorithm 3 from a fresh chain: dense pass at min(n, 24 // b), z-oversampled
        passes up to n - 1 (ceil(z*k) kept), k kept at n."""
        return self._check(self._lib.ig_intergrams(self._h, n, k, float(z)))

    def rewind(self):
        """Make the table retained before the last pass current again."""
        return self._check(self._lib.ig_rewind(self._h))

    def try_pass(self, n, k_keep):
        """ig_pass's return code (no exception)."""
        return int(self._lib.ig_pass(self._h, n, k_keep))

    def table_info(self):
        n, k = ctypes.c_uint32(), ctypes.c_uint64()
        self._check(self._lib.ig_table_info(self._h, ctypes.byref(n), ctypes.byref(k)))
        return n.value, k.value

    def topk(self, k=None):
        """(keys (k, 2) uint64 lo/hi, counts uint64) of the retained table, in order."""
        if k is None:
            k = self.table_info()[1]
        keys = np.zeros((max(k, 1), 2), np.uint64)
        counts = np.zeros(max(k, 1), np.uint64)
        kout = ctypes.c_uint64()
        self._check(self._lib.ig_topk(self._h, k, keys.ctypes.data, counts.ctypes.data, ctypes.byref(kout)))
        return keys[:kout.value], counts[:kout.value]

    def table(self):
        keys, counts = self.topk()
        return [(int(lo) | (int(hi) << 64), int(c)) for (lo, hi), c in zip(keys, counts)]

    def featurize(self, corpus_or_data, offsets=None, noalloc=False):
        """CSR rows (indptr uint64[m+1], indices int32[nnz]) of new sequences; ``noalloc`` calls
        ig_featurize_noalloc (same rows, no device allocation)."""
        fn = self._lib.ig_featurize_noalloc if noalloc else self._lib.ig_featurize
        data, offs = _as_host(corpus_or_data, offsets)
        data = np.ascontiguousarray(data, np.uint8)
        m = len(offs) - 1
        indptr = np.zeros(m + 1, np.uint64)
        nnz = ctypes.c_uint64()
        cap = 1 << 16
        while True:
            ind = np.zeros(max(cap, 1), np.int32)
            rc = fn(self._h, data.ctypes.data, data.nbytes, _u64p(offs), m, _u64p(indptr), ind.ctypes.data, cap,
                    ctypes.byref(nnz))
            if rc == IG_ETRUNC:
                cap = int(nnz.value)
                continue
            self._check(rc)
            return indptr, ind[:nnz.value]

    def featurize_loaded(self):
        """CSR rows (indptr uint64[m+1], indices int32[nnz]) of the loaded sequences themselves."""
        indptr = np.zeros(self._m + 1, np.uint64)
        nnz = ctypes.c_uint64()
        # cap 0 sizes the output (indptr and the total are filled, IG_ETRUNC when nnz > 0)
        rc = self._lib.ig_featurize_loaded(self._h, _u64p(indptr), None, 0, ctypes.byref(nnz))
        if rc != IG_ETRUNC:
            self._check(rc)
        ind = np.zeros(max(int(nnz.value), 1), np.int32)
        self._check(self._lib.ig_featurize_loaded(self._h, _u64p(indptr), ind.ctypes.data, int(nnz.value),
                                                  ctypes.byref(nnz)))
        return indptr, ind[:nnz.value]

    def autotune(self, n, k_keep):
        """Search the scan's launch shape on pass n (chain state unchanged); returns a report dict."""
        rep = ig_tune_report()
        self._check(self._lib.ig_autotune(self._h, n, k_keep, ctypes.byref(rep)))
        cands = [{"chunk_syms": c.chunk_syms, "block": c.block, "set_cap": c.set_cap, "wg_per_cu": c.wg_per_cu,
                  "map_slots_log2": c.map_slots_log2, "filter_max_words": c.filter_max_words, "pass_ms": c.pass_ms}
                 for c in rep.cand[:rep.n_candidates]]
        return {"candidates": cands, "best": cands[rep.best] if cands else None, "identical": bool(rep.identical),
                "from_cache": bool(rep.from_cache)}

    def launch(self):
        a, b, c, w = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        self._check(self._lib.ig_get_launch(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(w)))
        return {"chunk_syms": a.value, "block": b.value, "set_cap": c.value, "wg_per_cu": w.value}

    def set_launch(self, chunk_syms, block, set_cap, wg_per_cu=1):
        self._check(self._lib.ig_set_launch(self._h, chunk_syms, block, set_cap, wg_per_cu))

    def tables(self):
        """The table sizes (ig_get_tables) as a dict."""
        t = ig_table_shape()
        self._check(self._lib.ig_get_tables(self._h, ctypes.byref(t)))
        return {f: int(getattr(t, f)) for f, _ in ig_table_shape._fields_ if f != "reserved"}

    def set_tables(self, **kw):
        """Change some table sizes (ig_set_tables); the others keep their current values
        (sparse_slots and record_capacity default to 0: left as they are)."""
        cur = self.tables()
        cur["sparse_slots"] = cur["record_capacity"] = 0
        cur.update(kw)
        t = ig_table_shape(**cur)
        self._check(self._lib.ig_set_tables(self._h, ctypes.byref(t)))

    def measure_read_bw(self, nbytes=4 << 30, reps=5):
        """GB/s that the library's plain streaming-read kernel attains on this device."""
        out = ctypes.c_double()
        self._check(self._lib.ig_measure_read_bw(self._h, nbytes, reps, ctypes.byref(out)))
        return out.value

    def last_stats(self):
        st = ig_pass_stats()
        self._check(self._lib.ig_last_pass_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ig_pass_stats._fields_}

    # ------------------------------------------------------------------ serving
    def serve_start(self, max_inflight_bytes=1 << 30, n_streams=4, max_batch=64, queue_capacity=1 << 16):
        """Start the continuous-batching loop over the retained table."""
        cfg = ig_serve_config(max_inflight_bytes, n_streams, max_batch, queue_capacity)
        self._check(self._lib.ig_serve_start(self._h, ctypes.byref(cfg)))

    def submit(self, kind, data, offsets, tag, t_arrival=None):
        """Queue one request; returns IG_OK or IG_EBUSY (queue full), raises on bad arguments."""
        data = np.ascontiguousarray(data, np.uint8)
        offs = np.ascontiguousarray(offsets, np.uint64)
        if t_arrival is None:
            t_arrival = self._lib.ig_serve_now()
        rc = self._lib.ig_submit(self._h, kind, data.ctypes.data, data.nbytes, _u64p(offs), len(offs) - 1, tag,
                                 t_arrival)
        if rc not in (IG_OK, IG_EBUSY):
            raise IGError(rc, "ig_submit")
        return rc

    def poll(self, max_results=1024, cap=1 << 20):
        """Completed results, oldest first: dicts with tag, kind, status, t_arrival, t_done, cols, counts."""
        res = (ig_result * max(1, max_results))()
        while True:
            cols = np.zeros(max(cap, 1), np.int32)
            counts = np.zeros(max(cap, 1), np.uint64)
            offs = np.zeros(max_results + 1, np.uint64)
            nout = ctypes.c_uint64()
            rc = self._lib.ig_poll(self._h, res, max_results, cols.ctypes.data, counts.ctypes.data, cap,
                                   offs.ctypes.data, ctypes.byref(nout))
            if rc == IG_ETRUNC:
                cap = int(res[0].n)
                continue
            if rc:
                raise IGError(rc, "ig_poll")
            out = []
            for i in range(nout.value):
                r = res[i]
                a, z = int(offs[i]), int(offs[i + 1])
                out.append({"tag": r.tag, "kind": r.kind, "status": r.status, "t_arrival": r.t_arrival,
                            "t_done": r.t_done, "n": r.n, "cols": cols[a:z].copy(),
                            "counts": counts[a:z].copy() if r.kind == REQ_COUNT else None})
            return out

    def serve_now(self):
        """The library clock (seconds) that t_done is measured on."""
        return self._lib.ig_serve_now()

    def serve_stats(self):
        st = ig_serve_stats()
        self._check(self._lib.ig_serve_get_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ig_serve_stats._fields_}

    def serve_stop(self):
        """Drain in-flight work and stop the loop (results not yet polled are dropped)."""
        self._check(self._lib.ig_serve_stop(self._h))
