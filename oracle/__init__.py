"""CPU oracle for the Intergrams per-pass scan (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The library path never does.

``ig_oracle.cpp`` is the plain definition (Eq. 1 / Eq. 2, Algorithm 3);
``brute.py`` is an independent brute force used to pin it.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libig_oracle.so")
_lib = None

FREQ_DOC, FREQ_OCC = 0, 1
OK, EINVAL, ESTATE, ENOMEM, ETRUNC = 0, -1, -2, -3, -4


def build(force=False, out=None, defines=(), flags=()):
    """Compile the oracle with g++ (``defines`` is for planted-mistake tests, ``flags`` for the
    sanitizer build)."""
    so = out or _SO
    if force or not os.path.exists(so):
        tmp = so + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread"] + list(flags)
        cmd += ["-D%s" % d for d in defines]
        cmd += [os.path.join(_HERE, "ig_oracle.cpp"), "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, so)
    return so


def _bind(lib):
    u64, u32, i32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p
    lib.igo_create.argtypes = [i32, i32, i32]
    lib.igo_create.restype = vp
    lib.igo_destroy.argtypes = [vp]
    lib.igo_set_threads.argtypes = [vp, i32]
    lib.igo_load.argtypes = [vp, vp, u64, vp, u64]
    lib.igo_pass.argtypes = [vp, u32, u64]
    lib.igo_kept.argtypes = [vp]
    lib.igo_kept.restype = u64
    lib.igo_last_n.argtypes = [vp]
    lib.igo_last_n.restype = u32
    lib.igo_topk.argtypes = [vp, u64, vp, vp, vp]
    lib.igo_set_retained.argtypes = [vp, u32, vp, vp, u64]
    lib.igo_featurize.argtypes = [vp, vp, u64, vp, u64, vp, vp, u64, vp]
    return lib


def _load(path=None):
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        build()
        _lib = _bind(ctypes.CDLL(_SO))
    return _lib


def keys_to_int(lohi):
    """(k, 2) uint64 (lo, hi) -> list of Python ints."""
    return [int(lo) | (int(hi) << 64) for lo, hi in lohi]


class Oracle:
    """One oracle context: load a corpus, run passes, read the retained table."""

    def __init__(self, symbol_bits=8, freq=FREQ_DOC, nthreads=None, lib_path=None):
        self._lib = _load(lib_path)
        if nthreads is None:
            nthreads = min(16, os.cpu_count() or 1)
        self.nthreads = nthreads
        self.symbol_bits = symbol_bits
        self._h = self._lib.igo_create(symbol_bits, freq, nthreads)
        if not self._h:
            raise ValueError("bad oracle arguments")

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.igo_destroy(self._h)
            self._h = None

    def load(self, corpus):
        data = np.ascontiguousarray(corpus.data, np.uint8)
        offs = np.ascontiguousarray(corpus.offsets, np.uint64)
        rc = self._lib.igo_load(self._h, data.ctypes.data, data.nbytes, offs.ctypes.data, len(offs) - 1)
        if rc:
            raise ValueError("igo_load: %d" % rc)

    def pass_(self, n, k_keep):
        return int(self._lib.igo_pass(self._h, n, k_keep))

    def intergrams(self, corpus, n, k, z=1.0):
        """Algorithm 3 as a whole (Section 4), on a freshly loaded ``corpus``.

        P^(n0) is the top ceil(z*k) of all n0-grams (Algorithm 2 for bytes, n0 = 3; for
        b-bit symbols n0 is the largest length whose keys fit 24 bits, never above n); then
        for j = n0+1 .. n the j-grams whose (j-1)-prefix is in P^(j-1) are counted and
        ceil(z*k) are kept while j < n, k at j = n.  Returns the last pass's return code.
        """
        if not (z >= 1.0 and math.isfinite(z)) or k < 1 or n < 1:
            raise ValueError("need n >= 1, k >= 1, finite z >= 1")
        kz = math.ceil(z * float(k))
        n0 = min(n, 24 // self.symbol_bits)
        self.load(corpus)                   # the first pass after a load is unfiltered
        for j in range(n0, n + 1):
            rc = self.pass_(j, kz if j < n else k)
            if rc:
                return rc
        return 0

    def kept(self):
        return int(self._lib.igo_kept(self._h))

    def topk(self, k=None):
        """Ordered (keys as (k,2) uint64 lo/hi, counts uint64) of the retained table."""
        if k is None:
            k = self.kept()
        keys = np.zeros((max(k, 1), 2), np.uint64)
        counts = np.zeros(max(k, 1), np.uint64)
        kout = ctypes.c_uint64(0)
        rc = self._lib.igo_topk(self._h, k, keys.ctypes.data, counts.ctypes.data, ctypes.byref(kout))
        if rc:
            raise RuntimeError("igo_topk: %d" % rc)
        return keys[:kout.value], counts[:kout.value]

    def table(self):
        """Retained table as a list of (int key, count)."""
        keys, counts = self.topk()
        return list(zip(keys_to_int(keys), [int(c) for c in counts]))

    def set_retained(self, n, keys_int, counts):
        keys = np.array([[k & (2**64 - 1), k >> 64] for k in keys_int], np.uint64).reshape(-1, 2)
        cnt = np.asarray(counts, np.uint64)
        rc = self._lib.igo_set_retained(self._h, n, keys.ctypes.data, cnt.ctypes.data, len(cnt))
        if rc:
            raise ValueError("igo_set_retained: %d" % rc)

    def featurize(self, corpus):
        """CSR rows (indptr uint64[m+1], indices int32[nnz]) of ``corpus`` against the table."""
        data = np.ascontiguousarray(corpus.data, np.uint8)
        offs = np.ascontiguousarray(corpus.offsets, np.uint64)
        m = len(offs) - 1
        indptr = np.zeros(m + 1, np.uint64)
        cap = 1 << 16
        while True:
            ind = np.zeros(cap, np.int32)
            nnz = ctypes.c_uint64(0)
            rc = self._lib.igo_featurize(self._h, data.ctypes.data, data.nbytes, offs.ctypes.data, m,
                                         indptr.ctypes.data, ind.ctypes.data, cap, ctypes.byref(nnz))
            if rc == ETRUNC:
                cap = int(nnz.value)
                continue
            if rc:
                raise RuntimeError("igo_featurize: %d" % rc)
            return indptr, ind[:nnz.value]
