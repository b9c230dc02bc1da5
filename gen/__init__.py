"""Seeded synthetic workloads for the Intergrams hot path.

Generation is done by ``iggen.c`` (SplitMix64 streams keyed by seed, stream tag
and file index), so every corpus is reproducible and independent of thread
count.  This package holds no part of the method's arithmetic; the CPU oracle
and the HIP path both consume what it writes.
"""
import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libiggen.so")
_lib = None

BASE_SEED = 20251114


def build(force=False):
    """Compile ``libiggen.so`` with gcc (always, when ``force``)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread",
                               os.path.join(_HERE, "iggen.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        u64, i32, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
        lib.iggen_offsets.argtypes = [i32, u64, u64, vp]
        lib.iggen_fill.argtypes = [i32, u64, u64, vp, vp, i32]
        lib.iggen_data_bytes.argtypes = [i32, u64]
        lib.iggen_data_bytes.restype = u64
        lib.iggen_default_m.argtypes = [i32]
        lib.iggen_symbol_bits.argtypes = [i32]
        lib.iggen_req_open.argtypes = [u64, u64]
        lib.iggen_req_open.restype = vp
        lib.iggen_req_close.argtypes = [vp]
        lib.iggen_req_gap.argtypes = [vp, u64]
        lib.iggen_req_gap.restype = ctypes.c_double
        lib.iggen_req_len.argtypes = [vp, u64]
        lib.iggen_req_len.restype = u64
        lib.iggen_req_fill.argtypes = [vp, u64, vp]
        _lib = lib
    return _lib


@dataclass
class Corpus:
    """m sequences: ``data`` holds the symbol stream (bytes, or 2-bit symbols
    packed MSB first), ``offsets[i]..offsets[i+1]`` are file i's symbol range."""
    data: np.ndarray
    offsets: np.ndarray
    symbol_bits: int
    name: str = ""

    @property
    def m(self):
        return len(self.offsets) - 1

    @property
    def nbytes(self):
        return int(self.data.nbytes)

    def file(self, i):
        """Symbols of file i as a uint8 array (one symbol per element)."""
        a, b = int(self.offsets[i]), int(self.offsets[i + 1])
        if self.symbol_bits == 8:
            return self.data[a:b]
        return unpack2(self.data, a, b)

    def sha256(self):
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.offsets).tobytes())
        h.update(memoryview(self.data))
        return h.hexdigest()


def unpack2(data, a, b):
    """2-bit symbols [a, b) of a packed MSB-first stream."""
    if b <= a:
        return np.zeros(0, np.uint8)
    lo, hi = a // 4, (b + 3) // 4
    byts = data[lo:hi]
    syms = np.empty(len(byts) * 4, np.uint8)
    for j in range(4):
        syms[j::4] = (byts >> (6 - 2 * j)) & 3
    return syms[a - 4 * lo: b - 4 * lo]


def pack2(symbol_lists):
    """Pack lists of 2-bit symbols contiguously, MSB first; returns (data, offsets)."""
    offs = np.zeros(len(symbol_lists) + 1, np.uint64)
    for i, s in enumerate(symbol_lists):
        offs[i + 1] = offs[i] + len(s)
    total = int(offs[-1])
    allsym = np.zeros(((total + 3) // 4) * 4, np.uint8)
    if total:
        allsym[:total] = np.concatenate([np.asarray(s, np.uint8) for s in symbol_lists])
    data = np.zeros(len(allsym) // 4, np.uint8)
    for j in range(4):
        data |= (allsym[j::4] & 3) << (6 - 2 * j)
    return data, offs


def from_files(files, symbol_bits=8, name="custom"):
    """Corpus from a list of symbol sequences (bytes / lists / arrays)."""
    if symbol_bits == 8:
        arrs = [np.frombuffer(bytes(f), np.uint8) if isinstance(f, (bytes, bytearray)) else np.asarray(f, np.uint8)
                for f in files]
        offs = np.zeros(len(arrs) + 1, np.uint64)
        for i, a in enumerate(arrs):
            offs[i + 1] = offs[i] + len(a)
        data = np.concatenate(arrs) if arrs and offs[-1] else np.zeros(0, np.uint8)
        return Corpus(np.ascontiguousarray(data, np.uint8), offs, 8, name)
    if symbol_bits == 2:
        data, offs = pack2([f if isinstance(f, np.ndarray) else list(f) for f in files])
        return Corpus(data, offs, 2, name)
    raise ValueError("symbol_bits must be 8 or 2")


def default_m(cfg):
    return int(_load().iggen_default_m(cfg))


def workload(cfg, m=None, seed=None, nthreads=None):
    """Workload ``cfg`` (1..4); ``m`` < default gives the first m files of a
    scaled-down variant (same recipe; workload 3 scales its total with m)."""
    lib = _load()
    if cfg not in (1, 2, 3, 4):
        raise ValueError("workload must be 1..4")
    if m is None:
        m = default_m(cfg)
    if seed is None:
        seed = BASE_SEED + cfg
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
    offs = np.zeros(m + 1, np.uint64)
    if lib.iggen_offsets(cfg, seed, m, offs.ctypes.data) != 0:
        raise RuntimeError("iggen_offsets failed")
    nbytes = int(lib.iggen_data_bytes(cfg, int(offs[-1])))
    data = np.empty(max(nbytes, 1), np.uint8)[:nbytes]
    rc = lib.iggen_fill(cfg, seed, m, offs.ctypes.data, data.ctypes.data if nbytes else None, nthreads)
    if rc != 0:
        raise RuntimeError("iggen_fill failed: %d" % rc)
    return Corpus(data, offs, int(lib.iggen_symbol_bits(cfg)), "workload%d(m=%d,seed=%d)" % (cfg, m, seed))


class RequestStream:
    """Workload 5: request i is one binary-like file (motif library of workload 2)."""

    def __init__(self, seed=BASE_SEED + 5, lib_seed=BASE_SEED + 2):
        self._lib = _load()
        self._h = self._lib.iggen_req_open(seed, lib_seed)
        if not self._h:
            raise MemoryError("iggen_req_open")

    def close(self):
        if self._h:
            self._lib.iggen_req_close(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def gap(self, i):
        return float(self._lib.iggen_req_gap(self._h, i))

    def length(self, i):
        return int(self._lib.iggen_req_len(self._h, i))

    def file(self, i, out=None):
        n = self.length(i)
        buf = np.empty(n, np.uint8) if out is None else out[:n]
        self._lib.iggen_req_fill(self._h, i, buf.ctypes.data)
        return buf
