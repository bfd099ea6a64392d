"""CPU oracle for the exhaustive k-order epistasis scan -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports, links
or calls it, and it shares no code with the GPU library.

The arithmetic lives in ``epi_oracle.c`` (plain C99, per-individual walk,
double-precision mutual information, Sections 2.1-2.4 and Equations 1-3 of
the paper).  This module only compiles it with gcc and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "epi_oracle.c")
BUILD_DIR = os.path.join(_HERE, "_build")
LIB_PATH = os.path.join(BUILD_DIR, "liboracle.so")
CFLAGS = ["-O2", "-fno-tree-vectorize", "-std=gnu99", "-fPIC", "-shared", "-pthread"]

_lib = None
_lock = threading.Lock()


def build(source=SOURCE, out=LIB_PATH, extra_flags=()):
    """Compile the oracle into a shared library with gcc; returns the path."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, *extra_flags, source, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def _bind(lib):
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i32p = ctypes.POINTER(ctypes.c_int32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.oracle_binomial.restype = ctypes.c_uint64
    lib.oracle_binomial.argtypes = [ctypes.c_int64, ctypes.c_int64]
    lib.oracle_enumerate_count.restype = ctypes.c_uint64
    lib.oracle_enumerate_count.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.oracle_count_table.restype = ctypes.c_int
    lib.oracle_count_table.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int32, i32p, ctypes.c_int32, u64p]
    lib.oracle_genotype_rows.restype = ctypes.c_int
    lib.oracle_genotype_rows.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int32, i32p, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint32)]
    lib.oracle_mi.restype = ctypes.c_double
    lib.oracle_mi.argtypes = [u64p, ctypes.c_int32]
    lib.oracle_scan.restype = ctypes.c_int
    lib.oracle_scan.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32,
                                i32p, f64p, u64p, i32p, i32p]
    lib.oracle_digest.restype = ctypes.c_int
    lib.oracle_digest.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32, u64p, u64p]
    lib.oracle_score_list.restype = ctypes.c_int
    lib.oracle_score_list.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int32, ctypes.c_int32, i32p,
                                      ctypes.c_int32, f64p, u64p]
    return lib


def load(path=None):
    """Load (building first if needed) and return the ctypes library."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SOURCE):
                build()
            _lib = _bind(ctypes.CDLL(LIB_PATH))
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _as_inputs(G, y):
    G = np.ascontiguousarray(G, dtype=np.uint8)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    if G.ndim != 2 or y.ndim != 1 or G.shape[1] != y.shape[0]:
        raise ValueError("G must be (M, N) and y (N,)")
    return G, y


class Oracle:
    """Numpy-facing wrapper around one loaded oracle library."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    def binomial(self, n, k):
        return int(self.lib.oracle_binomial(int(n), int(k)))

    def enumerate_count(self, M, k):
        return int(self.lib.oracle_enumerate_count(int(M), int(k)))

    def count_table(self, G, y, combo):
        """Contingency table, shape (2, 3**k): row 0 cases, row 1 controls."""
        G, y = _as_inputs(G, y)
        c = np.ascontiguousarray(combo, dtype=np.int32)
        k = c.shape[0]
        out = np.zeros((2, 3**k), np.uint64)
        rc = self.lib.oracle_count_table(_ptr(G, ctypes.c_uint8), G.shape[1], _ptr(y, ctypes.c_uint8),
                                         G.shape[1], _ptr(c, ctypes.c_int32), k, _ptr(out, ctypes.c_uint64))
        if rc != 0:
            raise ValueError("genotype outside {0,1,2}")
        return out

    def genotype_rows(self, G, y, combo, words0, words1):
        """Genotype table, shape (3**k, words0 + words1) uint32: row x holds the
        cases with genotype combination x as a bitset over the cases (first
        words0 words), then the controls (words1 words)."""
        G, y = _as_inputs(G, y)
        c = np.ascontiguousarray(combo, dtype=np.int32)
        k = c.shape[0]
        out = np.zeros((3**k, words0 + words1), np.uint32)
        rc = self.lib.oracle_genotype_rows(_ptr(G, ctypes.c_uint8), G.shape[1], _ptr(y, ctypes.c_uint8),
                                           G.shape[1], _ptr(c, ctypes.c_int32), k, int(words0), int(words1),
                                           _ptr(out, ctypes.c_uint32))
        if rc != 0:
            raise ValueError("genotype outside {0,1,2} or a class wider than its words")
        return out

    def mi(self, table):
        t = np.ascontiguousarray(table, dtype=np.uint64).reshape(2, -1)
        k = int(round(np.log(t.shape[1]) / np.log(3)))
        if 3**k != t.shape[1]:
            raise ValueError("table width must be a power of 3")
        return float(self.lib.oracle_mi(_ptr(t, ctypes.c_uint64), k))

    def scan(self, G, y, order, top_k, rank_begin=0, rank_end=None, nthreads=0, tables=True):
        """Best ``top_k`` combinations of the lexicographic rank range.

        Returns dict with ``combos`` (n, k) int32, ``scores`` (n,) float64,
        ``tables`` (n, 2, 3**k) uint64 or None, ``threads``.
        """
        G, y = _as_inputs(G, y)
        M, N = G.shape
        total = self.binomial(M, order)
        end = total if rank_end is None else min(int(rank_end), total)
        combos = np.zeros((top_k, order), np.int32)
        scores = np.zeros(top_k, np.float64)
        tabs = np.zeros((top_k, 2, 3**order), np.uint64) if tables else None
        n_out = ctypes.c_int32(0)
        used = ctypes.c_int32(0)
        rc = self.lib.oracle_scan(_ptr(G, ctypes.c_uint8), N, _ptr(y, ctypes.c_uint8), M, N, order, top_k,
                                  int(rank_begin), int(end), int(nthreads), _ptr(combos, ctypes.c_int32),
                                  _ptr(scores, ctypes.c_double),
                                  _ptr(tabs, ctypes.c_uint64) if tables else None,
                                  ctypes.byref(n_out), ctypes.byref(used))
        if rc != 0:
            raise ValueError("oracle_scan rejected its input")
        n = n_out.value
        return {"combos": combos[:n], "scores": scores[:n], "tables": tabs[:n] if tables else None,
                "threads": used.value}

    def digest(self, G, y, order, rank_begin=0, rank_end=None, nthreads=0):
        """(count, digest) of the combinations of the lexicographic rank range:
        how many there are and the sum modulo 2^64 of each one's hash with its
        table (the completeness check of a scan)."""
        G, y = _as_inputs(G, y)
        M, N = G.shape
        total = self.binomial(M, order)
        end = total if rank_end is None else min(int(rank_end), total)
        count, dig = ctypes.c_uint64(0), ctypes.c_uint64(0)
        rc = self.lib.oracle_digest(_ptr(G, ctypes.c_uint8), N, _ptr(y, ctypes.c_uint8), M, N, order,
                                    int(rank_begin), int(end), int(nthreads), ctypes.byref(count), ctypes.byref(dig))
        if rc != 0:
            raise ValueError("oracle_digest rejected its input")
        return count.value, dig.value

    def score_list(self, G, y, combos):
        """Scores (n,) and tables (n, 2, 3**k) of explicit combinations."""
        G, y = _as_inputs(G, y)
        c = np.ascontiguousarray(combos, dtype=np.int32)
        n, k = c.shape
        scores = np.zeros(n, np.float64)
        tabs = np.zeros((n, 2, 3**k), np.uint64)
        rc = self.lib.oracle_score_list(_ptr(G, ctypes.c_uint8), G.shape[1], _ptr(y, ctypes.c_uint8),
                                        G.shape[1], k, _ptr(c, ctypes.c_int32), n,
                                        _ptr(scores, ctypes.c_double), _ptr(tabs, ctypes.c_uint64))
        if rc != 0:
            raise ValueError("genotype outside {0,1,2}")
        return scores, tabs


_default = None


def default():
    """Process-wide :class:`Oracle` on the default build."""
    global _default
    if _default is None:
        _default = Oracle()
    return _default
