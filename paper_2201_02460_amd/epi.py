"""Thin ctypes binding of ``libepi.so`` (declared in ``include/epi.h``).

Functions carry the C names and only marshal arguments: every step of the scan
runs in the library's HIP kernels.  Device inputs may be torch tensors (their
``data_ptr()`` is passed); streams may be ``torch.cuda.Stream`` objects, raw
``hipStream_t`` integers or ``None`` (the context's stream).

If the library is not built, :func:`lib` raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libepi.so")

EPI_OK = 0
EPI_EINVAL = -1
EPI_ENOMEM = -2
EPI_EDEVICE = -3
EPI_EUNSUPPORTED = -4
EPI_ENOTREADY = -5
EPI_ENOTFOUND = -6
EPI_MIN_ORDER = 2
EPI_MAX_ORDER = 8
EPI_SERVE_MAX_ORDER = 5
EPI_BLOCK_MFMA_FP4 = 16
EPI_BLOCK_MFMA_I8 = 32
EPI_BLOCK_MFMA_FP4_2J = 48
EPI_BLOCK_SEGMENTED = 64
EPI_BLOCK_ALL_CELLS = 81
EPI_NOALLOC_SCRATCH_BYTES = 134217728
EPI_MAX_TOP_K = 256

# Every function the header declares, with (restype, argtypes).
_c = ctypes
_i32, _i64, _u64, _vp = _c.c_int32, _c.c_int64, _c.c_uint64, _c.c_void_p
_P = _c.POINTER


class ScanDesc(_c.Structure):
    _fields_ = [("dataset_id", _i32), ("order", _i32), ("top_k", _i32), ("reserved", _i32)]


class ServerConfig(_c.Structure):
    _fields_ = [("max_active", _i32), ("rounds_in_flight", _i32), ("request_budget", _u64)]


SIGNATURES = {
    "epi_last_error": (_c.c_char_p, []),
    "epi_version": (_c.c_char_p, []),
    "epi_create": (_c.c_int, [_i32, _u64, _P(_vp)]),
    "epi_destroy": (_c.c_int, [_vp]),
    "epi_memory": (_c.c_int, [_vp, _P(_u64), _P(_u64)]),
    "epi_load_genotypes": (_c.c_int, [_vp, _vp, _i64, _vp, _i32, _i32, _P(_i32)]),
    "epi_load_genotypes_device": (_c.c_int, [_vp, _vp, _i64, _vp, _i32, _i32, _vp, _P(_i32)]),
    "epi_repack_device": (_c.c_int, [_vp, _i32, _vp, _i64, _vp, _vp]),
    "epi_unload": (_c.c_int, [_vp, _i32]),
    "epi_dataset_info": (_c.c_int, [_vp, _i32, _P(_i32), _P(_i32), _P(_i32), _P(_u64)]),
    "epi_scan": (_c.c_int, [_vp, _i32, _i32, _i32, _vp, _P(_i32)]),
    "epi_scan_batch": (_c.c_int, [_vp, _P(ScanDesc), _i32, _vp, _P(_i32)]),
    "epi_scan_orders": (_c.c_int, [_vp, _i32, _i32, _i32, _vp, _P(_i32)]),
    "epi_query": (_c.c_int, [_vp, _i32, _P(_i32)]),
    "epi_wait": (_c.c_int, [_vp, _i32]),
    "epi_results": (_c.c_int, [_vp, _i32, _i32, _vp, _vp, _vp, _P(_i32)]),
    "epi_scan_timing": (_c.c_int, [_vp, _i32, _P(_c.c_float)]),
    "epi_scan_info": (_c.c_int, [_vp, _i32, _P(_u64), _P(_i32), _P(_i32)]),
    "epi_release": (_c.c_int, [_vp, _i32]),
    "epi_scan_check": (_c.c_int, [_vp, _i32, _i32, _i32, _vp, _P(_i32)]),
    "epi_scan_digest": (_c.c_int, [_vp, _i32, _P(_u64), _P(_u64)]),
    "epi_scan_noalloc": (_c.c_int, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "epi_batch_create": (_c.c_int, [_vp, _P(ScanDesc), _i32, _i32, _i32, _P(_i32)]),
    "epi_batch_run": (_c.c_int, [_vp, _i32, _vp]),
    "epi_batch_wait": (_c.c_int, [_vp, _i32]),
    "epi_batch_results": (_c.c_int, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _P(_i32)]),
    "epi_batch_timing": (_c.c_int, [_vp, _i32, _P(_c.c_float)]),
    "epi_batch_destroy": (_c.c_int, [_vp, _i32]),
    "epi_autotune": (_c.c_int, [_vp, _i32, _i32, _P(_i32)]),
    "epi_autotune_report": (_c.c_int, [_vp, _i32, _i32, _i32, _vp, _vp, _P(_i32)]),
    "epi_set_prefix_block": (_c.c_int, [_vp, _i32, _i32, _i32]),
    "epi_genotype_tables": (_c.c_int, [_vp, _i32, _i32, _vp, _u64, _vp, _P(_c.c_float)]),
    "epi_contingency_tables": (_c.c_int, [_vp, _i32, _i32, _vp, _u64, _vp, _P(_c.c_float)]),
    "epi_mutual_information": (_c.c_int, [_vp, _i32, _i32, _vp, _u64, _vp, _P(_c.c_float)]),
    "epi_server_start": (_c.c_int, [_vp, _P(ServerConfig), _P(_i32)]),
    "epi_server_submit": (_c.c_int, [_vp, _i32, _i32, _i32, _i32, _P(_i32)]),
    "epi_server_poll": (_c.c_int, [_vp, _i32, _i32, _P(_i32)]),
    "epi_server_results": (_c.c_int, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _P(_i32), _P(_c.c_double)]),
    "epi_server_stats": (_c.c_int, [_vp, _i32, _P(_u64)]),
    "epi_server_stop": (_c.c_int, [_vp, _i32]),
}

_lib = None


class EpiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"epi error {code}: {msg}")
        self.code = code


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch bundles its own HIP runtime (same SONAME as the system one);
        # loading it first makes this library bind to that single runtime so
        # torch tensors, streams and this library share one device context.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2201_02460_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != EPI_OK:
        raise EpiError(rc, lib().epi_last_error().decode())
    return rc


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _ptr(x):
    """Device/host address of a torch tensor or numpy array."""
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    return int(x.ctypes.data)


def _cells(order):
    return 3**order


# ---- thin wrappers (same names as the C ABI) --------------------------------

def epi_version():
    return lib().epi_version().decode()


def epi_last_error():
    return lib().epi_last_error().decode()


def epi_create(device=0, hbm_budget_bytes=0):
    out = _vp()
    _check(lib().epi_create(device, hbm_budget_bytes, ctypes.byref(out)))
    return out


def epi_destroy(ctx):
    _check(lib().epi_destroy(ctx))


def epi_memory(ctx):
    used, budget = _u64(), _u64()
    _check(lib().epi_memory(ctx, ctypes.byref(used), ctypes.byref(budget)))
    return used.value, budget.value


def _host_inputs(geno, pheno):
    """Genotypes (M, N) and phenotypes (N,) as contiguous uint8 numpy arrays;
    other dtypes are refused rather than cast (a cast could wrap an invalid
    value into the valid range)."""
    g, p = np.asarray(geno), np.asarray(pheno)
    if g.dtype != np.uint8 or p.dtype != np.uint8:
        raise EpiError(EPI_EINVAL, "genotypes and phenotypes must be uint8 arrays")
    if g.ndim != 2 or p.ndim != 1 or p.shape[0] != g.shape[1]:
        raise EpiError(EPI_EINVAL, f"genotypes must be (M, N) and phenotypes (N,): got {g.shape} and {p.shape}")
    return np.ascontiguousarray(g), np.ascontiguousarray(p)


def _device_inputs(d_geno, d_pheno, shape=None):
    """Checks of device genotypes (M, N) uint8 with unit stride along the
    individuals and phenotypes (N,) uint8 contiguous: the library reads M
    rows of N bytes and N bytes through the raw pointers.  Returns (M, N, ld)."""
    import torch

    for t, what in ((d_geno, "genotypes"), (d_pheno, "phenotypes")):
        if not (isinstance(t, torch.Tensor) and t.is_cuda):
            raise EpiError(EPI_EINVAL, f"{what} must be a device tensor")
        if t.dtype != torch.uint8:
            raise EpiError(EPI_EINVAL, f"{what} must be uint8, got {t.dtype}")
    if d_geno.dim() != 2 or d_pheno.dim() != 1 or d_pheno.shape[0] != d_geno.shape[1]:
        raise EpiError(EPI_EINVAL, f"genotypes must be (M, N) and phenotypes (N,): got {tuple(d_geno.shape)} and "
                                   f"{tuple(d_pheno.shape)}")
    M, N = d_geno.shape
    if shape is not None and (M, N) != tuple(shape):
        raise EpiError(EPI_EINVAL, f"genotypes {M} x {N} differ from the dataset's {shape[0]} x {shape[1]}")
    if N > 1 and d_geno.stride(1) != 1:
        raise EpiError(EPI_EINVAL, "genotype rows must be contiguous (stride 1 along the individuals)")
    if M > 1 and d_geno.stride(0) < N:
        raise EpiError(EPI_EINVAL, "genotype rows overlap (row stride below N)")
    if not d_pheno.is_contiguous():
        raise EpiError(EPI_EINVAL, "phenotypes must be contiguous")
    return M, N, d_geno.stride(0) if M > 1 else N


def epi_load_genotypes(ctx, geno, pheno):
    g, p = _host_inputs(geno, pheno)
    M, N = g.shape
    out = _i32()
    _check(lib().epi_load_genotypes(ctx, _ptr(g), N, _ptr(p), M, N, ctypes.byref(out)))
    return out.value


def epi_load_genotypes_device(ctx, d_geno, d_pheno, stream=None):
    M, N, ld = _device_inputs(d_geno, d_pheno)
    out = _i32()
    _check(lib().epi_load_genotypes_device(ctx, _ptr(d_geno), ld, _ptr(d_pheno), M, N, _stream(stream),
                                           ctypes.byref(out)))
    return out.value


def epi_repack_device(ctx, dataset_id, d_geno, d_pheno, stream=None):
    info = epi_dataset_info(ctx, dataset_id)
    _, _, ld = _device_inputs(d_geno, d_pheno, (info["M"], info["N"]))
    _check(lib().epi_repack_device(ctx, dataset_id, _ptr(d_geno), ld, _ptr(d_pheno), _stream(stream)))


def epi_unload(ctx, dataset_id):
    _check(lib().epi_unload(ctx, dataset_id))


def epi_dataset_info(ctx, dataset_id):
    M, N, nc, b = _i32(), _i32(), _i32(), _u64()
    _check(lib().epi_dataset_info(ctx, dataset_id, ctypes.byref(M), ctypes.byref(N), ctypes.byref(nc),
                                  ctypes.byref(b)))
    return {"M": M.value, "N": N.value, "n_cases": nc.value, "device_bytes": b.value}


def epi_scan(ctx, dataset_id, order, top_k, stream=None):
    out = _i32()
    _check(lib().epi_scan(ctx, dataset_id, order, top_k, _stream(stream), ctypes.byref(out)))
    return out.value


def _descs(descs):
    arr = (ScanDesc * len(descs))()
    for i, d in enumerate(descs):
        arr[i] = ScanDesc(int(d[0]), int(d[1]), int(d[2]), 0)
    return arr


def epi_scan_batch(ctx, descs, stream=None):
    arr = _descs(descs)
    ids = (_i32 * len(descs))()
    _check(lib().epi_scan_batch(ctx, arr, len(descs), _stream(stream), ids))
    return list(ids)


def epi_scan_orders(ctx, dataset_id, max_order, top_k, stream=None):
    """Scans of every order 2 .. max_order in one pass; list of scan ids (order 2 first)."""
    ids = (_i32 * (max_order - 1))()
    _check(lib().epi_scan_orders(ctx, dataset_id, max_order, top_k, _stream(stream), ids))
    return list(ids)


def epi_query(ctx, scan_id):
    done = _i32()
    _check(lib().epi_query(ctx, scan_id, ctypes.byref(done)))
    return bool(done.value)


def epi_wait(ctx, scan_id):
    _check(lib().epi_wait(ctx, scan_id))


def _result_buffers(capacity, order):
    combos = np.zeros((capacity, order), np.int32)
    scores = np.zeros(capacity, np.float32)
    tables = np.zeros((capacity, 2, _cells(order)), np.uint32)
    return combos, scores, tables


def epi_results(ctx, scan_id, capacity, order, tables=True):
    """(combos (n, order) int32, scores (n,) float32, tables (n, 2, 3^order) uint32 or None)."""
    c, s, t = _result_buffers(capacity, order)
    n = _i32()
    _check(lib().epi_results(ctx, scan_id, capacity, _ptr(c), _ptr(s), _ptr(t) if tables else None,
                             ctypes.byref(n)))
    k = n.value
    return c[:k], s[:k], (t[:k] if tables else None)


def epi_scan_timing(ctx, scan_id):
    ms = (_c.c_float * 4)()
    _check(lib().epi_scan_timing(ctx, scan_id, ms))
    return list(ms)


def epi_scan_info(ctx, scan_id):
    n, v, np_ = _u64(), _i32(), _i32()
    _check(lib().epi_scan_info(ctx, scan_id, ctypes.byref(n), ctypes.byref(v), ctypes.byref(np_)))
    return {"n_combinations": n.value, "variant": v.value, "prefix_block": np_.value}


def epi_release(ctx, scan_id):
    _check(lib().epi_release(ctx, scan_id))


def epi_scan_check(ctx, dataset_id, order, top_k, stream=None):
    out = _i32()
    _check(lib().epi_scan_check(ctx, dataset_id, order, top_k, _stream(stream), ctypes.byref(out)))
    return out.value


def epi_scan_noalloc(ctx, dataset_id, order, top_k, d_combos, d_scores, d_tables, d_n, stream=None):
    """Enqueue an allocation-free scan writing into caller device tensors
    (int32 [top_k, order], float32 [top_k], uint32-sized [top_k, 2, 3^order]
    or None, int32 [1]); synchronise the stream before reading them."""
    _device_buffer(d_combos, 4, top_k * order, "combinations")
    _device_buffer(d_scores, 4, top_k, "scores")
    if d_tables is not None:
        _device_buffer(d_tables, 4, top_k * 2 * 3**order, "tables")
    _device_buffer(d_n, 4, 1, "count")
    _check(lib().epi_scan_noalloc(ctx, dataset_id, order, top_k, _stream(stream), _ptr(d_combos), _ptr(d_scores),
                                  _ptr(d_tables) if d_tables is not None else None, _ptr(d_n)))


def epi_scan_digest(ctx, scan_id):
    """(combinations scored, digest) of a finished scan from epi_scan_check."""
    n, d = _u64(), _u64()
    _check(lib().epi_scan_digest(ctx, scan_id, ctypes.byref(n), ctypes.byref(d)))
    return n.value, d.value


def epi_batch_create(ctx, descs, persistent=True, use_graph=True):
    arr = _descs(descs)
    out = _i32()
    _check(lib().epi_batch_create(ctx, arr, len(descs), int(persistent), int(use_graph), ctypes.byref(out)))
    return out.value


def epi_batch_run(ctx, batch_id, stream=None):
    _check(lib().epi_batch_run(ctx, batch_id, _stream(stream)))


def epi_batch_wait(ctx, batch_id):
    _check(lib().epi_batch_wait(ctx, batch_id))


def epi_batch_results(ctx, batch_id, index, capacity, order, tables=True):
    c, s, t = _result_buffers(capacity, order)
    n = _i32()
    _check(lib().epi_batch_results(ctx, batch_id, index, capacity, _ptr(c), _ptr(s), _ptr(t) if tables else None,
                                   ctypes.byref(n)))
    k = n.value
    return c[:k], s[:k], (t[:k] if tables else None)


def epi_batch_timing(ctx, batch_id):
    ms = _c.c_float()
    _check(lib().epi_batch_timing(ctx, batch_id, ctypes.byref(ms)))
    return ms.value


def epi_batch_destroy(ctx, batch_id):
    _check(lib().epi_batch_destroy(ctx, batch_id))


def epi_autotune(ctx, dataset_id, order):
    out = _i32()
    _check(lib().epi_autotune(ctx, dataset_id, order, ctypes.byref(out)))
    return out.value


def epi_autotune_report(ctx, dataset_id, order):
    """[(block, ns per scored combination)] of the last autotune of the order
    for the dataset's size bucket."""
    blocks = np.zeros(16, np.int32)
    ns = np.zeros(16, np.float64)
    n = _i32()
    _check(lib().epi_autotune_report(ctx, dataset_id, order, 16, _ptr(blocks), _ptr(ns), ctypes.byref(n)))
    k = min(n.value, 16)
    return [(int(b), float(t)) for b, t in zip(blocks[:k], ns[:k])]


def epi_set_prefix_block(ctx, dataset_id, order, block):
    _check(lib().epi_set_prefix_block(ctx, dataset_id, order, block))


def _device_buffer(t, itemsize, count, what):
    """Check that a torch tensor is a contiguous device buffer of at least
    count items of itemsize bytes (the library trusts the pointer it gets)."""
    if not (hasattr(t, "is_cuda") and t.is_cuda):
        raise EpiError(EPI_EINVAL, f"{what} must be a device tensor")
    if not t.is_contiguous():
        raise EpiError(EPI_EINVAL, f"{what} must be contiguous")
    if t.element_size() != itemsize or t.numel() < count:
        raise EpiError(EPI_EINVAL, f"{what} must hold {count} items of {itemsize} bytes")


def _combos_arg(d_combos):
    if d_combos.dim() != 2 or d_combos.dtype != _torch_int32():
        raise EpiError(EPI_EINVAL, "combinations must be an int32 [n, k] device tensor")
    n, k = d_combos.shape
    _device_buffer(d_combos, 4, n * k, "combinations")
    return n, k


def _torch_int32():
    import torch

    return torch.int32


def epi_genotype_tables(ctx, dataset_id, d_combos, d_rows):
    """Genotype rows of the combinations in d_combos (device int32 [n][k])
    into d_rows (device 32-bit [n][3^k][W]); returns the kernel time in ms."""
    n, k = _combos_arg(d_combos)
    info = epi_dataset_info(ctx, dataset_id)
    nc, nt = info["n_cases"], info["N"] - info["n_cases"]
    W = 4 * ((nc + 127) // 128) + 4 * ((nt + 127) // 128)
    _device_buffer(d_rows, 4, n * 3**k * W, "rows")
    ms = _c.c_float()
    _check(lib().epi_genotype_tables(ctx, dataset_id, k, _ptr(d_combos), n, _ptr(d_rows), _c.byref(ms)))
    return ms.value


def epi_contingency_tables(ctx, dataset_id, d_combos, d_tables):
    """Contingency tables (device 32-bit [n][2][3^k]) of d_combos; returns ms."""
    n, k = _combos_arg(d_combos)
    _device_buffer(d_tables, 4, n * 2 * 3**k, "tables")
    ms = _c.c_float()
    _check(lib().epi_contingency_tables(ctx, dataset_id, k, _ptr(d_combos), n, _ptr(d_tables), _c.byref(ms)))
    return ms.value


def epi_mutual_information(ctx, dataset_id, order, d_tables, d_mi):
    """MI (device float64 [n]) of n tables (device 32-bit [n][2][3^order]); returns ms."""
    n = d_tables.shape[0]
    _device_buffer(d_tables, 4, n * 2 * 3**order, "tables")
    _device_buffer(d_mi, 8, n, "mi")
    ms = _c.c_float()
    _check(lib().epi_mutual_information(ctx, dataset_id, order, _ptr(d_tables), n, _ptr(d_mi), _c.byref(ms)))
    return ms.value


def epi_server_start(ctx, max_active=64, rounds_in_flight=0, request_budget=0):
    cfg = ServerConfig(max_active, rounds_in_flight, request_budget)
    out = _i32()
    _check(lib().epi_server_start(ctx, ctypes.byref(cfg), ctypes.byref(out)))
    return out.value


def epi_server_submit(ctx, server_id, dataset_id, order, top_k):
    out = _i32()
    _check(lib().epi_server_submit(ctx, server_id, dataset_id, order, top_k, ctypes.byref(out)))
    return out.value


def epi_server_poll(ctx, server_id, request_id):
    st = _i32()
    _check(lib().epi_server_poll(ctx, server_id, request_id, ctypes.byref(st)))
    return st.value


def epi_server_results(ctx, server_id, request_id, capacity, order, tables=True):
    c, s, t = _result_buffers(capacity, order)
    n = _i32()
    lat = _c.c_double()
    _check(lib().epi_server_results(ctx, server_id, request_id, capacity, _ptr(c), _ptr(s),
                                    _ptr(t) if tables else None, ctypes.byref(n), ctypes.byref(lat)))
    k = n.value
    return c[:k], s[:k], (t[:k] if tables else None), lat.value


def epi_server_stats(ctx, server_id):
    out = (_u64 * 5)()
    _check(lib().epi_server_stats(ctx, server_id, out))
    keys = ("requests_done", "rounds", "combo_samples", "peak_request_bytes", "peak_active")
    return dict(zip(keys, list(out)))


def epi_server_stop(ctx, server_id):
    _check(lib().epi_server_stop(ctx, server_id))


# ---- convenience ------------------------------------------------------------

class Context:
    """Owns one ``epi_ctx``; methods wrap the calls above."""

    def __init__(self, device=0, hbm_budget_bytes=0):
        self.ctx = epi_create(device, hbm_budget_bytes)

    def close(self):
        if self.ctx:
            epi_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def load(self, geno, pheno):
        return epi_load_genotypes(self.ctx, geno, pheno)

    def scan(self, dataset_id, order, top_k, stream=None, tables=True):
        """Run one scan to completion; returns dict of combos, scores, tables, timing."""
        sid = epi_scan(self.ctx, dataset_id, order, top_k, stream)
        try:
            epi_wait(self.ctx, sid)
            c, s, t = epi_results(self.ctx, sid, top_k, order, tables)
            ms = epi_scan_timing(self.ctx, sid)
            info = epi_scan_info(self.ctx, sid)
        finally:
            epi_release(self.ctx, sid)
        return {"combos": c, "scores": s, "tables": t, "ms": ms, **info}
