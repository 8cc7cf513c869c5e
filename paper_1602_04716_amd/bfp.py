"""Python binding of libbfp (include/bfp.h): argument marshalling only.

Every function named ``bfp_*`` calls the C function of the same name; all
arithmetic and layout work happens in the library's HIP kernels.  Device
buffers are torch CUDA tensors (or raw integer device addresses); ``stream``
defaults to torch's current stream on the current device.  A non-OK status
raises :class:`BfpError`.  If ``libbfp.so`` has not been built, :func:`lib`
raises: there is no other execution path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfp.so")
# launch configurations measured by the autotuner on MI355X; BFP_TUNE_FILE
# overrides the path, and an empty BFP_TUNE_FILE keeps the built-in defaults
TUNE_TABLE = os.path.join(_HERE, "tuning", "gfx950.txt")

BFP_OK = 0
BFP_E_FORMAT, BFP_E_NULL, BFP_E_ALIGN, BFP_E_OP, BFP_E_HIP = -1, -2, -3, -4, -5
BFP_E_ARG, BFP_E_BUDGET, BFP_E_CANCELLED, BFP_E_TIMEOUT, BFP_E_BUSY = -6, -8, -11, -12, -13
BFP_RNE, BFP_RZ = 0, 1
BFP_ADD, BFP_SUB, BFP_MUL, BFP_DIV = 0, 1, 2, 3
OPS = {"add": BFP_ADD, "sub": BFP_SUB, "mul": BFP_MUL, "div": BFP_DIV}


class bfp_format(ctypes.Structure):
    _fields_ = [("e", ctypes.c_uint8), ("m", ctypes.c_uint8), ("round", ctypes.c_uint8),
                ("pad", ctypes.c_uint8)]

    def __repr__(self):
        return "bfp_format(e=%d, m=%d, round=%d)" % (self.e, self.m, self.round)


class bfp_launch(ctypes.Structure):
    _fields_ = [("words_per_lane", ctypes.c_int32), ("block", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("unroll", ctypes.c_int32)]

    def __repr__(self):
        return "bfp_launch(words_per_lane=%d, block=%d, blocks_per_cu=%d, unroll=%d)" % (
            self.words_per_lane, self.block, self.blocks_per_cu, max(1, self.unroll))


class bfp_task(ctypes.Structure):
    _fields_ = [("a", ctypes.c_void_p), ("b", ctypes.c_void_p), ("c", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("f", bfp_format), ("op", ctypes.c_int32)]


class bfp_completion(ctypes.Structure):
    _fields_ = [("req_id", ctypes.c_uint64), ("result", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("_pad", ctypes.c_uint32), ("n", ctypes.c_uint64), ("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_launch_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64)]


class bfp_request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("f", bfp_format), ("a", ctypes.c_uint64), ("b", ctypes.c_uint64),
                ("n", ctypes.c_uint64), ("arrival_ns", ctypes.c_int64)]


class bfp_server_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in (
        "budget", "used", "high_water", "submitted", "admitted", "completed", "ticks", "max_tick_requests",
        "max_inflight_ticks", "deferred_budget", "pending", "inflight", "deferred_frees", "cancelled",
        "timed_out", "live_vectors", "table_slots")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for (k, _t) in self._fields_}


class BfpError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s (%d)" % (where, lib().bfp_status_string(status).decode(), status))


_lib = None

_SIGS = {
    "bfp_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "bfp_version": (ctypes.c_char_p, []),
    "bfp_format_supported": (ctypes.c_int, [bfp_format]),
    "bfp_container_bytes": (ctypes.c_size_t, [bfp_format]),
    "bfp_plane_stride_words": (ctypes.c_uint64, [ctypes.c_uint64]),
    "bfp_bitslice_bytes": (ctypes.c_size_t, [bfp_format, ctypes.c_uint64]),
    "bfp_pack": (ctypes.c_int, [bfp_format, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    "bfp_unpack": (ctypes.c_int, [bfp_format, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                  ctypes.c_void_p]),
    "bfp_binop": (ctypes.c_int, [ctypes.c_int, bfp_format, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_uint64, ctypes.c_void_p]),
    "bfp_add": (ctypes.c_int, [bfp_format, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                               ctypes.c_void_p]),
    "bfp_sub": (ctypes.c_int, [bfp_format, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                               ctypes.c_void_p]),
    "bfp_mul": (ctypes.c_int, [bfp_format, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                               ctypes.c_void_p]),
    "bfp_div": (ctypes.c_int, [bfp_format, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                               ctypes.c_void_p]),
    "bfp_chain2": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, bfp_format, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    "bfp_axpy": (ctypes.c_int, [bfp_format, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_uint64, ctypes.c_void_p]),
    "bfp_int_container_bytes": (ctypes.c_size_t, [ctypes.c_int]),
    "bfp_int_bitslice_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_uint64]),
    "bfp_int_pack": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                    ctypes.c_void_p]),
    "bfp_int_unpack": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                      ctypes.c_void_p]),
    "bfp_int_binop": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    "bfp_binop_std": (ctypes.c_int, [ctypes.c_int, bfp_format, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    "bfp_launch_get": (ctypes.c_int, [ctypes.c_int, bfp_format, ctypes.POINTER(bfp_launch)]),
    "bfp_launch_set": (ctypes.c_int, [ctypes.c_int, bfp_format, ctypes.POINTER(bfp_launch)]),
    "bfp_launch_load": (ctypes.c_int, [ctypes.c_char_p]),
    "bfp_measure_copy": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_double)]),
    "bfp_launch_save": (ctypes.c_int, [ctypes.c_char_p]),
    "bfp_layout_method_set": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "bfp_layout_method_get": (ctypes.c_int, [ctypes.c_int, ctypes.c_int]),
    "bfp_autotune_layout": (ctypes.c_int, [ctypes.c_int, bfp_format, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p,
                                           ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]),
    "bfp_chain_launch_get": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, bfp_format, ctypes.POINTER(bfp_launch)]),
    "bfp_chain_launch_set": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, bfp_format, ctypes.POINTER(bfp_launch)]),
    "bfp_int_launch_get": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(bfp_launch)]),
    "bfp_int_launch_set": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(bfp_launch)]),
    "bfp_autotune_chain": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, bfp_format, ctypes.c_uint64, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.POINTER(bfp_launch),
                                          ctypes.POINTER(ctypes.c_double)]),
    "bfp_autotune_int": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.POINTER(bfp_launch),
                                        ctypes.POINTER(ctypes.c_double)]),
    "bfp_measure_hbm": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "bfp_flush_llc": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_void_p]),
    "bfp_wave_clock": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p]),
    "bfp_gate_count": (ctypes.c_long, [ctypes.c_int, bfp_format]),
    "bfp_autotune": (ctypes.c_int, [ctypes.c_int, bfp_format, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.POINTER(bfp_launch), ctypes.POINTER(ctypes.c_double)]),
    "bfp_batch_plan_create": (ctypes.c_int, [ctypes.POINTER(bfp_task), ctypes.c_uint32,
                                             ctypes.POINTER(ctypes.c_void_p)]),
    "bfp_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "bfp_batch_run_eager": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "bfp_batch_run_per_vector": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "bfp_batch_run_per_vector_graph": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "bfp_batch_plan_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                                           ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)]),
    "bfp_batch_plan_destroy": (None, [ctypes.c_void_p]),
    "bfp_batch_run_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]),
    "bfp_server_create": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "bfp_server_put": (ctypes.c_int, [ctypes.c_void_p, bfp_format, ctypes.c_void_p, ctypes.c_uint64,
                                      ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "bfp_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, bfp_format, ctypes.c_uint64,
                                         ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]),
    "bfp_server_cancel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "bfp_server_set_queue_timeout": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "bfp_server_set_tick_limit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "bfp_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(bfp_completion), ctypes.c_uint32,
                                       ctypes.POINTER(ctypes.c_uint32)]),
    "bfp_server_wait_idle": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "bfp_server_replay": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(bfp_request), ctypes.c_uint32,
                                         ctypes.POINTER(ctypes.c_uint64)]),
    "bfp_server_set_autofree": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "bfp_server_view": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_uint64)]),
    "bfp_server_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, bfp_format, ctypes.c_void_p,
                                      ctypes.c_void_p]),
    "bfp_server_free": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "bfp_server_stats_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(bfp_server_stats)]),
    "bfp_server_destroy": (None, [ctypes.c_void_p]),
}


def lib():
    """Load libbfp.so; raise if it is not built.

    torch is imported first when it is installed: PyTorch for ROCm ships its
    own HIP runtime, and libbfp.so must bind to that one.  Loaded the other
    way round, the process ends up with two HIP runtimes (the system one for
    libbfp.so, torch's for the tensors and streams passed to it), and the
    library's allocations and launches fail."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libbfp.so is not built (python -m paper_1602_04716_amd.build)")
        try:
            import torch  # noqa: F401  (binds the HIP runtime before libbfp.so loads)
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        table = os.environ.get("BFP_TUNE_FILE", TUNE_TABLE)
        if table and os.path.exists(table):
            _check(L.bfp_launch_load(table.encode()), "bfp_launch_load")
    return _lib


def declared_functions():
    return sorted(_SIGS)


def fmt(e: int, m: int, round: int = BFP_RNE) -> bfp_format:
    return bfp_format(e, m, round, 0)


def _op(op) -> int:
    return OPS[op] if isinstance(op, str) else int(op)


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    if not x.is_cuda:
        raise ValueError("expected a device tensor")
    if not x.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return x.data_ptr()


def _stream(s) -> int:
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _check(st: int, where: str):
    if st != BFP_OK:
        raise BfpError(st, where)


# ---- the C functions, same names -----------------------------------------
def bfp_status_string(s: int) -> str:
    return lib().bfp_status_string(s).decode()


def bfp_version() -> str:
    return lib().bfp_version().decode()


def bfp_format_supported(f: bfp_format) -> bool:
    return bool(lib().bfp_format_supported(f))


def bfp_container_bytes(f: bfp_format) -> int:
    return int(lib().bfp_container_bytes(f))


def bfp_plane_stride_words(n: int) -> int:
    return int(lib().bfp_plane_stride_words(n))


def bfp_bitslice_bytes(f: bfp_format, n: int) -> int:
    return int(lib().bfp_bitslice_bytes(f, n))


def bfp_pack(f, std_in, bs_out, n: int, stream=None):
    _check(lib().bfp_pack(f, _ptr(std_in), _ptr(bs_out), n, _stream(stream)), "bfp_pack")


def bfp_unpack(f, bs_in, std_out, n: int, stream=None):
    _check(lib().bfp_unpack(f, _ptr(bs_in), _ptr(std_out), n, _stream(stream)), "bfp_unpack")


def bfp_binop(op, f, a, b, c, n: int, stream=None):
    _check(lib().bfp_binop(_op(op), f, _ptr(a), _ptr(b), _ptr(c), n, _stream(stream)), "bfp_binop")


def bfp_add(f, a, b, c, n: int, stream=None):
    _check(lib().bfp_add(f, _ptr(a), _ptr(b), _ptr(c), n, _stream(stream)), "bfp_add")


def bfp_sub(f, a, b, c, n: int, stream=None):
    _check(lib().bfp_sub(f, _ptr(a), _ptr(b), _ptr(c), n, _stream(stream)), "bfp_sub")


def bfp_mul(f, a, b, c, n: int, stream=None):
    _check(lib().bfp_mul(f, _ptr(a), _ptr(b), _ptr(c), n, _stream(stream)), "bfp_mul")


def bfp_div(f, a, b, c, n: int, stream=None):
    _check(lib().bfp_div(f, _ptr(a), _ptr(b), _ptr(c), n, _stream(stream)), "bfp_div")


def bfp_chain2(op1, op2, f, a, b, c, d, n: int, stream=None):
    _check(lib().bfp_chain2(_op(op1), _op(op2), f, _ptr(a), _ptr(b), _ptr(c), _ptr(d), n, _stream(stream)),
           "bfp_chain2")


def bfp_axpy(f, alpha: int, x, y, d, n: int, stream=None):
    _check(lib().bfp_axpy(f, int(alpha), _ptr(x), _ptr(y), _ptr(d), n, _stream(stream)), "bfp_axpy")


INT_KINDS = {"wrap": 0, "satu": 1, "sats": 2}


def _kind(kind) -> int:
    return INT_KINDS[kind] if isinstance(kind, str) else int(kind)


def bfp_int_container_bytes(k: int) -> int:
    return int(lib().bfp_int_container_bytes(k))


def bfp_int_bitslice_bytes(k: int, n: int) -> int:
    return int(lib().bfp_int_bitslice_bytes(k, n))


def bfp_int_pack(k: int, std, bs, n: int, stream=None):
    _check(lib().bfp_int_pack(k, _ptr(std), _ptr(bs), n, _stream(stream)), "bfp_int_pack")


def bfp_int_unpack(k: int, bs, std, n: int, stream=None):
    _check(lib().bfp_int_unpack(k, _ptr(bs), _ptr(std), n, _stream(stream)), "bfp_int_unpack")


def bfp_int_binop(op, k: int, kind, a, b, c, n: int, stream=None):
    _check(lib().bfp_int_binop(_op(op), k, _kind(kind), _ptr(a), _ptr(b), _ptr(c), n, _stream(stream)),
           "bfp_int_binop")


def int_container_dtype(k: int):
    import torch
    return {1: torch.uint8, 2: torch.uint16, 4: torch.uint32}[1 if k <= 8 else (2 if k <= 16 else 4)]


def int_empty_bitslice(k: int, n: int, device="cuda"):
    """Uninitialised k-bit integer bitslice vector: (k, G_pad) uint32 planes."""
    import torch
    return torch.empty((k, bfp_plane_stride_words(n)), dtype=torch.uint32, device=device)


def int_pack(k: int, std, stream=None):
    out = int_empty_bitslice(k, std.numel(), std.device)
    bfp_int_pack(k, std, out, std.numel(), stream)
    return out


def int_unpack(k: int, bs, n: int, stream=None):
    import torch
    out = torch.empty(n, dtype=int_container_dtype(k), device=bs.device)
    bfp_int_unpack(k, bs, out, n, stream)
    return out


def bfp_binop_std(op, f, a, b, c, n: int, stream=None):
    _check(lib().bfp_binop_std(_op(op), f, _ptr(a), _ptr(b), _ptr(c), n, _stream(stream)), "bfp_binop_std")


def bfp_launch_get(op, f) -> bfp_launch:
    out = bfp_launch()
    _check(lib().bfp_launch_get(_op(op), f, ctypes.byref(out)), "bfp_launch_get")
    return out


def bfp_launch_set(op, f, words_per_lane: int, block: int, blocks_per_cu: int, unroll: int = 1):
    cfg = bfp_launch(words_per_lane, block, blocks_per_cu, unroll)
    _check(lib().bfp_launch_set(_op(op), f, ctypes.byref(cfg)), "bfp_launch_set")


BFP_TRANSPOSE_LANE, BFP_TRANSPOSE_XLANE = 0, 1
_DIRECTIONS = {"pack": 0, "unpack": 1}


def _dir(d) -> int:
    return _DIRECTIONS[d] if isinstance(d, str) else int(d)


def bfp_layout_method_set(direction, cbytes: int, method: int):
    _check(lib().bfp_layout_method_set(_dir(direction), cbytes, method), "bfp_layout_method_set")


def bfp_layout_method_get(direction, cbytes: int) -> int:
    r = lib().bfp_layout_method_get(_dir(direction), cbytes)
    _check(r if r < 0 else BFP_OK, "bfp_layout_method_get")
    return r


def bfp_autotune_layout(direction, f, n_probe: int = 1 << 24, reps: int = 5, stream=None):
    """Returns (best method, median microseconds); installs the best."""
    m, us = ctypes.c_int(), ctypes.c_double()
    _check(lib().bfp_autotune_layout(_dir(direction), f, n_probe, reps, _stream(stream), ctypes.byref(m),
                                     ctypes.byref(us)), "bfp_autotune_layout")
    return m.value, us.value


def bfp_chain_launch_get(op1, op2, f) -> bfp_launch:
    out = bfp_launch()
    _check(lib().bfp_chain_launch_get(_op(op1), _op(op2), f, ctypes.byref(out)), "bfp_chain_launch_get")
    return out


def bfp_chain_launch_set(op1, op2, f, block: int, blocks_per_cu: int):
    cfg = bfp_launch(1, block, blocks_per_cu, 1)
    _check(lib().bfp_chain_launch_set(_op(op1), _op(op2), f, ctypes.byref(cfg)), "bfp_chain_launch_set")


def bfp_int_launch_get(op, k: int, kind) -> bfp_launch:
    out = bfp_launch()
    _check(lib().bfp_int_launch_get(_op(op), k, _kind(kind), ctypes.byref(out)), "bfp_int_launch_get")
    return out


def bfp_int_launch_set(op, k: int, kind, block: int, blocks_per_cu: int):
    cur = bfp_int_launch_get(op, k, kind)
    cfg = bfp_launch(cur.words_per_lane, block, blocks_per_cu, 1)
    _check(lib().bfp_int_launch_set(_op(op), k, _kind(kind), ctypes.byref(cfg)), "bfp_int_launch_set")


def bfp_autotune_chain(op1, op2, f, n_probe: int = 1 << 24, reps: int = 7, stream=None):
    best, us = bfp_launch(), ctypes.c_double()
    _check(lib().bfp_autotune_chain(_op(op1), _op(op2), f, n_probe, reps, _stream(stream), ctypes.byref(best),
                                    ctypes.byref(us)), "bfp_autotune_chain")
    return best, us.value


def bfp_autotune_int(op, k: int, kind, n_probe: int = 1 << 24, reps: int = 7, stream=None):
    best, us = bfp_launch(), ctypes.c_double()
    _check(lib().bfp_autotune_int(_op(op), k, _kind(kind), n_probe, reps, _stream(stream), ctypes.byref(best),
                                  ctypes.byref(us)), "bfp_autotune_int")
    return best, us.value


def bfp_measure_copy(nbytes: int, reps: int = 10, stream=None) -> float:
    """Read + write GB/s of a plain 16-byte-vector device copy of nbytes."""
    g = ctypes.c_double()
    _check(lib().bfp_measure_copy(nbytes, reps, _stream(stream), ctypes.byref(g)), "bfp_measure_copy")
    return g.value


def bfp_measure_hbm(nbytes: int, mode: str, reps: int = 10, stream=None) -> dict:
    """Best read / write / copy / two-reads-one-write rate (GB/s, all bytes
    moved) over the probe's launch shapes."""
    g = ctypes.c_double()
    grid, block, unroll = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    m = {"read": 0, "write": 1, "copy": 2, "read2_write1": 3}[mode]
    _check(lib().bfp_measure_hbm(nbytes, m, reps, _stream(stream), ctypes.byref(g), ctypes.byref(grid),
                                 ctypes.byref(block), ctypes.byref(unroll)), "bfp_measure_hbm")
    return {"GB/s": g.value, "grid": grid.value, "block": block.value, "in_flight": unroll.value}


def bfp_flush_llc(nbytes: int = 1 << 30, stream=None):
    _check(lib().bfp_flush_llc(nbytes, _stream(stream)), "bfp_flush_llc")


def bfp_wave_clock(iters: int = 400000, stream=None):
    """Enqueue the one-wave calibration kernel (a dependent chain of `iters`
    fused multiply-adds) on `stream`."""
    _check(lib().bfp_wave_clock(iters, _stream(stream)), "bfp_wave_clock")


def bfp_launch_load(path: str):
    _check(lib().bfp_launch_load(path.encode()), "bfp_launch_load")


def bfp_launch_save(path: str):
    _check(lib().bfp_launch_save(path.encode()), "bfp_launch_save")


def bfp_autotune(op, f, n_probe: int = 1 << 24, words_per_lane_mask: int = 7, reps: int = 7, stream=None):
    """Returns (best bfp_launch, median microseconds); installs the best."""
    best = bfp_launch()
    us = ctypes.c_double()
    _check(lib().bfp_autotune(_op(op), f, n_probe, words_per_lane_mask, reps, _stream(stream), ctypes.byref(best),
                              ctypes.byref(us)), "bfp_autotune")
    return best, us.value


def bfp_gate_count(op, f) -> int:
    return int(lib().bfp_gate_count(_op(op), f))


def bfp_batch_plan_create(tasks) -> int:
    """tasks: sequence of (a, b, c, n, format, op); returns the plan handle."""
    arr = (bfp_task * len(tasks))()
    for i, (a, b, c, n, f, op) in enumerate(tasks):
        arr[i] = bfp_task(_ptr(a), _ptr(b), _ptr(c), n, f, _op(op))
    h = ctypes.c_void_p()
    _check(lib().bfp_batch_plan_create(arr, len(tasks), ctypes.byref(h)), "bfp_batch_plan_create")
    return h.value


def task_table(tasks, device="cuda"):
    """A device array of bfp_task for bfp_batch_run_noalloc: tasks as for
    bfp_batch_plan_create, (a, b, c, n, format, op)."""
    import torch
    arr = (bfp_task * len(tasks))()
    for i, (a, b, c, n, f, op) in enumerate(tasks):
        arr[i] = bfp_task(_ptr(a), _ptr(b), _ptr(c), n, f, _op(op))
    host = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8)
    return host.to(device)


def bfp_batch_run_noalloc(tasks_dev, count: int, status_dev, stream=None):
    """Run `count` tasks from a device task table (task_table) without any
    allocation; the check's status lands in status_dev (a device int32)."""
    _check(lib().bfp_batch_run_noalloc(_ptr(tasks_dev), count, _ptr(status_dev), _stream(stream)),
           "bfp_batch_run_noalloc")


def bfp_batch_run(plan: int, stream=None):
    _check(lib().bfp_batch_run(plan, _stream(stream)), "bfp_batch_run")


def bfp_batch_run_eager(plan: int, stream=None):
    _check(lib().bfp_batch_run_eager(plan, _stream(stream)), "bfp_batch_run_eager")


def bfp_batch_run_per_vector(plan: int, stream=None):
    _check(lib().bfp_batch_run_per_vector(plan, _stream(stream)), "bfp_batch_run_per_vector")


def bfp_batch_run_per_vector_graph(plan: int, stream=None):
    _check(lib().bfp_batch_run_per_vector_graph(plan, _stream(stream)), "bfp_batch_run_per_vector_graph")


def bfp_batch_plan_info(plan: int):
    nch, grid, words = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
    _check(lib().bfp_batch_plan_info(plan, ctypes.byref(nch), ctypes.byref(grid), ctypes.byref(words)),
           "bfp_batch_plan_info")
    return {"chunks": nch.value, "grid": grid.value, "words_per_operand": words.value}


def bfp_batch_plan_destroy(plan: int):
    lib().bfp_batch_plan_destroy(plan)


class BatchPlan:
    """Owns a plan and keeps the task tensors alive while it exists."""

    def __init__(self, tasks):
        self._keep = [(a, b, c) for (a, b, c, *_r) in tasks]
        self.handle = bfp_batch_plan_create(tasks)

    def run(self, stream=None):
        bfp_batch_run(self.handle, stream)

    def run_eager(self, stream=None):
        bfp_batch_run_eager(self.handle, stream)

    def run_per_vector(self, stream=None):
        bfp_batch_run_per_vector(self.handle, stream)

    def run_per_vector_graph(self, stream=None):
        bfp_batch_run_per_vector_graph(self.handle, stream)

    def info(self):
        return bfp_batch_plan_info(self.handle)

    def close(self):
        if self.handle:
            bfp_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bfp_server_create(budget_bytes: int, slots: int) -> int:
    h = ctypes.c_void_p()
    _check(lib().bfp_server_create(budget_bytes, slots, ctypes.byref(h)), "bfp_server_create")
    return h.value


def bfp_server_put(server: int, f, std_dev, n: int, stream=None) -> int:
    h = ctypes.c_uint64()
    _check(lib().bfp_server_put(server, f, _ptr(std_dev), n, _stream(stream), ctypes.byref(h)), "bfp_server_put")
    return h.value


def bfp_server_submit(server: int, op, f, a: int, b: int, n: int) -> int:
    rid = ctypes.c_uint64()
    _check(lib().bfp_server_submit(server, _op(op), f, a, b, n, ctypes.byref(rid)), "bfp_server_submit")
    return rid.value


def bfp_server_cancel(server: int, req_id: int):
    _check(lib().bfp_server_cancel(server, req_id), "bfp_server_cancel")


def bfp_server_set_tick_limit(server: int, max_bytes: int):
    _check(lib().bfp_server_set_tick_limit(server, max_bytes), "bfp_server_set_tick_limit")


def bfp_server_set_queue_timeout(server: int, timeout_ns: int):
    _check(lib().bfp_server_set_queue_timeout(server, timeout_ns), "bfp_server_set_queue_timeout")


def bfp_server_poll(server: int, max_items: int = 4096):
    buf = (bfp_completion * max_items)()
    cnt = ctypes.c_uint32()
    _check(lib().bfp_server_poll(server, buf, max_items, ctypes.byref(cnt)), "bfp_server_poll")
    return [buf[i] for i in range(cnt.value)]


def bfp_server_replay(server: int, reqs) -> int:
    """reqs: sequence of (op, format, a, b, n, arrival_ns); returns the first id."""
    arr = (bfp_request * len(reqs))()
    for i, (op, f, a, b, n, t) in enumerate(reqs):
        arr[i] = bfp_request(_op(op), f, a, b, n, int(t))
    first = ctypes.c_uint64()
    _check(lib().bfp_server_replay(server, arr, len(reqs), ctypes.byref(first)), "bfp_server_replay")
    return first.value


def bfp_server_set_autofree(server: int, on: bool):
    _check(lib().bfp_server_set_autofree(server, 1 if on else 0), "bfp_server_set_autofree")


def bfp_server_wait_idle(server: int, timeout_ms: int = 60000):
    _check(lib().bfp_server_wait_idle(server, timeout_ms), "bfp_server_wait_idle")


def bfp_server_view(server: int, handle: int):
    p, n = ctypes.c_void_p(), ctypes.c_uint64()
    _check(lib().bfp_server_view(server, handle, ctypes.byref(p), ctypes.byref(n)), "bfp_server_view")
    return p.value, n.value


def bfp_server_get(server: int, handle: int, f, std_dev_out, stream=None):
    _check(lib().bfp_server_get(server, handle, f, _ptr(std_dev_out), _stream(stream)), "bfp_server_get")


def bfp_server_free(server: int, handle: int):
    _check(lib().bfp_server_free(server, handle), "bfp_server_free")


def bfp_server_stats_get(server: int) -> dict:
    st = bfp_server_stats()
    _check(lib().bfp_server_stats_get(server, ctypes.byref(st)), "bfp_server_stats_get")
    return st.as_dict()


def bfp_server_destroy(server: int):
    lib().bfp_server_destroy(server)


# ---- conveniences over torch tensors ----------------------------------------
def container_dtype(f: bfp_format):
    import torch
    return {1: torch.uint8, 2: torch.uint16, 4: torch.uint32, 8: torch.uint64}[bfp_container_bytes(f)]


def empty_bitslice(f: bfp_format, n: int, device="cuda"):
    """Uninitialised bitslice vector: (B, G_pad) uint32 planes."""
    import torch
    B = 1 + f.e + f.m
    return torch.empty((B, bfp_plane_stride_words(n)), dtype=torch.uint32, device=device)


def pack(f: bfp_format, std, stream=None):
    out = empty_bitslice(f, std.numel(), std.device)
    bfp_pack(f, std, out, std.numel(), stream)
    return out


def unpack(f: bfp_format, bs, n: int, stream=None):
    import torch
    out = torch.empty(n, dtype=container_dtype(f), device=bs.device)
    bfp_unpack(f, bs, out, n, stream)
    return out
