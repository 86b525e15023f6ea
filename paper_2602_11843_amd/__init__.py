"""Truncated Neumann series S_k(A) by low-product radix kernels on MI355X.

Thin ctypes binding over ``libns.so`` (C ABI in ``include/ns.h``).  Every
step of the computation runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch supplies device memory and streams: tensors are
passed by ``data_ptr()`` and the current stream.  Importing this module fails
loudly if the library has not been built (``python -m
paper_2602_11843_amd.build``); there is no CPU fallback.
"""

import ctypes
import os
import threading
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libns.so")

# methods (enum ns_method)
NAIVE, BINARY, RADIX9, RADIX15, RADIX9_RESID, QUINARY, TERNARY, HENSEL, MIXED, RADIX15C = range(10)
METHODS = {"naive": NAIVE, "binary": BINARY, "radix9": RADIX9, "radix15": RADIX15,
           "radix9_resid": RADIX9_RESID, "quinary": QUINARY, "ternary": TERNARY,
           "hensel": HENSEL, "mixed": MIXED, "radix15c": RADIX15C}
# compute precision (enum ns_dtype)
F64, F32, SPLIT_BF16, F16_SCALED, F32_ACC64 = range(5)
DTYPES = {"f64": F64, "f32": F32, "split_bf16": SPLIT_BF16, "f16_scaled": F16_SCALED,
          "f32_acc64": F32_ACC64}
# residual-product modifiers, OR-ed into a dtype (see ns.h)
RESID_LAST = 0x100


def RESID_INT8(slices: int = 0) -> int:
    return 0x200 | (int(slices) << 12)


RESID_CRT = 0x400


def dtype_code(dtype) -> int:
    """The ns_dtype value of a dtype given as an int or as a name with
    optional residual modifiers: "split_bf16+last", "split_bf16+i8" (7
    slices), "f16_scaled+i8x5+last", "split_bf16+crt" (residues)."""
    if not isinstance(dtype, str):
        return int(dtype)
    base, *mods = dtype.split("+")
    if base not in DTYPES:
        raise ValueError(f"unknown dtype {dtype!r}")
    code = DTYPES[base]
    for m in mods:
        if m == "last":
            code |= RESID_LAST
        elif m == "i8":
            code |= RESID_INT8(0)
        elif m.startswith("i8x") and m[3:].isdigit():
            code |= RESID_INT8(int(m[3:]))
        elif m == "crt":
            code |= RESID_CRT
        else:
            raise ValueError(f"unknown residual modifier {m!r} in {dtype!r}")
    return code

MAX_LEVELS = 64


class NSError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status} ({msg})")
        self.status = status


class Report(ctypes.Structure):
    _fields_ = [
        ("k_eff", ctypes.c_int64),
        ("levels", ctypes.c_int32),
        ("gemms_performed", ctypes.c_int32),
        ("gemms_formula", ctypes.c_int32),
        ("nonfinite", ctypes.c_int32),
        ("n_internal", ctypes.c_int32),
        ("method", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("level_norm", ctypes.c_double * MAX_LEVELS),
        ("kernel_prefix_err", ctypes.c_double),
        ("spill15", ctypes.c_double),
        ("spill16", ctypes.c_double),
        ("product_launches", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {
            "k_eff": self.k_eff, "levels": self.levels,
            "gemms_performed": self.gemms_performed, "gemms_formula": self.gemms_formula,
            "nonfinite": bool(self.nonfinite), "n_internal": self.n_internal,
            "level_norm": [self.level_norm[i] for i in range(min(self.levels, MAX_LEVELS))]
            if self.method != NAIVE else [],
            "kernel_prefix_err": self.kernel_prefix_err,
            "spill15": self.spill15, "spill16": self.spill16,
            "product_launches": self.product_launches,
        }


# exported symbols and their signatures: (restype, argtypes)
_P, _I64, _I32, _D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
_SIGNATURES = {
    "ns_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int]),
    "ns_destroy": (ctypes.c_int, [_P]),
    "ns_plan": (ctypes.c_int, [_I64, ctypes.c_int, ctypes.POINTER(_I64), ctypes.POINTER(_I32),
                               ctypes.POINTER(_I32)]),
    "ns_workspace_bytes": (ctypes.c_int, [_I64, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "ns_eval": (ctypes.c_int, [_P, _I64, _I64, ctypes.c_int, ctypes.c_int, _P]),
    "ns_eval_ex": (ctypes.c_int, [_P, _P, _I64, _I64, _I64, ctypes.c_int, ctypes.c_int, _P, _I64,
                                  _P, ctypes.POINTER(Report)]),
    "ns_eval_noalloc": (ctypes.c_int, [_P, _I64, _I64, _I64, ctypes.c_int, ctypes.c_int, _P, _I64,
                                       _P, ctypes.POINTER(Report)]),
    "ns_eval_batched": (ctypes.c_int, [_P, _P, _P, _P, _P, _I32, _I64, ctypes.c_int, ctypes.c_int,
                                       _P, _P, ctypes.POINTER(Report)]),
    "ns_eval_batched_loop": (ctypes.c_int, [_P, _P, _P, _P, _I32, _I64, ctypes.c_int,
                                            ctypes.c_int, _P, _P]),
    "ns_autotune_batched": (ctypes.c_int, [_P, _P, _P, _P, _P, _I32, _I64, _P, _P,
                                           ctypes.POINTER(_I32)]),
    "ns_radix15_coeffs": (ctypes.c_int, [ctypes.POINTER(_D), ctypes.POINTER(_D),
                                         ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "ns_radix15c_coeffs": (ctypes.c_int, [ctypes.POINTER(_D), ctypes.POINTER(_D),
                                          ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "ns_set_product_timing": (ctypes.c_int, [_P, ctypes.c_int]),
    "ns_product_timing": (ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_D),
                                         ctypes.POINTER(_D), ctypes.c_int]),
    "ns_product_timing_dtype": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(_I32),
                                               ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "ns_product_timing_launches": (ctypes.c_int, [_P, _I32, ctypes.POINTER(ctypes.c_float),
                                                  ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "ns_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ns_last_error": (ctypes.c_char_p, []),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run `python -m paper_2602_11843_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(status: int, where: str):
    if status != 0:
        raise NSError(status, where, lib.ns_last_error().decode(errors="replace"))


# ---------------------------------------------------------------------------
# host-only helpers
# ---------------------------------------------------------------------------

def ns_plan(k: int, method):
    """(k_eff, levels, products) of the literal schedule."""
    m = METHODS.get(method, method)
    ke, lv, g = _I64(), _I32(), _I32()
    _check(lib.ns_plan(int(k), int(m), ctypes.byref(ke), ctypes.byref(lv), ctypes.byref(g)), "ns_plan")
    return ke.value, lv.value, g.value


def ns_workspace_bytes(n: int, method, dtype) -> int:
    b = ctypes.c_size_t()
    _check(lib.ns_workspace_bytes(int(n), int(METHODS.get(method, method)),
                                  int(dtype_code(dtype)), ctypes.byref(b)),
           "ns_workspace_bytes")
    return b.value


def ns_radix15_coeffs():
    """(28 coefficients, prefix error, a15, a16) of the library's radix-15 table."""
    c = (_D * 28)()
    pe, s15, s16 = _D(), _D(), _D()
    _check(lib.ns_radix15_coeffs(c, ctypes.byref(pe), ctypes.byref(s15), ctypes.byref(s16)),
           "ns_radix15_coeffs")
    return list(c), pe.value, s15.value, s16.value


def ns_radix15c_coeffs():
    """(28 coefficients, prefix error, a15, a16) of the contraction-aware table."""
    c = (_D * 28)()
    pe, s15, s16 = _D(), _D(), _D()
    _check(lib.ns_radix15c_coeffs(c, ctypes.byref(pe), ctypes.byref(s15), ctypes.byref(s16)),
           "ns_radix15c_coeffs")
    return list(c), pe.value, s15.value, s16.value


def ns_status_string(status: int) -> str:
    return lib.ns_status_string(int(status)).decode()


# ---------------------------------------------------------------------------
# device entry points (torch tensors for memory and streams)
# ---------------------------------------------------------------------------

class Handle:
    """Owns an ns_handle (workspace, timing, batched graphs) on one device.
    Calls on one handle must not overlap, and ctypes releases the GIL during
    a call, so every call through the handle holds its lock."""

    def __init__(self, device: int = 0):
        self.ptr = _P()
        self.lock = threading.Lock()
        _check(lib.ns_create(ctypes.byref(self.ptr), int(device)), "ns_create")
        self.device = device

    def close(self):
        if self.ptr:
            with self.lock:
                lib.ns_destroy(self.ptr)
                self.ptr = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ns_set_product_timing(self, enable: bool):
        with self.lock:
            _check(lib.ns_set_product_timing(self.ptr, int(bool(enable))), "ns_set_product_timing")

    def ns_product_timing(self, reset: bool = True):
        """(launches, summed kernel ms, summed algorithmic flops) since the last reset."""
        cnt, ms, fl = _I32(), _D(), _D()
        with self.lock:
            _check(lib.ns_product_timing(self.ptr, ctypes.byref(cnt), ctypes.byref(ms),
                                         ctypes.byref(fl), int(bool(reset))), "ns_product_timing")
        return cnt.value, ms.value, fl.value

    def ns_product_timing_launches(self):
        """[(ms, engine dtype value)] of every timed launch since the last reset, in order."""
        cnt = _I32()
        with self.lock:
            _check(lib.ns_product_timing_launches(self.ptr, 0, None, None, ctypes.byref(cnt)),
                   "ns_product_timing_launches")
            n = cnt.value
            ms = (ctypes.c_float * max(n, 1))()
            eng = (_I32 * max(n, 1))()
            _check(lib.ns_product_timing_launches(self.ptr, n, ms, eng, ctypes.byref(cnt)),
                   "ns_product_timing_launches")
        return [(ms[i], eng[i]) for i in range(n)]

    def ns_product_timing_dtype(self, dtype):
        """The same sums over one product engine's launches (named by dtype)."""
        cnt, ms, fl = _I32(), _D(), _D()
        with self.lock:
            _check(lib.ns_product_timing_dtype(self.ptr, int(dtype_code(dtype)),
                                               ctypes.byref(cnt), ctypes.byref(ms), ctypes.byref(fl)),
                   "ns_product_timing_dtype")
        return cnt.value, ms.value, fl.value


_handles = {}
_handles_lock = threading.Lock()


def default_handle(device: Optional[int] = None) -> Handle:
    import torch
    dev = torch.cuda.current_device() if device is None else device
    with _handles_lock:
        if dev not in _handles:
            _handles[dev] = Handle(dev)
        return _handles[dev]


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return _P(stream.cuda_stream)


def io_dtype(dtype):
    """torch element type of A and out for a compute precision."""
    import torch
    return torch.float32 if (dtype_code(dtype) & 0xff) == F32 else torch.float64


# Argument checks of the binding: the library receives bare pointers, so a
# tensor of the wrong element type or layout would be read as something else.
# Leading dimensions, sizes and overlap are checked again by the library.

def _cuda_tensor(name, T, dtype, device=None):
    import torch
    if not isinstance(T, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if T.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {T.dtype}")
    if not T.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if device is not None and T.device != device:
        raise ValueError(f"{name} must be on {device}, got {T.device}")


def _square(name, T, dtype, n=None, device=None, contiguous=False):
    _cuda_tensor(name, T, dtype, device)
    if T.dim() != 2 or T.shape[0] != T.shape[1] or (n is not None and T.shape[0] != n):
        raise ValueError(f"{name} must be a square matrix" + (f" of order {n}" if n is not None else ""))
    if T.stride(1) != 1 or (contiguous and not T.is_contiguous()):
        raise ValueError(f"{name} must be row-major" + (" and contiguous" if contiguous
                                                          else " with unit column stride"))


def _packed(A_packed, n_host, out_packed, offsets_dev=None, n_dev=None):
    import torch
    args = [("A_packed", A_packed, torch.float32), ("out_packed", out_packed, torch.float32),
            ("offsets_dev", offsets_dev, torch.int64), ("n_dev", n_dev, torch.int32)]
    args = [a for a in args if a[1] is not None]
    for name, T, dt in args:                       # element types first, then placement
        if not isinstance(T, torch.Tensor) or T.dtype != dt:
            raise TypeError(f"{name} must be a {dt} tensor")
    for name, T, dt in args:
        _cuda_tensor(name, T, dt, A_packed.device)
        if not T.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    if out_packed.numel() != A_packed.numel():
        raise ValueError("out_packed must have as many elements as A_packed")
    batch = len(n_host)
    for name, T in (("offsets_dev", offsets_dev), ("n_dev", n_dev)):
        if T is not None and T.numel() < batch:
            raise ValueError(f"{name} must have an entry per matrix")
    if batch and int((n_host.to(torch.int64) ** 2).sum()) > A_packed.numel():
        raise ValueError("A_packed holds fewer elements than the matrices need")


def ns_eval_ex(A, k: int, method="radix9", dtype="f64", out=None, handle: Optional[Handle] = None,
         stream=None, report: bool = False):
    """S_k(A) for a square CUDA tensor A (row-major, any leading dimension
    >= n via a 2-D stride).  Returns out (and the report dict if asked)."""
    import torch
    m = METHODS.get(method, method)
    d = dtype_code(dtype)
    _square("A", A, io_dtype(d))
    n = A.shape[0]
    if out is None:
        out = torch.empty((n, n), dtype=A.dtype, device=A.device)
    _square("out", out, A.dtype, n, A.device)
    h = handle or default_handle(A.device.index)
    rep = Report() if report else None
    with h.lock:
        _check(lib.ns_eval_ex(h.ptr, _P(A.data_ptr()), n, A.stride(0), int(k), int(m), int(d),
                              _P(out.data_ptr()), out.stride(0), _stream_ptr(stream),
                              ctypes.byref(rep) if rep is not None else None), "ns_eval_ex")
    return (out, rep.as_dict()) if report else out


NOALLOC_SCRATCH_BYTES = 64 << 20


def ns_eval_noalloc(A, k: int, method="radix9", dtype="f64", out=None, stream=None,
                    report: bool = False):
    """ns_eval_ex without a handle, on A's device, with the library's fixed
    device array as workspace (nothing is allocated by the library; `out`
    must be given by callers that cannot allocate either).  Calls that
    overlap on one GPU race on that array (see ns.h)."""
    import torch
    m = METHODS.get(method, method)
    d = dtype_code(dtype)
    _square("A", A, io_dtype(d))
    n = A.shape[0]
    if out is None:
        out = torch.empty((n, n), dtype=A.dtype, device=A.device)
    _square("out", out, A.dtype, n, A.device)
    rep = Report() if report else None
    with torch.cuda.device(A.device):
        _check(lib.ns_eval_noalloc(_P(A.data_ptr()), n, A.stride(0), int(k), int(m), int(d),
                                   _P(out.data_ptr()), out.stride(0), _stream_ptr(stream),
                                   ctypes.byref(rep) if rep is not None else None),
               "ns_eval_noalloc")
    return (out, rep.as_dict()) if report else out


def ns_eval(A, k: int, method="radix9", dtype="f64", out=None):
    """The short form (per-device default handle, null stream, lda = n)."""
    import torch
    m, d = METHODS.get(method, method), dtype_code(dtype)
    _square("A", A, io_dtype(d), contiguous=True)
    if out is None:
        out = torch.empty_like(A)
    _square("out", out, A.dtype, A.shape[0], A.device, contiguous=True)
    _check(lib.ns_eval(_P(A.data_ptr()), A.shape[0], int(k), int(m), int(d), _P(out.data_ptr())),
           "ns_eval")
    return out


def ns_eval_batched(A_packed, offsets_dev, n_dev, n_host, k: int, method="radix9", dtype="f32",
                 out_packed=None, handle: Optional[Handle] = None, stream=None,
                 report: bool = False):
    """Batched S_k over packed row-major float32 matrices (see ns.h).  The
    per-matrix n comes from n_host; n_dev is not read by the library and may
    be None."""
    import torch
    if out_packed is None:
        out_packed = torch.empty_like(A_packed)
    n_host = n_host.to(torch.int32).contiguous().cpu()
    _packed(A_packed, n_host, out_packed, offsets_dev, n_dev)
    h = handle or default_handle(A_packed.device.index)
    rep = Report() if report else None
    with h.lock:
        _check(lib.ns_eval_batched(h.ptr, _P(A_packed.data_ptr()), _P(offsets_dev.data_ptr()),
                                   _P(n_dev.data_ptr() if n_dev is not None else None),
                                   _P(n_host.data_ptr()), len(n_host), int(k),
                                   int(METHODS.get(method, method)), int(dtype_code(dtype)),
                                   _P(out_packed.data_ptr()), _stream_ptr(stream),
                                   ctypes.byref(rep) if rep is not None else None),
               "ns_eval_batched")
    return (out_packed, rep.as_dict()) if report else out_packed


def ns_eval_batched_loop(A_packed, offsets_host, n_host, k: int, method="radix9", dtype="f32",
                      out_packed=None, handle: Optional[Handle] = None, stream=None):
    """The per-matrix launch loop over the same packed layout."""
    import torch
    if out_packed is None:
        out_packed = torch.empty_like(A_packed)
    offs = offsets_host.to(torch.int64).contiguous().cpu()
    n_host = n_host.to(torch.int32).contiguous().cpu()
    _packed(A_packed, n_host, out_packed)
    if len(offs) < len(n_host):
        raise ValueError("offsets_host must have an entry per matrix")
    if len(n_host) and int((offs[:len(n_host)] + n_host.to(torch.int64) ** 2).max()) > A_packed.numel():
        raise ValueError("a matrix extends past the end of A_packed")
    h = handle or default_handle(A_packed.device.index)
    with h.lock:
        _check(lib.ns_eval_batched_loop(h.ptr, _P(A_packed.data_ptr()), _P(offs.data_ptr()),
                                        _P(n_host.data_ptr()), len(n_host), int(k),
                                        int(METHODS.get(method, method)),
                                        int(dtype_code(dtype)), _P(out_packed.data_ptr()),
                                        _stream_ptr(stream)), "ns_eval_batched_loop")
    return out_packed


def ns_autotune_batched(A_packed, offsets_dev, n_dev, n_host, k: int, out_packed,
                     handle: Optional[Handle] = None, stream=None) -> int:
    import torch
    n_host = n_host.to(torch.int32).contiguous().cpu()
    _packed(A_packed, n_host, out_packed, offsets_dev, n_dev)
    h = handle or default_handle(A_packed.device.index)
    cnt = _I32()
    with h.lock:
        _check(lib.ns_autotune_batched(h.ptr, _P(A_packed.data_ptr()), _P(offsets_dev.data_ptr()),
                                       _P(n_dev.data_ptr() if n_dev is not None else None),
                                       _P(n_host.data_ptr()), len(n_host),
                                       int(k), _P(out_packed.data_ptr()), _stream_ptr(stream),
                                       ctypes.byref(cnt)), "ns_autotune_batched")
    return cnt.value
