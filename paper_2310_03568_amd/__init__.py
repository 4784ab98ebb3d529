"""Python binding of libpcad: forward and reverse-mode adjoint of reduce,
inclusive scan and reduce-by-index on AMD Instinct MI355X (gfx950).

Every step runs in the HIP kernels of ``libpcad.so``; this module only
marshals torch tensors (device memory and streams) into the C-ABI calls of
``include/pcad.h``.  There is no CPU fallback: if the library is missing or
no GPU is present, calls raise.

Low level: ``pcad_*`` attributes are the C functions themselves (ctypes),
with the same names and arguments as the header.

High level (torch tensors on a ROCm device, float32 / int32, contiguous):
  reduce_fwd / reduce_vjp, scan_fwd / scan_vjp, rbi_fwd / rbi_vjp
and the autograd wrappers in ``paper_2310_03568_amd.autograd``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcad.so")

OPS = {"add": 0, "mul": 1, "min": 2, "max": 3, "linrec": 4, "mat2": 5, "sumprod": 6, "satadd": 7}
# floats per element of the values and of the results (sumprod: scalar values,
# scalar results -- the p of the lifted pair)
DIM = {"add": 1, "mul": 1, "min": 1, "max": 1, "linrec": 2, "mat2": 4, "sumprod": 1, "satadd": 1}
REDUCE, SCAN, RBI = 0, 1, 2
ACCUMULATE = 1

_lib = None


class PcadError(RuntimeError):
    pass


def lib():
    """The loaded libpcad (ctypes.CDLL).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PcadError(f"{LIB_PATH} is missing: build it with "
                            "`python -m paper_2310_03568_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I, I64, U, SZ = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint,
                            ctypes.c_size_t)
        PSZ = ctypes.POINTER(ctypes.c_size_t)
        sig = {
            "pcad_status_string": ([I], ctypes.c_char_p),
            "pcad_last_hip_error": ([], I),
            "pcad_version": ([], ctypes.c_char_p),
            "pcad_ws_status": ([P, I, P], I),
            "pcad_query": ([I, I, I64, I64, I64, U, PSZ, PSZ], I),
            "pcad_reduce_fwd": ([I, I64, I64, P, P, P, P, U, P, SZ, P], I),
            "pcad_reduce_vjp": ([I, I64, I64, P, P, P, P, P, P, U, P, SZ, P], I),
            "pcad_scan_fwd": ([I, I64, I64, P, P, P, P, P, U, P, SZ, P], I),
            "pcad_scan_vjp": ([I, I64, I64, P, P, P, P, P, P, P, U, P, SZ, P], I),
            "pcad_scan_vjp_checkpoint": ([I, I64, I64, P, P, P, P, P, P, P, P, U, P, SZ, P], I),
            "pcad_scan_vjp_noalloc": ([I, I64, I64, P, P, P, P, P, P, P, U, P], I),
            "pcad_rbi_fwd": ([I, I64, I64, I64, P, P, P, P, U, P, SZ, P], I),
            "pcad_rbi_vjp": ([I, I64, I64, I64, P, P, P, P, P, U, P, SZ, P], I),
            "pcad_plan_create": ([ctypes.POINTER(P), I64, P, I64, U], I),
            "pcad_plan_query": ([P, PSZ, PSZ, ctypes.POINTER(I64), ctypes.POINTER(I64)], I),
            "pcad_plan_bind": ([P, P, P, P, P, P, P, P, P, P, P, P, P, SZ, P], I),
            "pcad_plan_run": ([P, I, P], I),
            "pcad_plan_run_per_segment": ([P, I, P], I),
            "pcad_plan_destroy": ([P], None),
            "pcad_plan_last_hip_error": ([], I),
            "pcad_vquery": ([I, I, I64, I64, I64, I64, U, PSZ, PSZ, PSZ], I),
            "pcad_vreduce_fwd": ([I, I64, I64, I64, P, P, P, U, P, SZ, P, SZ, P], I),
            "pcad_vreduce_vjp": ([I, I64, I64, I64, P, P, P, P, U, P, SZ, P, SZ, P], I),
            "pcad_vscan_fwd": ([I, I64, I64, I64, P, P, P, U, P, SZ, P, SZ, P], I),
            "pcad_vscan_vjp": ([I, I64, I64, I64, P, P, P, P, U, P, SZ, P, SZ, P], I),
            "pcad_vrbi_fwd": ([I, I64, I64, I64, I64, P, P, P, P, U, P, SZ, P, SZ, P], I),
            "pcad_vrbi_vjp": ([I, I64, I64, I64, I64, P, P, P, P, P, U, P, SZ, P, SZ, P], I),
            "pcad_bds_query": ([I, I64, I64, I64, U, PSZ, PSZ, PSZ, PSZ], I),
            "pcad_bds_scan_fwd": ([I, I64, I64, I64, P, P, P, U, P, SZ, P, SZ, P], I),
            "pcad_bds_scan_vjp": ([I, I64, I64, I64, P, P, P, P, U, P, SZ, P, SZ, P], I),
            "pcad_matd_query": ([I, I64, I64, U, PSZ, PSZ], I),
            "pcad_matd_scan_fwd": ([I, I64, I64, P, P, P, U, P, SZ, P], I),
            "pcad_matd_scan_vjp": ([I, I64, I64, P, P, P, P, U, P, SZ, P], I),
            "pcad_matd_reduce_fwd": ([I, I64, I64, P, P, P, U, P, SZ, P], I),
            "pcad_matd_reduce_vjp": ([I, I64, I64, P, P, P, P, U, P, SZ, P], I),
            "pcad_i32_query": ([I, I, I64, I64, I64, PSZ], I),
            "pcad_i32_fwd": ([I, I, I64, I64, I64, P, P, P, P, SZ, P], I),
            "pcad_knob_count": ([], I),
            "pcad_knob_name": ([I], ctypes.c_char_p),
            "pcad_knob_get": ([ctypes.c_char_p, ctypes.POINTER(I64)], I),
            "pcad_knob_set": ([ctypes.c_char_p, I64], I),
            "pcad_knob_reset": ([], None),
            "pcad_stream_copy": ([P, P, SZ, P], I),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def __getattr__(name):
    if name.startswith("pcad_"):
        return getattr(lib(), name)
    raise AttributeError(name)


# PCAD_SYNC_CHECK=1: after every call, synchronise its stream and raise if a
# look-back wait of that call timed out (pcad_ws_status); off by default
# because it costs a host round trip per call
SYNC_CHECK = os.environ.get("PCAD_SYNC_CHECK", "0") == "1"
E_TIMEOUT = 8


def check(status: int, what: str = "", ws: Optional[torch.Tensor] = None):
    if status != 0:
        L = lib()
        msg = L.pcad_status_string(status).decode()
        hip = L.pcad_last_hip_error()
        raise PcadError(f"{what}: {msg} (status {status}, hip error {hip})")
    if SYNC_CHECK and ws is not None:
        ws_status(ws, what=what)


def ws_status(ws: torch.Tensor, clear: bool = True, what: str = "") -> int:
    """Status of the calls on workspace ``ws`` (synchronises its device's
    current stream): raises PcadError if a look-back wait timed out, which
    invalidates that call's results; clears the report when ``clear``."""
    st = lib().pcad_ws_status(_ptr(ws), 1 if clear else 0, _stream(ws.device))
    if st == E_TIMEOUT:
        raise PcadError(f"{what or 'pcad'}: {lib().pcad_status_string(st).decode()}")
    check(st, "pcad_ws_status")
    return st


def ws_status_all(clear: bool = True) -> int:
    """ws_status over every cached workspace; 0 when none reports a timeout."""
    for buf in list(_ws.values()):
        ws_status(buf, clear)
    return 0


# ---------------------------------------------------------------------------
# tuning knobs (launch parameters; results do not depend on them)
# ---------------------------------------------------------------------------
def knobs() -> dict:
    """Current value of every tuning knob, by name."""
    L = lib()
    out = {}
    for i in range(L.pcad_knob_count()):
        name = L.pcad_knob_name(i)
        v = ctypes.c_int64(0)
        check(L.pcad_knob_get(name, ctypes.byref(v)), "pcad_knob_get")
        out[name.decode()] = v.value
    return out


def set_knob(name: str, value: int):
    check(lib().pcad_knob_set(name.encode(), int(value)), f"pcad_knob_set({name}={value})")


def reset_knobs():
    lib().pcad_knob_reset()


def stream_copy(dst: torch.Tensor, src: torch.Tensor):
    """dst <- src byte for byte with the library's streaming copy (both
    contiguous device tensors of the same byte size, 16-byte aligned)."""
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise PcadError("stream_copy: contiguous device tensors required")
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise PcadError("stream_copy: byte sizes differ")
    check(lib().pcad_stream_copy(_ptr(src), _ptr(dst), nb, _stream(src.device)),
          "pcad_stream_copy")
    return dst


# ---------------------------------------------------------------------------
# workspace: one zero-initialised buffer per (device, stream), grown on demand
# ---------------------------------------------------------------------------
_ws = {}


def workspace(nbytes: int, device: torch.device, stream=None) -> torch.Tensor:
    stream = stream if stream is not None else torch.cuda.current_stream(device)
    key = (device.index, stream.cuda_stream)
    buf = _ws.get(key)
    if buf is None or buf.numel() < nbytes:
        size = max(int(nbytes), 4096)
        size = 1 << (size - 1).bit_length()
        buf = torch.zeros(size, dtype=torch.uint8, device=device)
        _ws[key] = buf
    return buf


def query(comb: int, op: str, batch: int, n: int, m: int = 0):
    s = ctypes.c_size_t(0)
    w = ctypes.c_size_t(0)
    check(lib().pcad_query(comb, OPS[op], batch, n, m, 0, ctypes.byref(s), ctypes.byref(w)),
          "pcad_query")
    return s.value, w.value


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


def _dev_check(*ts):
    for t in ts:
        if t is None:
            continue
        if not t.is_cuda:
            raise PcadError("pcad needs device tensors (no CPU path)")
        if not t.is_contiguous():
            raise PcadError("pcad needs contiguous tensors")


def _shape(op: str, x: torch.Tensor):
    """(batch, n) of a value tensor: (..., n) for scalar ops and linrec,
    (..., n, 4) for mat2."""
    if op == "mat2":
        if x.shape[-1] != 4:
            raise PcadError("mat2 expects a trailing dimension of 4")
        lead = x.shape[:-1]
    else:
        lead = x.shape
    n = lead[-1] if len(lead) else 1
    batch = 1
    for d in lead[:-1]:
        batch *= d
    return batch, n, tuple(lead[:-1])


# ---------------------------------------------------------------------------
# reduce
# ---------------------------------------------------------------------------
def reduce_fwd(op: str, x0: torch.Tensor, x1: Optional[torch.Tensor] = None):
    """Returns (y, saved).  y has shape lead + (d,) for linrec/mat2 (linrec:
    (A, y) of the composed linear function), lead otherwise."""
    _dev_check(x0, x1)
    batch, n, lead = _shape(op, x0)
    d = DIM[op]
    s_b, w_b = query(REDUCE, op, batch, n)
    dev = x0.device
    y = torch.empty(lead + ((d,) if d > 1 else ()), dtype=torch.float32, device=dev)
    saved = torch.empty(max(s_b, 16), dtype=torch.uint8, device=dev)
    ws = workspace(w_b, dev)
    check(lib().pcad_reduce_fwd(OPS[op], batch, n, _ptr(x0), _ptr(x1), _ptr(y), _ptr(saved), 0,
                                _ptr(ws), ws.numel(), _stream(dev)), "pcad_reduce_fwd", ws=ws)
    return y, saved


def reduce_vjp(op: str, x0, x1, saved, ybar, out=None, accumulate: bool = False):
    _dev_check(x0, x1, ybar)
    batch, n, lead = _shape(op, x0)
    s_b, w_b = query(REDUCE, op, batch, n)
    dev = x0.device
    if out is None:
        out = (torch.empty_like(x0), torch.empty_like(x1)) if op == "linrec" else (torch.empty_like(x0),)
    ws = workspace(w_b, dev)
    check(lib().pcad_reduce_vjp(OPS[op], batch, n, _ptr(x0), _ptr(x1), _ptr(saved),
                                _ptr(ybar.contiguous()), _ptr(out[0]),
                                _ptr(out[1]) if len(out) > 1 else None,
                                ACCUMULATE if accumulate else 0, _ptr(ws), ws.numel(),
                                _stream(dev)), "pcad_reduce_vjp", ws=ws)
    return out if op == "linrec" else out[0]


# ---------------------------------------------------------------------------
# scan
# ---------------------------------------------------------------------------
def scan_fwd(op: str, x0: torch.Tensor, x1: Optional[torch.Tensor] = None, want_A: bool = False,
             keep_saved: bool = True):
    """Returns (y, A, saved); A is the linrec cumulative multiplier when
    ``want_A`` (else None); saved (the tile prefixes) is None unless
    ``keep_saved`` (the checkpoint adjoint does not read it)."""
    _dev_check(x0, x1)
    batch, n, lead = _shape(op, x0)
    s_b, w_b = query(SCAN, op, batch, n)
    dev = x0.device
    y = torch.empty_like(x0)
    A = torch.empty_like(x0) if (op == "linrec" and want_A) else None
    saved = torch.empty(max(s_b, 16), dtype=torch.uint8, device=dev) if keep_saved else None
    ws = workspace(w_b, dev)
    check(lib().pcad_scan_fwd(OPS[op], batch, n, _ptr(x0), _ptr(x1), _ptr(y), _ptr(A),
                              _ptr(saved), 0, _ptr(ws), ws.numel(), _stream(dev)),
          "pcad_scan_fwd", ws=ws)
    return y, A, saved


def scan_vjp(op: str, x0, x1, saved, ybar, Abar=None, out=None, accumulate: bool = False):
    """Adjoint of the scan.  Returns a_bar, b_bar for linrec, else x_bar."""
    _dev_check(x0, x1, ybar, Abar)
    batch, n, lead = _shape(op, x0)
    s_b, w_b = query(SCAN, op, batch, n)
    dev = x0.device
    if out is None:
        out = (torch.empty_like(x0), torch.empty_like(x1)) if op == "linrec" else (torch.empty_like(x0),)
    ws = workspace(w_b, dev)
    check(lib().pcad_scan_vjp(OPS[op], batch, n, _ptr(x0), _ptr(x1), _ptr(saved), _ptr(ybar),
                              _ptr(Abar), _ptr(out[0]), _ptr(out[1]) if len(out) > 1 else None,
                              ACCUMULATE if accumulate else 0, _ptr(ws), ws.numel(),
                              _stream(dev)), "pcad_scan_vjp", ws=ws)
    return out if op == "linrec" else out[0]


def scan_vjp_checkpoint(op: str, x0, x1, y0, y1, ybar, Abar=None, out=None,
                        accumulate: bool = False):
    """Adjoint of the scan reading the forward outputs (y0; linrec: y and,
    with Abar, A) instead of recomputing prefixes.  x1 (linrec b) may be None."""
    _dev_check(x0, x1, y0, y1, ybar, Abar)
    batch, n, lead = _shape(op, x0)
    s_b, w_b = query(SCAN, op, batch, n)
    dev = x0.device
    if out is None:
        out = (torch.empty_like(x0), torch.empty_like(x0)) if op == "linrec" else (torch.empty_like(x0),)
    ws = workspace(w_b, dev)
    check(lib().pcad_scan_vjp_checkpoint(OPS[op], batch, n, _ptr(x0), _ptr(x1), _ptr(y0),
                                         _ptr(y1), _ptr(ybar), _ptr(Abar), _ptr(out[0]),
                                         _ptr(out[1]) if len(out) > 1 else None,
                                         ACCUMULATE if accumulate else 0, _ptr(ws), ws.numel(),
                                         _stream(dev)), "pcad_scan_vjp_checkpoint", ws=ws)
    return out if op == "linrec" else out[0]


# ---------------------------------------------------------------------------
# reduce-by-index
# ---------------------------------------------------------------------------
def _rbi_shape(op: str, v: torch.Tensor):
    """(batch, n, lead, d): v is (..., n) for + * min max and (..., n, d) for
    linrec (d = 2, pairs (a, b)) and mat2 (d = 4)."""
    d = DIM[op]
    if d == 1:
        batch, n, lead = _shape(op, v)
        return batch, n, lead, 1
    if v.shape[-1] != d or v.dim() < 2:
        raise PcadError(f"{op} reduce_by_index expects values of shape (..., n, {d})")
    lead = tuple(v.shape[:-2])
    batch = 1
    for x in lead:
        batch *= x
    return batch, v.shape[-2], lead, d


def rbi_fwd(op: str, idx: torch.Tensor, v: torch.Tensor, m: int):
    """Returns (hist, saved).  idx (..., n); v (..., n) or (..., n, d) for
    linrec (pairs (a, b)) and mat2; hist (..., m) or (..., m, d).
    saved: mul -> uint32 n0[batch*m] then float y_pos[batch*m];
    min/max -> int32 argk[batch*m]; sumprod -> float s[batch*m] (bin sums);
    then, where the sort-based path may run
    (the ordered operators always, the others beyond the LDS capacity),
    each row's sort (sorted keys and permutation) for the adjoint."""
    _dev_check(idx, v)
    batch, n, lead, d = _rbi_shape(op, v)
    s_b, w_b = query(RBI, op, batch, n, m)
    dev = v.device
    hist = torch.empty(lead + (m,) + ((d,) if d > 1 else ()), dtype=torch.float32, device=dev)
    saved = torch.empty(max(s_b, 16), dtype=torch.uint8, device=dev)
    ws = workspace(w_b, dev)
    check(lib().pcad_rbi_fwd(OPS[op], batch, n, m, _ptr(idx), _ptr(v), _ptr(hist), _ptr(saved), 0,
                             _ptr(ws), ws.numel(), _stream(dev)), "pcad_rbi_fwd", ws=ws)
    return hist, saved


def rbi_vjp(op: str, idx, v, m: int, saved, hbar, out=None, accumulate: bool = False):
    _dev_check(idx, v, hbar)
    batch, n, lead, d = _rbi_shape(op, v)
    s_b, w_b = query(RBI, op, batch, n, m)
    dev = v.device
    out = torch.empty_like(v) if out is None else out
    ws = workspace(w_b, dev)
    check(lib().pcad_rbi_vjp(OPS[op], batch, n, m, _ptr(idx), _ptr(v), _ptr(saved), _ptr(hbar),
                             _ptr(out), ACCUMULATE if accumulate else 0, _ptr(ws), ws.numel(),
                             _stream(dev)), "pcad_rbi_vjp", ws=ws)
    return out


def saved_argk(saved: torch.Tensor, batch: int, m: int) -> torch.Tensor:
    return saved[: batch * m * 4].view(torch.int32).view(batch, m)


def saved_mul(saved: torch.Tensor, batch: int, m: int):
    n0 = saved[: batch * m * 4].view(torch.int32).view(batch, m)
    yp = saved[batch * m * 4: batch * m * 8].view(torch.float32).view(batch, m)
    return n0, yp


# ---------------------------------------------------------------------------
# vectorised operators: elements are vectors of d floats (the last axis),
# combined component-wise; the library transposes into the scalar form
# ---------------------------------------------------------------------------
_tmp = {}


def scratch(nbytes: int, device: torch.device, stream=None) -> torch.Tensor:
    """The `tmp` buffer of the vectorised calls (no initialisation needed),
    one per (device, stream), grown on demand."""
    stream = stream if stream is not None else torch.cuda.current_stream(device)
    key = (device.index, stream.cuda_stream)
    buf = _tmp.get(key)
    if buf is None or buf.numel() < nbytes:
        size = 1 << (max(int(nbytes), 4096) - 1).bit_length()
        buf = torch.empty(size, dtype=torch.uint8, device=device)
        _tmp[key] = buf
    return buf


def vquery(comb: int, op: str, batch: int, n: int, d: int, m: int = 0):
    s, w, t = ctypes.c_size_t(0), ctypes.c_size_t(0), ctypes.c_size_t(0)
    check(lib().pcad_vquery(comb, OPS[op], batch, n, d, m, 0, ctypes.byref(s), ctypes.byref(w),
                            ctypes.byref(t)), "pcad_vquery")
    return s.value, w.value, t.value


def _vshape(x: torch.Tensor):
    """(batch, n, d, lead) of a tensor (..., n, d)."""
    if x.dim() < 2:
        raise PcadError("vectorised calls expect values of shape (..., n, d)")
    lead = tuple(x.shape[:-2])
    batch = 1
    for t in lead:
        batch *= t
    return batch, x.shape[-2], x.shape[-1], lead


def vreduce_fwd(op: str, x: torch.Tensor):
    """x (..., n, d) -> (y (..., d), saved): reduce with map2 op."""
    _dev_check(x)
    batch, n, d, lead = _vshape(x)
    s_b, w_b, t_b = vquery(REDUCE, op, batch, n, d)
    dev = x.device
    y = torch.empty(lead + (d,), dtype=torch.float32, device=dev)
    saved = torch.empty(max(s_b, 16), dtype=torch.uint8, device=dev)
    ws, tmp = workspace(w_b, dev), scratch(t_b, dev)
    check(lib().pcad_vreduce_fwd(OPS[op], batch, n, d, _ptr(x), _ptr(y), _ptr(saved), 0, _ptr(ws),
                                 ws.numel(), _ptr(tmp), tmp.numel(), _stream(dev)),
          "pcad_vreduce_fwd", ws=ws)
    return y, saved


def vreduce_vjp(op: str, x, saved, ybar, out=None, accumulate: bool = False):
    _dev_check(x, ybar)
    batch, n, d, lead = _vshape(x)
    s_b, w_b, t_b = vquery(REDUCE, op, batch, n, d)
    dev = x.device
    out = torch.empty_like(x) if out is None else out
    ws, tmp = workspace(w_b, dev), scratch(t_b, dev)
    check(lib().pcad_vreduce_vjp(OPS[op], batch, n, d, _ptr(x), _ptr(saved), _ptr(ybar.contiguous()),
                                 _ptr(out), ACCUMULATE if accumulate else 0, _ptr(ws), ws.numel(),
                                 _ptr(tmp), tmp.numel(), _stream(dev)), "pcad_vreduce_vjp", ws=ws)
    return out


def vscan_fwd(op: str, x: torch.Tensor):
    """x (..., n, d) -> (y (..., n, d), saved): inclusive scan with map2 op."""
    _dev_check(x)
    batch, n, d, lead = _vshape(x)
    s_b, w_b, t_b = vquery(SCAN, op, batch, n, d)
    dev = x.device
    y = torch.empty_like(x)
    saved = torch.empty(max(s_b, 16), dtype=torch.uint8, device=dev)
    ws, tmp = workspace(w_b, dev), scratch(t_b, dev)
    check(lib().pcad_vscan_fwd(OPS[op], batch, n, d, _ptr(x), _ptr(y), _ptr(saved), 0, _ptr(ws),
                               ws.numel(), _ptr(tmp), tmp.numel(), _stream(dev)), "pcad_vscan_fwd", ws=ws)
    return y, saved


def vscan_vjp(op: str, x, saved, ybar, out=None, accumulate: bool = False):
    _dev_check(x, ybar)
    batch, n, d, lead = _vshape(x)
    s_b, w_b, t_b = vquery(SCAN, op, batch, n, d)
    dev = x.device
    out = torch.empty_like(x) if out is None else out
    ws, tmp = workspace(w_b, dev), scratch(t_b, dev)
    check(lib().pcad_vscan_vjp(OPS[op], batch, n, d, _ptr(x), _ptr(saved), _ptr(ybar.contiguous()),
                               _ptr(out), ACCUMULATE if accumulate else 0, _ptr(ws), ws.numel(),
                               _ptr(tmp), tmp.numel(), _stream(dev)), "pcad_vscan_vjp", ws=ws)
    return out


# ---------------------------------------------------------------------------
# scans of d x d matrix products (d = 3, 5)
# ---------------------------------------------------------------------------
def matd_query(d: int, batch: int, n: int):
    s, w = ctypes.c_size_t(0), ctypes.c_size_t(0)
    check(lib().pcad_matd_query(d, batch, n, 0, ctypes.byref(s), ctypes.byref(w)),
          "pcad_matd_query")
    return s.value, w.value


def _mdshape(M: torch.Tensor):
    """(d, batch, n, lead) of matrices (..., n, d, d)."""
    if M.dim() < 3 or M.shape[-1] != M.shape[-2]:
        raise PcadError("matd calls expect matrices of shape (..., n, d, d)")
    lead = tuple(M.shape[:-3])
    batch = 1
    for t in lead:
        batch *= t
    return M.shape[-1], batch, M.shape[-3], lead


def matd_scan_fwd(M: torch.Tensor):
    """M (..., n, d, d) -> (P, saved), P_i = M_0 ... M_i along n."""
    _dev_check(M)
    d, batch, n, lead = _mdshape(M)
    s_b, w_b = matd_query(d, batch, n)
    dev = M.device
    P = torch.empty_like(M)
    saved = torch.empty(max(s_b, 16), dtype=torch.uint8, device=dev)
    ws = workspace(w_b, dev)
    check(lib().pcad_matd_scan_fwd(d, batch, n, _ptr(M), _ptr(P), _ptr(saved), 0, _ptr(ws),
                                   ws.numel(), _stream(dev)), "pcad_matd_scan_fwd", ws=ws)
    return P, saved


def matd_scan_vjp(M, saved, Pbar, out=None, accumulate: bool = False):
    """Adjoint of matd_scan_fwd: returns M_bar (shape of M)."""
    _dev_check(M)
    d, batch, n, lead = _mdshape(M)
    s_b, w_b = matd_query(d, batch, n)
    dev = M.device
    out = torch.empty_like(M) if out is None else out
    _dev_check(out)
    ws = workspace(w_b, dev)
    check(lib().pcad_matd_scan_vjp(d, batch, n, _ptr(M), _ptr(saved), _ptr(Pbar.contiguous()),
                                   _ptr(out), ACCUMULATE if accumulate else 0, _ptr(ws),
                                   ws.numel(), _stream(dev)), "pcad_matd_scan_vjp", ws=ws)
    return out


def _bdsshape(M: torch.Tensor):
    """M (..., n, k, q, q) -> (q, k, batch, n, lead)"""
    if M.dim() < 4 or M.shape[-1] != M.shape[-2]:
        raise PcadError("block-diagonal operands are (..., n, k, q, q)")
    lead = tuple(M.shape[:-4])
    batch = 1
    for t in lead:
        batch *= t
    return M.shape[-1], M.shape[-3], batch, M.shape[-4], lead


def bds_query(q: int, k: int, batch: int, n: int):
    s, w, tf, tv = (ctypes.c_size_t(0) for _ in range(4))
    check(lib().pcad_bds_query(q, k, batch, n, 0, ctypes.byref(s), ctypes.byref(w),
                               ctypes.byref(tf), ctypes.byref(tv)), "pcad_bds_query")
    return s.value, w.value, tf.value, tv.value


def bds_scan_fwd(M: torch.Tensor):
    """Scan of block-diagonal matrix products.  M (..., n, k, q, q): element
    i is the block-diagonal matrix diag(M[i, 0], ..., M[i, k-1]).  Returns
    (P, saved) with P[i, j] = M[0, j] M[1, j] ... M[i, j]."""
    _dev_check(M)
    q, k, batch, n, lead = _bdsshape(M)
    s_b, w_b, t_b, _ = bds_query(q, k, batch, n)
    dev = M.device
    P = torch.empty_like(M)
    saved = torch.empty(max(s_b, 16), dtype=torch.uint8, device=dev)
    ws, tmp = workspace(w_b, dev), scratch(t_b, dev)
    check(lib().pcad_bds_scan_fwd(q, k, batch, n, _ptr(M), _ptr(P), _ptr(saved), 0, _ptr(ws),
                                  ws.numel(), _ptr(tmp), tmp.numel(), _stream(dev)),
          "pcad_bds_scan_fwd", ws=ws)
    return P, saved


def bds_scan_vjp(M, saved, Pbar, out=None, accumulate: bool = False):
    """Adjoint of bds_scan_fwd: returns M_bar (shape of M)."""
    _dev_check(M, Pbar)
    q, k, batch, n, lead = _bdsshape(M)
    s_b, w_b, _, t_b = bds_query(q, k, batch, n)
    dev = M.device
    out = torch.empty_like(M) if out is None else out
    _dev_check(out)
    ws, tmp = workspace(w_b, dev), scratch(t_b, dev)
    check(lib().pcad_bds_scan_vjp(q, k, batch, n, _ptr(M), _ptr(saved), _ptr(Pbar.contiguous()),
                                  _ptr(out), ACCUMULATE if accumulate else 0, _ptr(ws), ws.numel(),
                                  _ptr(tmp), tmp.numel(), _stream(dev)), "pcad_bds_scan_vjp", ws=ws)
    return out


def matd_reduce_fwd(M: torch.Tensor):
    """M (..., n, d, d) -> (Y (..., d, d), saved), Y = M_0 ... M_{n-1}."""
    _dev_check(M)
    d, batch, n, lead = _mdshape(M)
    s_b, w_b = matd_query(d, batch, n)
    dev = M.device
    Y = torch.empty(lead + (d, d), dtype=torch.float32, device=dev)
    saved = torch.empty(max(s_b, 16), dtype=torch.uint8, device=dev)
    ws = workspace(w_b, dev)
    check(lib().pcad_matd_reduce_fwd(d, batch, n, _ptr(M), _ptr(Y), _ptr(saved), 0, _ptr(ws),
                                     ws.numel(), _stream(dev)), "pcad_matd_reduce_fwd", ws=ws)
    return Y, saved


def matd_reduce_vjp(M, saved, Ybar, out=None, accumulate: bool = False):
    """Adjoint of matd_reduce_fwd: returns M_bar (shape of M)."""
    _dev_check(M)
    d, batch, n, lead = _mdshape(M)
    s_b, w_b = matd_query(d, batch, n)
    dev = M.device
    out = torch.empty_like(M) if out is None else out
    _dev_check(out)
    ws = workspace(w_b, dev)
    check(lib().pcad_matd_reduce_vjp(d, batch, n, _ptr(M), _ptr(saved), _ptr(Ybar.contiguous()),
                                     _ptr(out), ACCUMULATE if accumulate else 0, _ptr(ws),
                                     ws.numel(), _stream(dev)), "pcad_matd_reduce_vjp", ws=ws)
    return out


# ---------------------------------------------------------------------------
# int32 forward combinators (+ * min max, wrapping mod 2^32)
# ---------------------------------------------------------------------------
def i32_fwd(comb: int, op: str, x: torch.Tensor, idx: Optional[torch.Tensor] = None, m: int = 0):
    """x int32 (..., n).  REDUCE -> (...,); SCAN -> (..., n); RBI -> (..., m)."""
    _dev_check(x, idx)
    if x.dtype != torch.int32 or (idx is not None and idx.dtype != torch.int32):
        raise PcadError("i32 calls take int32 tensors")
    lead = tuple(x.shape[:-1])
    n = x.shape[-1] if x.dim() else 1
    batch = 1
    for t in lead:
        batch *= t
    w = ctypes.c_size_t(0)
    check(lib().pcad_i32_query(comb, OPS[op], batch, n, m, ctypes.byref(w)), "pcad_i32_query")
    dev = x.device
    shape = {REDUCE: lead, SCAN: lead + (n,), RBI: lead + (m,)}[comb]
    y = torch.empty(shape, dtype=torch.int32, device=dev)
    ws = workspace(w.value, dev) if w.value else None
    check(lib().pcad_i32_fwd(comb, OPS[op], batch, n, m, _ptr(idx), _ptr(x), _ptr(y), _ptr(ws),
                             ws.numel() if ws is not None else 0, _stream(dev)), "pcad_i32_fwd", ws=ws)
    return y


def vrbi_fwd(op: str, idx: torch.Tensor, v: torch.Tensor, m: int):
    """idx (..., n), v (..., n, d) -> (hist (..., m, d), saved)."""
    _dev_check(idx, v)
    batch, n, d, lead = _vshape(v)
    s_b, w_b, t_b = vquery(RBI, op, batch, n, d, m)
    dev = v.device
    hist = torch.empty(lead + (m, d), dtype=torch.float32, device=dev)
    saved = torch.empty(max(s_b, 16), dtype=torch.uint8, device=dev)
    ws, tmp = workspace(w_b, dev), scratch(t_b, dev)
    check(lib().pcad_vrbi_fwd(OPS[op], batch, n, d, m, _ptr(idx), _ptr(v), _ptr(hist), _ptr(saved),
                              0, _ptr(ws), ws.numel(), _ptr(tmp), tmp.numel(), _stream(dev)),
          "pcad_vrbi_fwd", ws=ws)
    return hist, saved


def vrbi_vjp(op: str, idx, v, m: int, saved, hbar, out=None, accumulate: bool = False):
    _dev_check(idx, v, hbar)
    batch, n, d, lead = _vshape(v)
    s_b, w_b, t_b = vquery(RBI, op, batch, n, d, m)
    dev = v.device
    out = torch.empty_like(v) if out is None else out
    ws, tmp = workspace(w_b, dev), scratch(t_b, dev)
    check(lib().pcad_vrbi_vjp(OPS[op], batch, n, d, m, _ptr(idx), _ptr(v), _ptr(saved),
                              _ptr(hbar.contiguous()), _ptr(out), ACCUMULATE if accumulate else 0,
                              _ptr(ws), ws.numel(), _ptr(tmp), tmp.numel(), _stream(dev)),
          "pcad_vrbi_vjp", ws=ws)
    return out


# ---------------------------------------------------------------------------
# batched segmented plan
# ---------------------------------------------------------------------------
PHASE_FWD, PHASE_BWD, PHASE_BOTH = 1, 2, 3
PLAN_PER_SEGMENT = 1


class BatchedPlan:
    """Many ragged instances of (linear-recurrence scan -> min-by-index into
    m bins), forward and adjoint, each phase one hipGraph launch.

    ``offsets``: host int64 array of nseg+1 element offsets.  Buffers are
    allocated here (torch, on ``device``) and bound once; inputs are copied
    into them with :meth:`load`.
    """

    def __init__(self, offsets, m: int, device=None, per_segment: bool = False):
        import numpy as np
        self.device = torch.device(device or "cuda:0")
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.offsets = off
        self.nseg = off.shape[0] - 1
        self.m = int(m)
        h = ctypes.c_void_p()
        check(lib().pcad_plan_create(ctypes.byref(h), self.nseg, off.ctypes.data, self.m,
                                     PLAN_PER_SEGMENT if per_segment else 0), "pcad_plan_create")
        self._h = h
        s, w = ctypes.c_size_t(0), ctypes.c_size_t(0)
        n, it = ctypes.c_int64(0), ctypes.c_int64(0)
        check(lib().pcad_plan_query(h, ctypes.byref(s), ctypes.byref(w), ctypes.byref(n),
                                    ctypes.byref(it)), "pcad_plan_query")
        self.saved_bytes, self.ws_bytes, self.n, self.n_items = s.value, w.value, n.value, it.value
        dev, N, S, m = self.device, self.n, self.nseg, self.m
        f32 = dict(dtype=torch.float32, device=dev)
        self.a = torch.empty(max(N, 4), **f32)
        self.b = torch.empty(max(N, 4), **f32)
        self.idx = torch.empty(max(N, 4), dtype=torch.int32, device=dev)
        self.y = torch.empty(max(N, 4), **f32)
        self.ybar = torch.empty(max(N, 4), **f32)
        self.abar = torch.empty(max(N, 4), **f32)
        self.bbar = torch.empty(max(N, 4), **f32)
        self.h = torch.empty(S * m, **f32)
        self.hbar = torch.empty(S * m, **f32)
        self.argk = torch.empty(S * m, dtype=torch.int32, device=dev)
        self.saved = torch.empty(max(self.saved_bytes, 256), dtype=torch.uint8, device=dev)
        self.ws = torch.zeros(max(self.ws_bytes, 256), dtype=torch.uint8, device=dev)
        st = torch.cuda.current_stream(dev).cuda_stream
        check(lib().pcad_plan_bind(h, self.a.data_ptr(), self.b.data_ptr(), self.idx.data_ptr(),
                                   self.y.data_ptr(), self.h.data_ptr(), self.argk.data_ptr(),
                                   self.ybar.data_ptr(), self.hbar.data_ptr(),
                                   self.abar.data_ptr(), self.bbar.data_ptr(),
                                   self.saved.data_ptr(), self.ws.data_ptr(), self.ws.numel(), st),
              "pcad_plan_bind")

    def load(self, a=None, b=None, idx=None, ybar=None, hbar=None):
        """Copy host or device arrays into the bound input buffers."""
        for name, v in (("a", a), ("b", b), ("idx", idx), ("ybar", ybar), ("hbar", hbar)):
            if v is None:
                continue
            t = torch.as_tensor(v)
            dst = getattr(self, name)
            dst[: t.numel()].copy_(t.reshape(-1).to(dst.dtype), non_blocking=False)

    def run(self, phase: int = PHASE_BOTH):
        st = torch.cuda.current_stream(self.device).cuda_stream
        r = lib().pcad_plan_run(self._h, phase, st)
        if r != 0:
            raise PcadError(f"pcad_plan_run: status {r}, hip {lib().pcad_plan_last_hip_error()}")
        if SYNC_CHECK:
            ws_status(self.ws, what="pcad_plan_run")

    def run_per_segment(self, phase: int = PHASE_BOTH):
        st = torch.cuda.current_stream(self.device).cuda_stream
        r = lib().pcad_plan_run_per_segment(self._h, phase, st)
        if r != 0:
            raise PcadError(f"pcad_plan_run_per_segment: status {r}, hip {lib().pcad_plan_last_hip_error()}")

    def ws_error(self) -> int:
        """The error word of the plan's workspace (0 when no look-back wait
        of its launches timed out); see pcad_ws_status."""
        st = lib().pcad_ws_status(self.ws.data_ptr(), 0,
                                  torch.cuda.current_stream(self.device).cuda_stream)
        if st not in (0, E_TIMEOUT):
            check(st, "pcad_ws_status")
        return 0 if st == 0 else int(self.ws[:16].view(torch.int32)[2].item())

    def close(self):
        if getattr(self, "_h", None):
            lib().pcad_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
