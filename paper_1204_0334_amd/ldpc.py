"""Python binding of the C ABI in include/ldpc.h (ctypes).

Argument marshalling only: every step of decoding runs in the HIP library
libldpc_hip.so.  PyTorch supplies device memory (the LLR, output and
workspace tensors) and the current HIP stream.  If the library has not been
built, importing this module raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch first: its wheel carries its own HIP runtime (same soname as the system
# one).  Loading torch before the library makes the library bind to that
# runtime, so the process has one HIP runtime and torch's streams and memory
# are valid in the library's calls.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldpc_hip.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_1204_0334_amd.build.build()")

_lib = ctypes.CDLL(LIB_PATH)

_vp, _i32, _i64, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t

OK, EINVAL, EWORKSPACE, EHIP, EUNSUPPORTED, ENOMEM = 0, -1, -2, -3, -4, -5
GRAPH_QC, GRAPH_CONV = 0, 1
LAYOUT_G8, LAYOUT_G16, LAYOUT_G32, LAYOUT_G64, LAYOUT_G64F4, LAYOUT_G64F2 = 0, 1, 2, 3, 4, 5
LAYOUT_G8F2, LAYOUT_G8F4, LAYOUT_G16F2, LAYOUT_G16F4, LAYOUT_G32F2, LAYOUT_G32F4 = 6, 7, 8, 9, 10, 11
LAYOUT_NAMES = ["G8", "G16", "G32", "G64", "G64F4", "G64F2", "G8F2", "G8F4", "G16F2", "G16F4", "G32F2", "G32F4"]
PLAN_LAYOUTS = len(LAYOUT_NAMES)
LAYOUT_VN2, LAYOUT_VN4, LAYOUT_CN2, LAYOUT_CN4 = 16, 32, 64, 128
LAYOUT_SPLIT2, LAYOUT_SPLIT4, LAYOUT_SPLIT8 = 256, 512, 768


def layout_name(layout: int) -> str:
    v, c, h = (layout >> 4) & 3, (layout >> 6) & 3, (layout >> 8) & 3
    return (LAYOUT_NAMES[layout & 15] + ("" if v == 0 else f"/VN{1 << v}") + ("" if c == 0 else f"/CN{1 << c}")
            + ("" if h == 0 else f"/S{1 << h}"))
PLAN_MAX_CODES = 16
TIMING_CLASSES = 24
MAX_ITERS = 100000
NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024


class GraphInfo(ctypes.Structure):
    _fields_ = [("kind", _i32), ("n", _i32), ("m", _i32), ("E", _i32), ("dv_max", _i32), ("dc_max", _i32),
                ("J", _i32), ("L", _i32), ("p", _i32), ("ms", _i32), ("T", _i32), ("Jb", _i32), ("Lb", _i32),
                ("c", _i32), ("c_minus_b", _i32), ("positions", _i32), ("layers", _i32), ("blocks", _i32),
                ("design_rate", ctypes.c_double)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_create_qc = _sig("ldpc_graph_create_qc", _i32, [_vp, _i32, _i32, _i32, ctypes.POINTER(_vp)])
_create_cc = _sig("ldpc_graph_create_ldpccc_from_qc", _i32, [_vp, _i32, _i32, _i32, _i32, _i32, ctypes.POINTER(_vp)])
_create_sf = _sig("ldpc_graph_create_ldpccc_sf", _i32,
                  [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _i32, ctypes.POINTER(_vp)])
_get_info = _sig("ldpc_graph_get_info", _i32, [_vp, ctypes.POINTER(GraphInfo)])
_destroy = _sig("ldpc_graph_destroy", None, [_vp])
_ws_size = _sig("ldpc_workspace_size", _i32, [_vp, _i32, _i32, _i32, ctypes.POINTER(_sz)])
_decode = _sig("ldpc_decode", _i32, [_vp, _vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp])
_decode_path = _sig("ldpc_decode_path", _i32, [_vp, ctypes.POINTER(_i32)])
_decode_noalloc = _sig("ldpc_decode_noalloc", _i32, [_vp, _vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp])
_nms_decode = _sig("ldpc_nms_decode", _i32, [_vp, _vp, _i32, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp])
_nms_ws_size = _sig("ldpc_nms_train_workspace_size", _i32, [_vp, _i32, _i32, _i32, ctypes.POINTER(_sz)])
_nms_forward = _sig("ldpc_nms_train_forward", _i32, [_vp, _vp, _i32, _i32, _i32, _vp, _vp, _vp, _sz, _vp])
_nms_backward = _sig("ldpc_nms_train_backward", _i32, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _sz, _vp])
_plan_create = _sig("ldpc_plan_create", _i32, [_vp, _vp, _i32, _i32, _i32, ctypes.POINTER(_vp)])
_plan_destroy = _sig("ldpc_plan_destroy", None, [_vp])
_plan_ws_size = _sig("ldpc_plan_workspace_size", _i32, [_vp, ctypes.POINTER(_sz)])
_plan_set_layout = _sig("ldpc_plan_set_layout", _i32, [_vp, _i32, _i32])
_plan_get_layout = _sig("ldpc_plan_get_layout", _i32, [_vp, _i32, ctypes.POINTER(_i32)])
_plan_decode = _sig("ldpc_plan_decode", _i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp])
_plan_capture = _sig("ldpc_plan_capture", _i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp])
_plan_replay = _sig("ldpc_plan_replay", _i32, [_vp, _vp])
_plan_autotune = _sig("ldpc_plan_autotune", _i32,
                      [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _i32, _vp, ctypes.POINTER(ctypes.c_double)])
_plan_set_persistent = _sig("ldpc_plan_set_persistent", _i32, [_vp, _i32, _i64])
_plan_check = _sig("ldpc_plan_check", _i32, [_vp, _vp, _vp])
_decode_window = _sig("ldpc_decode_window", _i32, [_vp, _vp, _i32, _i32, _i32, _vp, _vp, _vp, _sz, _vp])
_decode_pipeline = _sig("ldpc_decode_pipeline", _i32, [_vp, _vp, _i32, _i32, _vp, _vp, _vp, _sz, _vp])
_awgn_llr = _sig("ldpc_awgn_llr", _i32, [_i64, _i32, ctypes.c_double, ctypes.c_uint64, _i64, _vp, _vp])
_count_errors = _sig("ldpc_count_errors", _i32, [_vp, _i32, _i64, _vp, _vp, _vp])
_status_str = _sig("ldpc_status_str", ctypes.c_char_p, [_i32])
_timing_enable = _sig("ldpc_timing_enable", _i32, [_i32])
_timing_read = _sig("ldpc_timing_read", _i32, [ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double), _i32])
_class_name = _sig("ldpc_kernel_class_name", ctypes.c_char_p, [_i32])

EXPORTED = ["ldpc_graph_create_qc", "ldpc_graph_create_ldpccc_from_qc", "ldpc_graph_create_ldpccc_sf",
            "ldpc_graph_get_info", "ldpc_graph_destroy", "ldpc_workspace_size", "ldpc_decode", "ldpc_decode_path",
            "ldpc_decode_noalloc",
            "ldpc_nms_decode", "ldpc_nms_train_workspace_size", "ldpc_nms_train_forward",
            "ldpc_nms_train_backward", "ldpc_plan_create", "ldpc_plan_destroy", "ldpc_plan_workspace_size",
            "ldpc_plan_set_layout", "ldpc_plan_get_layout", "ldpc_plan_decode", "ldpc_plan_capture",
            "ldpc_plan_replay", "ldpc_plan_autotune", "ldpc_plan_set_persistent", "ldpc_plan_check", "ldpc_decode_window", "ldpc_decode_pipeline", "ldpc_awgn_llr",
            "ldpc_count_errors", "ldpc_status_str", "ldpc_timing_enable", "ldpc_timing_read",
            "ldpc_kernel_class_name"]


class LdpcError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_str(status)} ({status})")
        self.status = status


def status_str(status: int) -> str:
    return _status_str(int(status)).decode()


def _check(status: int, what: str):
    if status != OK:
        raise LdpcError(status, what)


def _int32_table(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64).astype(np.int32))


class Graph:
    """Host graph handle (QC block code or terminated convolutional code)."""

    def __init__(self, handle):
        self._h = handle
        info = GraphInfo()
        _check(_get_info(self._h, ctypes.byref(info)), "ldpc_graph_get_info")
        self.info = {k: getattr(info, k) for k, _ in GraphInfo._fields_}

    @classmethod
    def qc(cls, shifts, p: int) -> "Graph":
        a = _int32_table(shifts)
        if a.ndim != 2:
            raise ValueError("shifts must be a 2-D table")
        h = _vp()
        _check(_create_qc(a.ctypes.data, a.shape[0], a.shape[1], int(p), ctypes.byref(h)), "ldpc_graph_create_qc")
        return cls(h)

    @classmethod
    def ldpccc_from_qc(cls, shifts, p: int, positions: int, terminate: bool = True) -> "Graph":
        a = _int32_table(shifts)
        if a.ndim != 2:
            raise ValueError("shifts must be a 2-D table")
        h = _vp()
        _check(_create_cc(a.ctypes.data, a.shape[0], a.shape[1], int(p), int(positions), int(bool(terminate)),
                          ctypes.byref(h)), "ldpc_graph_create_ldpccc_from_qc")
        return cls(h)

    @classmethod
    def ldpccc_sf(cls, sf, p: int, positions: int, terminate: bool = True) -> "Graph":
        a = _int32_table(sf)
        if a.ndim != 4:
            raise ValueError("sf must be [T][ms+1][Jb][Lb]")
        T, ms1, Jb, Lb = a.shape
        h = _vp()
        _check(_create_sf(a.ctypes.data, T, ms1 - 1, Jb, Lb, int(p), int(positions), int(bool(terminate)),
                          ctypes.byref(h)), "ldpc_graph_create_ldpccc_sf")
        return cls(h)

    @property
    def handle(self):
        return self._h

    @property
    def n(self) -> int:
        return self.info["n"]

    def workspace_size(self, gamma: int, max_iters: int = 1, window: int = 0) -> int:
        out = _sz()
        _check(_ws_size(self._h, int(gamma), int(max_iters), int(window), ctypes.byref(out)), "ldpc_workspace_size")
        return int(out.value)

    def close(self):
        h = getattr(self, "_h", None)
        if h and _destroy is not None:   # module globals may be gone at interpreter exit
            _destroy(h)
        self._h = None

    def __del__(self):
        self.close()


def _torch():
    return torch


def _stream_handle(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _on_stream(stream, fresh):
    """Prepare tensors allocated by this module (`fresh`: workspace, outputs)
    for use on `stream`.  They come from torch's caching allocator on the
    current stream; on another stream the enqueued work must first wait for
    the current stream (the memory may have been released by work still
    queued there) and the allocator must know the tensors are in use on that
    stream until its work is done (record_stream), or it could hand the
    memory out again while the decoder still reads or writes it."""
    if stream is None:
        return
    cur = torch.cuda.current_stream(stream.device)
    if stream == cur:
        return
    stream.wait_stream(cur)
    for t in fresh:
        t.record_stream(stream)


def _need(t, dtype, shape, what):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous {dtype} tensor of shape {tuple(shape)}")


def workspace(g: Graph, gamma: int, max_iters: int = 1, window: int = 0, device=None):
    torch = _torch()
    nbytes = g.workspace_size(gamma, max_iters, window)
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device or "cuda")


def decode(g: Graph, llr, max_iters: int, early_stop: bool = False, out=None, ws=None, stream=None):
    """Decode llr [gamma, n] (float32, device).  Returns (post, bits, iters,
    converged) device tensors; enqueued on `stream` (default: current)."""
    torch = _torch()
    if llr.dim() != 2:
        raise ValueError("llr must be [gamma, n]")
    gamma, n = llr.shape
    _need(llr, torch.float32, (gamma, g.n), "llr")
    dev = llr.device
    fresh = []
    if out is None:
        out = (torch.empty((gamma, n), dtype=torch.float32, device=dev),
               torch.empty((gamma, n), dtype=torch.uint8, device=dev),
               torch.empty((gamma,), dtype=torch.int32, device=dev),
               torch.empty((gamma,), dtype=torch.uint8, device=dev))
        fresh += list(out)
    post, bits, iters, conv = out
    _need(post, torch.float32, (gamma, n), "post")
    _need(bits, torch.uint8, (gamma, n), "bits")
    _need(iters, torch.int32, (gamma,), "iters")
    _need(conv, torch.uint8, (gamma,), "converged")
    if ws is None:
        ws = workspace(g, gamma, max_iters, 0, dev)
        fresh.append(ws)
    _on_stream(stream, fresh)
    _check(_decode(g.handle, llr.data_ptr(), gamma, int(max_iters), int(bool(early_stop)), post.data_ptr(),
                   bits.data_ptr(), iters.data_ptr(), conv.data_ptr(), ws.data_ptr(), ws.numel(),
                   _stream_handle(stream)), "ldpc_decode")
    return post, bits, iters, conv


def decode_path(g: Graph) -> str:
    """ldpc_decode_path: "onchip" when ldpc_decode decodes each frame of g on
    one compute unit on the current device, "packages" otherwise."""
    v = _i32(0)
    _check(_decode_path(g.handle, ctypes.byref(v)), "ldpc_decode_path")
    return "onchip" if v.value else "packages"


def decode_noalloc(g: Graph, llr, max_iters: int, early_stop: bool = False, out=None, stream=None):
    """ldpc_decode_noalloc: decode without a workspace; the library's static
    per-device array of NOALLOC_SCRATCH_BYTES serves as one (calls on one
    device must not overlap).  Outputs as for decode; pass `out` to keep this
    binding from allocating them."""
    if llr.dim() != 2:
        raise ValueError("llr must be [gamma, n]")
    gamma, n = llr.shape
    _need(llr, torch.float32, (gamma, g.n), "llr")
    fresh = []
    post, bits, iters, conv = _decode_outputs(llr, gamma, n, out, fresh)
    _on_stream(stream, fresh)
    _check(_decode_noalloc(g.handle, llr.data_ptr(), gamma, int(max_iters), int(bool(early_stop)), post.data_ptr(),
                           bits.data_ptr(), iters.data_ptr(), conv.data_ptr(), _stream_handle(stream)),
           "ldpc_decode_noalloc")
    return post, bits, iters, conv


def _decode_outputs(llr, gamma, n, out, fresh):
    dev = llr.device
    if out is None:
        out = (torch.empty((gamma, n), dtype=torch.float32, device=dev),
               torch.empty((gamma, n), dtype=torch.uint8, device=dev),
               torch.empty((gamma,), dtype=torch.int32, device=dev),
               torch.empty((gamma,), dtype=torch.uint8, device=dev))
        fresh += list(out)
    post, bits, iters, conv = out
    _need(post, torch.float32, (gamma, n), "post")
    _need(bits, torch.uint8, (gamma, n), "bits")
    _need(iters, torch.int32, (gamma,), "iters")
    _need(conv, torch.uint8, (gamma,), "converged")
    return out


def nms_decode(g: Graph, llr, weights, early_stop: bool = False, out=None, ws=None, stream=None):
    """Learned min-sum decoding of llr [gamma, n] with weights float32
    [iters, blocks, 2] (scale, offset per edge class: the graph's circulant
    blocks) on the device; iters = weights.shape[0].
    Returns (post, bits, iters, converged)."""
    if llr.dim() != 2:
        raise ValueError("llr must be [gamma, n]")
    gamma, n = llr.shape
    _need(llr, torch.float32, (gamma, g.n), "llr")
    T = int(weights.shape[0]) if weights.dim() == 3 else -1
    _need(weights, torch.float32, (T, g.info["blocks"], 2), "weights")
    fresh = []
    post, bits, iters, conv = _decode_outputs(llr, gamma, n, out, fresh)
    if ws is None:
        ws = workspace(g, gamma, T, 0, llr.device)
        fresh.append(ws)
    _on_stream(stream, fresh)
    _check(_nms_decode(g.handle, llr.data_ptr(), gamma, T, weights.data_ptr(), int(bool(early_stop)),
                       post.data_ptr(), bits.data_ptr(), iters.data_ptr(), conv.data_ptr(), ws.data_ptr(),
                       ws.numel(), _stream_handle(stream)), "ldpc_nms_decode")
    return post, bits, iters, conv


def nms_train_workspace_size(g: Graph, gamma: int, iters: int, ckpt_every: int) -> int:
    out = _sz()
    _check(_nms_ws_size(g.handle, int(gamma), int(iters), int(ckpt_every), ctypes.byref(out)),
           "ldpc_nms_train_workspace_size")
    return int(out.value)


def nms_train_workspace(g: Graph, gamma: int, iters: int, ckpt_every: int, device=None):
    size = nms_train_workspace_size(g, gamma, iters, ckpt_every)
    return torch.empty(max(size, 1), dtype=torch.uint8, device=device or "cuda")


def nms_train_forward(g: Graph, llr, weights, ckpt_every: int, ws, loss=None, stream=None):
    """Per-iteration losses float32 [iters] of the learned min-sum decoder on
    llr [gamma, n] (all-zero codeword); keeps checkpoints in `ws` for
    nms_train_backward."""
    gamma, n = llr.shape
    _need(llr, torch.float32, (gamma, g.n), "llr")
    T = int(weights.shape[0]) if weights.dim() == 3 else -1
    _need(weights, torch.float32, (T, g.info["blocks"], 2), "weights")
    fresh = []
    if loss is None:
        loss = torch.empty((T,), dtype=torch.float32, device=llr.device)
        fresh.append(loss)
    _need(loss, torch.float32, (T,), "loss")
    _on_stream(stream, fresh)
    _check(_nms_forward(g.handle, llr.data_ptr(), gamma, T, int(ckpt_every), weights.data_ptr(), loss.data_ptr(),
                        ws.data_ptr(), ws.numel(), _stream_handle(stream)), "ldpc_nms_train_forward")
    return loss


def nms_train_backward(g: Graph, gamma: int, weights, ckpt_every: int, dloss, ws, grad=None, stream=None):
    """Gradient float32 [iters, blocks, 2] of sum_t dloss[t] loss[t] with respect to
    the weights, after nms_train_forward on the same workspace."""
    T = int(weights.shape[0]) if weights.dim() == 3 else -1
    _need(weights, torch.float32, (T, g.info["blocks"], 2), "weights")
    _need(dloss, torch.float32, (T,), "dloss")
    fresh = []
    if grad is None:
        grad = torch.empty_like(weights)
        fresh.append(grad)
    _need(grad, torch.float32, tuple(weights.shape), "grad")
    _on_stream(stream, fresh)
    _check(_nms_backward(g.handle, int(gamma), T, int(ckpt_every), weights.data_ptr(), dloss.data_ptr(),
                         grad.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(stream)),
           "ldpc_nms_train_backward")
    return grad


def decode_window(g: Graph, llr, W: int, iters_per_window: int, out=None, ws=None, stream=None):
    """Sliding-window decoding of llr [gamma, positions * c].  Returns (post, bits)."""
    torch = _torch()
    if llr.dim() != 2:
        raise ValueError("llr must be [gamma, n]")
    gamma, n = llr.shape
    _need(llr, torch.float32, (gamma, g.n), "llr")
    dev = llr.device
    fresh = []
    if out is None:
        out = (torch.empty((gamma, n), dtype=torch.float32, device=dev),
               torch.empty((gamma, n), dtype=torch.uint8, device=dev))
        fresh += list(out)
    post, bits = out
    _need(post, torch.float32, (gamma, n), "post")
    _need(bits, torch.uint8, (gamma, n), "bits")
    if ws is None:
        ws = workspace(g, gamma, 1, W, dev)
        fresh.append(ws)
    _on_stream(stream, fresh)
    _check(_decode_window(g.handle, llr.data_ptr(), gamma, int(W), int(iters_per_window), post.data_ptr(),
                          bits.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(stream)),
           "ldpc_decode_window")
    return post, bits


def decode_pipeline(g: Graph, llr, iters: int, out=None, ws=None, stream=None):
    """Pipelined decoding (Algorithm 2) of llr [gamma, positions * c] with
    `iters` processors.  Returns (post, bits)."""
    if llr.dim() != 2:
        raise ValueError("llr must be [gamma, n]")
    gamma, n = llr.shape
    _need(llr, torch.float32, (gamma, g.n), "llr")
    dev = llr.device
    fresh = []
    if out is None:
        out = (torch.empty((gamma, n), dtype=torch.float32, device=dev),
               torch.empty((gamma, n), dtype=torch.uint8, device=dev))
        fresh += list(out)
    post, bits = out
    _need(post, torch.float32, (gamma, n), "post")
    _need(bits, torch.uint8, (gamma, n), "bits")
    if ws is None:
        ws = workspace(g, gamma, iters, 0, dev)
        fresh.append(ws)
    _on_stream(stream, fresh)
    _check(_decode_pipeline(g.handle, llr.data_ptr(), gamma, int(iters), post.data_ptr(), bits.data_ptr(),
                            ws.data_ptr(), ws.numel(), _stream_handle(stream)), "ldpc_decode_pipeline")
    return post, bits


def awgn_llr(n: int, gamma: int, sigma2: float, seed: int, frame0: int = 0, out=None, device=None, stream=None):
    """Channel LLRs of the all-zero codeword generated on the GPU: float32 [gamma, n]."""
    fresh = []
    if out is None:
        out = torch.empty((gamma, n), dtype=torch.float32, device=device or "cuda")
        fresh.append(out)
    _need(out, torch.float32, (gamma, n), "out")
    _on_stream(stream, fresh)
    _check(_awgn_llr(int(n), int(gamma), float(sigma2), int(seed) & 0xFFFFFFFFFFFFFFFF, int(frame0), out.data_ptr(),
                     _stream_handle(stream)), "ldpc_awgn_llr")
    return out


def count_errors(bits, frame_errors=None, totals=None, stream=None):
    """Bit errors per frame against the all-zero codeword; adds the batch's
    bit and frame errors to `totals` (int64 [2]) when given."""
    gamma, n = bits.shape
    _need(bits, torch.uint8, (gamma, n), "bits")
    fresh = []
    if frame_errors is None:
        frame_errors = torch.empty((gamma,), dtype=torch.int32, device=bits.device)
        fresh.append(frame_errors)
    _need(frame_errors, torch.int32, (gamma,), "frame_errors")
    if totals is not None:
        _need(totals, torch.int64, (2,), "totals")
    _on_stream(stream, fresh)
    _check(_count_errors(bits.data_ptr(), gamma, n, frame_errors.data_ptr(),
                         totals.data_ptr() if totals is not None else None, _stream_handle(stream)),
           "ldpc_count_errors")
    return frame_errors


def timing_enable(on: bool = True):
    _check(_timing_enable(int(bool(on))), "ldpc_timing_enable")


def timing_read() -> dict:
    """Per kernel class: (launches, summed device ms) since the last read."""
    cnt = (_i64 * TIMING_CLASSES)()
    ms = (ctypes.c_double * TIMING_CLASSES)()
    _check(_timing_read(cnt, ms, TIMING_CLASSES), "ldpc_timing_read")
    return {_class_name(c).decode(): (int(cnt[c]), float(ms[c])) for c in range(TIMING_CLASSES)}


class Plan:
    """Several QC graphs, each with its own batch size, decoded together by
    one check-node and one variable-node launch per iteration
    (`ldpc_plan_*`).  Buffers are lists of device tensors, one per code."""

    def __init__(self, graphs, gammas, max_iters: int, early_stop: bool = False):
        n = len(graphs)
        if n != len(gammas):
            raise ValueError("one batch size per graph")
        self.graphs = list(graphs)          # the plan refers to them
        self.gammas = [int(x) for x in gammas]
        self.max_iters = int(max_iters)
        hs = (_vp * max(n, 1))(*[g.handle for g in graphs])
        gs = (_i32 * max(n, 1))(*self.gammas)
        h = _vp()
        _check(_plan_create(hs, gs, n, self.max_iters, int(bool(early_stop)), ctypes.byref(h)), "ldpc_plan_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def workspace_size(self) -> int:
        out = _sz()
        _check(_plan_ws_size(self._h, ctypes.byref(out)), "ldpc_plan_workspace_size")
        return int(out.value)

    def workspace(self, device=None):
        return torch.empty(max(self.workspace_size(), 1), dtype=torch.uint8, device=device or "cuda")

    def set_layout(self, code: int, layout: int):
        _check(_plan_set_layout(self._h, int(code), int(layout)), "ldpc_plan_set_layout")

    def layout(self, code: int) -> int:
        out = _i32()
        _check(_plan_get_layout(self._h, int(code), ctypes.byref(out)), "ldpc_plan_get_layout")
        return int(out.value)

    def outputs(self, device=None):
        dev = device or "cuda"
        outs = []
        for g, gamma in zip(self.graphs, self.gammas):
            outs.append((torch.empty((gamma, g.n), dtype=torch.float32, device=dev),
                         torch.empty((gamma, g.n), dtype=torch.uint8, device=dev),
                         torch.empty((gamma,), dtype=torch.int32, device=dev),
                         torch.empty((gamma,), dtype=torch.uint8, device=dev)))
        return outs

    def _arrays(self, llrs, outs):
        n = len(self.graphs)
        if len(llrs) != n or len(outs) != n:
            raise ValueError("one llr tensor and one output tuple per code")
        for c, (g, gamma) in enumerate(zip(self.graphs, self.gammas)):
            _need(llrs[c], torch.float32, (gamma, g.n), f"llr[{c}]")
            post, bits, it, conv = outs[c]
            _need(post, torch.float32, (gamma, g.n), f"post[{c}]")
            _need(bits, torch.uint8, (gamma, g.n), f"bits[{c}]")
            _need(it, torch.int32, (gamma,), f"iters[{c}]")
            _need(conv, torch.uint8, (gamma,), f"converged[{c}]")

        def arr(ts):
            return (_vp * n)(*[t.data_ptr() for t in ts])
        return (arr(llrs), arr([o[0] for o in outs]), arr([o[1] for o in outs]), arr([o[2] for o in outs]),
                arr([o[3] for o in outs]))

    def decode(self, llrs, outs=None, ws=None, stream=None):
        """Decode llrs[c] [gamma_c, n_c]; returns [(post, bits, iters, converged)] per code."""
        fresh = []
        if outs is None:
            outs = self.outputs(llrs[0].device)
            fresh += [t for o in outs for t in o]
        if ws is None:
            ws = self.workspace(llrs[0].device)
            fresh.append(ws)
        a = self._arrays(llrs, outs)
        _on_stream(stream, fresh)
        _check(_plan_decode(self._h, *a, ws.data_ptr(), ws.numel(), _stream_handle(stream)), "ldpc_plan_decode")
        return outs

    def capture(self, llrs, outs, ws, stream=None):
        """Record the decode of these buffers into a HIP graph (runs nothing)."""
        a = self._arrays(llrs, outs)
        _check(_plan_capture(self._h, *a, ws.data_ptr(), ws.numel(), _stream_handle(stream)), "ldpc_plan_capture")

    def replay(self, stream=None):
        _check(_plan_replay(self._h, _stream_handle(stream)), "ldpc_plan_replay")

    def autotune(self, llrs, outs, ws, trials: int = 3, stream=None) -> float:
        """Coordinate descent over the codes' layouts, timing whole decodes of
        the plan on these buffers; returns the final time per decode (ms)."""
        a = self._arrays(llrs, outs)
        best = ctypes.c_double()
        _check(_plan_autotune(self._h, *a, ws.data_ptr(), ws.numel(), int(trials), _stream_handle(stream),
                              ctypes.byref(best)), "ldpc_plan_autotune")
        return float(best.value)

    def set_persistent(self, on: bool = True, wait_limit_us: int = 0):
        """Decode (and capture, autotune) as one persistent launch instead of
        the phase launches; wait_limit_us bounds each of its waits (0: 2 s)."""
        _check(_plan_set_persistent(self._h, int(bool(on)), int(wait_limit_us)), "ldpc_plan_set_persistent")

    def check(self, ws, stream=None):
        """Raise LdpcError(EHIP) if a persistent decode on `ws` had a wait
        expire since the last check (synchronises the stream)."""
        _check(_plan_check(self._h, ws.data_ptr(), _stream_handle(stream)), "ldpc_plan_check")

    def close(self):
        h = getattr(self, "_h", None)
        if h and _plan_destroy is not None:
            _plan_destroy(h)
        self._h = None

    def __del__(self):
        self.close()
