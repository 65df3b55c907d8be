"""ctypes binding of libffv.so (include/ffv.h): argument marshalling only.

Every step of the view-interpolation forward pass runs in the library's HIP
kernels; this module passes torch device pointers and a HIP stream through.
There is no fallback: if the library is missing the import of ``lib()``
raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libffv.so")

FFV_ABI_VERSION = 1
FFV_FP32, FFV_BF16, FFV_FP8_E4M3 = 0, 1, 2
PRECISIONS = {"fp32": FFV_FP32, "bf16": FFV_BF16, "fp8": FFV_FP8_E4M3}
FFV_OP_ACT_OUT = 0x100  # op_conv: output in the activation dtype

STATUS = {0: "FFV_OK", 1: "FFV_PENDING", -1: "FFV_ERR_ARG", -2: "FFV_ERR_OOM",
          -3: "FFV_ERR_BUDGET", -4: "FFV_ERR_DEVICE", -5: "FFV_ERR_WEIGHTS",
          -6: "FFV_ERR_TICKET", -7: "FFV_ERR_STATE"}

# Every symbol include/ffv.h declares.
EXPORTS = ["ffv_default_opts", "ffv_create_net", "ffv_destroy_net", "ffv_interpolate",
           "ffv_last_error", "ffv_calibrate", "ffv_register_camera", "ffv_submit", "ffv_submit_many", "ffv_poll", "ffv_serving_stats",
           "ffv_debug_tap", "ffv_set_debug", "ffv_set_profiling", "ffv_kernel_stats", "ffv_op_conv",
           "ffv_autotune", "ffv_save_tuning", "ffv_load_tuning", "ffv_interpolate_blend",
           "ffv_interpolate_recursive", "ffv_stitch_cluster", "ffv_debug_fault", "ffv_op_conv_noalloc",
           "ffv_lap_loss"]
FFV_OP_NOALLOC_SCRATCH_BYTES = 64 << 20


class FfvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class ffv_opts(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("device", ctypes.c_int32), ("graphs", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("workspace_bytes", ctypes.c_uint64),
                ("hbm_budget_bytes", ctypes.c_uint64), ("tick_ms", ctypes.c_float),
                ("max_batch_views", ctypes.c_int32)]


class ffv_request(ctypes.Structure):
    _fields_ = [("cam_left", ctypes.c_int32), ("cam_right", ctypes.c_int32),
                ("t", ctypes.c_float), ("out", ctypes.c_void_p), ("user_tag", ctypes.c_uint64)]


class ffv_timing(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double)]


class ffv_pair(ctypes.Structure):
    _fields_ = [("left", ctypes.c_void_p), ("right", ctypes.c_void_p),
                ("height", ctypes.c_int32), ("width", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libffv.so (built in-tree); raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2112_10603_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    c_int, c_void, c_f, c_sz = ctypes.c_int32, ctypes.c_void_p, ctypes.c_float, ctypes.c_size_t
    L.ffv_default_opts.argtypes = [ctypes.POINTER(ffv_opts)]
    L.ffv_default_opts.restype = None
    L.ffv_create_net.argtypes = [ctypes.c_char_p, ctypes.POINTER(ffv_opts), ctypes.POINTER(c_void)]
    L.ffv_create_net.restype = c_int
    L.ffv_destroy_net.argtypes = [c_void]
    L.ffv_destroy_net.restype = None
    L.ffv_interpolate.argtypes = [c_void, ctypes.POINTER(ffv_pair), c_int, ctypes.POINTER(c_f),
                                  c_int, c_void]
    L.ffv_interpolate.restype = c_int
    L.ffv_last_error.argtypes = []
    L.ffv_last_error.restype = ctypes.c_char_p
    L.ffv_debug_tap.argtypes = [c_void, ctypes.c_char_p, c_void, c_sz, ctypes.POINTER(c_int)]
    L.ffv_debug_tap.restype = c_int
    L.ffv_set_debug.argtypes = [c_void, c_int]
    L.ffv_set_debug.restype = c_int
    L.ffv_set_profiling.argtypes = [c_void, c_int]
    L.ffv_set_profiling.restype = c_int
    L.ffv_kernel_stats.argtypes = [c_void, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.ffv_kernel_stats.restype = c_int
    L.ffv_op_conv.argtypes = [c_int, c_void, c_int, c_int, c_int, c_int, c_void, c_void, c_int,
                              c_int, c_int, c_int, c_int, c_int, c_void, c_void]
    L.ffv_op_conv.restype = c_int
    L.ffv_op_conv_noalloc.argtypes = L.ffv_op_conv.argtypes
    L.ffv_op_conv_noalloc.restype = c_int
    L.ffv_lap_loss.argtypes = [c_void, c_void, c_int, c_int, c_int, c_void, c_void, c_void]
    L.ffv_lap_loss.restype = c_int
    L.ffv_autotune.argtypes = [c_void, ctypes.POINTER(ffv_pair), c_int, ctypes.POINTER(c_f), c_int,
                               c_void, ctypes.POINTER(c_int)]
    L.ffv_autotune.restype = c_int
    L.ffv_interpolate_blend.argtypes = [c_void, ctypes.POINTER(ffv_pair), c_int, ctypes.POINTER(c_f),
                                        c_int, c_void]
    L.ffv_interpolate_blend.restype = c_int
    L.ffv_interpolate_recursive.argtypes = [c_void, ctypes.POINTER(ffv_pair), c_int, c_int, c_void]
    L.ffv_interpolate_recursive.restype = c_int
    L.ffv_stitch_cluster.argtypes = [c_void, ctypes.POINTER(c_void), ctypes.POINTER(c_void), c_int,
                                     c_int, c_int, c_void, c_void]
    L.ffv_stitch_cluster.restype = c_int
    L.ffv_save_tuning.argtypes = [c_void, ctypes.c_char_p]
    L.ffv_save_tuning.restype = c_int
    L.ffv_load_tuning.argtypes = [c_void, ctypes.c_char_p, ctypes.POINTER(c_int)]
    L.ffv_load_tuning.restype = c_int
    L.ffv_calibrate.argtypes = [c_void, ctypes.POINTER(ffv_pair), c_f]
    L.ffv_calibrate.restype = c_int
    L.ffv_register_camera.argtypes = [c_void, c_int, c_void, c_int, c_int]
    L.ffv_register_camera.restype = c_int
    L.ffv_submit.argtypes = [c_void, ctypes.POINTER(ffv_request), ctypes.POINTER(ctypes.c_uint64)]
    L.ffv_submit.restype = c_int
    L.ffv_submit_many.argtypes = [c_void, ctypes.POINTER(ffv_request), c_int, ctypes.POINTER(ctypes.c_uint64)]
    L.ffv_submit_many.restype = c_int
    L.ffv_poll.argtypes = [c_void, ctypes.c_uint64, ctypes.POINTER(ffv_timing)]
    L.ffv_poll.restype = c_int
    L.ffv_serving_stats.argtypes = [c_void, ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_uint64)]
    L.ffv_serving_stats.restype = c_int
    L.ffv_debug_fault.argtypes = [ctypes.c_char_p]
    L.ffv_debug_fault.restype = c_int
    _lib = L
    return L


def _check(code: int) -> int:
    if code < 0:
        msg = lib().ffv_last_error()
        raise FfvError(code, msg.decode() if msg else "")
    return code


def _dev_f32(x: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float32:
        raise TypeError(f"{name} must be a float32 CUDA tensor")
    if not x.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    return x


class Net:
    """A loaded network on one GPU. ``precision`` is "fp32" or "bf16"."""

    def __init__(self, weights_path: str, precision: str = "fp32", device: int = 0,
                 workspace_bytes: int = 0, hbm_budget_bytes: int = 0, tick_ms: float = 5.0,
                 max_batch_views: int = 0, graphs: bool = True):
        L = lib()
        self.device = torch.device("cuda", device)
        # The library works on this stream; calls order it after the caller's
        # current stream.
        self.stream = torch.cuda.Stream(device=self.device)
        opts = ffv_opts()
        L.ffv_default_opts(ctypes.byref(opts))
        opts.precision = PRECISIONS[precision]
        opts.device = device
        opts.stream = self.stream.cuda_stream
        opts.workspace_bytes = workspace_bytes
        opts.hbm_budget_bytes = hbm_budget_bytes
        opts.tick_ms = tick_ms
        opts.max_batch_views = max_batch_views
        opts.graphs = 1 if graphs else 0
        h = ctypes.c_void_p()
        _check(L.ffv_create_net(os.fsencode(weights_path), ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self.precision = precision
        self._cam_shapes = {}  # registered camera id -> (H, W)

    def close(self):
        if getattr(self, "_h", None):
            lib().ffv_destroy_net(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def interpolate(self, pairs, ts, out: torch.Tensor | None = None) -> torch.Tensor:
        """``pairs``: list of (left, right) [3, H, W] float32 CUDA tensors.
        ``ts``: phases in [0, 1]. Returns [n_pairs, n_t, 3, H, W] float32."""
        arr, tarr, out = self._call_args(pairs, ts, out)
        _check(lib().ffv_interpolate(self._h, arr, len(arr), tarr, len(tarr), out.data_ptr()))
        return out

    def interpolate_blend(self, pairs, ts, out: torch.Tensor | None = None) -> torch.Tensor:
        """The Eq. 1 blend alone (no refinement), shaped as ``interpolate``."""
        arr, tarr, out = self._call_args(pairs, ts, out)
        _check(lib().ffv_interpolate_blend(self._h, arr, len(arr), tarr, len(tarr), out.data_ptr()))
        return out

    def interpolate_recursive(self, pairs, levels: int, out: torch.Tensor | None = None) -> torch.Tensor:
        """Recursive midpoints: [n_pairs, 2^levels - 1, 3, H, W], view k-1 at
        t = k / 2^levels."""
        n_views = (1 << levels) - 1
        arr, _, out = self._call_args(pairs, [0.5] * n_views, out)
        _check(lib().ffv_interpolate_recursive(self._h, arr, len(arr), levels, out.data_ptr()))
        return out

    def autotune(self, pairs, ts, out: torch.Tensor | None = None) -> int:
        """Run the call as ``interpolate`` does, then tune the conv tiles of
        its launches; returns the number of launch shapes tuned."""
        arr, tarr, out = self._call_args(pairs, ts, out)
        n = ctypes.c_int32(0)
        _check(lib().ffv_autotune(self._h, arr, len(arr), tarr, len(tarr), out.data_ptr(),
                                  ctypes.byref(n)))
        return n.value

    def save_tuning(self, path: str):
        _check(lib().ffv_save_tuning(self._h, os.fsencode(path)))

    def load_tuning(self, path: str) -> int:
        n = ctypes.c_int32(0)
        _check(lib().ffv_load_tuning(self._h, os.fsencode(path), ctypes.byref(n)))
        return n.value

    def _call_args(self, pairs, ts, out):
        pairs = list(pairs)
        ts = [float(t) for t in ts]
        if not pairs or not ts:
            raise ValueError("need at least one pair and one t")
        H, W = pairs[0][0].shape[-2:]
        arr = (ffv_pair * len(pairs))()
        for i, (l, r) in enumerate(pairs):
            _dev_f32(l, "left")
            _dev_f32(r, "right")
            if l.dim() != 3 or l.shape[0] != 3 or l.shape != r.shape:
                raise ValueError("views must be [3, H, W] and equal in shape")
            arr[i] = ffv_pair(l.data_ptr(), r.data_ptr(), int(l.shape[1]), int(l.shape[2]))
        if out is None:
            out = torch.empty((len(pairs), len(ts), 3, H, W), dtype=torch.float32,
                              device=pairs[0][0].device)
        _dev_f32(out, "out")
        if out.numel() != len(pairs) * len(ts) * 3 * H * W:
            raise ValueError("out has the wrong size")
        tarr = (ctypes.c_float * len(ts))(*ts)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        return arr, tarr, out

    def calibrate(self, left: torch.Tensor, right: torch.Tensor, t: float = 0.5):
        """FP8 nets: set the activation scales from one representative view."""
        _dev_f32(left, "left")
        _dev_f32(right, "right")
        pr = ffv_pair(left.data_ptr(), right.data_ptr(), int(left.shape[1]), int(left.shape[2]))
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        _check(lib().ffv_calibrate(self._h, ctypes.byref(pr), float(t)))

    # ---------------------------------------------------------------- serving
    def register_camera(self, cam_id: int, image: torch.Tensor):
        """Make ``image`` ([3, H, W] float32 CUDA) resident as camera ``cam_id``."""
        _dev_f32(image, "image")
        if image.dim() != 3 or image.shape[0] != 3:
            raise ValueError("image must be [3, H, W]")
        torch.cuda.current_stream(self.device).synchronize()
        _check(lib().ffv_register_camera(self._h, cam_id, image.data_ptr(), int(image.shape[1]),
                                         int(image.shape[2])))
        self._cam_shapes[cam_id] = (int(image.shape[1]), int(image.shape[2]))

    def submit(self, cam_left: int, cam_right: int, t: float, out: torch.Tensor,
               tag: int = 0) -> int:
        """Queue one view; ``out`` ([3, H, W] float32 CUDA) must stay alive
        until ``poll`` reports it done. Returns the ticket."""
        _dev_f32(out, "out")
        hw = self._cam_shapes.get(cam_left)
        if hw is not None and tuple(out.shape) != (3,) + hw:
            raise ValueError(f"out must be [3, {hw[0]}, {hw[1]}] for camera {cam_left}, got "
                             f"{list(out.shape)}")
        req = ffv_request(cam_left, cam_right, float(t), out.data_ptr(), tag)
        tk = ctypes.c_uint64()
        torch.cuda.current_stream(self.device).synchronize()
        _check(lib().ffv_submit(self._h, ctypes.byref(req), ctypes.byref(tk)))
        return tk.value

    def submit_many(self, reqs) -> list:
        """Queue several views at once: ``reqs`` holds (cam_left, cam_right,
        t, out) tuples, checked like ``submit``; none is queued if one is
        bad. The scheduler sees the whole burst together. Returns the
        tickets in order."""
        reqs = list(reqs)
        arr = (ffv_request * max(1, len(reqs)))()
        for i, (cl, cr, t, out) in enumerate(reqs):
            _dev_f32(out, "out")
            hw = self._cam_shapes.get(cl)
            if hw is not None and tuple(out.shape) != (3,) + hw:
                raise ValueError(f"request {i}: out must be [3, {hw[0]}, {hw[1]}] for camera {cl}, got "
                                 f"{list(out.shape)}")
            arr[i] = ffv_request(cl, cr, float(t), out.data_ptr(), 0)
        tks = (ctypes.c_uint64 * max(1, len(reqs)))()
        torch.cuda.current_stream(self.device).synchronize()
        _check(lib().ffv_submit_many(self._h, arr, len(reqs), tks))
        return [tks[i] for i in range(len(reqs))]

    def poll(self, ticket: int):
        """None while pending; the timing dict once the view is written.
        Raises FfvError (e.g. FFV_ERR_DEVICE, FFV_ERR_OOM) when the view's
        batch failed; the ticket is collected either way."""
        tm = ffv_timing()
        code = _check(lib().ffv_poll(self._h, ticket, ctypes.byref(tm)))
        if code == 1:
            return None
        return {"t_submit": tm.t_submit, "t_admit": tm.t_admit, "t_launch": tm.t_launch,
                "t_done": tm.t_done}

    def serving_stats(self):
        a, c, q = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        b = ctypes.c_uint64()
        _check(lib().ffv_serving_stats(self._h, ctypes.byref(a), ctypes.byref(c), ctypes.byref(q),
                                       ctypes.byref(b)))
        return {"admitted": a.value, "completed": c.value, "queued": q.value,
                "bytes_in_use": b.value}

    def set_debug(self, on: bool = True):
        _check(lib().ffv_set_debug(self._h, 1 if on else 0))

    def debug_tap(self, name: str) -> torch.Tensor:
        cap = 1 << 26
        buf = torch.empty(cap, dtype=torch.float32, device=self.device)
        dims = (ctypes.c_int32 * 3)()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        _check(lib().ffv_debug_tap(self._h, name.encode(), buf.data_ptr(), cap, dims))
        c, h, w = dims[0], dims[1], dims[2]
        return buf[: c * h * w].view(c, h, w).clone()

    def set_profiling(self, on: bool = True):
        _check(lib().ffv_set_profiling(self._h, 1 if on else 0))

    def kernel_stats(self, name: str):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        work = ctypes.c_double()
        _check(lib().ffv_kernel_stats(self._h, name.encode(), ctypes.byref(n), ctypes.byref(ms),
                                      ctypes.byref(work)))
        return {"launches": n.value, "ms": ms.value, "work": work.value}


def debug_fault(spec: str | None):
    """Arm the library's fault-injection hook ("alloc:N", "launch:N"), or
    disarm it with None (tests of the error paths)."""
    _check(lib().ffv_debug_fault(spec.encode() if spec else None))


def op_conv(x: torch.Tensor, weight, bias, stride: int = 1, transposed: bool = False,
            relu: bool = False, precision: str = "fp32", n_tile: int = 0,
            tile_w: int = 0, act_out: bool = False, noalloc: bool = False) -> torch.Tensor:
    """One conv layer through the library's implicit-GEMM kernel.
    ``x``: [n, cin, h, w] float32 CUDA; ``weight``/``bias``: host arrays in
    the weights-file layout; ``n_tile``/``tile_w``: kernel variant (0 =
    default); ``act_out``: the layer writes activation-dtype output, as in
    the network, returned widened to float32; ``noalloc``: call
    ffv_op_conv_noalloc (device buffers in the library's fixed scratch
    array) instead of ffv_op_conv."""
    import numpy as np
    _dev_f32(x, "x")
    n, cin, h, w = x.shape
    wt = np.ascontiguousarray(weight, dtype=np.float32)
    bs = np.ascontiguousarray(bias, dtype=np.float32)
    cout = wt.shape[1] if transposed else wt.shape[0]
    if transposed:
        ho, wo = 2 * h, 2 * w
    else:
        ho, wo = (h - 1) // stride + 1, (w - 1) // stride + 1
    y = torch.empty((n, cout, ho, wo), dtype=torch.float32, device=x.device)
    s = torch.cuda.current_stream(x.device)
    fn = lib().ffv_op_conv_noalloc if noalloc else lib().ffv_op_conv
    _check(fn(PRECISIONS[precision] | (FFV_OP_ACT_OUT if act_out else 0), x.data_ptr(), n, cin, h, w,
              wt.ctypes.data, bs.ctypes.data, cout, stride, 1 if transposed else 0,
              1 if relu else 0, n_tile, tile_w, y.data_ptr(), s.cuda_stream))
    return y


def lap_loss(x: torch.Tensor, gt: torch.Tensor, grad: bool = False):
    """Eq. 3 Laplacian-pyramid loss of each image in ``x`` against ``gt``
    ([n, 3, H, W] float32 CUDA): a float32 tensor [n], and with ``grad`` also
    d loss / d x [n, 3, H, W]."""
    _dev_f32(x, "x")
    _dev_f32(gt, "gt")
    if x.dim() != 4 or x.shape[1] != 3 or x.shape != gt.shape:
        raise ValueError("x and gt must both be [n, 3, H, W]")
    n, _, H, W = x.shape
    loss = torch.empty(n, dtype=torch.float32, device=x.device)
    g = torch.empty_like(x) if grad else None
    s = torch.cuda.current_stream(x.device)
    _check(lib().ffv_lap_loss(x.data_ptr(), gt.data_ptr(), n, H, W, loss.data_ptr(),
                              g.data_ptr() if grad else None, s.cuda_stream))
    return (loss, g) if grad else loss


def stitch_cluster(real_view: torch.Tensor, left, right, out: torch.Tensor | None = None) -> torch.Tensor:
    """Cluster frame [3, H, 3W] = [left block | real view | right block] of
    the library's stitch kernel; ``left``/``right``: lists of g*g [3, H, W]
    float32 CUDA views."""
    _dev_f32(real_view, "real_view")
    left, right = list(left), list(right)
    _, H, W = real_view.shape
    for v in left + right:
        _dev_f32(v, "view")
        if v.shape != real_view.shape:
            raise ValueError("views must match the real view's shape")
    if out is None:
        out = torch.empty((3, H, 3 * W), dtype=torch.float32, device=real_view.device)
    _dev_f32(out, "out")
    la = (ctypes.c_void_p * max(1, len(left)))(*[v.data_ptr() for v in left])
    ra = (ctypes.c_void_p * max(1, len(right)))(*[v.data_ptr() for v in right])
    s = torch.cuda.current_stream(real_view.device)
    _check(lib().ffv_stitch_cluster(real_view.data_ptr(), la, ra, len(left), H, W, out.data_ptr(),
                                    s.cuda_stream))
    return out
