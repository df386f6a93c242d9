"""Tensor-level helpers over the C entry points (PyTorch supplies device memory
and the current stream; all computation is in the HIP library)."""
from __future__ import annotations

import ctypes

from . import _binding as B


def _torch():
    import torch
    return torch


def _check_tensor(t, name, shape=None, device=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name} is on cuda:{t.device.index}, expected cuda:{device}")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous float32")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _device():
    return _torch().cuda.current_device()


def _quiesce(device) -> bool:
    """Waits for the device's queued work, so that a plan's code and memory
    are freed only once no launch can still use them. False while the
    current stream captures a graph (the handle is then kept, not freed)."""
    torch = _torch()
    if torch.cuda.is_current_stream_capturing():
        return False
    torch.cuda.synchronize(device)
    return True


def _stream(stream):
    if stream is None:
        return _torch().cuda.current_stream().cuda_stream
    return int(getattr(stream, "cuda_stream", stream))


class Plan:
    """A compiled configuration for one (out_h, out_w, filt_h, filt_w) shape."""

    def __init__(self, out_h, out_w, filt_h, filt_w, config=None):
        self.shape = B.shape(out_h, out_w, filt_h, filt_w)
        self._device = _device()
        self.handle = B.conv2d_plan(self.shape, config)
        cfg, src = B.conv2d_plan_config(self.handle)
        self.config = cfg.tuple()
        self.source = {0: "default", 1: "tuned", 2: "given", 3: "tuned-older-kernel",
                       4: "tuned-other-shape"}.get(src, str(src))

    def __call__(self, inp, filt, out=None, stream=None):
        torch = _torch()
        H, W, fh, fw = self.shape.tuple()
        _check_tensor(inp, "inp", (H + fh - 1, W + fw - 1), self._device)
        _check_tensor(filt, "filt", (fh, fw), self._device)
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=inp.device)
        _check_tensor(out, "out", (H, W), self._device)
        B.conv2d_run(self.handle, inp.data_ptr(), filt.data_ptr(), out.data_ptr(), _stream(stream))
        return out

    def close(self):
        """Frees the plan once its device has finished the queued work."""
        if self.handle and _quiesce(self._device):
            B.conv2d_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_plans: dict = {}


def conv2d(inp, filt, config=None, out=None, stream=None):
    """One convolution; plans are cached per (device, shape, config). A plan
    whose filter goes to constant memory copies the filter into its module's
    one constant array before each launch, so two streams must not share it:
    such plans are cached per stream as well."""
    fh, fw = filt.shape
    H, W = inp.shape[0] - fh + 1, inp.shape[1] - fw + 1
    key = (_device(), H, W, fh, fw, None if config is None else tuple(B.config(config).tuple()))
    st = _stream(stream)
    plan = _plans.get(key)
    if plan is None:
        plan = _plans[key] = Plan(H, W, fh, fw, config)
        plan._first_stream = st
    if plan.config[5] == 1 and plan._first_stream != st:
        skey = key + (st,)
        plan = _plans.get(skey)
        if plan is None:
            plan = _plans[skey] = Plan(H, W, fh, fw, _plans[key].config)
    return plan(inp, filt, out=out, stream=stream)


def reference(inp, filt, out=None, stream=None):
    """The library's plain reference kernel (one thread per output)."""
    torch = _torch()
    dev = _device()
    _check_tensor(inp, "inp", device=dev)
    _check_tensor(filt, "filt", device=dev)
    if inp.dim() != 2 or filt.dim() != 2:
        raise ValueError("inp and filt must be 2-D")
    fh, fw = filt.shape
    H, W = inp.shape[0] - fh + 1, inp.shape[1] - fw + 1
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=inp.device)
    _check_tensor(out, "out", (H, W), dev)
    B.conv2d_reference(B.shape(H, W, fh, fw), inp.data_ptr(), filt.data_ptr(), out.data_ptr(), _stream(stream))
    return out


class Batch:
    """Many convolutions (uneven sizes, mixed filter sizes) run by one graph launch."""

    def __init__(self, shapes, flags=0):
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self._device = _device()
        self.handle = B.conv2d_batch_plan(self.shapes, flags)
        self.info = B.conv2d_batch_info(self.handle)

    def __call__(self, inputs, filters, outputs=None, stream=None):
        torch = _torch()
        if len(inputs) != len(self.shapes) or len(filters) != len(self.shapes):
            raise ValueError("one input and one filter per problem")
        if outputs is None:
            outputs = [torch.empty((H, W), dtype=torch.float32, device=inputs[0].device)
                       for (H, W, _, _) in self.shapes]
        for k, (H, W, fh, fw) in enumerate(self.shapes):
            _check_tensor(inputs[k], f"inputs[{k}]", (H + fh - 1, W + fw - 1), self._device)
            _check_tensor(filters[k], f"filters[{k}]", (fh, fw), self._device)
            _check_tensor(outputs[k], f"outputs[{k}]", (H, W), self._device)
        B.conv2d_batch_run(self.handle, [t.data_ptr() for t in inputs], [t.data_ptr() for t in filters],
                           [t.data_ptr() for t in outputs], _stream(stream))
        return outputs

    def bind(self, inputs, filters, outputs):
        """Checks the tensors once and returns a callable run(stream=None)
        that enqueues the batch on them with no per-call Python checks (the
        library still compares the pointers with the last upload). The
        tensors must stay alive while the callable is used."""
        if len(inputs) != len(self.shapes) or len(filters) != len(self.shapes) or len(outputs) != len(self.shapes):
            raise ValueError("one input, filter and output per problem")
        for k, (H, W, fh, fw) in enumerate(self.shapes):
            _check_tensor(inputs[k], f"inputs[{k}]", (H + fh - 1, W + fw - 1), self._device)
            _check_tensor(filters[k], f"filters[{k}]", (fh, fw), self._device)
            _check_tensor(outputs[k], f"outputs[{k}]", (H, W), self._device)
        n = len(self.shapes)
        keep = (list(inputs), list(filters), list(outputs))
        arrays = [(ctypes.c_void_p * n)(*[t.data_ptr() for t in ts]) for ts in keep]
        run = B.lib.conv2d_batch_run

        def bound(stream=None):
            # the handle is read at each call: after close() it is None, which
            # the library rejects
            B.check(run(self.handle, *arrays, _stream(stream)), "conv2d_batch_run")
            return keep[2]
        return bound

    def close(self):
        """Frees the batch once its device has finished the queued work."""
        if self.handle and _quiesce(self._device):
            B.conv2d_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hotspot:
    """A compiled hotspot configuration for one rows x cols grid (the tuned
    winner of the hotspot winners cache when one exists, else the default)."""

    def __init__(self, rows, cols, config=None):
        self.shape = B.hotspot_shape(rows, cols)
        self._device = _device()
        self.handle = B.hotspot_plan(self.shape, config)
        self.config, tuned = B.hotspot_plan_config(self.handle)
        self.source = "given" if config is not None else {1: "tuned", 2: "tuned-other-grid"}.get(tuned, "default")
        self._work = None

    def __call__(self, temp, power, steps, coeffs, out=None, stream=None):
        """The grid after `steps` steps; coeffs = (cc, gx, gy, gz, t_amb).
        Calls of one Hotspot object share its work grid: calls on different
        streams must not overlap."""
        torch = _torch()
        shp = (self.shape.rows, self.shape.cols)
        _check_tensor(temp, "temp", shp, self._device)
        _check_tensor(power, "power", shp, self._device)
        if out is None:
            out = torch.empty(shp, dtype=torch.float32, device=temp.device)
        _check_tensor(out, "out", shp, self._device)
        work = 0
        if steps > self.config[4]:
            if self._work is None or self._work.device != temp.device:
                self._work = torch.empty(shp, dtype=torch.float32, device=temp.device)
            work = self._work.data_ptr()
        B.hotspot_run(self.handle, temp.data_ptr(), power.data_ptr(), out.data_ptr(), work, steps,
                      B.hotspot_coeffs(*coeffs), _stream(stream))
        return out

    def close(self):
        """Frees the plan once its device has finished the queued work."""
        if self.handle and _quiesce(self._device):
            B.hotspot_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reference_hotspot(temp, power, steps, coeffs, out=None, stream=None):
    """The library's one-step-per-launch hotspot reference."""
    torch = _torch()
    dev = _device()
    _check_tensor(temp, "temp", device=dev)
    if temp.dim() != 2:
        raise ValueError("temp must be 2-D")
    rows, cols = temp.shape
    _check_tensor(power, "power", (rows, cols), dev)
    if out is None:
        out = torch.empty((rows, cols), dtype=torch.float32, device=temp.device)
    _check_tensor(out, "out", (rows, cols), dev)
    # torch's caching allocator keeps the work buffer's memory for this
    # stream until the stream has passed the launches
    work = torch.empty((rows, cols), dtype=torch.float32, device=temp.device) if steps > 1 else None
    B.hotspot_reference(B.hotspot_shape(rows, cols), temp.data_ptr(), power.data_ptr(), out.data_ptr(),
                        0 if work is None else work.data_ptr(), steps, B.hotspot_coeffs(*coeffs), _stream(stream))
    return out
