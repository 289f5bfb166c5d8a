"""ctypes binding of libconet.so: argument marshalling only.

PyTorch supplies device memory (the model workspace, inputs and outputs) and the
stream; every step of the receiver runs in the library's HIP kernels. There is no
fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libconet.so")

CONET_FP32, CONET_BF16, CONET_FP8E4M3 = 0, 1, 2
DTYPES = {"f32": CONET_FP32, "fp32": CONET_FP32, "bf16": CONET_BF16, "fp8": CONET_FP8E4M3}
STATUS = {0: "OK", 1: "EINVAL", 2: "ESHAPE", 3: "ENOMEM", 4: "EDEVICE", 5: "EBUSY", 6: "ETIMEOUT", 7: "ESTATE"}

# Every symbol include/conet.h declares.
EXPORTS = ("conet_weight_count", "conet_workspace_bytes", "conet_create", "conet_set_act_scales",
           "conet_calibrate", "conet_get_act_scales", "conet_forward", "conet_forward_ragged", "conet_forward_profiled",
           "conet_forward_noalloc", "conet_forward_noalloc_capacity", "conet_forward_grid",
           "conet_block_tile_width", "conet_mfma_peak", "conet_mfma_dot", "conet_featurise", "conet_featurise_var", "conet_simulate",
           "conet_graph_create", "conet_graph_launch", "conet_graph_destroy",
           "conet_serve_create", "conet_serve_submit", "conet_serve_wait", "conet_serve_get_stats",
           "conet_serve_reset_stats", "conet_serve_pause", "conet_serve_destroy", "conet_backward", "conet_grads",
           "conet_master_weights", "conet_adam_step", "conet_get_weights", "conet_save_train_state",
           "conet_load_train_state", "conet_bce", "conet_destroy",
           "conet_last_error")


class ConetError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class conet_config(ctypes.Structure):
    _fields_ = [("branches", ctypes.c_int32), ("blocks", ctypes.c_int32), ("channels", ctypes.c_int32),
                ("in_channels", ctypes.c_int32), ("bits_per_symbol", ctypes.c_int32),
                ("fuse_mask", ctypes.c_uint32), ("ln_eps", ctypes.c_float), ("dtype", ctypes.c_int32),
                ("train", ctypes.c_int32), ("max_res", ctypes.c_int64), ("fusion_op", ctypes.c_int32),
                ("feedback", ctypes.c_int32), ("norm", ctypes.c_int32), ("support_blocks", ctypes.c_int32),
                ("block_type", ctypes.c_int32)]


class conet_sim_config(ctypes.Structure):
    _fields_ = [("F", ctypes.c_int32), ("T", ctypes.c_int32), ("n_rx", ctypes.c_int32),
                ("bits_per_symbol", ctypes.c_int32), ("n_taps", ctypes.c_int32), ("max_doppler_hz", ctypes.c_float),
                ("snr_lo_db", ctypes.c_float), ("snr_hi_db", ctypes.c_float), ("seed", ctypes.c_uint64)]


class conet_request(ctypes.Structure):
    _fields_ = [("n_prb", ctypes.c_int32), ("n_rx", ctypes.c_int32), ("bits_per_symbol", ctypes.c_int32),
                ("T", ctypes.c_int32), ("x_host", ctypes.c_void_p), ("llr_host", ctypes.c_void_p),
                ("tag", ctypes.c_uint64), ("input", ctypes.c_int32)]


class conet_serve_stats(ctypes.Structure):
    _fields_ = [("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double), ("mean_us", ctypes.c_double),
                ("max_us", ctypes.c_double), ("res_per_s", ctypes.c_double), ("mean_batch_requests", ctypes.c_double),
                ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("lane_res", ctypes.c_int64), ("mean_queue_us", ctypes.c_double), ("mean_prep_us", ctypes.c_double),
                ("mean_device_us", ctypes.c_double), ("mean_scatter_us", ctypes.c_double),
                ("mean_h2d_us", ctypes.c_double), ("mean_forward_us", ctypes.c_double), ("mean_d2h_us", ctypes.c_double),
                ("direct_inputs", ctypes.c_uint64), ("direct_outputs", ctypes.c_uint64),
                ("slowest_queue_us", ctypes.c_double), ("slowest_prep_us", ctypes.c_double),
                ("slowest_device_us", ctypes.c_double), ("slowest_scatter_us", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libconet.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2510_12739_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    cfgp = ctypes.POINTER(conet_config)
    fp = ctypes.POINTER(ctypes.c_float)
    lib.conet_weight_count.argtypes = [cfgp]; lib.conet_weight_count.restype = sz
    lib.conet_workspace_bytes.argtypes = [cfgp]; lib.conet_workspace_bytes.restype = sz
    lib.conet_create.argtypes = [cfgp, fp, sz, vp, sz, ctypes.POINTER(vp)]; lib.conet_create.restype = i32
    lib.conet_set_act_scales.argtypes = [vp, fp, sz]; lib.conet_set_act_scales.restype = i32
    lib.conet_get_act_scales.argtypes = [vp, fp, sz]; lib.conet_get_act_scales.restype = i32
    lib.conet_calibrate.argtypes = [vp, vp, i32, i32, i32, vp]; lib.conet_calibrate.restype = i32
    lib.conet_forward.argtypes = [vp, vp, i32, i32, i32, vp, i32, vp]; lib.conet_forward.restype = i32
    lib.conet_forward_ragged.argtypes = [vp, vp, i32, i32, ctypes.POINTER(i32), vp, vp]
    lib.conet_forward_ragged.restype = i32
    lib.conet_forward_profiled.argtypes = [vp, vp, i32, i32, i32, vp, fp, ctypes.POINTER(i32), i32, vp]
    lib.conet_forward_profiled.restype = i32
    lib.conet_forward_noalloc.argtypes = [vp, vp, i32, i32, i32, vp, vp]; lib.conet_forward_noalloc.restype = i32
    lib.conet_forward_noalloc_capacity.argtypes = [vp]; lib.conet_forward_noalloc_capacity.restype = i64
    lib.conet_block_tile_width.argtypes = [vp]; lib.conet_block_tile_width.restype = i32
    dp = ctypes.POINTER(ctypes.c_double)
    lib.conet_mfma_peak.argtypes = [i32, i32, dp, dp, vp]; lib.conet_mfma_peak.restype = i32
    lib.conet_mfma_dot.argtypes = [i32, i32, vp, vp, ctypes.POINTER(ctypes.c_float)]; lib.conet_mfma_dot.restype = i32
    lib.conet_featurise.argtypes = [vp, i32, i32, i32, i32, i32, vp, vp]; lib.conet_featurise.restype = i32
    lib.conet_forward_grid.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp]; lib.conet_forward_grid.restype = i32
    lib.conet_simulate.argtypes = [ctypes.POINTER(conet_sim_config), ctypes.c_int64, i32, vp, vp, vp, vp]
    lib.conet_simulate.restype = i32
    lib.conet_graph_create.argtypes = [vp, vp, i32, i32, i32, vp, ctypes.POINTER(vp)]
    lib.conet_graph_create.restype = i32
    lib.conet_graph_launch.argtypes = [vp, vp]; lib.conet_graph_launch.restype = i32
    lib.conet_graph_destroy.argtypes = [vp]; lib.conet_graph_destroy.restype = i32
    lib.conet_featurise_var.argtypes = [vp, vp, i32, i32, i32, i32, i32, vp, vp]; lib.conet_featurise_var.restype = i32
    lib.conet_serve_create.argtypes = [vp, sz, i32, i32, i32, ctypes.POINTER(vp)]
    lib.conet_serve_create.restype = i32
    lib.conet_serve_submit.argtypes = [vp, ctypes.POINTER(conet_request), ctypes.POINTER(ctypes.c_uint64)]
    lib.conet_serve_submit.restype = i32
    lib.conet_serve_wait.argtypes = [vp, ctypes.c_uint64, i64, ctypes.POINTER(ctypes.c_double)]
    lib.conet_serve_wait.restype = i32
    lib.conet_serve_get_stats.argtypes = [vp, ctypes.POINTER(conet_serve_stats)]
    lib.conet_serve_get_stats.restype = i32
    lib.conet_serve_reset_stats.argtypes = [vp]; lib.conet_serve_reset_stats.restype = i32
    lib.conet_serve_pause.argtypes = [vp, i32]; lib.conet_serve_pause.restype = i32
    lib.conet_serve_destroy.argtypes = [vp]; lib.conet_serve_destroy.restype = i32
    lib.conet_backward.argtypes = [vp, vp, vp]; lib.conet_backward.restype = i32
    lib.conet_grads.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(sz)]; lib.conet_grads.restype = i32
    lib.conet_master_weights.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(sz)]
    lib.conet_master_weights.restype = i32
    lib.conet_adam_step.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]
    lib.conet_adam_step.restype = i32
    lib.conet_get_weights.argtypes = [vp, fp, sz]; lib.conet_get_weights.restype = i32
    lib.conet_save_train_state.argtypes = [vp, fp, fp, fp, sz, ctypes.POINTER(i32)]
    lib.conet_save_train_state.restype = i32
    lib.conet_load_train_state.argtypes = [vp, fp, fp, fp, sz, i32]; lib.conet_load_train_state.restype = i32
    lib.conet_bce.argtypes = [vp, vp, vp, vp, i32, i32, i32, i64, vp, vp, vp]; lib.conet_bce.restype = i32
    lib.conet_destroy.argtypes = [vp]; lib.conet_destroy.restype = i32
    lib.conet_last_error.argtypes = []; lib.conet_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(st: int):
    if st != 0:
        raise ConetError(st, load().conet_last_error().decode())


FUSIONS = {"product": 0, "sum": 1, "concat": 2}
NORMS = {"ln": 0, "bn": 1}
BLOCKS = {"standard": 0, "ds": 1}


def make_config(K: int, L: int, C: int, C_in: int, m: int, dtype: str = "bf16", fuse_mask: int = -1,
                max_res: int = 1 << 20, ln_eps: float = 1e-5, train: bool = False, fusion: str = "product",
                feedback: bool = False, norm: str = "ln", support_blocks: int = 0,
                block: str = "standard") -> conet_config:
    """fuse_mask -1: fusion after every block the support branches have (support_blocks, or L)."""
    Ls = L if support_blocks <= 0 else support_blocks
    mask = ((1 << Ls) - 1) if fuse_mask < 0 else int(fuse_mask)
    return conet_config(K, L, C, C_in, m, mask, ln_eps, DTYPES[dtype], 1 if train else 0, int(max_res),
                        FUSIONS[fusion], 1 if feedback else 0, NORMS[norm], int(support_blocks), BLOCKS[block])


def weight_count(cfg: conet_config) -> int:
    return int(load().conet_weight_count(ctypes.byref(cfg)))


def workspace_bytes(cfg: conet_config) -> int:
    return int(load().conet_workspace_bytes(ctypes.byref(cfg)))


def _stream_ptr(stream) -> ctypes.c_void_p:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Conet:
    """A CoNet-Rx model resident on the current GPU.

    The workspace (filters in fragment order, vectors, activations for up to max_res
    REs) is one torch uint8 tensor owned by this object.
    """

    def __init__(self, K: int, L: int, C: int, C_in: int, m: int, blob: np.ndarray, dtype: str = "bf16",
                 fuse_mask: int = -1, max_res: int = 1 << 20, device=None, train: bool = False,
                 fusion: str = "product", feedback: bool = False, norm: str = "ln", support_blocks: int = 0,
                 block: str = "standard"):
        import torch
        self.lib = load()
        self.train = train
        self.cfg = make_config(K, L, C, C_in, m, dtype, fuse_mask, max_res, train=train, fusion=fusion,
                               feedback=feedback, norm=norm, support_blocks=support_blocks, block=block)
        self.K, self.L, self.C, self.C_in, self.m, self.dtype = K, L, C, C_in, m, dtype
        n = weight_count(self.cfg)
        if n == 0:
            raise ConetError(1, self.lib.conet_last_error().decode())
        blob = np.ascontiguousarray(blob, dtype=np.float32)
        if blob.size != n:
            raise ValueError(f"blob has {blob.size} values, configuration needs {n}")
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        nbytes = workspace_bytes(self.cfg)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib.conet_create(ctypes.byref(self.cfg), blob.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                         n, ctypes.c_void_p(self.workspace.data_ptr()), nbytes, ctypes.byref(handle)))
        self.handle = handle

    @property
    def n_scales(self) -> int:
        return 1 + 2 * self.K * self.L

    def set_act_scales(self, scales: Sequence[float]):
        s = np.ascontiguousarray(scales, dtype=np.float32)
        _check(self.lib.conet_set_act_scales(self.handle, s.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), s.size))

    def get_act_scales(self) -> np.ndarray:
        s = np.zeros(self.n_scales, dtype=np.float32)
        _check(self.lib.conet_get_act_scales(self.handle, s.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), s.size))
        return s

    def calibrate(self, x, stream=None):
        B, T, F, _ = x.shape
        _check(self.lib.conet_calibrate(self.handle, ctypes.c_void_p(x.data_ptr()), B, T, F, _stream_ptr(stream)))

    def _check_x(self, x):
        import torch
        if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
            raise ValueError("x must be a contiguous float32 CUDA tensor")
        if x.shape[-1] != self.C_in:
            raise ValueError(f"x has {x.shape[-1]} channels, model expects {self.C_in}")

    def forward(self, x, out=None, stream=None, save: bool = False):
        """x: [B, T, F, C_in] float32 on the GPU -> LLR [B, T, F, m] float32 (enqueued on the stream).

        save=True (train models) keeps the activations for backward(); x must stay alive."""
        import torch
        self._check_x(x)
        B, T, F, _ = x.shape
        if out is None:
            out = torch.empty((B, T, F, self.m), dtype=torch.float32, device=x.device)
        _check(self.lib.conet_forward(self.handle, ctypes.c_void_p(x.data_ptr()), B, T, F,
                                      ctypes.c_void_p(out.data_ptr()), 1 if save else 0, _stream_ptr(stream)))
        if save:
            self._saved_x = x
        return out

    def forward_noalloc(self, x, out, stream=None):
        """conet_forward_noalloc: the forward with its activation buffers in the library's static
        device array (no allocation; `out` must be given). Calls on one GPU must not overlap."""
        self._check_x(x)
        B, T, F, _ = x.shape
        _check(self.lib.conet_forward_noalloc(self.handle, ctypes.c_void_p(x.data_ptr()), B, T, F,
                                              ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    @property
    def noalloc_capacity(self) -> int:
        return int(self.lib.conet_forward_noalloc_capacity(self.handle))

    # ---- training
    def _view(self, fn):
        import torch
        p, n = ctypes.c_void_p(), ctypes.c_size_t()
        _check(fn(self.handle, ctypes.byref(p), ctypes.byref(n)))
        off = p.value - self.workspace.data_ptr()
        return self.workspace[off:off + 4 * n.value].view(torch.float32)

    def grads(self):
        """Gradient buffer (device FP32, blob order; overwritten by backward())."""
        return self._view(self.lib.conet_grads)

    def master(self):
        """FP32 master weights (device, blob order)."""
        return self._view(self.lib.conet_master_weights)

    def backward(self, dllr, stream=None):
        _check(self.lib.conet_backward(self.handle, ctypes.c_void_p(dllr.data_ptr()), _stream_ptr(stream)))
        return self.grads()

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(self.lib.conet_adam_step(self.handle, lr, beta1, beta2, eps, _stream_ptr(stream)))

    def get_weights(self) -> np.ndarray:
        w = np.zeros(weight_count(self.cfg), dtype=np.float32)
        _check(self.lib.conet_get_weights(self.handle, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w.size))
        return w

    def save_train_state(self):
        """Checkpoint: (master weights, Adam first moment, second moment, Adam steps taken), host copies."""
        n = weight_count(self.cfg)
        bufs = [np.zeros(n, dtype=np.float32) for _ in range(3)]
        steps = ctypes.c_int32()
        fp = ctypes.POINTER(ctypes.c_float)
        _check(self.lib.conet_save_train_state(self.handle, *[b.ctypes.data_as(fp) for b in bufs], n,
                                               ctypes.byref(steps)))
        return bufs[0], bufs[1], bufs[2], int(steps.value)

    def load_train_state(self, master, m, v, steps: int):
        """Resume from save_train_state() of a model with the same configuration."""
        fp = ctypes.POINTER(ctypes.c_float)
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (master, m, v)]
        _check(self.lib.conet_load_train_state(self.handle, *[a.ctypes.data_as(fp) for a in arrs], arrs[0].size,
                                               int(steps)))

    def bce(self, llr, bits, data_mask, n_data_per_slot: int, stream=None):
        """Bitwise BCE on device: returns (loss tensor [1], dllr)."""
        import torch
        B, T, F, _ = llr.shape
        dllr = torch.empty_like(llr)
        loss = torch.empty(1, dtype=torch.float32, device=llr.device)
        _check(self.lib.conet_bce(self.handle, ctypes.c_void_p(llr.data_ptr()), ctypes.c_void_p(bits.data_ptr()),
                                  ctypes.c_void_p(data_mask.data_ptr()), B, T, F, int(n_data_per_slot),
                                  ctypes.c_void_p(dllr.data_ptr()), ctypes.c_void_p(loss.data_ptr()),
                                  _stream_ptr(stream)))
        return loss, dllr

    __call__ = forward

    @property
    def block_tile_width(self) -> int:
        """Subcarriers per fused residual-block tile of inference forwards (0: two conv launches per block)."""
        return int(self.lib.conet_block_tile_width(self.handle))

    def forward_profiled(self, x, out=None, stream=None, units: bool = False):
        """forward() with per-stage HIP event timing: returns (llr, stage_ms[1 + 3L]), plus the
        per-stage conv-branch units when units=True."""
        import torch
        self._check_x(x)
        B, T, F, _ = x.shape
        if out is None:
            out = torch.empty((B, T, F, self.m), dtype=torch.float32, device=x.device)
        ms = np.zeros(1 + 3 * self.L, dtype=np.float32)
        un = np.zeros(1 + 3 * self.L, dtype=np.int32)
        _check(self.lib.conet_forward_profiled(self.handle, ctypes.c_void_p(x.data_ptr()), B, T, F,
                                               ctypes.c_void_p(out.data_ptr()),
                                               ms.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                               un.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ms.size,
                                               _stream_ptr(stream)))
        return (out, ms, un) if units else (out, ms)

    def forward_grid(self, y, out=None, stream=None):
        """conet_forward_grid: y is the received grid, a contiguous float32 CUDA tensor
        [B][T][F][n_rx][2]; the input layer forms the features while staging. Returns LLRs
        [B][T][F][m]."""
        import torch
        if not (y.is_cuda and y.dtype == torch.float32 and y.is_contiguous() and y.dim() == 5 and y.shape[-1] == 2):
            raise ValueError("y must be a contiguous float32 CUDA tensor [B][T][F][n_rx][2]")
        B, T, F, n_rx, _ = y.shape
        if out is None:
            out = torch.empty((B, T, F, self.m), dtype=torch.float32, device=y.device)
        _check(self.lib.conet_forward_grid(self.handle, ctypes.c_void_p(y.data_ptr()), B, T, F, n_rx,
                                           ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def record(self, x, out):
        """conet_graph_create: the forward of x into out recorded as a HIP graph; returns a
        ForwardGraph whose launch() recomputes out from x's current contents."""
        self._check_x(x)
        B, T, F, _ = x.shape
        h = ctypes.c_void_p()
        _check(self.lib.conet_graph_create(self.handle, ctypes.c_void_p(x.data_ptr()), B, T, F,
                                           ctypes.c_void_p(out.data_ptr()), ctypes.byref(h)))
        return ForwardGraph(self, h, x, out)

    def forward_ragged(self, x_packed, T: int, F_list: Sequence[int], out=None, stream=None):
        """Slots of different widths packed back to back: x_packed [sum T*F_s, C_in]."""
        import torch
        self._check_x(x_packed)
        F_arr = (ctypes.c_int32 * len(F_list))(*[int(f) for f in F_list])
        n_re = int(sum(F_list)) * T
        if out is None:
            out = torch.empty((n_re, self.m), dtype=torch.float32, device=x_packed.device)
        _check(self.lib.conet_forward_ragged(self.handle, ctypes.c_void_p(x_packed.data_ptr()), len(F_list), T, F_arr,
                                             ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def close(self):
        if getattr(self, "handle", None):
            self.lib.conet_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pinned_array(shape, dtype=np.float32) -> np.ndarray:
    """A zeroed numpy array in page-locked host memory (torch's pinned allocator); the array
    keeps that memory alive."""
    import torch
    tdt = {np.dtype(np.float32): torch.float32, np.dtype(np.uint8): torch.uint8}[np.dtype(dtype)]
    n = int(np.prod(shape))
    return torch.zeros(n, dtype=tdt, pin_memory=True).numpy().reshape(shape)


class ForwardGraph:
    """A recorded forward (conet_graph_*): keeps its model and buffers alive."""

    def __init__(self, model, handle, x, out):
        self.model, self.handle, self.x, self.out = model, handle, x, out

    def launch(self, stream=None):
        _check(self.model.lib.conet_graph_launch(self.handle, _stream_ptr(stream)))
        return self.out

    def close(self):
        if getattr(self, "handle", None):
            self.model.lib.conet_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server over a Conet model (lanes = HIP streams with own buffers).

    submit() copies nothing: the feature and LLR arrays are held until wait() returns. Arrays
    from pinned_array() are page-locked: the server reads and writes them by DMA, with no host
    copy (inputs: grids, and features with all C_in channels).
    """

    def __init__(self, model: Conet, mem_budget: int = 8 << 30, n_streams: int = 2, max_batch_res: int = 1 << 20,
                 max_queue: int = 4096):
        self.lib = load()
        self.model = model
        h = ctypes.c_void_p()
        _check(self.lib.conet_serve_create(model.handle, int(mem_budget), n_streams, int(max_batch_res),
                                           int(max_queue), ctypes.byref(h)))
        self.handle = h
        self._held = {}

    def submit(self, x: np.ndarray, n_prb: int, n_rx: int, m: int, out: Optional[np.ndarray] = None, T: int = 14,
               grid: bool = False):
        """x: float32 features [T, 12*n_prb, 4*n_rx], or with grid=True the received grid
        [T, 12*n_prb, n_rx, 2] (Re, Im; featurised on the GPU). Returns (ticket, llr array [T, F, m])."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        F = 12 * n_prb
        want = (T, F, n_rx, 2) if grid else (T, F, 4 * n_rx)
        if x.shape != want:
            raise ValueError(f"x has shape {x.shape}, expected {want}")
        if out is None:
            out = np.empty((T, F, m), dtype=np.float32)
        elif out.dtype != np.float32 or not out.flags.c_contiguous or out.shape != (T, F, m):
            raise ValueError(f"out must be a C-contiguous float32 array of shape {(T, F, m)}")
        req = conet_request(n_prb, n_rx, m, T, x.ctypes.data, out.ctypes.data, 0, 1 if grid else 0)
        t = ctypes.c_uint64()
        _check(self.lib.conet_serve_submit(self.handle, ctypes.byref(req), ctypes.byref(t)))
        self._held[t.value] = (x, out)
        return t.value, out

    def wait(self, ticket: int, timeout_us: int = -1) -> float:
        lat = ctypes.c_double()
        st = self.lib.conet_serve_wait(self.handle, ctypes.c_uint64(ticket), int(timeout_us), ctypes.byref(lat))
        if st != 6:                      # ETIMEOUT keeps the buffers held for a later wait
            self._held.pop(ticket, None)
        _check(st)
        return lat.value

    def stats(self) -> dict:
        s = conet_serve_stats()
        _check(self.lib.conet_serve_get_stats(self.handle, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in conet_serve_stats._fields_}

    def reset_stats(self):
        _check(self.lib.conet_serve_reset_stats(self.handle))

    def pause(self, paused: bool = True):
        _check(self.lib.conet_serve_pause(self.handle, 1 if paused else 0))

    def close(self):
        if getattr(self, "handle", None):
            _check(self.lib.conet_serve_destroy(self.handle))
            self.handle = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def conet_function():
    """torch.autograd.Function over a train-mode Conet: forward saves activations, backward
    runs the library's hand-written reverse mode and returns the parameter gradient."""
    import torch

    class ConetFunction(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x, params, model):
            ctx.model = model
            return model.forward(x, save=True)

        @staticmethod
        def backward(ctx, dllr):
            g = ctx.model.backward(dllr.contiguous())
            return None, g.clone(), None

    return ConetFunction


def mfma_peak(dtype: str = "bf16", iters: int = 0, stream=None):
    """Measured dense MFMA TFLOP/s and shader clock (GHz) on the current device (conet_mfma_peak)."""
    lib = load()
    code = DTYPES[dtype]
    if iters <= 0:
        iters = 50_000 if dtype == "f32" else 100_000
    tf, ghz = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib.conet_mfma_peak(code, iters, ctypes.byref(tf), ctypes.byref(ghz), _stream_ptr(stream)))
    return tf.value, ghz.value


def mfma_dot(dtype: str, shape: int, a, b) -> float:
    """conet_mfma_dot: sum of a[k] b[k] by one matrix instruction (dtype "bf16": a, b are float
    values rounded to BF16; "fp8": a, b are e4m3fn byte codes)."""
    lib = load()
    if dtype == "bf16":
        def bits(v):
            u = np.asarray(v, np.float32).view(np.uint32).astype(np.uint64)
            return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)
        ca, cb = bits(a), bits(b)
    else:
        ca, cb = np.asarray(a, np.uint8), np.asarray(b, np.uint8)
    ca, cb = np.ascontiguousarray(ca), np.ascontiguousarray(cb)
    out = ctypes.c_float()
    _check(lib.conet_mfma_dot(DTYPES[dtype], int(shape), ca.ctypes.data_as(ctypes.c_void_p),
                              cb.ctypes.data_as(ctypes.c_void_p), ctypes.byref(out)))
    return float(np.float32(out.value))


def featurise(y, C_in: int, out=None, stream=None, variances=None):
    """conet_featurise: y is a contiguous float32 CUDA tensor [B][T][F][n_rx][2]; returns the
    float32 features [B][T][F][C_in] (LS at the pilots + linear interpolation). With variances
    (float32 CUDA [B][2]: noise and interference variance per slot), conet_featurise_var: the
    last 8 channels carry them."""
    import torch
    if not (y.is_cuda and y.dtype == torch.float32 and y.is_contiguous() and y.dim() == 5 and y.shape[-1] == 2):
        raise ValueError("y must be a contiguous float32 CUDA tensor [B][T][F][n_rx][2]")
    B, T, F, n_rx, _ = y.shape
    if out is None:
        out = torch.empty((B, T, F, C_in), dtype=torch.float32, device=y.device)
    if variances is None:
        _check(load().conet_featurise(ctypes.c_void_p(y.data_ptr()), B, T, F, n_rx, C_in,
                                      ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    else:
        if not (variances.is_cuda and variances.dtype == torch.float32 and variances.is_contiguous()
                and tuple(variances.shape) == (B, 2)):
            raise ValueError("variances must be a contiguous float32 CUDA tensor [B][2]")
        _check(load().conet_featurise_var(ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(variances.data_ptr()), B, T,
                                          F, n_rx, C_in, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def simulate(F: int, n_rx: int, bits_per_symbol: int, first_slot: int, B: int, n_taps: int = 8,
             max_doppler_hz: float = 400.0, snr_db=(-5.0, 25.0), seed: int = 0, T: int = 14, out=None, stream=None):
    """conet_simulate: slots first_slot .. first_slot + B - 1 generated on the current GPU.
    Returns (y float32 [B][T][F][n_rx][2], bits uint8 [B][T][F][m], noise_var float32 [B]);
    `out` may pass those three tensors to fill."""
    import torch
    cfg = conet_sim_config(F, T, n_rx, bits_per_symbol, n_taps, max_doppler_hz, snr_db[0], snr_db[1], seed)
    if out is None:
        dev = torch.device("cuda", torch.cuda.current_device())
        out = (torch.empty((B, T, F, n_rx, 2), dtype=torch.float32, device=dev),
               torch.empty((B, T, F, bits_per_symbol), dtype=torch.uint8, device=dev),
               torch.empty((B,), dtype=torch.float32, device=dev))
    y, bits, nv = out
    _check(load().conet_simulate(ctypes.byref(cfg), int(first_slot), B, ctypes.c_void_p(y.data_ptr()),
                                 ctypes.c_void_p(bits.data_ptr()), ctypes.c_void_p(nv.data_ptr()), _stream_ptr(stream)))
    return y, bits, nv
