"""Python binding of libko_nn.so (include/ko_nn.h): the learned surrogate.

Argument marshalling only: tokens, forward, backward and Adam run in the
library's gfx950 kernels; features and the lower bound are host functions of
the library.  PyTorch supplies device memory and the current stream.  Fails
loudly when libko_nn.so has not been built.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from . import KoError, gpu_model, kernel_array, _stream_handle  # (does not load libko.so)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_NN_PATH = os.path.join(_HERE, "libko_nn.so")
if not os.path.exists(LIB_NN_PATH):
    raise ImportError(f"{LIB_NN_PATH} is missing: build it with `python paper_1511_07983_amd/build.py`")
# Load PyTorch's HIP runtime first: libko_nn.so must bind to the same
# libamdhip64 instance that owns the device memory and streams it is given.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_NN_PATH)

N_FEAT = 8
N_POS = 17
UNPLACED = 16
D_IN = 32
D_HID = 256
MAX_TOKENS = 16

EXPORTED = ("ko_nn_num_params", "ko_nn_state_bytes", "ko_nn_work_bytes", "ko_nn_load", "ko_nn_read",
            "ko_nn_features", "ko_nn_lower_bound", "ko_nn_tokens", "ko_nn_targets", "ko_nn_within_set_ranks",
            "ko_nn_forward",
            "ko_nn_backward", "ko_nn_adam", "ko_nn_layer1_table", "ko_nn_score_work_bytes",
            "ko_nn_forward_positions", "ko_nn_score", "ko_nn_beam_expand", "ko_nn_beam_cap", "ko_nn_beam_gather",
            "ko_nn_train_step", "ko_nn_batch", "ko_nn_step_capture", "ko_nn_graph_launch", "ko_nn_graph_destroy",
            "ko_nn_split_table_bytes", "ko_nn_split_table", "ko_nn_score_split", "ko_nn_score_split_acc",
            "ko_nn_last_error")

_vp = ctypes.c_void_p
_lib.ko_nn_num_params.restype = ctypes.c_size_t
_lib.ko_nn_state_bytes.restype = ctypes.c_size_t
_lib.ko_nn_work_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
_lib.ko_nn_work_bytes.restype = ctypes.c_size_t
_lib.ko_nn_load.argtypes = [_vp, _vp, _vp]
_lib.ko_nn_read.argtypes = [_vp, ctypes.c_int32, _vp, _vp]
_lib.ko_nn_features.argtypes = [_vp, _vp, ctypes.c_int32, _vp]
_lib.ko_nn_lower_bound.argtypes = [_vp, _vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
_lib.ko_nn_tokens.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp]
_lib.ko_nn_targets.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int32, _vp, _vp]
_lib.ko_nn_forward.argtypes = [_vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp]
_lib.ko_nn_backward.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp]
_lib.ko_nn_adam.argtypes = [_vp, ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                            ctypes.c_float, _vp]
_lib.ko_nn_layer1_table.argtypes = [_vp, _vp, ctypes.c_int32, _vp, _vp]
_lib.ko_nn_within_set_ranks.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp]
_lib.ko_nn_score_work_bytes.argtypes = [ctypes.c_int32]
_lib.ko_nn_score_work_bytes.restype = ctypes.c_size_t
_lib.ko_nn_forward_positions.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp]
_lib.ko_nn_score.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp]
_lib.ko_nn_beam_expand.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp]
_lib.ko_nn_beam_cap.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_uint64,
                                _vp]
_lib.ko_nn_beam_gather.argtypes = [_vp, ctypes.c_int32, _vp, _vp, ctypes.c_int32, _vp, _vp]
_lib.ko_nn_train_step.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp]
_lib.ko_nn_batch.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp]
_lib.ko_nn_step_capture.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32,
                                    _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]
_lib.ko_nn_graph_launch.argtypes = [_vp, _vp]
_lib.ko_nn_graph_destroy.argtypes = [_vp]
_lib.ko_nn_split_table_bytes.argtypes = [ctypes.c_int32]
_lib.ko_nn_split_table_bytes.restype = ctypes.c_size_t
_lib.ko_nn_split_table.argtypes = [_vp, _vp, ctypes.c_int32, _vp, _vp]
_lib.ko_nn_score_split.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp]
_lib.ko_nn_score_split_acc.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_int32,
                                       _vp, _vp]
_lib.ko_nn_last_error.restype = ctypes.c_char_p
for _f in ("ko_nn_load", "ko_nn_read", "ko_nn_features", "ko_nn_lower_bound", "ko_nn_tokens", "ko_nn_targets",
           "ko_nn_forward", "ko_nn_backward", "ko_nn_adam", "ko_nn_layer1_table", "ko_nn_within_set_ranks",
           "ko_nn_forward_positions", "ko_nn_score", "ko_nn_beam_expand", "ko_nn_beam_cap", "ko_nn_beam_gather",
           "ko_nn_train_step", "ko_nn_batch", "ko_nn_step_capture", "ko_nn_graph_launch", "ko_nn_graph_destroy",
           "ko_nn_split_table", "ko_nn_score_split", "ko_nn_score_split_acc"):
    getattr(_lib, _f).restype = ctypes.c_int


def _check(rc):
    if rc != 0:
        raise KoError(rc, _lib.ko_nn_last_error().decode())


def beam_expand(prefix, n: int, stream=None):
    """Candidates of one beam step: prefix (device uint8 [W, d]) -> (positions
    [W (n - d), n] uint8, candidates [W (n - d)] int32 = parent << 8 | kernel)."""
    W, d = prefix.shape
    C = W * (n - d)
    pos = torch.empty((C, n), dtype=torch.uint8, device=prefix.device)
    cand = torch.empty(C, dtype=torch.int32, device=prefix.device)
    _check(_lib.ko_nn_beam_expand(prefix.data_ptr() if d else None, W, d, n, pos.data_ptr(), cand.data_ptr(),
                                  _stream_handle(stream)))
    return pos, cand


def beam_cap(scores, W: int, m: int, cap: int = 0, temperature: float = 0.0, seed: int = 0, stream=None):
    """Diversity rules on a step's scores (device float32 [W * m], in place)."""
    _check(_lib.ko_nn_beam_cap(scores.data_ptr(), W, m, int(cap), float(temperature),
                               int(seed) & ((1 << 64) - 1), _stream_handle(stream)))
    return scores


def beam_gather(prefix, cand, idx, stream=None):
    """Next prefixes: device uint8 [keep, d + 1] from the chosen candidates idx (device int64)."""
    W, d = prefix.shape
    keep = idx.numel()
    out = torch.empty((keep, d + 1), dtype=torch.uint8, device=cand.device)
    _check(_lib.ko_nn_beam_gather(prefix.data_ptr() if d else None, d, cand.data_ptr(), idx.data_ptr(), keep,
                                  out.data_ptr(), _stream_handle(stream)))
    return out


# struct ko_nn_sched (include/ko_nn.h), 48 bytes
SCHED_DTYPE = np.dtype([("step", "<i4"), ("warmup", "<i4"), ("total", "<i4"), ("per_epoch", "<i4"),
                        ("lr", "<f4"), ("lr_final", "<f4"), ("beta1", "<f4"), ("beta2", "<f4"), ("eps", "<f4"),
                        ("reserved", "<i4", (3,))])
assert SCHED_DTYPE.itemsize == 48


def sched(*, lr: float, warmup: int = 0, total: int = 1, lr_final: float = 1.0, per_epoch: int = 1, step: int = 0,
          beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, device="cuda:0"):
    """A device ko_nn_sched (uint8 tensor of 48 bytes): Adam's hyper-parameters
    and rate schedule, read and advanced by train steps on the device."""
    if per_epoch < 1 or total < 1 or warmup < 0 or step < 0:
        raise ValueError("need per_epoch >= 1, total >= 1, warmup >= 0 and step >= 0")
    h = np.zeros(1, dtype=SCHED_DTYPE)
    h["step"], h["warmup"], h["total"], h["per_epoch"] = step, warmup, total, per_epoch
    h["lr"], h["lr_final"], h["beta1"], h["beta2"], h["eps"] = lr, lr_final, beta1, beta2, eps
    return torch.from_numpy(h.view(np.uint8).copy()).to(device)


def sched_read(sched_dev) -> dict:
    """The fields of a device ko_nn_sched (host copy; waits for the device)."""
    h = sched_dev.cpu().numpy().view(SCHED_DTYPE)[0]
    return {k: h[k].item() for k in SCHED_DTYPE.names if k != "reserved"}


class StepGraph:
    """An instantiated HIP graph of one training step (ko_nn_step_capture)."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep  # every buffer the graph reads or writes must outlive it

    def launch(self, stream=None):
        _check(_lib.ko_nn_graph_launch(self._h, _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.ko_nn_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def num_params() -> int:
    return int(_lib.ko_nn_num_params())


def features(gpu, kernels) -> np.ndarray:
    """Per-kernel features [n, 8] (float32), computed by the library on the host."""
    g = gpu_model(gpu)
    k = kernel_array(kernels)
    out = np.zeros((len(k), N_FEAT), dtype=np.float32)
    _check(_lib.ko_nn_features(ctypes.addressof(g), k.ctypes.data, len(k), out.ctypes.data))
    return out


def lower_bound(gpu, kernels) -> int:
    g = gpu_model(gpu)
    k = kernel_array(kernels)
    lb = ctypes.c_int64(0)
    _check(_lib.ko_nn_lower_bound(ctypes.addressof(g), k.ctypes.data, len(k), ctypes.byref(lb)))
    return int(lb.value)


def within_set_ranks(values, n_sets: int, per_set: int, stream=None):
    """Device int64 ranks of each set's samples (see ko_nn_within_set_ranks)."""
    import torch
    ranks = torch.empty(n_sets * per_set, dtype=torch.int64, device=values.device)
    _check(_lib.ko_nn_within_set_ranks(values.data_ptr(), n_sets, per_set, ranks.data_ptr(),
                                       _stream_handle(stream)))
    return ranks


class Surrogate:
    """Device state (weights, gradients, Adam moments) plus a workspace."""

    def __init__(self, params=None, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.state = torch.zeros(int(_lib.ko_nn_state_bytes()), dtype=torch.uint8, device=self.device)
        self._work = None
        self._work_key = None
        self._score_work = None
        if params is not None:
            self.load(params)

    def _workspace(self, B, n):
        need = int(_lib.ko_nn_work_bytes(B, n))
        if self._work is None or self._work.numel() < need:
            self._work = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        return self._work

    def load(self, params, stream=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != num_params():
            raise ValueError(f"expected {num_params()} parameters, got {p.size}")
        _check(_lib.ko_nn_load(self.state.data_ptr(), p.ctypes.data, _stream_handle(stream)))

    def read(self, which: str = "weights", stream=None) -> np.ndarray:
        """Host copy of the weights, "grads" or Adam's moments "m" and "v"."""
        code = {"weights": 0, "grads": 1, "m": 2, "v": 3}[which]
        out = np.zeros(num_params(), dtype=np.float32)
        _check(_lib.ko_nn_read(self.state.data_ptr(), code, out.ctypes.data, _stream_handle(stream)))
        return out

    def tokens(self, feat, pos, set_of=None, rows=None, B=None, stream=None, out=None):
        """feat: device float32 [S, n, 8]; pos: device uint8 [R, n]; set_of: device
        int32 [R]; rows: device int64 [B] (sample b uses row rows[b]; default b)."""
        torch = self.torch
        n = pos.shape[1]
        if B is None:
            B = rows.shape[0] if rows is not None else pos.shape[0]
        x = out if out is not None else torch.empty((B, n, D_IN), dtype=torch.int16, device=self.device)
        _check(_lib.ko_nn_tokens(feat.data_ptr(), set_of.data_ptr() if set_of is not None else None,
                                 pos.data_ptr(), rows.data_ptr() if rows is not None else None, B, n,
                                 x.data_ptr(), _stream_handle(stream)))
        return x

    def targets(self, makespans, center, scale, set_of=None, rows=None, B=None, stream=None, out=None):
        """t[b] = (makespans[r] - center[s]) / scale[s] (device float32 [B]); r = rows[b], s = set_of[r]."""
        torch = self.torch
        if B is None:
            B = rows.shape[0] if rows is not None else makespans.shape[0]
        t = out if out is not None else torch.empty(B, dtype=torch.float32, device=self.device)
        _check(_lib.ko_nn_targets(makespans.data_ptr(), set_of.data_ptr() if set_of is not None else None,
                                  center.data_ptr(), scale.data_ptr(),
                                  rows.data_ptr() if rows is not None else None, B, t.data_ptr(),
                                  _stream_handle(stream)))
        return t

    def forward(self, x, stream=None):
        torch = self.torch
        B, n, _ = x.shape
        y = torch.empty(B, dtype=torch.float32, device=self.device)
        _check(_lib.ko_nn_forward(self.state.data_ptr(), x.data_ptr(), B, n, y.data_ptr(),
                                  self._workspace(B, n).data_ptr(), _stream_handle(stream)))
        return y

    def backward(self, x, t, stream=None):
        torch = self.torch
        B, n, _ = x.shape
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _check(_lib.ko_nn_backward(self.state.data_ptr(), x.data_ptr(), t.data_ptr(), B, n,
                                   loss.data_ptr(), self._workspace(B, n).data_ptr(),
                                   _stream_handle(stream)))
        return loss

    def layer1_table(self, feat, stream=None):
        """feat: device float32 [n, 8] of one set -> device float32 table [n, 17, 256]."""
        n = feat.shape[0]
        table = self.torch.empty((n, N_POS, D_HID), dtype=self.torch.float32, device=self.device)
        _check(_lib.ko_nn_layer1_table(self.state.data_ptr(), feat.data_ptr(), n, table.data_ptr(),
                                       _stream_handle(stream)))
        return table

    def forward_positions(self, table, pos, y=None, stream=None):
        """pos: device uint8 [B, n] (position of each kernel) -> y [B]."""
        torch = self.torch
        B, n = pos.shape
        if y is None:
            y = torch.empty(B, dtype=torch.float32, device=self.device)
        need = int(_lib.ko_nn_score_work_bytes(B))
        if self._score_work is None or self._score_work.numel() < need:
            self._score_work = torch.empty(need, dtype=torch.uint8, device=self.device)
        _check(_lib.ko_nn_forward_positions(self.state.data_ptr(), table.data_ptr(), pos.data_ptr(), B, n,
                                            y.data_ptr(), self._score_work.data_ptr(),
                                            _stream_handle(stream)))
        return y

    def score(self, feat, pos, y=None, stream=None):
        """feat: device float32 [n, 8] of one set; pos: device uint8 [B, n]
        (position of each kernel) -> y [B], in one fused kernel (ko_nn_score)."""
        torch = self.torch
        B, n = pos.shape
        if y is None:
            y = torch.empty(B, dtype=torch.float32, device=self.device)
        _check(_lib.ko_nn_score(self.state.data_ptr(), feat.data_ptr(), pos.data_ptr(), B, n, y.data_ptr(),
                                _stream_handle(stream)))
        return y

    def split_table(self, feat, stream=None):
        """feat: device float32 [n, 8] of one set -> its scoring operand pack
        for score_split (device int16, flat: the split layer-1 table's BF16
        high and low parts [256, KP] and the BF16 W2 and W3, each in MFMA
        fragment order, as include/ko_nn.h describes)."""
        n = feat.shape[0]
        split = self.torch.empty(int(_lib.ko_nn_split_table_bytes(n)) // 2, dtype=self.torch.int16,
                                 device=self.device)
        _check(_lib.ko_nn_split_table(self.state.data_ptr(), feat.data_ptr(), n, split.data_ptr(),
                                      _stream_handle(stream)))
        return split

    def score_split(self, split, pos, y=None, scale: float = 1.0, accumulate: bool = False, stream=None):
        """pos: device uint8 [B, n] -> y [B], the pooling on the matrix cores
        from the set's split table: y = scale * score, or y + scale * score
        with accumulate (ko_nn_score_split_acc)."""
        B, n = pos.shape
        if split.numel() * 2 != int(_lib.ko_nn_split_table_bytes(n)):
            raise ValueError("the split table was made for another number of kernels")
        if y is None:
            if accumulate:
                raise ValueError("accumulate needs y")
            y = self.torch.empty(B, dtype=self.torch.float32, device=self.device)
        _check(_lib.ko_nn_score_split_acc(self.state.data_ptr(), split.data_ptr(), pos.data_ptr(), B, n,
                                          float(scale), 1 if accumulate else 0, y.data_ptr(),
                                          _stream_handle(stream)))
        return y

    def train_step(self, x, t, sched_dev, loss=None, stream=None):
        """Forward, loss, gradients and Adam (rate and step from the device
        schedule, which advances) in one stream-ordered call; returns the loss."""
        torch = self.torch
        B, n, _ = x.shape
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _check(_lib.ko_nn_train_step(self.state.data_ptr(), x.data_ptr(), t.data_ptr(), B, n,
                                     sched_dev.data_ptr(), loss.data_ptr(), self._workspace(B, n).data_ptr(),
                                     _stream_handle(stream)))
        return loss

    def batch(self, feat, pos, set_of, makespans, center, scale, perm, sched_dev, B: int, x=None, t=None,
              stream=None):
        """The minibatch of the schedule's next step (ko_nn_batch): tokens x [B, n, 32]
        and targets t [B] for rows perm[(step mod per_epoch) B + b]."""
        torch = self.torch
        n = pos.shape[1]
        if perm.numel() < B * int(sched_read(sched_dev)["per_epoch"]):
            raise ValueError("perm must hold per_epoch * B rows")
        x = x if x is not None else torch.empty((B, n, D_IN), dtype=torch.int16, device=self.device)
        t = t if t is not None else torch.empty(B, dtype=torch.float32, device=self.device)
        _check(_lib.ko_nn_batch(feat.data_ptr(), set_of.data_ptr() if set_of is not None else None, pos.data_ptr(),
                                makespans.data_ptr(), center.data_ptr(), scale.data_ptr(), perm.data_ptr(),
                                sched_dev.data_ptr(), B, n, x.data_ptr(), t.data_ptr(), _stream_handle(stream)))
        return x, t

    def capture_step(self, feat, pos, set_of, makespans, center, scale, perm, sched_dev, B: int, *, stream,
                     x=None, t=None, loss=None):
        """A HIP graph of batch + train_step (ko_nn_step_capture); each replay is
        the next training step.  stream: a created torch stream."""
        torch = self.torch
        n = pos.shape[1]
        if perm.numel() < B * int(sched_read(sched_dev)["per_epoch"]):
            raise ValueError("perm must hold per_epoch * B rows")
        x = x if x is not None else torch.empty((B, n, D_IN), dtype=torch.int16, device=self.device)
        t = t if t is not None else torch.empty(B, dtype=torch.float32, device=self.device)
        loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=self.device)
        work = self._workspace(B, n)
        g = ctypes.c_void_p()
        _check(_lib.ko_nn_step_capture(self.state.data_ptr(), feat.data_ptr(),
                                       set_of.data_ptr() if set_of is not None else None, pos.data_ptr(),
                                       makespans.data_ptr(), center.data_ptr(), scale.data_ptr(), perm.data_ptr(),
                                       sched_dev.data_ptr(), B, n, x.data_ptr(), t.data_ptr(), loss.data_ptr(),
                                       work.data_ptr(), _stream_handle(stream), ctypes.byref(g)))
        graph = StepGraph(g, (self.state, feat, pos, set_of, makespans, center, scale, perm, sched_dev, x, t, loss,
                              work))
        graph.x, graph.t, graph.loss = x, t, loss
        return graph

    def adam(self, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(_lib.ko_nn_adam(self.state.data_ptr(), step, lr, beta1, beta2, eps,
                               _stream_handle(stream)))
