"""Python binding of libko.so (include/ko.h): exact kernel-launch-order evaluation.

Argument marshalling only.  Every step of the evaluation runs in the library:
the launch-order heuristic on the host, the makespan enumeration, statistics
and histograms in its gfx950 kernels.  PyTorch supplies device memory and the
current HIP stream.  Importing this package fails loudly when libko.so has not
been built (``python paper_1511_07983_amd/build.py``); there is no fallback.

Names mirror the C ABI: ko_heuristic_order, ko_count_orders,
ko_simulate_batch, ko_simulate_batch_noalloc, ko_rank_percentile, ko_sync, ko_shutdown, ko_last_error.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libko.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1511_07983_amd/build.py`")


KO_OK = 0
KO_EINVAL = -1
KO_ERANGE = -2
KO_ENOMEM = -3
KO_EHIP = -4

KO_ORDERS_ALL = 0
KO_ORDERS_RANK_RANGE = 1
KO_ORDERS_EXPLICIT = 2
KO_ORDERS_SAMPLED = 3

KO_HEUR_PER_BLOCK = 1
KO_HEUR_FULL_SORT = 2

EXPORTED = ("ko_heuristic_order", "ko_count_orders", "ko_simulate_batch", "ko_simulate_batch_noalloc",
            "ko_rank_percentile",
            "ko_sync", "ko_shutdown", "ko_plan_create", "ko_plan_info", "ko_plan_launch", "ko_plan_status",
            "ko_plan_engine",
            "ko_plan_destroy", "ko_graph_capture", "ko_graph_launch", "ko_graph_destroy",
            "ko_sample_orders", "ko_topk_f32", "ko_kth_smallest_i64", "ko_sort_i64", "ko_stats_i64",
            "ko_simulate_rounds",
            "ko_set_kernel_timing", "ko_last_kernel_ms", "ko_hw_vgprs", "ko_hw_time_orders",
            "ko_hw_last_error", "ko_last_error")


class KoGpuModel(ctypes.Structure):
    _fields_ = [("n_cu", ctypes.c_int32), ("wave_size", ctypes.c_int32),
                ("wave_cu", ctypes.c_int32), ("blk_cu", ctypes.c_int32),
                ("reg_cu", ctypes.c_int64), ("lds_cu", ctypes.c_int64),
                ("rb_milli", ctypes.c_int32), ("mem_blocks", ctypes.c_int32)]


class KoKernel(ctypes.Structure):
    _fields_ = [("n_tblk", ctypes.c_int64), ("n_inst", ctypes.c_int64),
                ("lds_blk", ctypes.c_int64), ("waves_blk", ctypes.c_int32),
                ("regs_thr", ctypes.c_int32), ("r_milli", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class KoSetStats(ctypes.Structure):
    _fields_ = [("min_makespan", ctypes.c_int64), ("max_makespan", ctypes.c_int64),
                ("argmin", ctypes.c_uint64), ("argmax", ctypes.c_uint64),
                ("n_less", ctypes.c_uint64), ("n_equal", ctypes.c_uint64),
                ("n_greater", ctypes.c_uint64), ("n_orders", ctypes.c_uint64)]


class KoRankResult(ctypes.Structure):
    _fields_ = [("makespan", ctypes.c_int64), ("min_makespan", ctypes.c_int64),
                ("max_makespan", ctypes.c_int64), ("n_less", ctypes.c_uint64),
                ("n_equal", ctypes.c_uint64), ("n_greater", ctypes.c_uint64),
                ("n_total", ctypes.c_uint64), ("pct_inclusive", ctypes.c_double),
                ("pct_strict", ctypes.c_double), ("pct_mid", ctypes.c_double)]


# simulation engines (ko_launch_config.engine); all give identical results
ENGINE_AUTO, ENGINE_WAVE, ENGINE_LANES = 0, 1, 2


class KoLaunchConfig(ctypes.Structure):
    _fields_ = [("chunk_log2", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("engine", ctypes.c_int32), ("lane_entries", ctypes.c_int32)]


class KoOrderSpec(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("rank_lo_hi", ctypes.POINTER(ctypes.c_uint64)),
                ("orders_dev", ctypes.c_void_p),
                ("orders_per_set", ctypes.POINTER(ctypes.c_int64)),
                ("seed", ctypes.c_uint64)]


# numpy views of the ABI records (same layout as the C structs)
SET_STATS_DTYPE = np.dtype([("min_makespan", "<i8"), ("max_makespan", "<i8"), ("argmin", "<u8"),
                            ("argmax", "<u8"), ("n_less", "<u8"), ("n_equal", "<u8"),
                            ("n_greater", "<u8"), ("n_orders", "<u8")])
KERNEL_DTYPE = np.dtype([("n_tblk", "<i8"), ("n_inst", "<i8"), ("lds_blk", "<i8"),
                         ("waves_blk", "<i4"), ("regs_thr", "<i4"), ("r_milli", "<i4"),
                         ("reserved", "<i4")])

_i32p = ctypes.POINTER(ctypes.c_int32)
_u64p = ctypes.POINTER(ctypes.c_uint64)

_lib = None


def _L():
    """libko.so, loaded on first use (the package can be imported without loading it)."""
    global _lib
    if _lib is None:
        # PyTorch's HIP runtime must be loaded first so that libko.so binds to
        # the libamdhip64 instance that owns the caller's memory and streams
        import torch  # noqa: F401
        lib = ctypes.CDLL(LIB_PATH)
        lib.ko_heuristic_order.argtypes = [ctypes.POINTER(KoGpuModel), ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_uint32, _i32p, _i32p]
        lib.ko_heuristic_order.restype = ctypes.c_int
        lib.ko_count_orders.argtypes = [_i32p, ctypes.c_int32, ctypes.POINTER(KoOrderSpec), _u64p, _u64p]
        lib.ko_count_orders.restype = ctypes.c_int
        lib.ko_simulate_batch.argtypes = [ctypes.POINTER(KoGpuModel), ctypes.c_void_p, _i32p,
                                           ctypes.c_int32, ctypes.POINTER(KoOrderSpec), ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_int32, ctypes.c_void_p]
        lib.ko_simulate_batch.restype = ctypes.c_int
        lib.ko_simulate_batch_noalloc.argtypes = lib.ko_simulate_batch.argtypes
        lib.ko_simulate_batch_noalloc.restype = ctypes.c_int
        lib.ko_rank_percentile.argtypes = [ctypes.POINTER(KoGpuModel), ctypes.c_void_p, ctypes.c_int32,
                                            _i32p, ctypes.c_uint64, ctypes.c_uint64,
                                            ctypes.POINTER(KoRankResult), ctypes.c_void_p]
        lib.ko_rank_percentile.restype = ctypes.c_int
        lib.ko_sync.argtypes = [ctypes.c_void_p]
        lib.ko_sync.restype = ctypes.c_int
        lib.ko_shutdown.argtypes = []
        lib.ko_shutdown.restype = ctypes.c_int
        vp = ctypes.c_void_p
        lib.ko_plan_create.argtypes = [ctypes.POINTER(KoGpuModel), vp, _i32p, ctypes.c_int32,
                                        ctypes.POINTER(KoOrderSpec), ctypes.POINTER(KoLaunchConfig),
                                        ctypes.POINTER(vp)]
        lib.ko_plan_info.argtypes = [vp, _u64p, _u64p, _u64p, _i32p]
        lib.ko_plan_launch.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int32, vp]
        lib.ko_plan_status.argtypes = [vp, vp]
        lib.ko_plan_engine.argtypes = [vp, _i32p, _i32p, _u64p, _u64p, vp]
        lib.ko_plan_destroy.argtypes = [vp]
        lib.ko_graph_capture.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int32, vp, ctypes.POINTER(vp)]
        lib.ko_graph_launch.argtypes = [vp, vp]
        lib.ko_graph_destroy.argtypes = [vp]
        for f in ("ko_plan_create", "ko_plan_info", "ko_plan_launch", "ko_plan_status", "ko_plan_engine",
                  "ko_plan_destroy",
                  "ko_graph_capture", "ko_graph_launch", "ko_graph_destroy"):
            getattr(lib, f).restype = ctypes.c_int
        lib.ko_sample_orders.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]
        lib.ko_sample_orders.restype = ctypes.c_int
        lib.ko_simulate_rounds.argtypes = [ctypes.POINTER(KoGpuModel), ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p,
                                            ctypes.c_void_p]
        lib.ko_simulate_rounds.restype = ctypes.c_int
        lib.ko_topk_f32.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]
        lib.ko_topk_f32.restype = ctypes.c_int
        lib.ko_kth_smallest_i64.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                             ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint64),
                                             ctypes.c_void_p]
        lib.ko_kth_smallest_i64.restype = ctypes.c_int
        lib.ko_sort_i64.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]
        lib.ko_sort_i64.restype = ctypes.c_int
        lib.ko_stats_i64.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p]
        lib.ko_stats_i64.restype = ctypes.c_int
        lib.ko_hw_vgprs.argtypes = [ctypes.c_int32, _i32p]
        lib.ko_hw_vgprs.restype = ctypes.c_int
        lib.ko_hw_time_orders.argtypes = [ctypes.c_void_p, ctypes.c_int32, _i32p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
        lib.ko_hw_time_orders.restype = ctypes.c_int
        lib.ko_hw_last_error.argtypes = []
        lib.ko_hw_last_error.restype = ctypes.c_char_p
        lib.ko_set_kernel_timing.argtypes = [ctypes.c_int32]
        lib.ko_set_kernel_timing.restype = ctypes.c_int
        lib.ko_last_kernel_ms.argtypes = [ctypes.POINTER(ctypes.c_float)]
        lib.ko_last_kernel_ms.restype = ctypes.c_int
        lib.ko_last_error.argtypes = []
        lib.ko_last_error.restype = ctypes.c_char_p
        _lib = lib
    return _lib


class KoError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{message} (code {code})")
        self.code = code


def ko_last_error() -> str:
    return _L().ko_last_error().decode()


def _check(rc: int):
    if rc != KO_OK:
        raise KoError(rc, ko_last_error())


def gpu_model(model) -> KoGpuModel:
    """A KoGpuModel from a mapping or an object with the same field names
    (mem_blocks, the memory-contention parameter, is optional: 0 = none)."""
    if isinstance(model, KoGpuModel):
        return model
    if isinstance(model, dict):
        get, mem = model.get, model.get("mem_blocks", 0)
    else:
        get, mem = (lambda f: getattr(model, f)), getattr(model, "mem_blocks", 0)
    return KoGpuModel(int(get("n_cu")), int(get("wave_size")), int(get("wave_cu")),
                      int(get("blk_cu")), int(get("reg_cu")), int(get("lds_cu")),
                      int(get("rb_milli")), int(mem))


def kernel_array(kernels) -> np.ndarray:
    """ko_kernel records (KERNEL_DTYPE) from a structured array or a list of mappings."""
    if isinstance(kernels, np.ndarray) and kernels.dtype == KERNEL_DTYPE:
        return np.ascontiguousarray(kernels)
    if isinstance(kernels, np.ndarray) and kernels.dtype.names:
        rows = [{f: kernels[f][i] for f in kernels.dtype.names} for i in range(len(kernels))]
    else:
        rows = list(kernels)
    out = np.zeros(len(rows), dtype=KERNEL_DTYPE)
    for i, r in enumerate(rows):
        for f in ("n_tblk", "n_inst", "lds_blk", "waves_blk", "regs_thr", "r_milli"):
            out[f][i] = int(r[f])
    return out


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev_ptr(t, dtype, numel: int, name: str):
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {numel}")
    return t.data_ptr()


def ko_heuristic_order(gpu, kernels, flags: int = 0, *, with_rounds: bool = False):
    """Launch order of Algorithm 1 (host).  Returns the order, or (order, rounds)."""
    g = gpu_model(gpu)
    k = kernel_array(kernels)
    n = len(k)
    order = np.zeros(max(n, 1), dtype=np.int32)
    rounds = np.zeros(max(n, 1), dtype=np.int32)
    _check(_L().ko_heuristic_order(ctypes.byref(g), k.ctypes.data if n else None, n, flags,
                                   order.ctypes.data_as(_i32p), rounds.ctypes.data_as(_i32p)))
    if with_rounds:
        return order[:n].tolist(), rounds[:n].tolist()
    return order[:n].tolist()


class OrderSpec:
    """Which orders of each set to evaluate (mirrors ko_order_spec)."""

    def __init__(self, mode: int, rank_lo_hi=None, orders_dev=None, orders_per_set=None,
                 seed: int = 0):
        self.mode = mode
        self._rank = None if rank_lo_hi is None else np.ascontiguousarray(rank_lo_hi, dtype=np.uint64).ravel()
        self._per = None if orders_per_set is None else np.ascontiguousarray(orders_per_set, dtype=np.int64)
        self.orders_dev = orders_dev
        self.seed = int(seed) & ((1 << 64) - 1)

    def c_struct(self) -> KoOrderSpec:
        s = KoOrderSpec()
        s.mode = self.mode
        s.reserved = 0
        s.rank_lo_hi = self._rank.ctypes.data_as(_u64p) if self._rank is not None else None
        if self.orders_dev is not None:
            s.orders_dev = _dev_ptr(self.orders_dev, __import__("torch").uint8, 0, "orders_dev")
        s.orders_per_set = (self._per.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
                            if self._per is not None else None)
        s.seed = self.seed
        return s

    @staticmethod
    def all():
        return OrderSpec(KO_ORDERS_ALL)

    @staticmethod
    def rank_range(lo_hi):
        return OrderSpec(KO_ORDERS_RANK_RANGE, rank_lo_hi=lo_hi)

    @staticmethod
    def explicit(orders_dev, orders_per_set):
        return OrderSpec(KO_ORDERS_EXPLICIT, orders_dev=orders_dev, orders_per_set=orders_per_set)

    @staticmethod
    def sampled(orders_per_set, seed: int):
        return OrderSpec(KO_ORDERS_SAMPLED, orders_per_set=orders_per_set, seed=seed)


def _offsets(set_offsets) -> np.ndarray:
    return np.ascontiguousarray(set_offsets, dtype=np.int32)


def ko_count_orders(set_offsets, spec: OrderSpec):
    """(per-set order counts, total) for a batch."""
    off = _offsets(set_offsets)
    n_sets = len(off) - 1
    per = np.zeros(max(n_sets, 1), dtype=np.uint64)
    total = np.zeros(1, dtype=np.uint64)
    sp = spec.c_struct()
    _check(_L().ko_count_orders(off.ctypes.data_as(_i32p), n_sets, ctypes.byref(sp),
                                per.ctypes.data_as(_u64p), total.ctypes.data_as(_u64p)))
    return per[:n_sets], int(total[0])


def ko_simulate_batch(gpu, kernels, set_offsets, spec: OrderSpec, *, ref_makespan=None,
                      makespans=None, stats=None, hist=None, n_bins: int = 0, stream=None):
    """Enqueue the evaluation of a batch on the current HIP stream (asynchronous).

    ``kernels``/``set_offsets`` are host data; ``ref_makespan`` (int64[n_sets]),
    ``makespans`` (int64[total]), ``stats`` (uint8[n_sets*64] or a tensor of
    n_sets*8 int64) and ``hist`` (int64[n_sets*n_bins], read as uint64) are
    device tensors or None.
    """
    return _simulate_batch("ko_simulate_batch", gpu, kernels, set_offsets, spec, ref_makespan, makespans,
                           stats, hist, n_bins, stream)


def ko_simulate_batch_noalloc(gpu, kernels, set_offsets, spec: OrderSpec, *, ref_makespan=None,
                              makespans=None, stats=None, hist=None, n_bins: int = 0, stream=None):
    """ko_simulate_batch without any device allocation: the library's static
    per-GPU scratch holds the batch's tables (synchronous; KoError with
    KO_ERANGE when a batch does not fit it).  Arguments as ko_simulate_batch."""
    return _simulate_batch("ko_simulate_batch_noalloc", gpu, kernels, set_offsets, spec, ref_makespan,
                           makespans, stats, hist, n_bins, stream)


def _simulate_batch(entry, gpu, kernels, set_offsets, spec, ref_makespan, makespans, stats, hist, n_bins,
                    stream):
    import torch
    g = gpu_model(gpu)
    k = kernel_array(kernels)
    off = _offsets(set_offsets)
    n_sets = len(off) - 1
    sp = spec.c_struct()
    per, total = ko_count_orders(off, spec) if n_sets >= 1 else (None, 0)
    if spec.mode == KO_ORDERS_EXPLICIT and spec.orders_dev is not None:
        need = int(sum(int(per[s]) * int(off[s + 1] - off[s]) for s in range(n_sets)))
        if spec.orders_dev.numel() < need:
            raise ValueError(f"orders_dev holds {spec.orders_dev.numel()} bytes, needs {need}")
    ref_p = _dev_ptr(ref_makespan, torch.int64, n_sets, "ref_makespan")
    ms_p = _dev_ptr(makespans, torch.int64, total, "makespans")
    st_p = _dev_ptr(stats, torch.int64, 8 * n_sets, "stats")
    h_p = _dev_ptr(hist, torch.int64, n_sets * max(n_bins, 0), "hist")
    _check(getattr(_L(), entry)(ctypes.byref(g), k.ctypes.data if len(k) else None,
                                off.ctypes.data_as(_i32p), n_sets, ctypes.byref(sp), ref_p,
                                ms_p, st_p, h_p, n_bins, _stream_handle(stream)))
    return per, total


def stats_records(stats_tensor) -> np.ndarray:
    """Host copy of a device stats tensor as SET_STATS_DTYPE records."""
    return stats_tensor.detach().cpu().numpy().view(SET_STATS_DTYPE)


def ko_rank_percentile(gpu, kernels, order, n_samples: int = 0, seed: int = 0, stream=None) -> dict:
    """Makespan and percentile rank of one order (synchronous)."""
    g = gpu_model(gpu)
    k = kernel_array(kernels)
    o = np.ascontiguousarray(order, dtype=np.int32)
    res = KoRankResult()
    _check(_L().ko_rank_percentile(ctypes.byref(g), k.ctypes.data if len(k) else None, len(k),
                                   o.ctypes.data_as(_i32p), int(n_samples), int(seed) & ((1 << 64) - 1),
                                   ctypes.byref(res), _stream_handle(stream)))
    return {f: getattr(res, f) for f, _ in KoRankResult._fields_}


def _outputs(ref_makespan, makespans, stats, hist, n_bins, total, n_sets):
    import torch
    ref_p = _dev_ptr(ref_makespan, torch.int64, n_sets, "ref_makespan")
    ms_p = _dev_ptr(makespans, torch.int64, total, "makespans")
    st_p = _dev_ptr(stats, torch.int64, 8 * n_sets, "stats")
    h_p = _dev_ptr(hist, torch.int64, n_sets * max(n_bins, 1), "hist") if hist is not None else None
    return ref_p, ms_p, st_p, h_p


class Plan:
    """A batch prepared once (ko_plan_create) and launched many times."""

    def __init__(self, gpu, kernels, set_offsets, spec: "OrderSpec", chunk_log2: int = 0, wg_per_cu: int = 0,
                 engine: int = ENGINE_AUTO, lane_entries: int = 0):
        g = gpu_model(gpu)
        k = kernel_array(kernels)
        off = np.ascontiguousarray(set_offsets, dtype=np.int32)
        self.n_sets = len(off) - 1
        self._spec = spec.c_struct()  # keeps the rank table alive during create
        cfg = KoLaunchConfig(int(chunk_log2), int(wg_per_cu), int(engine), int(lane_entries))
        h = ctypes.c_void_p()
        _check(_L().ko_plan_create(ctypes.byref(g), k.ctypes.data if len(k) else None, off.ctypes.data_as(_i32p),
                                   self.n_sets, ctypes.byref(self._spec), ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._keep = spec  # an explicit order tensor must outlive the plan
        tot, items, chunk = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        grid = ctypes.c_int32()
        _check(_L().ko_plan_info(h, ctypes.byref(tot), ctypes.byref(items), ctypes.byref(chunk),
                                 ctypes.byref(grid)))
        self.total_orders, self.work_items, self.chunk, self.grid = tot.value, items.value, chunk.value, grid.value

    def launch(self, *, ref_makespan=None, makespans=None, stats=None, hist=None, n_bins: int = 0, stream=None):
        p = _outputs(ref_makespan, makespans, stats, hist, n_bins, self.total_orders, self.n_sets)
        _check(_L().ko_plan_launch(self._h, *p, int(n_bins), _stream_handle(stream)))

    def status(self, stream=None):
        _check(_L().ko_plan_status(self._h, _stream_handle(stream)))

    def engine(self, stream=None):
        """(engine, group entries per lane, orders and whole work items the last
        launch passed from the lane engine to the wave engine); waits for the stream."""
        e, ent, sp, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(_L().ko_plan_engine(self._h, ctypes.byref(e), ctypes.byref(ent), ctypes.byref(sp), ctypes.byref(n),
                                   _stream_handle(stream)))
        return e.value, ent.value, sp.value, n.value

    def capture(self, *, stream, ref_makespan=None, makespans=None, stats=None, hist=None, n_bins: int = 0):
        """A HIP graph of one launch with these outputs (stream: a created torch stream)."""
        p = _outputs(ref_makespan, makespans, stats, hist, n_bins, self.total_orders, self.n_sets)
        g = ctypes.c_void_p()
        _check(_L().ko_graph_capture(self._h, *p, int(n_bins), _stream_handle(stream), ctypes.byref(g)))
        return Graph(g, self, (ref_makespan, makespans, stats, hist))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _L().ko_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """An instantiated HIP graph of one plan launch (ko_graph_capture)."""

    def __init__(self, handle, plan, outputs):
        self._h = handle
        self._plan = plan        # the plan and the outputs must outlive the graph
        self._outputs = outputs

    def launch(self, stream=None):
        _check(_L().ko_graph_launch(self._h, _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _L().ko_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ko_sample_orders(n: int, set_index: int, seed: int, count: int, *, first: int = 0, indices=None,
                     orders=None, positions=None, stream=None):
    """Write the SAMPLED-mode orders (uint8 [count][n]) and/or their inverses
    (positions) into device tensors; samples first..first+count-1, or the
    sample numbers in `indices` (int64/uint64 device tensor)."""
    import torch
    o = _dev_ptr(orders, torch.uint8, count * n, "orders") if orders is not None else None
    p = _dev_ptr(positions, torch.uint8, count * n, "positions") if positions is not None else None
    ix = None
    if indices is not None:
        if indices.dtype not in (torch.int64, torch.uint64):
            raise TypeError("indices must be a 64-bit integer tensor")
        ix = _dev_ptr(indices, indices.dtype, count, "indices")
    _check(_L().ko_sample_orders(int(n), int(set_index), int(seed) & ((1 << 64) - 1), int(first), ix,
                                 int(count), o, p, _stream_handle(stream)))


def ko_simulate_rounds(gpu, kernels, orders=None, makespans=None, *, first: int = 0, count=None, stream=None):
    """Round-synchronous makespans (execution rounds of Section 2) of the launch
    orders in the uint8 device tensor orders [count, n], or with orders=None of
    the lexicographic ranks first .. first+count-1; writes and returns the int64
    device tensor makespans [count].  Asynchronous on the stream."""
    import torch
    g = gpu_model(gpu)
    k = kernel_array(kernels)
    n = len(k)
    if orders is not None:
        if orders.dim() != 2 or orders.shape[1] != n:
            raise ValueError("orders must be [count, n]")
        count = orders.shape[0]
        o = _dev_ptr(orders, torch.uint8, count * n, "orders")
        dev = orders.device
    else:
        if count is None:
            raise ValueError("count is required when orders is None")
        o = None
        dev = makespans.device if makespans is not None else torch.device("cuda", torch.cuda.current_device())
    if makespans is None:
        makespans = torch.empty(int(count), dtype=torch.int64, device=dev)
    m = _dev_ptr(makespans, torch.int64, int(count), "makespans")
    _check(_L().ko_simulate_rounds(ctypes.byref(g), k.ctypes.data if n else None, n, o, int(first), int(count),
                                   m, _stream_handle(stream)))
    return makespans


def ko_topk_f32(y, k: int, *, idx_out=None, val_out=None, stream=None):
    """The k smallest of the float32 device tensor y, ascending by (value, index).
    Returns (idx int64 tensor, val float32 tensor) on y's device."""
    import torch
    count = y.numel()
    if idx_out is None:
        idx_out = torch.empty(k, dtype=torch.int64, device=y.device)
    if val_out is None:
        val_out = torch.empty(k, dtype=torch.float32, device=y.device)
    _check(_L().ko_topk_f32(_dev_ptr(y, torch.float32, count, "y"), count, int(k),
                            _dev_ptr(idx_out, torch.int64, k, "idx_out"),
                            _dev_ptr(val_out, torch.float32, k, "val_out"), _stream_handle(stream)))
    return idx_out, val_out


def ko_kth_smallest_i64(v, k: int, stream=None, *, with_count: bool = False):
    """The k-th smallest (1-based) of the int64 device tensor v (synchronous);
    with_count=True returns (value, number of elements <= value)."""
    import torch
    out = ctypes.c_int64(0)
    le = ctypes.c_uint64(0)
    _check(_L().ko_kth_smallest_i64(_dev_ptr(v, torch.int64, v.numel(), "v"), v.numel(), int(k),
                                    ctypes.byref(out), ctypes.byref(le), _stream_handle(stream)))
    return (int(out.value), int(le.value)) if with_count else int(out.value)


def ko_sort_i64(v, *, sorted_out=None, index_out=None, want_index: bool = True, stream=None):
    """Stable ascending sort of the int64 device tensor v on the device
    (synchronous): (sorted values, index in v of each) as device tensors
    (int64, and uint64 read as int64); ties keep their order in v."""
    import torch
    n = v.numel()
    if sorted_out is None:
        sorted_out = torch.empty(n, dtype=torch.int64, device=v.device)
    if index_out is None and want_index:
        index_out = torch.empty(n, dtype=torch.int64, device=v.device)
    _check(_L().ko_sort_i64(_dev_ptr(v, torch.int64, n, "v"), n, _dev_ptr(sorted_out, torch.int64, n, "sorted_out"),
                            _dev_ptr(index_out, torch.int64, n, "index_out"), _stream_handle(stream)))
    return sorted_out, index_out


def ko_stats_i64(v, *, ref=None, stats=None, stream=None):
    """Device statistics of the int64 device tensor v (asynchronous): min/max
    with smallest indices and the counts against ref (an int64[1] device tensor
    or None), into stats (int64[8] device tensor, created if None; read it
    with stats_records).  Returns stats."""
    import torch
    n = v.numel()
    if stats is None:
        stats = torch.empty(8, dtype=torch.int64, device=v.device)
    _check(_L().ko_stats_i64(_dev_ptr(v, torch.int64, n, "v") if n else None, n,
                             _dev_ptr(ref, torch.int64, 1, "ref"), _dev_ptr(stats, torch.int64, 8, "stats"),
                             _stream_handle(stream)))
    return stats


def ranking_curve(makespans, stream=None):
    """Figure 1's ranking curve of a full enumeration: the makespans of all
    orders in ascending order and the lexicographic rank of each (ties by
    smaller rank), both device tensors."""
    return ko_sort_i64(makespans, stream=stream)


def median_gain(makespans, t_alg: int, stream=None) -> float:
    """The gain over a random order that Algorithm 1's order reaches with
    probability at least one half (Section 6): g such that at least half of
    all orders have a makespan >= (1 + g) * t_alg, i.e. the makespan of
    ascending place floor(N/2) over t_alg, minus 1.  The selection runs on
    the device (ko_kth_smallest_i64)."""
    n = makespans.numel()
    m = ko_kth_smallest_i64(makespans, n // 2 + 1, stream=stream)
    return m / float(t_alg) - 1.0


def ko_hw_vgprs(regs_thr: int) -> int:
    out = ctypes.c_int32(0)
    rc = _L().ko_hw_vgprs(int(regs_thr), ctypes.byref(out))
    if rc:
        raise KoError(rc, _L().ko_hw_last_error().decode())
    return int(out.value)


def ko_hw_time_orders(kernels, orders, scale: int, reps: int = 2) -> np.ndarray:
    """Measured makespans (ms) of the given orders of a kernel set (see ko.h)."""
    k = kernel_array(kernels)
    o = np.ascontiguousarray(orders, dtype=np.int32)
    if o.ndim == 1:
        o = o[None, :]
    out = np.zeros(len(o), dtype=np.float64)
    rc = _L().ko_hw_time_orders(k.ctypes.data, len(k), o.ctypes.data_as(_i32p), len(o), int(scale), int(reps),
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc:
        raise KoError(rc, _L().ko_hw_last_error().decode())
    return out


def ko_sync(stream=None):
    _check(_L().ko_sync(_stream_handle(stream)))


def ko_shutdown():
    _check(_L().ko_shutdown())


def ko_set_kernel_timing(enable: bool):
    """Time the simulate kernel of later ko_simulate_batch calls (current device)."""
    _check(_L().ko_set_kernel_timing(1 if enable else 0))


def ko_last_kernel_ms() -> float:
    """Duration (ms) of the simulate kernel of the last timed call; waits for it."""
    ms = ctypes.c_float(0.0)
    _check(_L().ko_last_kernel_ms(ctypes.byref(ms)))
    return float(ms.value)


def library_handle():
    return _L()
