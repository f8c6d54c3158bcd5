"""Thin Python binding of libewahthr.so (include/ewahthr.h): argument marshalling only.

Every step of the query runs in the HIP kernels of the library; PyTorch only
provides device memory (tensors whose data_ptr is handed over) and streams.
Names follow the C ABI without the `ewah_` prefix.  If the native library is
missing this module raises on import: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libewahthr.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")

# One HIP runtime per process: PyTorch ships its own libamdhip64, so it is
# loaded first and the library binds to that already-loaded runtime.
try:
    import torch  # noqa: F401
except ImportError:  # a C-ABI user without PyTorch gets the system runtime
    torch = None

_L = ctypes.CDLL(LIB_PATH)
_vp, _u32, _u64, _i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int

OK, EINVAL, EFORMAT, ENOMEM, ENOSPC, EDEVICE = 0, -1, -2, -3, -4, -5


class View(ctypes.Structure):
    _fields_ = [("words", _vp), ("n_words", _u64), ("n_bits", _u64)]


class Stats(ctypes.Structure):
    _fields_ = [(n, _u64) for n in ("n_bits", "n_words", "n_markers", "n_literals", "one_fill_words",
                                    "popcount", "run_count", "index_bytes")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class Query(ctypes.Structure):
    _fields_ = [("idx", _vp), ("n", _u32), ("T", _u32), ("out_words_dev", _vp), ("out_cap", _u64),
                ("out_n_words_dev", _vp), ("variant", _u32)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("grid", _u32), ("use_graph", _i32)]


def _sig(name, res, args):
    f = getattr(_L, name)
    f.restype = res
    f.argtypes = args
    return f


_init = _sig("ewah_init", _i32, [_i32])
_last_error = _sig("ewah_last_error", ctypes.c_char_p, [])
_register_many = _sig("ewah_register_many", _i32, [ctypes.POINTER(View), _u32, _i32, ctypes.POINTER(_vp)])
_release = _sig("ewah_release", None, [_vp])
_get_stats = _sig("ewah_get_stats", _i32, [_vp, ctypes.POINTER(Stats)])
_device_words = _sig("ewah_device_words", _vp, [_vp])
_output_bound = _sig("ewah_output_bound", _u64, [_u64, _u64])
_threshold_v = _sig("ewah_threshold_v", _i32, [ctypes.POINTER(_vp), _u32, _u32, _vp, _u64, _vp, _u32, _vp])
_threshold_noalloc = _sig("ewah_threshold_noalloc", _i32, [ctypes.POINTER(_vp), _u32, _u32, _vp, _u64, _vp, _vp])
_symmetric = _sig("ewah_symmetric", _i32, [ctypes.POINTER(_vp), _u32, _vp, _u32, _vp, _u64, _vp, _vp])
_count_histogram = _sig("ewah_count_histogram", _i32, [ctypes.POINTER(_vp), _u32, _vp, _vp])
_opt_threshold = _sig("ewah_opt_threshold", _i32, [ctypes.POINTER(_vp), _u32, _u64, _vp, _u64, _vp,
                                                   ctypes.POINTER(_u32), _vp])
_variant_code = _sig("ewah_variant_code", _u32, [_i32, _u32, _u32])
_variant_code_ex = _sig("ewah_variant_code_ex", _u32, [_i32, _u32, _u32, _i32])
_default_variant = _sig("ewah_default_variant", _u32, [])
_batch_plan = _sig("ewah_batch_plan", _i32, [ctypes.POINTER(_vp), _u32, ctypes.POINTER(Query), _u32,
                                             ctypes.POINTER(BatchConfig), ctypes.POINTER(_vp)])
_batch_run = _sig("ewah_batch_run", _i32, [_vp, _vp])
_batch_set_variants = _sig("ewah_batch_set_variants", _i32, [_vp, _vp])
_batch_set_grid = _sig("ewah_batch_set_grid", _i32, [_vp, _u32])
_batch_set_win_batch = _sig("ewah_batch_set_win_batch", _i32, [_vp, _u32])
_batch_set_prepass = _sig("ewah_batch_set_prepass", _i32, [_vp, _i32])
_batch_free = _sig("ewah_batch_free", None, [_vp])
_device_errors = _sig("ewah_device_errors", _i32, [ctypes.POINTER(_u32)])
_num_cus = _sig("ewah_num_cus", _u32, [])
_query_features = _sig("ewah_query_features", _i32, [ctypes.POINTER(_vp), _u32, _vp, _vp, _vp, _u32, _vp, _vp])
_batch_features = _sig("ewah_batch_features", _i32, [_vp, _vp, _vp])
_batch_select = _sig("ewah_batch_select", _i32, [_vp, _vp, _u32, _vp, _vp])
_batch_get_variants = _sig("ewah_batch_get_variants", _i32, [_vp, _vp])
_batch_time_queries = _sig("ewah_batch_time_queries", _i32, [_vp, _u32, _vp, _vp])
_batch_select_model = _sig("ewah_batch_select_model", _i32, [_vp, _vp, _i32, _vp])
_variant_code_full = _sig("ewah_variant_code_full", _u32, [_i32, _u32, _u32, _i32, _u32])


class TrainConfig(ctypes.Structure):
    _fields_ = [("epochs", _u32), ("batch", _u32), ("lr", ctypes.c_float), ("seed", _u64)]


_selector_load = _sig("ewah_selector_load", _i32, [ctypes.c_char_p, ctypes.POINTER(_vp)])
_selector_save = _sig("ewah_selector_save", _i32, [_vp, ctypes.c_char_p])
_selector_free = _sig("ewah_selector_free", None, [_vp])
_selector_num_arms = _sig("ewah_selector_num_arms", _u32, [_vp])
_selector_arm_codes = _sig("ewah_selector_arm_codes", _i32, [_vp, _vp])
_selector_train = _sig("ewah_selector_train", _i32, [_vp, _vp, _u32, _u32, _vp, ctypes.POINTER(TrainConfig),
                                                     ctypes.POINTER(_vp)])
_selector_train_loss = _sig("ewah_selector_train_loss", ctypes.c_float, [_vp])
_selector_predict = _sig("ewah_selector_predict", _i32, [_vp, _i32, _vp, _u32, _vp, _vp])
SELECT_MLP, SELECT_RULES = 0, 1
_mlp_create = _sig("ewah_mlp_create", _i32, [_u32, _u64, ctypes.POINTER(_vp)])
_mlp_free = _sig("ewah_mlp_free", None, [_vp])
_mlp_num_params = _sig("ewah_mlp_num_params", _u64, [_u32])
_mlp_get_params = _sig("ewah_mlp_get_params", _i32, [_vp, _vp, _u64])
_mlp_set_params = _sig("ewah_mlp_set_params", _i32, [_vp, _vp, _u64])
_mlp_forward = _sig("ewah_mlp_forward", _i32, [_vp, _vp, _u32, _vp, _vp])
_mlp_grad = _sig("ewah_mlp_grad", _i32, [_vp, _vp, _vp, _u32, _vp, _vp, _vp])
_mlp_train_step = _sig("ewah_mlp_train_step", _i32, [_vp, _vp, _vp, _u32, ctypes.c_float, _vp, _vp])
_mlp_last_error = _sig("ewah_mlp_last_error", ctypes.c_char_p, [])

EXPORTED = ["ewah_init", "ewah_last_error", "ewah_register", "ewah_register_many", "ewah_release",
            "ewah_get_stats", "ewah_device_words", "ewah_output_bound", "ewah_threshold", "ewah_threshold_v", "ewah_threshold_noalloc",
            "ewah_symmetric", "ewah_opt_threshold", "ewah_count_histogram",
            "ewah_variant_code", "ewah_variant_code_ex", "ewah_default_variant", "ewah_batch_plan", "ewah_batch_run",
            "ewah_batch_set_variants", "ewah_batch_set_grid", "ewah_batch_set_win_batch", "ewah_batch_set_prepass",
            "ewah_batch_free", "ewah_device_errors",
            "ewah_num_cus", "ewah_query_features", "ewah_batch_features", "ewah_batch_select",
            "ewah_batch_get_variants", "ewah_batch_time_queries", "ewah_batch_select_model",
            "ewah_variant_code_full", "ewah_selector_load", "ewah_selector_save", "ewah_selector_free",
            "ewah_selector_num_arms", "ewah_selector_arm_codes", "ewah_selector_train", "ewah_selector_train_loss",
            "ewah_selector_predict", "ewah_mlp_create", "ewah_mlp_free", "ewah_mlp_num_params",
            "ewah_mlp_get_params", "ewah_mlp_set_params", "ewah_mlp_forward", "ewah_mlp_grad",
            "ewah_mlp_train_step", "ewah_mlp_last_error"]


class EwahError(RuntimeError):
    def __init__(self, code, where):
        msg = _last_error().decode(errors="replace")
        super().__init__(f"{where}: status {code}: {msg}")
        self.code = code


def _check(code, where):
    if code != OK:
        raise EwahError(code, where)


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)   # torch.cuda.Stream: a hipStream_t on ROCm


def init(device: int = 0):
    _check(_init(device), "init")


def num_cus() -> int:
    return int(_num_cus())


def output_bound(n_bits: int, sum_input_words: int) -> int:
    return int(_output_bound(n_bits, sum_input_words))


def variant_code(dense: bool, walk: int, litwalk: int, looped: bool = False, gate: int = 0) -> int:
    if gate:
        return int(_variant_code_full(1 if dense else 0, walk, litwalk, 1 if looped else 0, gate))
    if looped:
        return int(_variant_code_ex(1 if dense else 0, walk, litwalk, 1))
    return int(_variant_code(1 if dense else 0, walk, litwalk))


def default_variant() -> int:
    return int(_default_variant())


class Bitmap:
    """A registered bitmap (library-owned device copy + indexes)."""
    __slots__ = ("_h", "n_bits", "n_words")

    def __init__(self, handle, n_bits, n_words):
        self._h = handle
        self.n_bits = n_bits
        self.n_words = n_words

    @property
    def handle(self):
        return self._h

    def stats(self) -> dict:
        s = Stats()
        _check(_get_stats(self._h, ctypes.byref(s)), "get_stats")
        return s.as_dict()

    def device_words_ptr(self) -> int:
        return int(_device_words(self._h))

    def release(self):
        if self._h:
            _release(self._h)
            self._h = None


def register_many(streams, n_bits: int, on_device: bool = False) -> list:
    """Register EWAH streams (np.uint64 host arrays, or device pointers with on_device)."""
    count = len(streams)
    if count == 0:
        return []
    views = (View * count)()
    keep = []
    for i, s in enumerate(streams):
        if on_device:
            ptr, n = s
        else:
            a = np.ascontiguousarray(np.asarray(s, dtype=np.uint64))
            keep.append(a)
            ptr, n = (a.ctypes.data if len(a) else None), len(a)
        views[i].words = ptr
        views[i].n_words = n
        views[i].n_bits = n_bits
    outs = (_vp * count)()
    _check(_register_many(views, count, 1 if on_device else 0, outs), "register_many")
    res = []
    for i in range(count):
        res.append(Bitmap(outs[i], n_bits, views[i].n_words))
    return res


def register(stream, n_bits: int) -> Bitmap:
    return register_many([stream], n_bits)[0]


class Inputs:
    """The inputs of a query marshalled once (the C array of handles), for callers that run
    many queries over the same list; every query function takes it in place of a list."""

    def __init__(self, bitmaps):
        self.bitmaps = list(bitmaps)
        self.n = len(self.bitmaps)
        self.arr = (_vp * max(self.n, 1))(*[b.handle for b in self.bitmaps])

    def __len__(self):
        return self.n

    def __getitem__(self, i):
        return self.bitmaps[i]

    def __iter__(self):
        return iter(self.bitmaps)


def _handles(bitmaps):
    if isinstance(bitmaps, Inputs):
        return bitmaps.arr, bitmaps.n
    n = len(bitmaps)
    return (_vp * max(n, 1))(*[b.handle for b in bitmaps]), n


def threshold(bitmaps, T: int, out_words_ptr: int, out_cap: int, out_n_ptr: int, stream=None, variant: int = 0):
    """Enqueue one T-of-N query; outputs are device pointers (e.g. tensor.data_ptr())."""
    arr, n = _handles(bitmaps)
    _check(_threshold_v(arr, n, T, out_words_ptr, out_cap, out_n_ptr, variant, _stream_ptr(stream)), "threshold")


def threshold_noalloc(bitmaps, T: int, out_words_ptr: int, out_cap: int, out_n_ptr: int, stream=None):
    """As threshold, through the entry point that allocates nothing (its scratch is a static
    device array shared by every call on the GPU: calls that overlap race)."""
    arr, n = _handles(bitmaps)
    _check(_threshold_noalloc(arr, n, T, out_words_ptr, out_cap, out_n_ptr, _stream_ptr(stream)), "threshold_noalloc")


def symmetric(bitmaps, f, out_words_ptr: int, out_cap: int, out_n_ptr: int, stream=None):
    """Enqueue one query of a symmetric function: output row i is f[c_i], c_i = number of inputs
    with row i set; f is a sequence of len(bitmaps) + 1 truth values (counts 0..N)."""
    arr, n = _handles(bitmaps)
    tab = (ctypes.c_uint8 * max(len(f), 1))(*[1 if v else 0 for v in f])
    _check(_symmetric(arr, n, tab, len(f), out_words_ptr, out_cap, out_n_ptr, _stream_ptr(stream)), "symmetric")


def opt_threshold(bitmaps, K: int, out_words_ptr: int, out_cap: int, out_n_ptr: int, stream=None) -> int:
    """Largest T whose T-of-N result has at least K rows; its result is enqueued to the outputs.
    Returns T (the call waits for it)."""
    arr, n = _handles(bitmaps)
    t = _u32(0)
    _check(_opt_threshold(arr, n, K, out_words_ptr, out_cap, out_n_ptr, ctypes.byref(t), _stream_ptr(stream)),
           "opt_threshold")
    return int(t.value)


def count_histogram(bitmaps, stream=None) -> np.ndarray:
    """hist[c] = rows set in exactly c of the inputs, c = 0..len(bitmaps) (the call waits)."""
    arr, n = _handles(bitmaps)
    hist = np.zeros(n + 1, dtype=np.uint64)
    _check(_count_histogram(arr, n, hist.ctypes.data, _stream_ptr(stream)), "count_histogram")
    return hist


class Batch:
    """A planned batch of queries run by one persistent, optionally graph-captured launch."""

    def __init__(self, pool, queries, out_ptrs, out_caps, out_n_ptrs, variants=None, grid=0, use_graph=True):
        nq = len(queries)
        pool_arr = (_vp * len(pool))(*[b.handle for b in pool])
        qs = (Query * nq)()
        self._idx = []
        for i, (idx, T) in enumerate(queries):
            a = np.ascontiguousarray(np.asarray(idx, dtype=np.uint32))
            self._idx.append(a)
            qs[i].idx = a.ctypes.data
            qs[i].n = len(a)
            qs[i].T = T
            qs[i].out_words_dev = out_ptrs[i]
            qs[i].out_cap = out_caps[i]
            qs[i].out_n_words_dev = out_n_ptrs[i]
            qs[i].variant = 0 if variants is None else int(variants[i])
        cfg = BatchConfig(grid, 1 if use_graph else 0)
        h = _vp()
        _check(_batch_plan(pool_arr, len(pool), qs, nq, ctypes.byref(cfg), ctypes.byref(h)), "batch_plan")
        self._h = h
        self.nq = nq
        self.grid = grid          # 0: the library default (as many workgroups as are resident at once)
        self.win_batch = 6
        self.prepass = None       # None: the library default (on for batches of at least 65,536 items)

    def run(self, stream=None):
        _check(_batch_run(self._h, _stream_ptr(stream)), "batch_run")

    def set_variants(self, variants):
        a = np.ascontiguousarray(np.asarray(variants, dtype=np.uint32))
        assert len(a) == self.nq
        _check(_batch_set_variants(self._h, a.ctypes.data), "batch_set_variants")

    def set_grid(self, grid: int):
        _check(_batch_set_grid(self._h, grid), "batch_set_grid")
        self.grid = grid

    def set_win_batch(self, win_batch: int):
        _check(_batch_set_win_batch(self._h, win_batch), "batch_set_win_batch")
        self.win_batch = win_batch

    def set_prepass(self, on: bool):
        _check(_batch_set_prepass(self._h, 1 if on else 0), "batch_set_prepass")
        self.prepass = bool(on)

    def features(self, feat_ptr: int, stream=None):
        _check(_batch_features(self._h, feat_ptr, _stream_ptr(stream)), "batch_features")

    def select(self, pred_ptr: int, arm_codes, stream=None):
        a = np.ascontiguousarray(np.asarray(arm_codes, dtype=np.uint32))
        self._codes = a
        _check(_batch_select(self._h, pred_ptr, len(a), a.ctypes.data, _stream_ptr(stream)), "batch_select")

    def set_arm_codes(self, arm_codes):
        self._codes = np.ascontiguousarray(np.asarray(arm_codes, dtype=np.uint32))

    def select_async(self, pred_ptr: int, stream=None):
        """Device argmin over pred [nq][K] with the arm codes set by set_arm_codes."""
        a = self._codes
        _check(_batch_select(self._h, pred_ptr, len(a), a.ctypes.data, _stream_ptr(stream)), "batch_select")

    def time_queries(self, reps: int = 2, stream=None) -> np.ndarray:
        """Per-query busy time inside the batch (us), min over reps eager runs."""
        out = np.zeros(self.nq, dtype=np.float32)
        _check(_batch_time_queries(self._h, reps, out.ctypes.data, _stream_ptr(stream)), "batch_time_queries")
        return out

    def select_model(self, selector, mode: int = 0, stream=None):
        """Features -> selector prediction -> per-query argmin into the batch (device, asynchronous)."""
        _check(_batch_select_model(self._h, selector.handle, mode, _stream_ptr(stream)), "batch_select_model")

    def get_variants(self) -> np.ndarray:
        out = np.zeros(self.nq, dtype=np.uint32)
        _check(_batch_get_variants(self._h, out.ctypes.data), "batch_get_variants")
        return out

    def free(self):
        if self._h:
            _batch_free(self._h)
            self._h = None


class Selector:
    """Handle of a library selector: learned cost model plus rule set (ewah_selector_*)."""

    def __init__(self, handle):
        self._h = handle
        self.n_arms = int(_selector_num_arms(handle))

    @property
    def handle(self):
        return self._h

    @classmethod
    def load(cls, path: str) -> "Selector":
        h = _vp()
        _check(_selector_load(os.fsencode(path), ctypes.byref(h)), "selector_load")
        return cls(h)

    @classmethod
    def train(cls, feat, log2_time, arm_codes, epochs: int = 0, batch: int = 0, lr: float = 0.0,
              seed: int = 0) -> "Selector":
        F = np.ascontiguousarray(np.asarray(feat, dtype=np.float32))
        Y = np.ascontiguousarray(np.asarray(log2_time, dtype=np.float32))
        C = np.ascontiguousarray(np.asarray(arm_codes, dtype=np.uint32))
        assert F.ndim == 2 and F.shape[1] == 16 and Y.shape == (F.shape[0], len(C))
        cfg = TrainConfig(epochs, batch, lr, seed)
        h = _vp()
        _check(_selector_train(F.ctypes.data, Y.ctypes.data, F.shape[0], len(C), C.ctypes.data, ctypes.byref(cfg),
                               ctypes.byref(h)), "selector_train")
        return cls(h)

    def save(self, path: str):
        _check(_selector_save(self._h, os.fsencode(path)), "selector_save")

    def arm_codes(self) -> np.ndarray:
        out = np.zeros(self.n_arms, dtype=np.uint32)
        _check(_selector_arm_codes(self._h, out.ctypes.data), "selector_arm_codes")
        return out

    def train_loss(self) -> float:
        return float(_selector_train_loss(self._h))

    def predict(self, feat_ptr: int, n: int, pred_ptr: int, mode: int = 0, stream=None):
        _check(_selector_predict(self._h, mode, feat_ptr, n, pred_ptr, _stream_ptr(stream)), "selector_predict")

    def free(self):
        if self._h:
            _selector_free(self._h)
            self._h = None


def query_features(pool, queries, feat_ptr: int, stream=None):
    """Device features [nq][16] of queries (idx, T) over registered pool bitmaps."""
    pool_arr = (_vp * len(pool))(*[b.handle for b in pool])
    offs = np.zeros(len(queries) + 1, dtype=np.uint32)
    for i, (idx, _) in enumerate(queries):
        offs[i + 1] = offs[i] + len(idx)
    idx = np.ascontiguousarray(np.concatenate([np.asarray(q[0], dtype=np.uint32) for q in queries])
                               if queries else np.zeros(0, dtype=np.uint32))
    T = np.ascontiguousarray(np.array([q[1] for q in queries], dtype=np.uint32))
    _check(_query_features(pool_arr, len(pool), idx.ctypes.data, offs.ctypes.data, T.ctypes.data, len(queries),
                           feat_ptr, _stream_ptr(stream)), "query_features")


class MLPError(RuntimeError):
    pass


def _mcheck(code, where):
    if code != OK:
        raise MLPError(f"{where}: status {code}: {_mlp_last_error().decode(errors='replace')}")


class MLP:
    """Handle of the library's FP32 16 -> 64 -> 64 -> n_out MLP (device-resident parameters)."""

    def __init__(self, n_out: int, seed: int = 1):
        h = _vp()
        _mcheck(_mlp_create(n_out, seed, ctypes.byref(h)), "mlp_create")
        self._h = h
        self.n_out = n_out
        self.n_params = int(_mlp_num_params(n_out))

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.n_params, dtype=np.float32)
        _mcheck(_mlp_get_params(self._h, a.ctypes.data, self.n_params), "mlp_get_params")
        return a

    def set_params(self, p) -> None:
        a = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        assert a.size == self.n_params
        _mcheck(_mlp_set_params(self._h, a.ctypes.data, self.n_params), "mlp_set_params")

    def forward(self, x_ptr: int, batch: int, y_ptr: int, stream=None):
        _mcheck(_mlp_forward(self._h, x_ptr, batch, y_ptr, _stream_ptr(stream)), "mlp_forward")

    def grad(self, x_ptr: int, t_ptr: int, batch: int, g_ptr: int, loss_ptr: int, stream=None):
        _mcheck(_mlp_grad(self._h, x_ptr, t_ptr, batch, g_ptr, loss_ptr, _stream_ptr(stream)), "mlp_grad")

    def train_step(self, x_ptr: int, t_ptr: int, batch: int, lr: float, loss_ptr: int, stream=None):
        _mcheck(_mlp_train_step(self._h, x_ptr, t_ptr, batch, lr, loss_ptr, _stream_ptr(stream)), "mlp_train_step")

    def free(self):
        if self._h:
            _mlp_free(self._h)
            self._h = None


def device_errors() -> int:
    v = _u32(0)
    _check(_device_errors(ctypes.byref(v)), "device_errors")
    return int(v.value)
