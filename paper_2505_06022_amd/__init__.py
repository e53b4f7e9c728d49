"""Python binding of libccl (ctypes): argument marshalling only.

Every function here has the name of the C entry point it calls (see
``include/ccl.h``) and does nothing but convert arguments; all device work
runs in the library's HIP kernels.  If ``libccl.so`` has not been built the
first call raises: there is no fallback path.

PyTorch is used only by the helpers in ``fields`` for device memory and
streams; this module imports it lazily.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "libccl.so"

CCL_OK = 0
CCL_E_INVALID = -1
CCL_E_RANGE = -2
CCL_E_HIP = -3
CCL_E_UNSUPPORTED = -4
CCL_E_NOMEM = -5
CCL_E_STATE = -6
CCL_E_TIMEOUT = -7

CCL_MAX_DIMS = 3
CCL_MAX_CHUNKS = 64
CCL_MAX_DEPTH = 8

ONE_TO_ONE, NEIGHBORHOOD, ALL, FIXED, SLICE = 0, 1, 2, 3, 4

_I64x3 = ctypes.c_int64 * 3


class ccl_subrange(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32), ("offset", _I64x3), ("range", _I64x3)]

    def box(self):
        d = self.dims
        return (tuple(self.offset[:d]), tuple(self.range[:d]))


class ccl_chunk(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32), ("offset", _I64x3), ("range", _I64x3),
                ("global_offset", _I64x3), ("global_range", _I64x3)]

    def box(self):
        d = self.dims
        return (tuple(self.offset[:d]), tuple(self.range[:d]))


class ccl_range_mapper(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("extent", _I64x3), ("offset", _I64x3),
                ("dim", ctypes.c_int32)]


class ccl_chunk_buffer(ctypes.Structure):
    _fields_ = [("base", ctypes.c_void_p), ("region", ccl_subrange), ("pitch", _I64x3)]


class ccl_accessor(ctypes.Structure):
    _fields_ = [("mapper", ccl_range_mapper), ("mode", ctypes.c_int32),
                ("buffer_range", _I64x3), ("bufs", ctypes.c_void_p)]


class ccl_kernel_fn(ctypes.Structure):
    _fields_ = [("fn", ctypes.c_int32), ("a", ctypes.c_float), ("dim", ctypes.c_int32)]


CCL_ACCESS_READ, CCL_ACCESS_WRITE, CCL_ACCESS_READ_WRITE = 1, 2, 3
CCL_FN_SAXPY, CCL_FN_SUM_ALONG = 0, 1


class ccl_transfer(ctypes.Structure):
    _fields_ = [("owner", ctypes.c_int32), ("reader", ctypes.c_int32), ("box", ccl_subrange)]


class ccl_wave_params(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32), ("r2", ctypes.c_double),
                ("temporal_depth", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("dtype", ctypes.c_int32)]


CCL_DTYPE_F32, CCL_DTYPE_F64, CCL_DTYPE_BF16, CCL_DTYPE_F16 = 0, 1, 2, 3
DTYPES = {"f32": CCL_DTYPE_F32, "f64": CCL_DTYPE_F64, "bf16": CCL_DTYPE_BF16,
          "f16": CCL_DTYPE_F16}
DTYPE_BYTES = {CCL_DTYPE_F32: 4, CCL_DTYPE_F64: 8, CCL_DTYPE_BF16: 2, CCL_DTYPE_F16: 2}


class ccl_batch_grid(ctypes.Structure):
    _fields_ = [("ny", ctypes.c_int64), ("nx", ctypes.c_int64), ("pitch", ctypes.c_int64),
                ("steps", ctypes.c_int32), ("temporal_depth", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("r2", ctypes.c_float),
                ("buf", ctypes.c_void_p * 4)]


CCL_BATCH_NO_GRAPH = 1
CCL_BATCH_PER_GRID = 2


class ccl_tune_config(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32), ("shape", _I64x3), ("nchunks", ctypes.c_int32),
                ("temporal_depth", ctypes.c_int32), ("tile_rows", ctypes.c_int32)]


class ccl_tune_sample(ctypes.Structure):
    _fields_ = [("seconds_per_step", ctypes.c_double), ("joules_per_step", ctypes.c_double),
                ("window_seconds", ctypes.c_double), ("runs_in_window", ctypes.c_int32)]


CCL_MLP_IN, CCL_MLP_HIDDEN, CCL_MLP_OUT, CCL_MLP_NPARAMS = 12, 64, 2, 5122
CCL_MLP_PARAMS, CCL_MLP_GRADS, CCL_MLP_LOSS = 0, 1, 2


class CclError(RuntimeError):
    def __init__(self, fn: str, status: int, message: str):
        super().__init__(f"{fn} failed with status {status}: {message}")
        self.status = status
        self.message = message


# Every symbol include/ccl.h declares, with (restype, argtypes).
_P = ctypes.POINTER
_SIGS = {
    "ccl_version": (ctypes.c_char_p, []),
    "ccl_last_error": (ctypes.c_char_p, []),
    "ccl_split_range": (ctypes.c_int32, [_P(ccl_subrange), ctypes.c_int32, ctypes.c_int32,
                                         _P(ccl_chunk)]),
    "ccl_split_grid": (ctypes.c_int32, [_P(ccl_subrange), _P(ctypes.c_int32), _P(ccl_chunk)]),
    "ccl_region_of": (ctypes.c_int32, [_P(ccl_chunk), _P(ccl_range_mapper), _P(ctypes.c_int64),
                                       _P(ccl_subrange)]),
    "ccl_transfers": (ctypes.c_int32, [ctypes.c_int32, _P(ccl_chunk), _P(ccl_range_mapper),
                                       _P(ctypes.c_int64), _P(ccl_transfer), ctypes.c_int32,
                                       _P(ctypes.c_int32)]),
    "ccl_halo_exchange": (ctypes.c_int32, [ctypes.c_int32, _P(ccl_chunk), _P(ccl_range_mapper),
                                           _P(ccl_chunk_buffer), ctypes.c_int32,
                                           ctypes.c_void_p]),
    "ccl_halo_pack": (ctypes.c_int32, [ctypes.c_int32, _P(ccl_subrange), _P(ccl_chunk_buffer),
                                       ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "ccl_halo_unpack": (ctypes.c_int32, [ctypes.c_int32, _P(ccl_subrange),
                                         _P(ccl_chunk_buffer), ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "ccl_wave_step": (ctypes.c_int32, [_P(ccl_wave_params), ctypes.c_int32, _P(ccl_chunk),
                                       _P(ccl_chunk_buffer), _P(ccl_chunk_buffer),
                                       _P(ccl_chunk_buffer), _P(ccl_chunk_buffer),
                                       ctypes.c_int32, ctypes.c_void_p]),
    "ccl_energy_read": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_void_p, _P(ctypes.c_double),
                                         _P(ctypes.c_uint64)]),
    "ccl_energy_backend": (ctypes.c_char_p, [ctypes.c_int32]),
    "ccl_parallel_for": (ctypes.c_int32, [_P(ccl_kernel_fn), ctypes.c_int32, _P(ccl_chunk),
                                          ctypes.c_int32, _P(ccl_accessor), ctypes.c_void_p]),
    "ccl_saxpy": (ctypes.c_int32, [ctypes.c_int64, ctypes.c_float, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ccl_wave_energy": (ctypes.c_int32, [ctypes.c_int32, _P(ctypes.c_int64), _P(ctypes.c_int64),
                                         ctypes.c_int32, ctypes.c_double, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ccl_batch_create": (ctypes.c_int32, [ctypes.c_int32, _P(ccl_batch_grid), ctypes.c_int32,
                                          _P(ctypes.c_void_p)]),
    "ccl_batch_run": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "ccl_batch_check": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "ccl_batch_set_wait_limit": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64]),
    "ccl_batch_result": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, _P(ctypes.c_int32),
                                          _P(ctypes.c_int32)]),
    "ccl_batch_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "ccl_batch_run_static": (ctypes.c_int32, [ctypes.c_int32, _P(ccl_batch_grid),
                                              _P(ctypes.c_int32), _P(ctypes.c_int32),
                                              _P(ctypes.c_int32), ctypes.c_void_p]),
    "ccl_autotune_measure": (ctypes.c_int32, [ctypes.c_int32, _P(ccl_tune_config), ctypes.c_float,
                                              ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                              ctypes.c_int32, ctypes.c_void_p,
                                              _P(ccl_tune_sample)]),
    "ccl_wave_plan_rows": (ctypes.c_int32, [_P(ccl_tune_config), _P(ctypes.c_int32)]),
    "ccl_wave_slots": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, _P(ctypes.c_int64)]),
    "ccl_costmodel_features": (ctypes.c_int32, [ctypes.c_int32, _P(ccl_tune_config),
                                                _P(ctypes.c_float)]),
    "ccl_mlp_create": (ctypes.c_int32, [_P(ctypes.c_float), _P(ctypes.c_void_p)]),
    "ccl_mlp_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "ccl_mlp_get": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, _P(ctypes.c_float)]),
    "ccl_mlp_forward": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "ccl_mlp_grad": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "ccl_mlp_grad_weighted": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p]),
    "ccl_mlp_adam": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float, ctypes.c_void_p]),
    "ccl_mlp_train": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_float, ctypes.c_void_p]),
    "ccl_mlp_pick": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_float, ctypes.c_float, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "ccl_mlp_rank": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_float, ctypes.c_float, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "ccl_autotune_candidates": (ctypes.c_int32, [ctypes.c_int32, _P(ctypes.c_int64),
                                                 ctypes.c_int32, ctypes.c_int32,
                                                 _P(ccl_tune_config), _P(ctypes.c_int32)]),
    "ccl_autotune_sweep": (ctypes.c_int32, [ctypes.c_int32, _P(ctypes.c_int64), ctypes.c_int32,
                                            ctypes.c_float, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_void_p, ctypes.c_int32, _P(ccl_tune_config),
                                            _P(ccl_tune_sample), _P(ctypes.c_int32),
                                            _P(ctypes.c_int32)]),
    "ccl_timing_enable": (ctypes.c_int32, [ctypes.c_int32]),
    "ccl_timing_query": (ctypes.c_int32, [ctypes.c_int32, _P(ctypes.c_int64),
                                          _P(ctypes.c_double)]),
}

CCL_KERNEL_STENCIL, CCL_KERNEL_HALO, CCL_KERNEL_SAXPY, CCL_KERNEL_BATCH = 0, 1, 2, 3

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libccl.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2505_06022_amd.build` "
                "(there is no fallback implementation)")
        L = ctypes.CDLL(str(LIB_PATH))
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(fn: str, st: int):
    if st != CCL_OK:
        raise CclError(fn, st, lib().ccl_last_error().decode())


def _stream(stream):
    """hipStream_t as a void*: None -> the current torch stream, int/ptr as is."""
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return stream


def _i64(vals, n=3):
    a = _I64x3()
    for i, v in enumerate(list(vals)[:n]):
        a[i] = int(v)
    return a


def make_subrange(offset, rng) -> ccl_subrange:
    s = ccl_subrange()
    s.dims = len(rng)
    s.offset = _i64(offset)
    s.range = _i64(rng)
    return s


def make_mapper(kind: int, extent=(0, 0, 0), offset=(0, 0, 0), dim: int = 0) -> ccl_range_mapper:
    """extent: NEIGHBORHOOD's growth per side or FIXED's box extent; offset:
    FIXED's box origin; dim: the dimension SLICE takes whole."""
    m = ccl_range_mapper()
    m.kind = int(kind)
    m.extent = _i64(extent)
    m.offset = _i64(offset)
    m.dim = int(dim)
    return m


def _mapper(kind, extent) -> ccl_range_mapper:
    """A mapper given as a ccl_range_mapper, or as (kind, extent)."""
    return kind if isinstance(kind, ccl_range_mapper) else make_mapper(kind, extent)


def ccl_version() -> str:
    return lib().ccl_version().decode()


def ccl_last_error() -> str:
    return lib().ccl_last_error().decode()


def ccl_split_range(offset, rng, nchunks: int, split_dim: int = 0):
    out = (ccl_chunk * max(1, nchunks))()
    r = make_subrange(offset, rng)
    _check("ccl_split_range", lib().ccl_split_range(ctypes.byref(r), nchunks, split_dim, out))
    return out


def ccl_split_grid(offset, rng, counts):
    """Chunks of the block split with counts[d] pieces along dimension d."""
    total = 1
    for c in counts:
        total *= max(1, int(c))
    out = (ccl_chunk * total)()
    r = make_subrange(offset, rng)
    cn = (ctypes.c_int32 * 3)(*[int(c) for c in counts], *([1] * (3 - len(counts))))
    _check("ccl_split_grid", lib().ccl_split_grid(ctypes.byref(r), cn, out))
    return out


def ccl_region_of(chunk: ccl_chunk, kind: int, extent, buffer_range) -> ccl_subrange:
    m = _mapper(kind, extent)
    br = _i64(buffer_range)
    out = ccl_subrange()
    _check("ccl_region_of", lib().ccl_region_of(ctypes.byref(chunk), ctypes.byref(m), br,
                                                ctypes.byref(out)))
    return out


def ccl_transfers(chunks, kind: int, extent, buffer_range):
    m = _mapper(kind, extent)
    br = _i64(buffer_range)
    n = ctypes.c_int32(0)
    st = lib().ccl_transfers(len(chunks), chunks, ctypes.byref(m), br, None, 0, ctypes.byref(n))
    if st not in (CCL_OK, CCL_E_RANGE):
        _check("ccl_transfers", st)
    out = (ccl_transfer * max(1, n.value))()
    _check("ccl_transfers", lib().ccl_transfers(len(chunks), chunks, ctypes.byref(m), br, out,
                                                n.value, ctypes.byref(n)))
    return list(out)[: n.value]


def ccl_halo_exchange(chunks, kind: int, extent, bufs, elem_bytes: int = 4, stream=None):
    m = _mapper(kind, extent)
    _check("ccl_halo_exchange", lib().ccl_halo_exchange(len(chunks), chunks, ctypes.byref(m),
                                                        bufs, elem_bytes, _stream(stream)))


def ccl_halo_pack(boxes, srcs, elem_bytes: int, staging_ptr: int, stream=None):
    bx = (ccl_subrange * len(boxes))(*boxes)
    _check("ccl_halo_pack", lib().ccl_halo_pack(len(boxes), bx, srcs, elem_bytes,
                                                ctypes.c_void_p(staging_ptr), _stream(stream)))


def ccl_halo_unpack(boxes, dsts, elem_bytes: int, staging_ptr: int, stream=None):
    bx = (ccl_subrange * len(boxes))(*boxes)
    _check("ccl_halo_unpack", lib().ccl_halo_unpack(len(boxes), bx, dsts, elem_bytes,
                                                    ctypes.c_void_p(staging_ptr),
                                                    _stream(stream)))


def make_wave_params(dims: int, r2: float, temporal_depth: int = 1, tile_rows: int = 0,
                     dtype: str = "f32"):
    """dtype: "f32", "f64", "bf16" or "f16" (the buffers' element type)."""
    p = ccl_wave_params()
    p.dims, p.r2, p.temporal_depth, p.tile_rows, p.flags = dims, r2, temporal_depth, tile_rows, 0
    p.dtype = DTYPES[dtype]
    return p


def ccl_wave_step(params: ccl_wave_params, chunks, u_prev, u_cur, w_prev, w_cur, nsteps: int,
                  stream=None):
    """Advances nsteps; the four ccl_chunk_buffer arrays are rotated in place."""
    _check("ccl_wave_step", lib().ccl_wave_step(ctypes.byref(params), len(chunks), chunks,
                                                u_prev, u_cur, w_prev, w_cur, int(nsteps),
                                                _stream(stream)))


def ccl_energy_read(device: int = 0, stream=None):
    """(joules, timestamp_ns).  ``stream`` (torch stream or hipStream_t int)
    is synchronised first when given; None reads without synchronising."""
    j = ctypes.c_double(0.0)
    ts = ctypes.c_uint64(0)
    s = _stream(stream) if stream is not None else None
    _check("ccl_energy_read", lib().ccl_energy_read(device, s, ctypes.byref(j), ctypes.byref(ts)))
    return j.value, ts.value


def ccl_energy_backend(device: int = 0) -> str:
    return lib().ccl_energy_backend(device).decode()


def make_accessor(mapper: ccl_range_mapper, mode: int, buffer_range, bufs) -> ccl_accessor:
    """`bufs`: a ctypes array of ccl_chunk_buffer, one per chunk (kept alive
    by the returned object)."""
    a = ccl_accessor()
    a.mapper = mapper
    a.mode = int(mode)
    a.buffer_range = _i64(buffer_range)
    a.bufs = ctypes.cast(bufs, ctypes.c_void_p)
    a._keep = bufs
    return a


def ccl_parallel_for(fn: int, chunks, accessors, a: float = 0.0, dim: int = 0, stream=None):
    k = ccl_kernel_fn()
    k.fn, k.a, k.dim = int(fn), float(a), int(dim)
    arr = (ccl_accessor * len(accessors))(*accessors)
    _check("ccl_parallel_for", lib().ccl_parallel_for(ctypes.byref(k), len(chunks), chunks,
                                                      len(accessors), arr, _stream(stream)))


def ccl_saxpy(n: int, a: float, x_ptr: int, y_ptr: int, z_ptr: int, stream=None):
    _check("ccl_saxpy", lib().ccl_saxpy(int(n), float(a), ctypes.c_void_p(x_ptr),
                                        ctypes.c_void_p(y_ptr), ctypes.c_void_p(z_ptr),
                                        _stream(stream)))


def ccl_wave_energy(shape, pitch, dtype: str, r2: float, u_new_ptr: int, u_old_ptr: int,
                    out_ptr: int, stream=None):
    """Discrete leapfrog energy of (u^{n+1}, u^n) held in one device buffer
    each; written as one double to the device pointer `out_ptr`.  `pitch`:
    element strides of the outer dimensions; `dtype`: "f32", "f64", "bf16"
    or "f16"."""
    dims = len(shape)
    sh = (ctypes.c_int64 * 3)(*[int(v) for v in shape])
    pt = (ctypes.c_int64 * 3)(*([int(v) for v in pitch] + [0] * (3 - len(pitch))))
    _check("ccl_wave_energy", lib().ccl_wave_energy(
        dims, sh, pt, DTYPES[dtype], float(r2), ctypes.c_void_p(u_new_ptr),
        ctypes.c_void_p(u_old_ptr), ctypes.c_void_p(out_ptr), _stream(stream)))


def ccl_timing_enable(on: bool = True):
    _check("ccl_timing_enable", lib().ccl_timing_enable(1 if on else 0))


def ccl_timing_query(kernel: int):
    """(launches, total_ms) of the recorded launches of one kernel family."""
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check("ccl_timing_query", lib().ccl_timing_query(int(kernel), ctypes.byref(n),
                                                      ctypes.byref(ms)))
    return n.value, ms.value


def ccl_batch_create(grids, flags: int = 0) -> ctypes.c_void_p:
    arr = (ccl_batch_grid * len(grids))(*grids)
    h = ctypes.c_void_p()
    _check("ccl_batch_create", lib().ccl_batch_create(len(grids), arr, int(flags),
                                                      ctypes.byref(h)))
    return h


def ccl_batch_run(h, stream=None):
    _check("ccl_batch_run", lib().ccl_batch_run(h, _stream(stream)))


def ccl_batch_check(h, stream=None):
    _check("ccl_batch_check", lib().ccl_batch_check(h, _stream(stream)))


def ccl_batch_set_wait_limit(h, microseconds: int):
    _check("ccl_batch_set_wait_limit", lib().ccl_batch_set_wait_limit(h, int(microseconds)))


def ccl_batch_result(h, grid: int):
    p = ctypes.c_int32(0)
    c = ctypes.c_int32(0)
    _check("ccl_batch_result", lib().ccl_batch_result(h, int(grid), ctypes.byref(p),
                                                      ctypes.byref(c)))
    return p.value, c.value


def ccl_batch_destroy(h):
    _check("ccl_batch_destroy", lib().ccl_batch_destroy(h))


CCL_BATCH_STATIC_BYTES = 4 << 20


def ccl_batch_run_static(grids, stream=None, check: bool = False):
    """One persistent run of `grids` (a list of ccl_batch_grid) with the
    library's static device tables (no device allocation).  Returns the
    (prev, cur) buffer index of every grid; with `check`, the call also
    synchronises the stream and raises on a dependency-wait timeout."""
    n = len(grids)
    arr = (ccl_batch_grid * n)(*grids)
    prev = (ctypes.c_int32 * n)()
    cur = (ctypes.c_int32 * n)()
    failed = ctypes.c_int32(0)
    _check("ccl_batch_run_static",
           lib().ccl_batch_run_static(n, arr, prev, cur, ctypes.byref(failed) if check else None,
                                      _stream(stream)))
    return list(zip(prev, cur))


def make_tune_config(shape, nchunks: int, temporal_depth: int, tile_rows: int = 0):
    c = ccl_tune_config()
    c.dims = len(shape)
    c.shape = _i64(shape)
    c.nchunks, c.temporal_depth, c.tile_rows = int(nchunks), int(temporal_depth), int(tile_rows)
    return c


def ccl_autotune_measure(cfgs, r2: float, steps: int, reps: int = 3,
                         energy_window_s: float = 0.0, device: int = 0, stream=None):
    arr = (ccl_tune_config * len(cfgs))(*cfgs)
    out = (ccl_tune_sample * len(cfgs))()
    _check("ccl_autotune_measure",
           lib().ccl_autotune_measure(len(cfgs), arr, float(r2), int(steps), int(reps),
                                      float(energy_window_s), int(device), _stream(stream), out))
    return list(out)


CCL_OBJECTIVE_TIME, CCL_OBJECTIVE_ENERGY, CCL_OBJECTIVE_EDP = 0, 1, 2
OBJECTIVE_CODES = {"time": CCL_OBJECTIVE_TIME, "energy": CCL_OBJECTIVE_ENERGY,
                   "edp": CCL_OBJECTIVE_EDP}


def ccl_autotune_candidates(shape, nchunks: int = 0):
    """The library's candidate configs for a domain shape (K, tile rows, T;
    only K == nchunks when nchunks > 0)."""
    dims = len(shape)
    sh = (ctypes.c_int64 * 3)(*([int(v) for v in shape] + [0] * (3 - dims)))
    n = ctypes.c_int32(0)
    st = lib().ccl_autotune_candidates(dims, sh, int(nchunks), 0, None, ctypes.byref(n))
    if st not in (CCL_OK, CCL_E_RANGE):
        _check("ccl_autotune_candidates", st)
    out = (ccl_tune_config * max(1, n.value))()
    _check("ccl_autotune_candidates", lib().ccl_autotune_candidates(
        dims, sh, int(nchunks), n.value, out, ctypes.byref(n)))
    return list(out)[:n.value]


def ccl_autotune_sweep(shape, nchunks: int, r2: float, steps: int, reps: int = 3,
                       energy_window_s: float = 0.0, objective: str = "time", device: int = 0,
                       stream=None):
    """Every candidate of the shape (K == nchunks when nchunks > 0) measured;
    returns (configs, samples, index of the best by `objective`)."""
    dims = len(shape)
    sh = (ctypes.c_int64 * 3)(*([int(v) for v in shape] + [0] * (3 - dims)))
    cap = len(ccl_autotune_candidates(shape, nchunks))
    cfgs = (ccl_tune_config * max(1, cap))()
    out = (ccl_tune_sample * max(1, cap))()
    n, best = ctypes.c_int32(0), ctypes.c_int32(-1)
    _check("ccl_autotune_sweep", lib().ccl_autotune_sweep(
        dims, sh, int(nchunks), float(r2), int(steps), int(reps), float(energy_window_s),
        OBJECTIVE_CODES[objective], int(device), _stream(stream), cap, cfgs, out,
        ctypes.byref(n), ctypes.byref(best)))
    return list(cfgs)[:n.value], list(out)[:n.value], best.value


def ccl_wave_plan_rows(cfg) -> int:
    r = ctypes.c_int32(0)
    _check("ccl_wave_plan_rows", lib().ccl_wave_plan_rows(ctypes.byref(cfg), ctypes.byref(r)))
    return r.value


def ccl_wave_slots(dims: int, T: int) -> int:
    v = ctypes.c_int64(0)
    _check("ccl_wave_slots", lib().ccl_wave_slots(dims, T, ctypes.byref(v)))
    return v.value


def ccl_costmodel_features(cfgs):
    import numpy as np
    arr = (ccl_tune_config * len(cfgs))(*cfgs)
    x = np.zeros((len(cfgs), CCL_MLP_IN), dtype=np.float32)
    _check("ccl_costmodel_features", lib().ccl_costmodel_features(
        len(cfgs), arr, x.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return x


def ccl_mlp_create(params):
    import numpy as np
    p = np.ascontiguousarray(params, dtype=np.float32).ravel()
    if p.size != CCL_MLP_NPARAMS:
        raise ValueError(f"expected {CCL_MLP_NPARAMS} parameters, got {p.size}")
    h = ctypes.c_void_p()
    _check("ccl_mlp_create", lib().ccl_mlp_create(p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                  ctypes.byref(h)))
    return h


def ccl_mlp_destroy(h):
    _check("ccl_mlp_destroy", lib().ccl_mlp_destroy(h))


def ccl_mlp_get(h, what: int):
    import numpy as np
    out = np.zeros(1 if what == CCL_MLP_LOSS else CCL_MLP_NPARAMS, dtype=np.float32)
    _check("ccl_mlp_get", lib().ccl_mlp_get(h, int(what),
                                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out


def ccl_mlp_forward(h, n: int, x_ptr: int, y_ptr: int, stream=None):
    _check("ccl_mlp_forward", lib().ccl_mlp_forward(h, int(n), ctypes.c_void_p(x_ptr),
                                                    ctypes.c_void_p(y_ptr), _stream(stream)))


def ccl_mlp_grad(h, n: int, x_ptr: int, t_ptr: int, stream=None):
    _check("ccl_mlp_grad", lib().ccl_mlp_grad(h, int(n), ctypes.c_void_p(x_ptr),
                                              ctypes.c_void_p(t_ptr), _stream(stream)))


def ccl_mlp_grad_weighted(h, n: int, x_ptr: int, t_ptr: int, w_ptr: int, stream=None):
    _check("ccl_mlp_grad_weighted", lib().ccl_mlp_grad_weighted(
        h, int(n), ctypes.c_void_p(x_ptr), ctypes.c_void_p(t_ptr),
        ctypes.c_void_p(w_ptr) if w_ptr else None, _stream(stream)))


def ccl_mlp_adam(h, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check("ccl_mlp_adam", lib().ccl_mlp_adam(h, float(lr), float(beta1), float(beta2),
                                              float(eps), _stream(stream)))


def ccl_mlp_train(h, n: int, x_ptr: int, t_ptr: int, epochs: int, lr: float = 1e-3,
                  stream=None, w_ptr: int = 0):
    _check("ccl_mlp_train", lib().ccl_mlp_train(h, int(n), ctypes.c_void_p(x_ptr),
                                                ctypes.c_void_p(t_ptr),
                                                ctypes.c_void_p(w_ptr) if w_ptr else None,
                                                int(epochs), float(lr), _stream(stream)))


def ccl_mlp_rank(h, n: int, x_ptr: int, w_time: float, w_energy: float, k: int,
                 order_ptr: int, stream=None):
    _check("ccl_mlp_rank", lib().ccl_mlp_rank(h, int(n), ctypes.c_void_p(x_ptr), float(w_time),
                                              float(w_energy), int(k),
                                              ctypes.c_void_p(order_ptr), _stream(stream)))


def ccl_mlp_pick(h, n: int, x_ptr: int, w_time: float, w_energy: float, scores_ptr: int,
                 best_ptr: int, stream=None):
    _check("ccl_mlp_pick", lib().ccl_mlp_pick(h, int(n), ctypes.c_void_p(x_ptr), float(w_time),
                                              float(w_energy),
                                              ctypes.c_void_p(scores_ptr) if scores_ptr else None,
                                              ctypes.c_void_p(best_ptr), _stream(stream)))
