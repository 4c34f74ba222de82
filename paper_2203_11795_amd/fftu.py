"""ctypes binding of libfftu (include/fftu.h): argument marshalling only.

Every step of the transform runs in the HIP kernels of libfftu.so; this module
only passes device pointers, sizes and streams. PyTorch supplies device memory
and streams. If the library is missing, loading fails loudly -- there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfftu.so")

FORWARD = -1
INVERSE = 1
C64 = 1
C128 = 2
MAX_DIMS = 8
NOALLOC_MAX_BYTES = 64 << 20     # FFTU_NOALLOC_MAX_BYTES: the fixed workspace of fftu_execute_noalloc

STATUS = {0: "FFTU_SUCCESS", 1: "FFTU_ERROR_INVALID_VALUE", 2: "FFTU_ERROR_NOT_DIVISIBLE",
          3: "FFTU_ERROR_UNSUPPORTED", 4: "FFTU_ERROR_OUT_OF_MEMORY", 5: "FFTU_ERROR_DEVICE"}

# Every entry point declared in include/fftu.h.
EXPORTS = ["fftu_version", "fftu_status_string", "fftu_last_error", "fftu_check", "fftu_describe", "fftu_plan",
           "fftu_get_plan_info", "fftu_plan_device_bytes", "fftu_execute", "fftu_plan_external", "fftu_execute_ws", "fftu_execute_noalloc", "fftu_plan_real",
           "fftu_plan_r2r",
           "fftu_stage_local_fft",
           "fftu_stage_twiddle", "fftu_stage_exchange", "fftu_stage_remaining_fft", "fftu_stage_superstep", "fftu_timing_begin",
           "fftu_timing_end", "fftu_set_tuning", "fftu_get_tuning", "fftu_launch_name", "fftu_plan_batch", "fftu_execute_batch", "fftu_batch_error",
           "fftu_plan_batch_external", "fftu_batch_workspace_bytes", "fftu_batch_staging_bytes", "fftu_execute_batch_ws",
           "fftu_graph_capture", "fftu_graph_launch", "fftu_graph_destroy", "fftu_fill_uniform", "fftu_plan_convolution",
           "fftu_execute_convolution", "fftu_pointwise_mul", "fftu_destroy"]

TUNE = {"line_strided_logw": 0, "line_contig_logw": 1, "line_pad": 2, "max_lds_kb": 3, "fuse_last": 4, "pair": 5,
        "mixed_radix": 6, "mixed_tile_log": 7}


class FftuError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = int(status)
        super().__init__(f"{where}: {STATUS.get(self.status, self.status)}")


class PlanInfo(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("N", ctypes.c_int64), ("P", ctypes.c_int64), ("M", ctypes.c_int64),
                ("s0_kernels", ctypes.c_int32), ("exchange_fused", ctypes.c_int32),
                ("s2_kernels", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_uint64), ("table_bytes", ctypes.c_uint64),
                ("supersteps", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfftu.so and declare the signatures. Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libfftu.so is not built ({path}); run `python -m paper_2203_11795_amd.build`")
    lib = ctypes.CDLL(path)
    i64p = ctypes.POINTER(ctypes.c_int64)
    vp = ctypes.c_void_p
    lib.fftu_version.restype = ctypes.c_char_p
    lib.fftu_version.argtypes = []
    lib.fftu_status_string.restype = ctypes.c_char_p
    lib.fftu_status_string.argtypes = [ctypes.c_int]
    lib.fftu_last_error.restype = ctypes.c_int
    lib.fftu_last_error.argtypes = []
    lib.fftu_check.restype = ctypes.c_int
    lib.fftu_check.argtypes = [ctypes.c_int, i64p, i64p, ctypes.c_int, ctypes.c_int]
    lib.fftu_describe.restype = ctypes.c_int
    lib.fftu_describe.argtypes = [ctypes.c_int, i64p, i64p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(PlanInfo)]
    lib.fftu_plan.restype = vp
    lib.fftu_plan.argtypes = [ctypes.c_int, i64p, i64p, ctypes.c_int, ctypes.c_int]
    lib.fftu_get_plan_info.restype = ctypes.c_int
    lib.fftu_get_plan_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.fftu_plan_device_bytes.restype = ctypes.c_size_t
    lib.fftu_plan_device_bytes.argtypes = [vp]
    for name in ["fftu_execute", "fftu_stage_local_fft", "fftu_stage_twiddle", "fftu_stage_exchange",
                 "fftu_stage_remaining_fft"]:
        fn = getattr(lib, name)
        fn.restype = ctypes.c_int
        fn.argtypes = [vp, vp, vp, vp]
    lib.fftu_stage_superstep.restype = ctypes.c_int
    lib.fftu_stage_superstep.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    lib.fftu_plan_external.restype = vp
    lib.fftu_plan_external.argtypes = [ctypes.c_int, i64p, i64p, ctypes.c_int, ctypes.c_int]
    lib.fftu_plan_real.restype = vp
    lib.fftu_plan_real.argtypes = [ctypes.c_int, i64p, i64p, ctypes.c_int, ctypes.c_int]
    lib.fftu_plan_r2r.restype = vp
    lib.fftu_plan_r2r.argtypes = [ctypes.c_int, i64p, i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.fftu_execute_ws.restype = ctypes.c_int
    lib.fftu_execute_ws.argtypes = [vp, vp, vp, vp, vp]
    lib.fftu_execute_noalloc.restype = ctypes.c_int
    lib.fftu_execute_noalloc.argtypes = [vp, vp, vp, vp]
    lib.fftu_timing_begin.restype = ctypes.c_int
    lib.fftu_timing_begin.argtypes = [vp, ctypes.c_int]
    lib.fftu_timing_end.restype = ctypes.c_int
    lib.fftu_timing_end.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.fftu_set_tuning.restype = ctypes.c_int
    lib.fftu_set_tuning.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.fftu_get_tuning.restype = ctypes.c_int
    lib.fftu_get_tuning.argtypes = [ctypes.c_int]
    lib.fftu_launch_name.restype = ctypes.c_char_p
    lib.fftu_launch_name.argtypes = [vp, ctypes.c_int]
    ptr_arr = ctypes.POINTER(ctypes.c_void_p)
    lib.fftu_plan_batch.restype = vp
    lib.fftu_plan_batch.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(i64p),
                                    ctypes.POINTER(i64p), ctypes.c_int, ctypes.c_int]
    lib.fftu_execute_batch.restype = ctypes.c_int
    lib.fftu_execute_batch.argtypes = [vp, ptr_arr, ptr_arr, vp]
    lib.fftu_plan_batch_external.restype = vp
    lib.fftu_plan_batch_external.argtypes = lib.fftu_plan_batch.argtypes
    lib.fftu_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.fftu_batch_workspace_bytes.argtypes = [vp]
    lib.fftu_batch_staging_bytes.restype = ctypes.c_size_t
    lib.fftu_batch_staging_bytes.argtypes = [vp]
    lib.fftu_execute_batch_ws.restype = ctypes.c_int
    lib.fftu_execute_batch_ws.argtypes = [vp, ptr_arr, ptr_arr, vp, vp, vp]
    lib.fftu_batch_error.restype = ctypes.c_int
    lib.fftu_batch_error.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    lib.fftu_graph_capture.restype = vp
    lib.fftu_graph_capture.argtypes = [vp, ctypes.c_int, ptr_arr, ptr_arr]
    lib.fftu_graph_launch.restype = ctypes.c_int
    lib.fftu_graph_launch.argtypes = [vp, vp]
    lib.fftu_graph_destroy.restype = None
    lib.fftu_graph_destroy.argtypes = [vp]
    lib.fftu_fill_uniform.restype = ctypes.c_int
    lib.fftu_fill_uniform.argtypes = [vp, ctypes.c_int64, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint64, vp]
    lib.fftu_plan_convolution.restype = vp
    lib.fftu_plan_convolution.argtypes = [ctypes.c_int, i64p, i64p, ctypes.c_int]
    lib.fftu_execute_convolution.restype = ctypes.c_int
    lib.fftu_execute_convolution.argtypes = [vp, vp, vp, vp, vp]
    lib.fftu_pointwise_mul.restype = ctypes.c_int
    lib.fftu_pointwise_mul.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_int, ctypes.c_double, vp]
    lib.fftu_destroy.restype = None
    lib.fftu_destroy.argtypes = [vp]
    _lib = lib
    return lib


def _arr(vals):
    vals = [int(v) for v in vals]
    return (ctypes.c_int64 * len(vals))(*vals)


def _dtype_code(dtype) -> int:
    name = str(dtype)
    if name.endswith("complex128"):
        return C128
    if name.endswith("complex64"):
        return C64
    if dtype in (C64, C128):
        return int(dtype)
    raise ValueError(f"dtype must be complex64 or complex128, got {dtype!r}")


def check(n, p, dtype="complex128", direction=FORWARD) -> int:
    """Host-only validation (fftu_check); returns the status code."""
    lib = load_library()
    return int(lib.fftu_check(len(n), _arr(n), _arr(p), _dtype_code(dtype), int(direction)))


def describe(n, p, dtype="complex128", direction=FORWARD) -> dict:
    """Host-only planner dry run (fftu_describe)."""
    lib = load_library()
    info = PlanInfo()
    st = lib.fftu_describe(len(n), _arr(n), _arr(p), _dtype_code(dtype), int(direction), ctypes.byref(info))
    if st != 0:
        raise FftuError(st, "fftu_describe")
    return info.as_dict()


def set_tuning(name: str, value: int) -> None:
    """Set a planner knob (see fftu_tune_param in include/fftu.h); -1 restores the default."""
    st = load_library().fftu_set_tuning(TUNE[name], int(value))
    if st != 0:
        raise FftuError(st, f"fftu_set_tuning({name}={value})")


def get_tuning(name: str) -> int:
    return int(load_library().fftu_get_tuning(TUNE[name]))


def fill_uniform(out, key0: int, key1: int, counter_base: int = 0, stream=None):
    """Fill the contiguous complex device tensor `out` with Philox4x32-10 values in
    [-1, 1) (fftu_fill_uniform): element e from counter counter_base + e under the
    key (key0, key1). Asynchronous on `stream` (default: the current stream)."""
    import torch
    if not isinstance(out, torch.Tensor) or not out.is_cuda or not out.is_contiguous():
        raise TypeError("out must be a contiguous device tensor")
    if out.dtype == torch.complex64:
        code = C64
    elif out.dtype == torch.complex128:
        code = C128
    else:
        raise TypeError("out must be complex64 or complex128")
    if stream is None:
        stream = torch.cuda.current_stream(out.device)
    st = load_library().fftu_fill_uniform(ctypes.c_void_p(out.data_ptr()), out.numel(), code,
                                          int(key0) & 0xFFFFFFFF, int(key1) & 0xFFFFFFFF, int(counter_base),
                                          ctypes.c_void_p(int(stream.cuda_stream)))
    if st != 0:
        raise FftuError(st, "fftu_fill_uniform")
    return out


class Plan:
    """A plan for the cyclic-to-cyclic d-D FFT (Algorithm 2.3) of an n-array on a p-grid.

    Buffers are torch tensors on the plan's device holding N complex elements
    in the cyclic buffer layout (processor-major; see include/fftu.h).
    """

    def __init__(self, n, p, dtype="complex128", direction=FORWARD, external=False):
        """external=True: fftu_plan_external (no device memory of its own; run it
        with a workspace, see execute_ws)."""
        self.n = tuple(int(v) for v in n)
        self.p = tuple(int(v) for v in p)
        if len(self.n) != len(self.p):
            raise ValueError("n and p must have the same length")
        self.dtype_code = _dtype_code(dtype)
        self.direction = int(direction)
        self.external = bool(external)
        self._lib = load_library()
        make = self._lib.fftu_plan_external if self.external else self._lib.fftu_plan
        h = make(len(self.n), _arr(self.n), _arr(self.p), self.dtype_code, self.direction)
        if not h:
            raise FftuError(self._lib.fftu_last_error(), "fftu_plan_external" if self.external else "fftu_plan")
        self._h = ctypes.c_void_p(h)
        self.N = 1
        for v in self.n:
            self.N *= v

    # -- introspection
    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        info = PlanInfo()
        st = self._lib.fftu_get_plan_info(self._h, ctypes.byref(info))
        if st != 0:
            raise FftuError(st, "fftu_get_plan_info")
        return info.as_dict()

    def launch_names(self):
        """Profiler names of the kernels one execution launches, in order."""
        n = self.info()["launches"]
        return [self._lib.fftu_launch_name(self._h, i).decode() for i in range(n)]

    def device_bytes(self) -> int:
        return int(self._lib.fftu_plan_device_bytes(self._h))

    @property
    def torch_dtype(self):
        import torch
        return torch.complex128 if self.dtype_code == C128 else torch.complex64

    # -- execution on raw pointers (device addresses, hipStream_t)
    def execute_ptr(self, in_ptr: int, out_ptr: int, stream: int = 0, entry: str = "fftu_execute") -> None:
        fn = getattr(self._lib, entry)
        st = fn(self._h, ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr), ctypes.c_void_p(stream))
        if st != 0:
            raise FftuError(st, entry)

    def execute_ws_ptr(self, in_ptr: int, out_ptr: int, ws_ptr: int, stream: int = 0) -> None:
        st = self._lib.fftu_execute_ws(self._h, ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr),
                                       ctypes.c_void_p(ws_ptr), ctypes.c_void_p(stream))
        if st != 0:
            raise FftuError(st, "fftu_execute_ws")

    @property
    def workspace_bytes(self) -> int:
        return self.N * (16 if self.dtype_code == C128 else 8)

    # -- execution on torch tensors
    def _check_tensor(self, t, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a device tensor")
        if t.dtype != self.torch_dtype or t.numel() != self.N or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.torch_dtype} tensor of {self.N} elements")

    def _run(self, entry, x, out, stream):
        import torch
        self._check_tensor(x, "input")
        if out is None:
            out = torch.empty_like(x)
        self._check_tensor(out, "output")
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        self.execute_ptr(x.data_ptr(), out.data_ptr(), int(stream.cuda_stream), entry)
        return out

    def __call__(self, x, out=None, stream=None, workspace=None):
        """out = F(x) (forward) or F^{-1}(x) (inverse), asynchronously on `stream`.
        workspace: a device tensor of at least workspace_bytes (required for an
        external plan; fftu_execute_ws)."""
        if workspace is None:
            return self._run("fftu_execute", x, out, stream)
        import torch
        self._check_tensor(x, "input")
        if out is None:
            out = torch.empty_like(x)
        self._check_tensor(out, "output")
        if not workspace.is_cuda or workspace.numel() * workspace.element_size() < self.workspace_bytes:
            raise ValueError(f"workspace must be a device tensor of at least {self.workspace_bytes} bytes")
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        self.execute_ws_ptr(x.data_ptr(), out.data_ptr(), workspace.data_ptr(), int(stream.cuda_stream))
        return out

    def execute_noalloc(self, x, out, stream=None):
        """out = F(x) with the library's fixed device workspace (fftu_execute_noalloc):
        nothing is allocated, by the library or here."""
        self._check_tensor(x, "input")
        self._check_tensor(out, "output")
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(x.device)
        self.execute_ptr(x.data_ptr(), out.data_ptr(), int(stream.cuda_stream), "fftu_execute_noalloc")
        return out

    def stage(self, name: str, x, out=None, stream=None):
        """Run one superstep: 'local_fft', 'twiddle', 'exchange' or 'remaining_fft'."""
        if name not in ("local_fft", "twiddle", "exchange", "remaining_fft"):
            raise ValueError(f"unknown stage {name!r}")
        return self._run(f"fftu_stage_{name}", x, out, stream)

    def superstep(self, phase: int, part: int, x, out=None, stream=None):
        """One step of the transform (fftu_stage_superstep): part 0 = computation
        phase `phase`'s local FFTs, 1 = superstep `phase`'s twiddle, 2 = its Put."""
        import torch
        self._check_tensor(x, "input")
        if out is None:
            out = torch.empty_like(x)
        self._check_tensor(out, "output")
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        st = self._lib.fftu_stage_superstep(self._h, int(phase), int(part), ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(int(stream.cuda_stream)))
        if st != 0:
            raise FftuError(st, "fftu_stage_superstep")
        return out

    # -- per-kernel timing with HIP events on the execution stream
    def timing_begin(self, max_calls: int) -> None:
        st = self._lib.fftu_timing_begin(self._h, int(max_calls))
        if st != 0:
            raise FftuError(st, "fftu_timing_begin")

    def timing_end(self):
        """Mean milliseconds of each launch position over the recorded calls, and the call count."""
        cap = 64
        buf = (ctypes.c_float * cap)()
        nk, nc = ctypes.c_int(0), ctypes.c_int(0)
        st = self._lib.fftu_timing_end(self._h, buf, cap, ctypes.byref(nk), ctypes.byref(nc))
        if st != 0:
            raise FftuError(st, "fftu_timing_end")
        return [float(buf[i]) for i in range(min(nk.value, cap))], nc.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fftu_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class RealPlan(Plan):
    """The transform of a real array (fftu_plan_real). Forward: a real tensor of N
    values (float64 for dtype complex128, float32 for complex64; the packed cyclic
    layout) to a complex tensor of N/2 + N/n_d elements (the half spectrum cyclic
    over p, then the Nyquist plane). Inverse: the other way, times 1/N."""

    def __init__(self, n, p, dtype="complex128", direction=FORWARD):
        self.n = tuple(int(v) for v in n)
        self.p = tuple(int(v) for v in p)
        if len(self.n) != len(self.p):
            raise ValueError("n and p must have the same length")
        self.dtype_code = _dtype_code(dtype)
        self.direction = int(direction)
        self.external = False
        self._lib = load_library()
        h = self._lib.fftu_plan_real(len(self.n), _arr(self.n), _arr(self.p), self.dtype_code, self.direction)
        if not h:
            raise FftuError(self._lib.fftu_last_error(), "fftu_plan_real")
        self._h = ctypes.c_void_p(h)
        self.N = _prod(self.n)
        self.complex_elems = self.N // 2 + self.N // self.n[-1]

    @property
    def real_dtype(self):
        import torch
        return torch.float64 if self.dtype_code == C128 else torch.float32

    def _sides(self):
        fwd = self.direction == FORWARD
        in_side = (self.real_dtype, self.N) if fwd else (self.torch_dtype, self.complex_elems)
        out_side = (self.torch_dtype, self.complex_elems) if fwd else (self.real_dtype, self.N)
        return in_side, out_side

    def _check_io(self, x, out):
        import torch
        (in_dt, in_n), (out_dt, out_n) = self._sides()
        for t, dt, n, name in ((x, in_dt, in_n, "input"), (out, out_dt, out_n, "output")):
            if t is None:
                continue
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or t.numel() != n \
                    or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {dt} device tensor of {n} elements")

    def __call__(self, x, out=None, stream=None):
        import torch
        self._check_io(x, out)
        (_, _), (out_dt, out_n) = self._sides()
        if out is None:
            out = torch.empty(out_n, dtype=out_dt, device=x.device)
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        self.execute_ptr(x.data_ptr(), out.data_ptr(), int(stream.cuda_stream), "fftu_execute")
        return out


R2R_KIND = {"dct": 0, "dst": 1}      # fftu_r2r_kind


class R2RPlan(Plan):
    """The DCT-II / DST-II (forward) or its exact inverse (fftu_plan_r2r): N reals
    (float64 for dtype complex128, float32 for complex64) on both sides. Forward:
    the signal in the zig-zag cyclic layout to the coefficients cyclic over p;
    inverse: the other way."""

    def __init__(self, n, p, kind="dct", dtype="complex128", direction=FORWARD):
        self.n = tuple(int(v) for v in n)
        self.p = tuple(int(v) for v in p)
        if len(self.n) != len(self.p):
            raise ValueError("n and p must have the same length")
        if kind not in R2R_KIND:
            raise ValueError(f"kind must be one of {sorted(R2R_KIND)}")
        self.kind = kind
        self.dtype_code = _dtype_code(dtype)
        self.direction = int(direction)
        self.external = False
        self._lib = load_library()
        h = self._lib.fftu_plan_r2r(len(self.n), _arr(self.n), _arr(self.p), self.dtype_code, R2R_KIND[kind],
                                    self.direction)
        if not h:
            raise FftuError(self._lib.fftu_last_error(), "fftu_plan_r2r")
        self._h = ctypes.c_void_p(h)
        self.N = _prod(self.n)

    @property
    def real_dtype(self):
        import torch
        return torch.float64 if self.dtype_code == C128 else torch.float32

    def _check_io(self, x, out):
        import torch
        for t, name in ((x, "input"), (out, "output")):
            if t is None:
                continue
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != self.real_dtype or \
                    t.numel() != self.N or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {self.real_dtype} device tensor of {self.N} elements")

    def __call__(self, x, out=None, stream=None):
        import torch
        self._check_io(x, out)
        if out is None:
            out = torch.empty(self.N, dtype=self.real_dtype, device=x.device)
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        self.execute_ptr(x.data_ptr(), out.data_ptr(), int(stream.cuda_stream), "fftu_execute")
        return out


class ConvolutionPlan(Plan):
    """Circular convolution in the cyclic layout (fftu_plan_convolution): as a Plan
    it is the forward transform (use it to transform a filter once);
    convolve(x, filter_hat) = F^{-1}(F(x) . filter_hat)."""

    def __init__(self, n, p, dtype="complex128"):
        self.n = tuple(int(v) for v in n)
        self.p = tuple(int(v) for v in p)
        if len(self.n) != len(self.p):
            raise ValueError("n and p must have the same length")
        self.dtype_code = _dtype_code(dtype)
        self.direction = FORWARD
        self.external = False
        self._lib = load_library()
        h = self._lib.fftu_plan_convolution(len(self.n), _arr(self.n), _arr(self.p), self.dtype_code)
        if not h:
            raise FftuError(self._lib.fftu_last_error(), "fftu_plan_convolution")
        self._h = ctypes.c_void_p(h)
        self.N = _prod(self.n)

    def convolve(self, x, filter_hat, out=None, stream=None):
        import torch
        self._check_tensor(x, "input")
        self._check_tensor(filter_hat, "filter_hat")
        if out is None:
            out = torch.empty_like(x)
        self._check_tensor(out, "output")
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        st = self._lib.fftu_execute_convolution(self._h, ctypes.c_void_p(x.data_ptr()),
                                                ctypes.c_void_p(filter_hat.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                                ctypes.c_void_p(int(stream.cuda_stream)))
        if st != 0:
            raise FftuError(st, "fftu_execute_convolution")
        return out


def pointwise_mul(a, b, out=None, scale: float = 1.0, stream=None):
    """out = a * b * scale elementwise on device (fftu_pointwise_mul); out may be a or b."""
    import torch
    if a.dtype != b.dtype or a.numel() != b.numel() or not (a.is_cuda and b.is_cuda):
        raise ValueError("a and b must be device tensors of one complex dtype and size")
    if out is None:
        out = torch.empty_like(a)
    code = C128 if a.dtype == torch.complex128 else C64 if a.dtype == torch.complex64 else None
    if code is None or out.dtype != a.dtype or out.numel() != a.numel():
        raise ValueError("complex64 or complex128 tensors of one size")
    if stream is None:
        stream = torch.cuda.current_stream(a.device)
    st = load_library().fftu_pointwise_mul(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()), a.numel(), code, float(scale),
                                           ctypes.c_void_p(int(stream.cuda_stream)))
    if st != 0:
        raise FftuError(st, "fftu_pointwise_mul")
    return out


def _ptrs(values):
    return (ctypes.c_void_p * len(values))(*[ctypes.c_void_p(int(v)) for v in values])


class BatchPlan:
    """Many independent transforms of uneven shapes in one persistent launch
    (fftu_plan_batch / fftu_execute_batch). shapes[i] and grids[i] give n and p
    of transform i; all share dtype and direction."""

    def __init__(self, shapes, grids, dtype="complex64", direction=FORWARD, external=False):
        """external=True: fftu_plan_batch_external (no device memory of its own; run
        it with execute_ws and a workspace and page-locked staging buffer)."""
        self.external = bool(external)
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.grids = [tuple(int(v) for v in g) for g in grids]
        if len(self.shapes) != len(self.grids) or not self.shapes:
            raise ValueError("shapes and grids must be non-empty lists of equal length")
        self.dtype_code = _dtype_code(dtype)
        self.direction = int(direction)
        self._lib = load_library()
        count = len(self.shapes)
        ds = (ctypes.c_int * count)(*[len(s) for s in self.shapes])
        self._keep = [_arr(s) for s in self.shapes] + [_arr(g) for g in self.grids]
        i64p = ctypes.POINTER(ctypes.c_int64)
        ns = (i64p * count)(*[ctypes.cast(a, i64p) for a in self._keep[:count]])
        ps = (i64p * count)(*[ctypes.cast(a, i64p) for a in self._keep[count:]])
        make = self._lib.fftu_plan_batch_external if self.external else self._lib.fftu_plan_batch
        h = make(count, ds, ns, ps, self.dtype_code, self.direction)
        if not h:
            raise FftuError(self._lib.fftu_last_error(),
                            "fftu_plan_batch_external" if self.external else "fftu_plan_batch")
        self._h = ctypes.c_void_p(h)
        self.sizes = [_prod(s) for s in self.shapes]

    @property
    def torch_dtype(self):
        import torch
        return torch.complex128 if self.dtype_code == C128 else torch.complex64

    def execute_ptrs(self, in_ptrs, out_ptrs, stream: int = 0) -> None:
        st = self._lib.fftu_execute_batch(self._h, _ptrs(in_ptrs), _ptrs(out_ptrs), ctypes.c_void_p(stream))
        if st != 0:
            raise FftuError(st, "fftu_execute_batch")

    def check_buffers(self, xs, outs):
        """Inputs and outputs: one contiguous device tensor of the planned size and
        dtype per transform (the library checks alignment and overlaps)."""
        for name, ts in (("inputs", xs), ("outputs", outs)):
            if len(ts) != len(self.sizes):
                raise ValueError(f"one {name[:-1]} tensor per transform")
            for t, n in zip(ts, self.sizes):
                if not t.is_cuda or t.dtype != self.torch_dtype or t.numel() != n or not t.is_contiguous():
                    raise ValueError(f"{name} must be contiguous {self.torch_dtype} device tensors "
                                     f"of the planned sizes")

    def __call__(self, xs, outs=None, stream=None):
        import torch
        if len(xs) != len(self.sizes):
            raise ValueError("one input tensor per transform")
        if outs is None:
            outs = [torch.empty_like(x) for x in xs]
        self.check_buffers(xs, outs)
        if stream is None:
            stream = torch.cuda.current_stream(xs[0].device)
        self.execute_ptrs([x.data_ptr() for x in xs], [o.data_ptr() for o in outs], int(stream.cuda_stream))
        return outs

    @property
    def workspace_bytes(self) -> int:
        """Device bytes execute_ws needs (external batches)."""
        return int(self._lib.fftu_batch_workspace_bytes(self._h))

    @property
    def staging_bytes(self) -> int:
        """Page-locked host bytes execute_ws writes (external batches)."""
        return int(self._lib.fftu_batch_staging_bytes(self._h))

    def execute_ws_ptrs(self, in_ptrs, out_ptrs, workspace_ptr: int, staging_ptr: int, stream: int = 0) -> None:
        st = self._lib.fftu_execute_batch_ws(self._h, _ptrs(in_ptrs), _ptrs(out_ptrs), ctypes.c_void_p(workspace_ptr),
                                             ctypes.c_void_p(staging_ptr), ctypes.c_void_p(stream))
        if st != 0:
            raise FftuError(st, "fftu_execute_batch_ws")

    def execute_ws(self, xs, outs, workspace, staging, stream=None):
        """outs[i] = F(xs[i]) with a device workspace tensor (>= workspace_bytes) and a
        pinned host tensor (>= staging_bytes) that stays untouched until the
        enqueued copy has run."""
        import torch
        self.check_buffers(xs, outs)
        if not workspace.is_cuda or workspace.numel() * workspace.element_size() < self.workspace_bytes:
            raise ValueError(f"workspace must be a device tensor of at least {self.workspace_bytes} bytes")
        if staging.is_cuda or not staging.is_pinned() or staging.numel() * staging.element_size() < self.staging_bytes:
            raise ValueError(f"staging must be a pinned host tensor of at least {self.staging_bytes} bytes")
        if stream is None:
            stream = torch.cuda.current_stream(xs[0].device)
        self.execute_ws_ptrs([x.data_ptr() for x in xs], [o.data_ptr() for o in outs], workspace.data_ptr(),
                             staging.data_ptr(), int(stream.cuda_stream))
        return outs

    def error_flag(self) -> int:
        v = ctypes.c_int(0)
        st = self._lib.fftu_batch_error(self._h, ctypes.byref(v))
        if st != 0:
            raise FftuError(st, "fftu_batch_error")
        return v.value

    def timing_begin(self, max_calls: int) -> None:
        st = self._lib.fftu_timing_begin(self._h, int(max_calls))
        if st != 0:
            raise FftuError(st, "fftu_timing_begin")

    def timing_end(self):
        buf = (ctypes.c_float * 8)()
        nk, nc = ctypes.c_int(0), ctypes.c_int(0)
        st = self._lib.fftu_timing_end(self._h, buf, 8, ctypes.byref(nk), ctypes.byref(nc))
        if st != 0:
            raise FftuError(st, "fftu_timing_end")
        return [float(buf[i]) for i in range(nk.value)], nc.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fftu_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _prod(vals):
    r = 1
    for v in vals:
        r *= int(v)
    return r


class Graph:
    """A captured HIP graph of one execution (fftu_graph_capture): replay with launch()."""

    def __init__(self, plan, xs, outs):
        self._lib = load_library()
        self.plan = plan                 # the plan must outlive the graph
        if isinstance(plan, BatchPlan):
            plan.check_buffers(xs, outs)
            count = len(xs)
        else:
            if hasattr(plan, "_check_io"):        # real and DCT / DST plans: their own sides
                plan._check_io(xs, outs)
            else:
                plan._check_tensor(xs, "input")
                plan._check_tensor(outs, "output")
            count = 0
            xs, outs = [xs], [outs]
        self._bufs = (xs, outs)
        h = self._lib.fftu_graph_capture(plan.handle if not isinstance(plan, BatchPlan) else plan._h, count,
                                         _ptrs([x.data_ptr() for x in xs]), _ptrs([o.data_ptr() for o in outs]))
        if not h:
            raise FftuError(self._lib.fftu_last_error(), "fftu_graph_capture")
        self._h = ctypes.c_void_p(h)

    def launch(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        st = self._lib.fftu_graph_launch(self._h, ctypes.c_void_p(int(stream.cuda_stream)))
        if st != 0:
            raise FftuError(st, "fftu_graph_launch")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fftu_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
