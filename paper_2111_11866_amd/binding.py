"""ctypes binding of libsubsurf4d.so (argument marshalling only).

Every numerical step runs in the HIP library; this module only passes device
pointers of torch tensors, the current HIP stream and parameter structs, and
turns negative status codes into exceptions.  If the library has not been
built, importing works but every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libsubsurf4d.so")

OK, NOT_CONVERGED = 0, 1
EINVAL, ESHAPE, EWORKSPACE, ENONFINITE, EDEVICE = -1, -2, -3, -4, -5
U8, F32, F64 = 0, 1, 2
FP64, MIXED = 0, 1

CENTRE_DTYPE = np.dtype([("x", "<f4"), ("y", "<f4"), ("z", "<f4"), ("frame", "<i4")])

EXPORTED = (
    "subsurf4d_workspace_bytes", "subsurf4d_prepare_g", "subsurf4d_init_u", "subsurf4d_rescale",
    "subsurf4d_assemble", "subsurf4d_step", "subsurf4d_solve", "subsurf4d_status_string",
    "subsurf4d_last_error", "subsurf4d_version", "subsurf4d_timing", "subsurf4d_copy_probe",
    "subsurf4d_batch_workspace_bytes", "subsurf4d_batch_table_bytes", "subsurf4d_step_batched",
    "subsurf4d_prepare_workspace_bytes", "subsurf4d_prepare_batched", "subsurf4d_step_dirichlet",
    "subsurf4d_step_noalloc", "subsurf4d_stream_probe", "subsurf4d_track_workspace_bytes", "subsurf4d_track",
    "subsurf4d_track_join",
)

NOALLOC_SCRATCH_BYTES = 128 << 20     # SUBSURF4D_NOALLOC_SCRATCH_BYTES


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 4), ("h", ctypes.c_double)]


class PrepareParamsC(ctypes.Structure):
    _fields_ = [("K", ctypes.c_double), ("delta", ctypes.c_double), ("vartheta", ctypes.c_double),
                ("lam", ctypes.c_double), ("ball_r", ctypes.c_double), ("smooth_tau", ctypes.c_double),
                ("smooth_steps", ctypes.c_int32), ("smooth_max_iter", ctypes.c_int32),
                ("smooth_omega", ctypes.c_double), ("smooth_tol", ctypes.c_double),
                ("image_scale", ctypes.c_double)]


class StepParamsC(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("tau", ctypes.c_double), ("omega", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("rescale", ctypes.c_int32), ("precision", ctypes.c_int32), ("ball_r", ctypes.c_double),
                ("refine_tol", ctypes.c_double), ("inner_sweeps", ctypes.c_int32),
                ("fixed_iters", ctypes.c_int32), ("iter_hint", ctypes.c_int32), ("flags", ctypes.c_int32)]


FLAG_NO_GRAPH = 1
FLAG_SWEEP_FLAT = 2
FLAG_SWEEP_MARCH = 4
FLAG_ASYNC = 8
FLAG_SHORT_LAST_PASS = 16


class BatchJobC(ctypes.Structure):
    _fields_ = [("grid", Grid), ("G", ctypes.c_void_p), ("u", ctypes.c_void_p), ("owner", ctypes.c_void_p),
                ("centres", ctypes.c_void_p), ("n_centres", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


class BatchPrepareJobC(ctypes.Structure):
    _fields_ = [("grid", Grid), ("image", ctypes.c_void_p), ("image_dtype", ctypes.c_int32),
                ("n_centres", ctypes.c_int32), ("centres", ctypes.c_void_p), ("n_seeds", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("seeds", ctypes.c_void_p), ("G", ctypes.c_void_p),
                ("owner", ctypes.c_void_p), ("u", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


class CellC(ctypes.Structure):
    _fields_ = [("name", ctypes.c_int32), ("frame", ctypes.c_int32), ("centre", ctypes.c_int32),
                ("dist2", ctypes.c_int32), ("prev", ctypes.c_int32), ("kind", ctypes.c_int32)]


CELL_DTYPE = np.dtype([("name", "<i4"), ("frame", "<i4"), ("centre", "<i4"), ("dist2", "<i4"), ("prev", "<i4"),
                       ("kind", "<i4")])


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("outer_iterations", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("bnorm", ctypes.c_double)]

    def as_dict(self):
        return dict(status=self.status, iterations=self.iterations, outer=self.outer_iterations,
                    rel_res=self.rel_residual, bnorm=self.bnorm)


@dataclass(frozen=True)
class PrepareParams:
    K: float = 1000.0
    delta: float = 0.5
    vartheta: float = 0.5
    lam: float = 0.5
    ball_r: float = 8.0
    smooth_tau: float = 0.1
    smooth_steps: int = 1
    smooth_max_iter: int = 10000
    smooth_omega: float = 0.0          # <= 0: optimal omega for the heat system
    smooth_tol: float = 1e-13
    image_scale: float = 1.0

    def c(self) -> PrepareParamsC:
        return PrepareParamsC(self.K, self.delta, self.vartheta, self.lam, self.ball_r, self.smooth_tau,
                              self.smooth_steps, self.smooth_max_iter, self.smooth_omega, self.smooth_tol,
                              self.image_scale)


@dataclass(frozen=True)
class StepParams:
    eps: float = 1e-3
    tau: float = 0.5
    omega: float = 1.5
    tol: float = 1e-8
    max_iter: int = 10000
    check_every: int = 1
    rescale: bool = True
    precision: int = FP64
    ball_r: float = 8.0
    refine_tol: float = 1e-10
    inner_sweeps: int = 8
    fixed_iters: int = 0
    iter_hint: int = 0
    flags: int = 0

    def c(self) -> StepParamsC:
        return StepParamsC(self.eps, self.tau, self.omega, self.tol, self.max_iter, self.check_every,
                           int(bool(self.rescale)), self.precision, self.ball_r, self.refine_tol,
                           self.inner_sweeps, self.fixed_iters, self.iter_hint, self.flags)


class Subsurf4dError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"subsurf4d status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        P, I, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
        L.subsurf4d_workspace_bytes.argtypes = [ctypes.POINTER(Grid), I, I]
        L.subsurf4d_workspace_bytes.restype = SZ
        L.subsurf4d_prepare_g.argtypes = [ctypes.POINTER(Grid), P, I, P, I, ctypes.POINTER(PrepareParamsC),
                                          P, P, P, SZ, P]
        L.subsurf4d_init_u.argtypes = [ctypes.POINTER(Grid), P, I, D, D, P, P]
        L.subsurf4d_rescale.argtypes = [ctypes.POINTER(Grid), P, I, D, P, P, P, SZ, P]
        L.subsurf4d_assemble.argtypes = [ctypes.POINTER(Grid), P, P, ctypes.POINTER(StepParamsC), P, P, P]
        L.subsurf4d_step.argtypes = [ctypes.POINTER(Grid), P, P, I, P, P, ctypes.POINTER(StepParamsC),
                                     ctypes.POINTER(Result), P, SZ, P]
        L.subsurf4d_step_dirichlet.argtypes = [ctypes.POINTER(Grid), P, P, P, I, P, P,
                                               ctypes.POINTER(StepParamsC), ctypes.POINTER(Result), P, SZ, P]
        L.subsurf4d_step_noalloc.argtypes = [ctypes.POINTER(Grid), P, P, I, P, P, ctypes.POINTER(StepParamsC),
                                             ctypes.POINTER(Result), P]
        L.subsurf4d_solve.argtypes = [ctypes.POINTER(Grid), P, P, P, ctypes.POINTER(StepParamsC),
                                      ctypes.POINTER(Result), P, SZ, P]
        L.subsurf4d_status_string.argtypes = [ctypes.c_int]
        L.subsurf4d_status_string.restype = ctypes.c_char_p
        L.subsurf4d_last_error.restype = ctypes.c_char_p
        L.subsurf4d_version.restype = ctypes.c_char_p
        L.subsurf4d_timing.argtypes = [I, P, P, P, P]
        L.subsurf4d_timing.restype = None
        L.subsurf4d_copy_probe.argtypes = [P, P, SZ, I, P, P]
        L.subsurf4d_stream_probe.argtypes = [P, P, SZ, I, I, I, P, P]
        L.subsurf4d_batch_workspace_bytes.argtypes = [ctypes.POINTER(Grid), I]
        L.subsurf4d_batch_workspace_bytes.restype = SZ
        L.subsurf4d_prepare_workspace_bytes.argtypes = [ctypes.POINTER(Grid), I]
        L.subsurf4d_prepare_workspace_bytes.restype = SZ
        L.subsurf4d_batch_table_bytes.argtypes = [I]
        L.subsurf4d_batch_table_bytes.restype = SZ
        L.subsurf4d_step_batched.argtypes = [ctypes.POINTER(BatchJobC), I, ctypes.POINTER(StepParamsC),
                                             ctypes.POINTER(Result), P, SZ, P]
        L.subsurf4d_prepare_batched.argtypes = [ctypes.POINTER(BatchPrepareJobC), I,
                                                ctypes.POINTER(PrepareParamsC), D, D, D,
                                                ctypes.POINTER(ctypes.c_int32), P, SZ, P]
        L.subsurf4d_track_workspace_bytes.argtypes = [ctypes.POINTER(Grid), I]
        L.subsurf4d_track_workspace_bytes.restype = SZ
        L.subsurf4d_track.argtypes = [ctypes.POINTER(Grid), P, D, P, P, ctypes.POINTER(CellC), I,
                                      ctypes.POINTER(ctypes.c_int32), P, SZ, P]
        L.subsurf4d_track_join.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(CellC), I, D]
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        raise Subsurf4dError(rc, lib().subsurf4d_last_error().decode())
    return rc


def _p(t, name="tensor", dtype=None, nbytes=0):
    """Device pointer of a torch tensor (or None), after checking that the
    library may use it: a contiguous CUDA tensor of the expected dtype (a
    torch dtype name such as "float64") holding at least `nbytes` bytes.  The
    library only sees the address, so a host tensor or a short buffer would
    make a kernel fault; here it raises ValueError instead."""
    if t is None:
        return None
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{name}: expected a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensors passed to the library must be contiguous")
    if dtype is not None and str(t.dtype) != "torch." + dtype:
        raise ValueError(f"{name}: expected torch.{dtype}, got {t.dtype}")
    if _nb(t) < nbytes:
        raise ValueError(f"{name}: {_nb(t)} bytes, the call needs {nbytes}")
    return ctypes.c_void_p(t.data_ptr())


def _nb(t):
    """Byte size of a tensor (0 for None)."""
    return 0 if t is None else t.numel() * t.element_size()


def _cells(n):
    """(interior, padded) cell counts of grid n."""
    n1, n2, n3, n4 = (int(v) for v in n)
    return n1 * n2 * n3 * n4, (n1 + 2) * (n2 + 2) * (n3 + 2) * (n4 + 2)


def _stream(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def grid(n, h=1.0) -> Grid:
    return Grid((ctypes.c_int32 * 4)(*[int(v) for v in n]), float(h))


def padded_shape(n):
    n1, n2, n3, n4 = n
    return (n4 + 2, n3 + 2, n2 + 2, n1 + 2)


def interior_shape(n):
    n1, n2, n3, n4 = n
    return (n4, n3, n2, n1)


def centres_tensor(centres, device="cuda"):
    """Structured centre array (x, y, z float32, frame int32) -> device bytes."""
    import torch

    a = np.ascontiguousarray(np.asarray(centres, dtype=CENTRE_DTYPE))
    if a.size == 0:
        return torch.zeros(16, dtype=torch.uint8, device=device), 0
    return torch.from_numpy(a.view(np.uint8).copy()).to(device), int(a.size)


def workspace_bytes(n, n_centres=0, precision=FP64) -> int:
    return int(lib().subsurf4d_workspace_bytes(ctypes.byref(grid(n)), int(n_centres), int(precision)))


def alloc_workspace(n, n_centres=0, precision=FP64, device="cuda"):
    import torch

    nb = workspace_bytes(n, n_centres, precision)
    if nb == 0:
        raise Subsurf4dError(ESHAPE, "unsupported grid")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def prepare_g(n, h, image, centres, n_centres, params: PrepareParams, G, owner, ws, stream=None):
    import torch

    dt = {torch.uint8: U8, torch.float32: F32, torch.float64: F64}[image.dtype]
    ni, npd = _cells(n)
    return _check(lib().subsurf4d_prepare_g(ctypes.byref(grid(n, h)), _p(image, "image", None,
                                                                          ni * image.element_size()), dt,
                                             _p(centres, "centres", None, 16 * int(n_centres)),
                                             int(n_centres), ctypes.byref(params.c()),
                                             _p(G, "G", "float64", 32 * npd), _p(owner, "owner", "int32", 4 * ni),
                                             _p(ws, "workspace"), _nb(ws), _stream(stream)))


def init_u(n, h, seeds, n_seeds, v, R, u, stream=None):
    ni, npd = _cells(n)
    return _check(lib().subsurf4d_init_u(ctypes.byref(grid(n, h)), _p(seeds, "seeds", None, 16 * int(n_seeds)),
                                          int(n_seeds), float(v), float(R), _p(u, "u", "float64", 8 * npd),
                                          _stream(stream)))


def rescale(n, h, centres, n_centres, ball_r, owner, u, ws, stream=None):
    ni, npd = _cells(n)
    return _check(lib().subsurf4d_rescale(ctypes.byref(grid(n, h)), _p(centres, "centres", None, 16 * int(n_centres)),
                                           int(n_centres), float(ball_r), _p(owner, "owner", "int32", 4 * ni),
                                           _p(u, "u", "float64", 8 * npd), _p(ws, "workspace"), _nb(ws),
                                           _stream(stream)))


def assemble(n, h, G, u, params: StepParams, coef, b, stream=None):
    ni, npd = _cells(n)
    return _check(lib().subsurf4d_assemble(ctypes.byref(grid(n, h)), _p(G, "G", "float64", 32 * npd),
                                            _p(u, "u", "float64", 8 * npd), ctypes.byref(params.c()),
                                            _p(coef, "coef", "float64", 64 * ni), _p(b, "b", "float64", 8 * ni),
                                            _stream(stream)))


def _step_ptrs(n, G, centres, n_centres, owner, u):
    ni, npd = _cells(n)
    return (_p(G, "G", "float64", 32 * npd), _p(centres, "centres", None, 16 * int(n_centres)),
            _p(owner, "owner", "int32", 4 * ni), _p(u, "u", "float64", 8 * npd))


def step(n, h, G, centres, n_centres, owner, u, params: StepParams, ws, stream=None) -> dict:
    res = Result()
    pG, pc, po, pu = _step_ptrs(n, G, centres, n_centres, owner, u)
    _check(lib().subsurf4d_step(ctypes.byref(grid(n, h)), pG, pc, int(n_centres), po, pu,
                                ctypes.byref(params.c()), ctypes.byref(res), _p(ws, "workspace"), _nb(ws),
                                _stream(stream)))
    return res.as_dict()


def step_noalloc(n, h, G, centres, n_centres, owner, u, params: StepParams, stream=None) -> dict:
    """subsurf4d_step on the library's fixed device scratch (no workspace
    argument; no device memory is allocated by the call)."""
    res = Result()
    pG, pc, po, pu = _step_ptrs(n, G, centres, n_centres, owner, u)
    _check(lib().subsurf4d_step_noalloc(ctypes.byref(grid(n, h)), pG, pc, int(n_centres), po, pu,
                                        ctypes.byref(params.c()), ctypes.byref(res), _stream(stream)))
    return res.as_dict()


def step_dirichlet(n, h, G, ub, centres, n_centres, owner, u, params: StepParams, ws, stream=None) -> dict:
    """One step whose new level takes its Dirichlet data from ub's ghost layer."""
    res = Result()
    pG, pc, po, pu = _step_ptrs(n, G, centres, n_centres, owner, u)
    pub = _p(ub, "u_dirichlet", "float64", 8 * _cells(n)[1])
    _check(lib().subsurf4d_step_dirichlet(ctypes.byref(grid(n, h)), pG, pub, pc, int(n_centres), po, pu,
                                          ctypes.byref(params.c()), ctypes.byref(res), _p(ws, "workspace"),
                                          _nb(ws), _stream(stream)))
    return res.as_dict()


def solve(n, h, coef, b, u, params: StepParams, ws, stream=None) -> dict:
    res = Result()
    ni, npd = _cells(n)
    _check(lib().subsurf4d_solve(ctypes.byref(grid(n, h)), _p(coef, "coef", "float64", 64 * ni),
                                 _p(b, "b", "float64", 8 * ni), _p(u, "u", "float64", 8 * npd),
                                 ctypes.byref(params.c()), ctypes.byref(res), _p(ws, "workspace"), _nb(ws),
                                 _stream(stream)))
    return res.as_dict()


RESULT_BYTES = ctypes.sizeof(Result)


def result_tensor(device="cuda"):
    """Device buffer for the outcome of an enqueue-only call."""
    import torch

    return torch.zeros(RESULT_BYTES, dtype=torch.uint8, device=device)


def result_dict(t) -> dict:
    """Outcome written by an enqueue-only call (copies to the host, which
    waits for the call's work)."""
    raw = bytes(t.cpu().numpy().tobytes())
    return Result.from_buffer_copy(raw).as_dict()


def step_async(n, h, G, centres, n_centres, owner, u, params: StepParams, ws, result=None, stream=None):
    """Enqueue-only subsurf4d_step (SUBSURF4D_FLAG_ASYNC): nothing is
    synchronised; `result` (device tensor of RESULT_BYTES bytes, or None)
    receives the outcome when the stream reaches it."""
    from dataclasses import replace

    sp = replace(params, flags=params.flags | FLAG_ASYNC)
    pG, pc, po, pu = _step_ptrs(n, G, centres, n_centres, owner, u)
    pres = _p(result, "result", "uint8", RESULT_BYTES)
    _check(lib().subsurf4d_step(ctypes.byref(grid(n, h)), pG, pc, int(n_centres), po, pu, ctypes.byref(sp.c()),
                                ctypes.cast(pres, ctypes.POINTER(Result)) if pres is not None else None,
                                _p(ws, "workspace"), _nb(ws), _stream(stream)))


def solve_async(n, h, coef, b, u, params: StepParams, ws, result=None, stream=None):
    """Enqueue-only subsurf4d_solve (SUBSURF4D_FLAG_ASYNC)."""
    from dataclasses import replace

    sp = replace(params, flags=params.flags | FLAG_ASYNC)
    ni, npd = _cells(n)
    pres = _p(result, "result", "uint8", RESULT_BYTES)
    _check(lib().subsurf4d_solve(ctypes.byref(grid(n, h)), _p(coef, "coef", "float64", 64 * ni),
                                 _p(b, "b", "float64", 8 * ni), _p(u, "u", "float64", 8 * npd),
                                 ctypes.byref(sp.c()),
                                 ctypes.cast(pres, ctypes.POINTER(Result)) if pres is not None else None,
                                 _p(ws, "workspace"), _nb(ws), _stream(stream)))


def stream_probe(src, dst, reads, writes=1, reps=10, stream=None) -> float:
    """Mean ms of one pass over `reads` chunks of src, each the size of dst:
    writes=1: dst = their element-wise sum; writes=0: reads only, dst[:g]
    receives per-block partial sums (g = stream_probe_blocks(dst))."""
    ms = ctypes.c_double(0.0)
    nbytes = _nb(dst)
    _check(lib().subsurf4d_stream_probe(_p(src, "src", None, reads * nbytes), _p(dst, "dst"), nbytes, int(reads),
                                        int(writes), int(reps), ctypes.byref(ms), _stream(stream)))
    return ms.value


def stream_probe_blocks(dst) -> int:
    """Blocks of a stream-probe launch over chunks of dst's size (partial sums
    written by a read-only pass)."""
    n = _nb(dst) // 16
    return min(65536, -(-n // 1024))


def timing(op: int = 3) -> dict:
    """Sweep instrumentation: op 0 disable, 1 enable, 2 reset, 3 read."""
    ms = ctypes.c_double(0.0)
    la, up, so = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    lib().subsurf4d_timing(int(op), ctypes.byref(ms), ctypes.byref(la), ctypes.byref(up), ctypes.byref(so))
    return dict(sweep_ms=ms.value, sweep_launches=la.value, voxel_updates=up.value, solves=so.value)


def copy_probe(src, dst, reps=10, stream=None) -> float:
    """Mean ms of one 16-byte-access copy of src into dst (same byte size)."""
    ms = ctypes.c_double(0.0)
    nbytes = _nb(src)
    _check(lib().subsurf4d_copy_probe(_p(src, "src"), _p(dst, "dst", None, nbytes), nbytes, int(reps),
                                      ctypes.byref(ms), _stream(stream)))
    return ms.value


def prepare_workspace_bytes(n, n_centres=0) -> int:
    return int(lib().subsurf4d_prepare_workspace_bytes(ctypes.byref(grid(n)), int(n_centres)))


def batch_workspace_bytes(n, n_centres=0, h=1.0) -> int:
    return int(lib().subsurf4d_batch_workspace_bytes(ctypes.byref(grid(n, h)), int(n_centres)))


def batch_table_bytes(n_jobs) -> int:
    return int(lib().subsurf4d_batch_table_bytes(int(n_jobs)))


def _batch_job_c(j):
    """The checked descriptor of a batched job.  It is kept on the job object
    and reused while the job's tensors keep their addresses and sizes and its
    shape is unchanged, so a step of many windows does not re-check every
    tensor of every window."""
    key = (tuple(None if t is None else (t.data_ptr(), t.numel()) for t in (j.G, j.u, j.owner, j.centres, j.bws)),
           tuple(j.n), float(j.h), int(j.nc))
    cached = getattr(j, "_ss4_batch_c", None)
    if cached is not None and cached[0] == key:
        return cached[1]
    pG, pc, po, pu = _step_ptrs(j.n, j.G, j.centres, j.nc, j.owner, j.u)
    c = BatchJobC(grid(j.n, j.h), pG, pu, po, pc, int(j.nc), 0, _p(j.bws, "batch workspace"), _nb(j.bws))
    try:
        j._ss4_batch_c = (key, c)
    except AttributeError:
        pass
    return c


def step_batched(jobs, params: StepParams, table, stream=None):
    """jobs: sequence of objects with n, h, G, u, owner, centres, nc, bws (batch workspace).
    Returns (status, list of per-job result dicts)."""
    arr = (BatchJobC * len(jobs))()
    for q, j in enumerate(jobs):
        arr[q] = _batch_job_c(j)
    res = (Result * len(jobs))()
    rc = _check(lib().subsurf4d_step_batched(arr, len(jobs), ctypes.byref(params.c()), res,
                                              _p(table, "table"), _nb(table), _stream(stream)))
    return rc, [r.as_dict() for r in res]


def prepare_batched(jobs, pp: PrepareParams, v, R, ball_r, table, stream=None):
    """Batched preparation (owner map, G, u0 rescaled) of Job objects created
    with batch=True.  Returns (status, per-job statuses)."""
    import torch

    arr = (BatchPrepareJobC * len(jobs))()
    for q, j in enumerate(jobs):
        dt = {torch.uint8: U8, torch.float32: F32, torch.float64: F64}[j.image.dtype]
        ni, _ = _cells(j.n)
        pG, pc, po, pu = _step_ptrs(j.n, j.G, j.centres, j.nc, j.owner, j.u)
        arr[q] = BatchPrepareJobC(grid(j.n, j.h), _p(j.image, "image", None, ni * j.image.element_size()), dt,
                                  int(j.nc), pc, int(j.ns), 0, _p(j.seeds, "seeds", None, 16 * int(j.ns)),
                                  pG, po, pu, _p(j.bws, "batch workspace"), _nb(j.bws))
    st = (ctypes.c_int32 * len(jobs))()
    rc = _check(lib().subsurf4d_prepare_batched(arr, len(jobs), ctypes.byref(pp.c()), float(v), float(R),
                                                 float(ball_r), st, _p(table, "table"), _nb(table),
                                                 _stream(stream)))
    return rc, list(st)


def track(n, u, level, capacity=1 << 16, join_radius=None, label=None, dist2=None, ws=None, stream=None):
    """Cells of the segmentation u (device, padded) with their centres and
    backward links (subsurf4d_track), optionally joined into trajectories
    (subsurf4d_track_join with `join_radius`).  Returns (cells as a numpy
    record array, label tensor, dist2 tensor)."""
    import torch

    ni, npd = _cells(n)
    dev = u.device
    label = torch.empty(interior_shape(n), dtype=torch.int32, device=dev) if label is None else label
    dist2 = torch.empty(interior_shape(n), dtype=torch.int32, device=dev) if dist2 is None else dist2
    if ws is None:
        nb = int(lib().subsurf4d_track_workspace_bytes(ctypes.byref(grid(n)), int(capacity)))
        if nb == 0:
            raise Subsurf4dError(ESHAPE, "unsupported grid for tracking")
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    cells = (CellC * max(int(capacity), 1))()
    k = ctypes.c_int32(0)
    _check(lib().subsurf4d_track(ctypes.byref(grid(n)), _p(u, "u", "float64", 8 * npd), float(level),
                                 _p(label, "label", "int32", 4 * ni), _p(dist2, "dist2", "int32", 4 * ni), cells,
                                 int(capacity), ctypes.byref(k), _p(ws, "workspace"), _nb(ws), _stream(stream)))
    if join_radius is not None:
        _check(lib().subsurf4d_track_join(ctypes.byref(grid(n)), cells, k.value, float(join_radius)))
    out = np.frombuffer(ctypes.string_at(ctypes.addressof(cells), k.value * ctypes.sizeof(CellC)),
                        dtype=CELL_DTYPE).copy()
    return out, label, dist2


def version() -> str:
    return lib().subsurf4d_version().decode()


class Job:
    """Device-resident state of one segmentation job (image, G, owner map, u,
    workspace), with the pipeline of the implementation overview (Sec. 3.5):
    prepare -> initial function -> rescale -> steps.  Memory comes from torch."""

    def __init__(self, n, image_np, centres, seeds, h=1.0, precision=FP64, device="cuda", batch=False,
                 shared_ws=None):
        import torch

        self.n, self.h, self.device = tuple(int(v) for v in n), float(h), device
        self.image = torch.from_numpy(np.ascontiguousarray(image_np)).to(device)
        self.centres, self.nc = centres_tensor(centres, device)
        self.seeds, self.ns = centres_tensor(seeds, device)
        self.G = torch.empty((4,) + padded_shape(self.n), dtype=torch.float64, device=device)
        self.owner = torch.empty(interior_shape(self.n), dtype=torch.int32, device=device)
        self.u = torch.empty(padded_shape(self.n), dtype=torch.float64, device=device)
        # full single-job workspace, a caller-shared one (e.g. one preparation
        # workspace reused by many batched windows), or none (shared_ws=False:
        # a batched job prepared with prepare_batched)
        if shared_ws is False:
            self.ws = None
        else:
            self.ws = shared_ws if shared_ws is not None else alloc_workspace(self.n, self.nc, precision, device)
        self.bws = None
        if batch:
            import torch

            self.bws = torch.empty(batch_workspace_bytes(self.n, self.nc, self.h), dtype=torch.uint8,
                                   device=device)
        self.last_iters = 0

    def prepare(self, pp: PrepareParams):
        return prepare_g(self.n, self.h, self.image, self.centres, self.nc, pp, self.G, self.owner, self.ws)

    def init(self, v=1.0, R=0.0, ball_r=8.0, do_rescale=True):
        init_u(self.n, self.h, self.seeds, self.ns, v, R, self.u)
        if do_rescale:
            rescale(self.n, self.h, self.centres, self.nc, ball_r, self.owner, self.u, self.ws)

    def save(self, path):
        """Checkpoint of the job's device state (u, G, owner map) to one .npz
        file; with the image, centres and seeds it is all a job needs to
        resume."""
        np.savez(path, u=self.u.cpu().numpy(), G=self.G.cpu().numpy(), owner=self.owner.cpu().numpy(),
                 n=np.asarray(self.n), h=np.asarray(self.h))

    def load(self, path):
        """Resume from a checkpoint written by save() for the same grid."""
        import torch

        with np.load(path, allow_pickle=False) as z:
            if tuple(int(v) for v in z["n"]) != self.n or float(z["h"]) != self.h:
                raise ValueError("checkpoint of another grid")
            self.u.copy_(torch.from_numpy(z["u"]))
            self.G.copy_(torch.from_numpy(z["G"]))
            self.owner.copy_(torch.from_numpy(z["owner"]))

    def step(self, sp: StepParams):
        from dataclasses import replace

        if sp.iter_hint == 0 and self.last_iters:
            sp = replace(sp, iter_hint=self.last_iters)
        r = step(self.n, self.h, self.G, self.centres, self.nc, self.owner, self.u, sp, self.ws)
        self.last_iters = r["iterations"]
        return r
