"""Python binding of libfarpca.so (argument marshalling only).

The names follow the C-ABI in include/farpca.h: farpca_plan, farpca_run,
farpca_free, farpca_omega, farpca_sketch, farpca_gemm_nn, farpca_gemm_tn,
farpca_gemm_bf16_nn, farpca_gemm_bf16_tn, farpca_gemm_f32s_nn, farpca_gemm_f32s_tn, farpca_eig.  Device buffers are torch tensors on the current HIP device;
every step of the method runs in the library's kernels.  ``solve`` is a
convenience wrapper that allocates the caller-owned buffers the C-ABI asks for.

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfarpca.so")

SKETCH_IDS = {"gaussian": 0, "std_bernoulli": 1, "sparse_sign": 2, "sparse_gaussian": 3,
              "bernoulli": 4}
DTYPE_IDS = {"f32": 0, "bf16": 1}
STATUS_OK = 0
STATUS_NOT_CONVERGED = 1

EXPORTED = ["farpca_plan", "farpca_run", "farpca_run_static", "farpca_begin", "farpca_step",
            "farpca_step_async", "farpca_step_poll", "farpca_loop_bytes", "farpca_begin_loop",
            "farpca_grow", "farpca_final_bytes", "farpca_finish_final", "farpca_finish", "farpca_free", "farpca_status_str", "farpca_omega",
            "farpca_sketch", "farpca_gemm_scratch_bytes", "farpca_gemm_nn", "farpca_gemm_tn",
            "farpca_gemm_bf16_scratch_bytes", "farpca_gemm_bf16_nn", "farpca_gemm_bf16_tn",
            "farpca_gemm_f32s_nn", "farpca_gemm_f32s_tn",
            "farpca_eig_scratch_bytes", "farpca_eig", "farpca_profile_enable", "farpca_profile_get",
            "farpca_request_footprint", "farpca_server_create", "farpca_server_submit",
            "farpca_server_poll", "farpca_server_release", "farpca_server_fetch",
            "farpca_server_stats", "farpca_server_memory", "farpca_server_destroy"]
PROF_CLASSES = {"sketch": 0, "gemm_tn": 1, "gemm_nn": 2, "eig": 3, "gemm_c": 4}


class FarpcaParams(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
                ("a_dtype", ctypes.c_int32), ("sketch", ctypes.c_int32), ("tol", ctypes.c_double),
                ("rank", ctypes.c_int64), ("block", ctypes.c_int32), ("power", ctypes.c_int32),
                ("max_blocks", ctypes.c_int64), ("sketch_p", ctypes.c_double),
                ("sketch_zeta", ctypes.c_int32), ("a_layout", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class FarpcaInfo(ctypes.Structure):
    _fields_ = [("rank_l", ctypes.c_int64), ("rank_out", ctypes.c_int64),
                ("blocks", ctypes.c_int32), ("status", ctypes.c_int32),
                ("norm_a2", ctypes.c_double), ("err_indicator", ctypes.c_double),
                ("eig_sweeps", ctypes.c_int32), ("dropped", ctypes.c_int32),
                ("rank_trunc", ctypes.c_int64), ("eig_converged", ctypes.c_int32),
                ("reserved1", ctypes.c_int32)]


class FarpcaResult(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("info", FarpcaInfo), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("dU", ctypes.c_void_p), ("dS", ctypes.c_void_p),
                ("dV", ctypes.c_void_p), ("ld", ctypes.c_int64), ("m", ctypes.c_int64),
                ("n", ctypes.c_int64)]


class FarpcaError(RuntimeError):
    pass


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libfarpca.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FarpcaError(f"{path} not found: build it with `python -c 'import __graft_entry__ as g; "
                          "g.build()'` (hipcc, gfx950)")
    # torch brings its own HIP runtime (same soname, found by name only once it is
    # loaded): load it first so that this library binds to it instead of loading
    # a second runtime, whose streams and pointers torch's would not know.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
    lib.farpca_plan.argtypes = [ctypes.POINTER(FarpcaParams), ctypes.POINTER(vp),
                                ctypes.POINTER(i64), ctypes.POINTER(sz)]
    lib.farpca_plan.restype = ctypes.c_int
    lib.farpca_run.argtypes = [vp, vp, vp, sz, vp, vp, vp, ctypes.POINTER(FarpcaInfo), vp, vp]
    lib.farpca_run.restype = ctypes.c_int
    lib.farpca_run_static.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(FarpcaInfo), vp, vp]
    lib.farpca_run_static.restype = ctypes.c_int
    lib.farpca_begin.argtypes = [vp, vp, vp, sz, vp, vp]
    lib.farpca_begin.restype = ctypes.c_int
    lib.farpca_step.argtypes = [vp, vp]
    lib.farpca_step.restype = ctypes.c_int
    lib.farpca_step_async.argtypes = [vp, vp]
    lib.farpca_step_async.restype = ctypes.c_int
    lib.farpca_step_poll.argtypes = [vp, ctypes.c_int]
    lib.farpca_step_poll.restype = ctypes.c_int
    lib.farpca_loop_bytes.argtypes = [vp, i64]
    lib.farpca_loop_bytes.restype = sz
    lib.farpca_begin_loop.argtypes = [vp, vp, vp, sz, i64, vp, vp]
    lib.farpca_begin_loop.restype = ctypes.c_int
    lib.farpca_grow.argtypes = [vp, vp, sz, i64, vp]
    lib.farpca_grow.restype = ctypes.c_int
    lib.farpca_final_bytes.argtypes = [vp]
    lib.farpca_final_bytes.restype = sz
    lib.farpca_finish_final.argtypes = [vp, vp, sz, vp, i64, vp, vp, i64, ctypes.POINTER(FarpcaInfo), vp]
    lib.farpca_finish_final.restype = ctypes.c_int
    lib.farpca_finish.argtypes = [vp, vp, vp, vp, ctypes.POINTER(FarpcaInfo), vp]
    lib.farpca_finish.restype = ctypes.c_int
    lib.farpca_free.argtypes = [vp]
    lib.farpca_free.restype = None
    lib.farpca_status_str.argtypes = [ctypes.c_int]
    lib.farpca_status_str.restype = ctypes.c_char_p
    lib.farpca_omega.argtypes = [vp, i64, vp, sz, vp, vp, vp, vp]
    lib.farpca_omega.restype = ctypes.c_int
    lib.farpca_sketch.argtypes = [vp, vp, i64, vp, sz, vp, vp]
    lib.farpca_sketch.restype = ctypes.c_int
    lib.farpca_gemm_scratch_bytes.argtypes = [i64]
    lib.farpca_gemm_scratch_bytes.restype = sz
    lib.farpca_gemm_bf16_scratch_bytes.argtypes = [i64, i64]
    lib.farpca_gemm_bf16_scratch_bytes.restype = sz
    for name in ("farpca_gemm_nn", "farpca_gemm_tn", "farpca_gemm_bf16_nn", "farpca_gemm_bf16_tn",
                 "farpca_gemm_f32s_nn", "farpca_gemm_f32s_tn"):
        f = getattr(lib, name)
        f.argtypes = [vp, i64, vp, i64, vp, i64, i64, i64, i64, vp, vp]
        f.restype = ctypes.c_int
    lib.farpca_eig_scratch_bytes.argtypes = [i64]
    lib.farpca_eig_scratch_bytes.restype = sz
    lib.farpca_eig.argtypes = [vp, i64, vp, vp, vp, ctypes.c_double, ctypes.POINTER(ctypes.c_int), vp]
    lib.farpca_eig.restype = ctypes.c_int
    lib.farpca_profile_enable.argtypes = [ctypes.c_int]
    lib.farpca_profile_enable.restype = None
    lib.farpca_profile_get.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]
    lib.farpca_profile_get.restype = ctypes.c_int
    lib.farpca_request_footprint.argtypes = [ctypes.POINTER(FarpcaParams)]
    lib.farpca_request_footprint.restype = sz
    lib.farpca_server_create.argtypes = [sz, ctypes.c_int, ctypes.c_double, ctypes.POINTER(vp)]
    lib.farpca_server_create.restype = ctypes.c_int
    lib.farpca_server_submit.argtypes = [vp, ctypes.POINTER(FarpcaParams), vp, ctypes.c_uint64]
    lib.farpca_server_submit.restype = ctypes.c_int
    lib.farpca_server_poll.argtypes = [vp, ctypes.POINTER(FarpcaResult), ctypes.c_int, ctypes.c_int]
    lib.farpca_server_poll.restype = ctypes.c_int
    lib.farpca_server_release.argtypes = [vp, ctypes.c_uint64]
    lib.farpca_server_release.restype = ctypes.c_int
    lib.farpca_server_fetch.argtypes = [vp, ctypes.POINTER(FarpcaResult), vp, i64, vp, vp, i64, vp]
    lib.farpca_server_fetch.restype = ctypes.c_int
    lib.farpca_server_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(sz)]
    lib.farpca_server_stats.restype = ctypes.c_int
    lib.farpca_server_memory.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz),
                                         ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.farpca_server_memory.restype = ctypes.c_int
    lib.farpca_server_destroy.argtypes = [vp]
    lib.farpca_server_destroy.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None) -> ctypes.c_void_p:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check(rc: int, what: str) -> int:
    if rc < 0:
        msg = load_library().farpca_status_str(rc).decode()
        raise FarpcaError(f"{what} failed: {rc} ({msg})")
    return rc


LAYOUT_IDS = {"row": 0, "col": 1}


def make_params(m, n, lda=None, *, tol=0.0, rank=0, block=0, power=1, sketch="sparse_sign",
                p=0.0, zeta=0, seed=0, max_blocks=0, a_dtype="f32", layout="row") -> FarpcaParams:
    if lda is None:
        lda = m if layout == "col" else n
    return FarpcaParams(m=m, n=n, lda=lda, a_dtype=DTYPE_IDS[a_dtype],
                        sketch=SKETCH_IDS[sketch], tol=tol, rank=rank, block=block, power=power,
                        max_blocks=max_blocks, sketch_p=p, sketch_zeta=zeta,
                        a_layout=LAYOUT_IDS[layout], seed=seed)


@dataclass
class Plan:
    handle: ctypes.c_void_p
    l_max: int
    workspace_bytes: int
    params: FarpcaParams

    def free(self):
        if self.handle:
            load_library().farpca_free(self.handle)
            self.handle = ctypes.c_void_p()


def farpca_plan(params: FarpcaParams) -> Plan:
    lib = load_library()
    h = ctypes.c_void_p()
    lmax = ctypes.c_int64()
    ws = ctypes.c_size_t()
    _check(lib.farpca_plan(ctypes.byref(params), ctypes.byref(h), ctypes.byref(lmax), ctypes.byref(ws)),
           "farpca_plan")
    return Plan(h, lmax.value, ws.value, params)


def farpca_free(plan: Plan) -> None:
    plan.free()


def farpca_run(plan: Plan, A, work, U, S, V, ehist=None, stream=None):
    """Enqueue and run; returns (status, FarpcaInfo)."""
    lib = load_library()
    info = FarpcaInfo()
    rc = lib.farpca_run(plan.handle, _ptr(A), _ptr(work), work.numel() * work.element_size(),
                        _ptr(U), _ptr(S), _ptr(V), ctypes.byref(info),
                        _ptr(ehist) if ehist is not None else None, _stream(stream))
    _check(rc, "farpca_run")
    return rc, info


# workspace of farpca_run_static inside the library (FARPCA_STATIC_SCRATCH_BYTES)
STATIC_SCRATCH_BYTES = 64 << 20


def farpca_run_static(plan: Plan, A, U, S, V, ehist=None, stream=None):
    """farpca_run on the library's own static workspace (no allocation by the
    call); returns (status, FarpcaInfo)."""
    lib = load_library()
    info = FarpcaInfo()
    rc = lib.farpca_run_static(plan.handle, _ptr(A), _ptr(U), _ptr(S), _ptr(V), ctypes.byref(info),
                               _ptr(ehist) if ehist is not None else None, _stream(stream))
    _check(rc, "farpca_run_static")
    return rc, info


def farpca_begin(plan: Plan, A, work, ehist=None, stream=None) -> int:
    """Step a0 of a run driven block by block (see farpca_step / farpca_finish)."""
    lib = load_library()
    return _check(lib.farpca_begin(plan.handle, _ptr(A), _ptr(work), work.numel() * work.element_size(),
                                   _ptr(ehist) if ehist is not None else None, _stream(stream)),
                  "farpca_begin")


def farpca_step(plan: Plan, stream=None) -> int:
    """One block and the stop test: 1 if another block is needed, else 0."""
    return _check(load_library().farpca_step(plan.handle, _stream(stream)), "farpca_step")


def farpca_step_async(plan: Plan, stream=None) -> int:
    """Enqueue the next block (1), or 0 if the run needs none."""
    return _check(load_library().farpca_step_async(plan.handle, _stream(stream)), "farpca_step_async")


def farpca_step_poll(plan: Plan, wait: bool = False) -> int:
    """2 while the pending block runs (wait=False), else 1 (another block) or 0 (stop)."""
    return _check(load_library().farpca_step_poll(plan.handle, 1 if wait else 0), "farpca_step_poll")


def farpca_loop_bytes(plan: Plan, cap_blocks: int) -> int:
    return int(load_library().farpca_loop_bytes(plan.handle, cap_blocks))


def farpca_begin_loop(plan: Plan, A, loop, cap_blocks: int, ehist=None, stream=None) -> int:
    """farpca_begin on a loop part with room for cap_blocks blocks."""
    return _check(load_library().farpca_begin_loop(plan.handle, _ptr(A), _ptr(loop),
                                                   loop.numel() * loop.element_size(), cap_blocks,
                                                   _ptr(ehist) if ehist is not None else None,
                                                   _stream(stream)), "farpca_begin_loop")


def farpca_grow(plan: Plan, loop, cap_blocks: int, stream=None) -> int:
    """Move a run (between blocks) to a larger loop part."""
    return _check(load_library().farpca_grow(plan.handle, _ptr(loop), loop.numel() * loop.element_size(),
                                             cap_blocks, _stream(stream)), "farpca_grow")


def farpca_final_bytes(plan: Plan) -> int:
    return int(load_library().farpca_final_bytes(plan.handle))


def farpca_finish_final(plan: Plan, final, U, S, V, stream=None):
    """farpca_finish with a separate final part; U, V row-major with any leading dimension
    >= rank_out; returns (status, FarpcaInfo)."""
    lib = load_library()
    info = FarpcaInfo()
    rc = lib.farpca_finish_final(plan.handle, _ptr(final), final.numel() * final.element_size(),
                                 _ptr(U), U.stride(0), _ptr(S), _ptr(V), V.stride(0),
                                 ctypes.byref(info), _stream(stream))
    _check(rc, "farpca_finish_final")
    return rc, info


def farpca_finish(plan: Plan, U, S, V, stream=None):
    """Final decomposition of a run begun with farpca_begin; returns (status, FarpcaInfo)."""
    lib = load_library()
    info = FarpcaInfo()
    rc = lib.farpca_finish(plan.handle, _ptr(U), _ptr(S), _ptr(V), ctypes.byref(info), _stream(stream))
    _check(rc, "farpca_finish")
    return rc, info


def farpca_omega(plan: Plan, block_j: int, work, mask, neg, dense, stream=None) -> int:
    lib = load_library()
    return _check(lib.farpca_omega(plan.handle, block_j, _ptr(work), work.numel(), _ptr(mask), _ptr(neg),
                                   _ptr(dense), _stream(stream)), "farpca_omega")


def farpca_sketch(plan: Plan, A, block_j: int, work, S, stream=None) -> int:
    lib = load_library()
    return _check(lib.farpca_sketch(plan.handle, _ptr(A), block_j, _ptr(work), work.numel(), _ptr(S),
                                    _stream(stream)), "farpca_sketch")


def farpca_gemm_scratch_bytes(M: int) -> int:
    return int(load_library().farpca_gemm_scratch_bytes(M))


def farpca_gemm_nn(A, X, C, M, N, K, part, lda=None, ldx=None, ldc=None, stream=None) -> int:
    lib = load_library()
    return _check(lib.farpca_gemm_nn(_ptr(A), lda or A.stride(0), _ptr(X), ldx or X.stride(0), _ptr(C),
                                     ldc or C.stride(0), M, N, K, _ptr(part), _stream(stream)),
                  "farpca_gemm_nn")


def farpca_gemm_tn(A, Y, C, M, N, K, part, lda=None, ldy=None, ldc=None, stream=None) -> int:
    lib = load_library()
    return _check(lib.farpca_gemm_tn(_ptr(A), lda or A.stride(0), _ptr(Y), ldy or Y.stride(0), _ptr(C),
                                     ldc or C.stride(0), M, N, K, _ptr(part), _stream(stream)),
                  "farpca_gemm_tn")


def farpca_gemm_bf16_scratch_bytes(M: int, K: int) -> int:
    return int(load_library().farpca_gemm_bf16_scratch_bytes(M, K))


def farpca_gemm_bf16_nn(A, X, C, M, N, K, scratch, lda=None, ldx=None, ldc=None,
                        stream=None) -> int:
    """A: BF16 (torch.bfloat16 or int16/uint16 bit patterns), X, C: FP32."""
    lib = load_library()
    return _check(lib.farpca_gemm_bf16_nn(_ptr(A), lda or A.stride(0), _ptr(X), ldx or X.stride(0),
                                          _ptr(C), ldc or C.stride(0), M, N, K, _ptr(scratch),
                                          _stream(stream)), "farpca_gemm_bf16_nn")


def farpca_gemm_bf16_tn(A, Y, C, M, N, K, scratch, lda=None, ldy=None, ldc=None,
                        stream=None) -> int:
    lib = load_library()
    return _check(lib.farpca_gemm_bf16_tn(_ptr(A), lda or A.stride(0), _ptr(Y), ldy or Y.stride(0),
                                          _ptr(C), ldc or C.stride(0), M, N, K, _ptr(scratch),
                                          _stream(stream)), "farpca_gemm_bf16_tn")


def farpca_gemm_f32s_nn(A, X, C, M, N, K, scratch, lda=None, ldx=None, ldc=None,
                        stream=None) -> int:
    """A, X, C: FP32; scratch: farpca_gemm_bf16_scratch_bytes(M, K) bytes."""
    lib = load_library()
    return _check(lib.farpca_gemm_f32s_nn(_ptr(A), lda or A.stride(0), _ptr(X), ldx or X.stride(0),
                                          _ptr(C), ldc or C.stride(0), M, N, K, _ptr(scratch),
                                          _stream(stream)), "farpca_gemm_f32s_nn")


def farpca_gemm_f32s_tn(A, Y, C, M, N, K, scratch, lda=None, ldy=None, ldc=None,
                        stream=None) -> int:
    lib = load_library()
    return _check(lib.farpca_gemm_f32s_tn(_ptr(A), lda or A.stride(0), _ptr(Y), ldy or Y.stride(0),
                                          _ptr(C), ldc or C.stride(0), M, N, K, _ptr(scratch),
                                          _stream(stream)), "farpca_gemm_f32s_tn")


def farpca_eig_scratch_bytes(l: int) -> int:
    return int(load_library().farpca_eig_scratch_bytes(l))


def farpca_eig(K, W, V, work, rel=0.0, stream=None):
    """(sweeps, converged) of the FP64 block-Jacobi eigensolver on K (relative
    off-diagonal test rel; 0 selects 1e-14)."""
    lib = load_library()
    conv = ctypes.c_int()
    sweeps = _check(lib.farpca_eig(_ptr(K), K.shape[0], _ptr(W), _ptr(V), _ptr(work), rel,
                                   ctypes.byref(conv), _stream(stream)), "farpca_eig")
    return sweeps, bool(conv.value)


def farpca_profile_enable(on: bool) -> None:
    load_library().farpca_profile_enable(1 if on else 0)


def farpca_profile_get(cls: str):
    """(total_ms, launches) of a kernel class since profiling was enabled."""
    t = ctypes.c_double()
    c = ctypes.c_int64()
    _check(load_library().farpca_profile_get(PROF_CLASSES[cls], ctypes.byref(t), ctypes.byref(c)),
           "farpca_profile_get")
    return t.value, c.value


@dataclass
class SolveResult:
    U: object
    S: object
    V: object
    info: FarpcaInfo
    status: int
    e_history: object


def alloc_outputs(plan: Plan, device="cuda"):
    import torch
    p = plan.params
    work = torch.empty(plan.workspace_bytes + 256, dtype=torch.uint8, device=device)
    off = (-work.data_ptr()) % 256
    work = work[off:off + plan.workspace_bytes]
    U = torch.empty((p.m, plan.l_max), dtype=torch.float32, device=device)
    S = torch.empty((plan.l_max,), dtype=torch.float64, device=device)
    V = torch.empty((p.n, plan.l_max), dtype=torch.float32, device=device)
    b = p.block or min(max(20, min(p.m, p.n) // 100), 50)
    eh = torch.zeros((plan.l_max // max(1, b) + 1,), dtype=torch.float64, device=device)
    return work, U, S, V, eh


def solve(A, *, tol=0.0, rank=0, block=0, power=1, sketch="sparse_sign", p=0.0, zeta=0, seed=0,
          max_blocks=0, stream=None) -> SolveResult:
    """Run the whole method on a CUDA tensor A (m x n): row-major float32, or
    bfloat16 for the precision form; or column-major float32 (a transposed
    view such as B.t() of a contiguous B), which the sparse sketch reads by
    columns."""
    import torch
    if A.dtype not in (torch.float32, torch.bfloat16) or not A.is_cuda or A.dim() != 2:
        raise FarpcaError("A must be a 2-D float32 or bfloat16 tensor on the GPU")
    m, n = A.shape
    dt = "bf16" if A.dtype == torch.bfloat16 else "f32"
    if A.stride(1) == 1:
        layout, lda = "row", A.stride(0)
    elif A.stride(0) == 1 and dt == "f32":
        layout, lda = "col", A.stride(1)
    else:
        raise FarpcaError("A must be row-major (float32/bfloat16) or column-major (float32)")
    prm = make_params(m, n, lda, tol=tol, rank=rank, block=block, power=power, sketch=sketch,
                      p=p, zeta=zeta, seed=seed, max_blocks=max_blocks, a_dtype=dt, layout=layout)
    plan = farpca_plan(prm)
    try:
        work, U, S, V, eh = alloc_outputs(plan, A.device)
        status, info = farpca_run(plan, A, work, U, S, V, eh, stream)
        k = info.rank_out
        nb = info.blocks
        return SolveResult(U[:, :k], S[:k], V[:, :k], info, status, eh[:nb])
    finally:
        plan.free()


# ---------------------------------------------------------------- serving
def farpca_request_footprint(params: FarpcaParams) -> int:
    return int(load_library().farpca_request_footprint(ctypes.byref(params)))


class Server:
    """farpca_server_* (continuous batching on one GPU): submit requests whose A
    is resident, poll finished results, fetch them into caller tensors, release."""

    def __init__(self, pool_bytes: int, slots: int = 4, starve_s: float = 0.25):
        self._lib = load_library()
        self.handle = ctypes.c_void_p()
        _check(self._lib.farpca_server_create(pool_bytes, slots, starve_s, ctypes.byref(self.handle)),
               "farpca_server_create")
        self._pending = {}      # tag -> (params, A) kept alive until the result is polled

    def submit(self, params: FarpcaParams, A, tag: int) -> None:
        _check(self._lib.farpca_server_submit(self.handle, ctypes.byref(params), _ptr(A), tag),
               "farpca_server_submit")
        self._pending[tag] = (params, A)

    def poll(self, max_out: int = 64, wait_ms: int = 0):
        buf = (FarpcaResult * max_out)()
        k = _check(self._lib.farpca_server_poll(self.handle, buf, max_out, wait_ms), "farpca_server_poll")
        out = [buf[i] for i in range(k)]
        for r in out:
            self._pending.pop(r.tag, None)
        return out

    def fetch(self, res: FarpcaResult, U=None, S=None, V=None, stream=None) -> None:
        _check(self._lib.farpca_server_fetch(self.handle, ctypes.byref(res),
                                             _ptr(U) if U is not None else None,
                                             U.stride(0) if U is not None else 0,
                                             _ptr(S) if S is not None else None,
                                             _ptr(V) if V is not None else None,
                                             V.stride(0) if V is not None else 0, _stream(stream)),
               "farpca_server_fetch")

    def release(self, tag: int) -> None:
        _check(self._lib.farpca_server_release(self.handle, tag), "farpca_server_release")

    def stats(self):
        q, r, f = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        _check(self._lib.farpca_server_stats(self.handle, ctypes.byref(q), ctypes.byref(r), ctypes.byref(f)),
               "farpca_server_stats")
        return q.value, r.value, f.value

    def memory(self):
        """(bytes granted now, most granted so far, loop parts grown, solves put back)."""
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        g, p = ctypes.c_int64(), ctypes.c_int64()
        _check(self._lib.farpca_server_memory(self.handle, ctypes.byref(a), ctypes.byref(b),
                                              ctypes.byref(g), ctypes.byref(p)), "farpca_server_memory")
        return a.value, b.value, g.value, p.value

    def close(self) -> None:
        if self.handle:
            self._lib.farpca_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()
            self._pending.clear()
