"""ctypes binding of librs.so (include/rs.h).

Argument marshalling only: every step of the RS path runs in the HIP library.
Importing this module raises if the library has not been built; there is no
CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
from typing import Optional, Sequence

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librs.so")

RS_OK, RS_E_INVALID, RS_E_NOMEM, RS_E_DEVICE, RS_E_RANK_CAP, RS_E_UNSUPPORTED = range(6)
KERNELS = {"newton": 0, "yukawa": 1, "newton+yukawa": 2}
PRECS = {"fp64": 0, "mixed_fp16": 1, "mixed_bf16": 2, "fp32": 3}
GRAMS = {"identity": 0, "gemm": 1}
RULES = {"literal": 0, "expsinc": 1}
SKETCHES = {"gram": 0, "side": 1}


class RSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_STATUS = {0: "RS_OK", 1: "RS_E_INVALID", 2: "RS_E_NOMEM", 3: "RS_E_DEVICE",
           4: "RS_E_RANK_CAP", 5: "RS_E_UNSUPPORTED"}


class rs_grid(C.Structure):
    _fields_ = [("b", C.c_double), ("n", C.c_int64)]


class rs_fdesc(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("lambda_", C.c_double), ("R", C.c_int32),
                ("R_l", C.c_int32), ("n_s", C.c_int32), ("delta_rel", C.c_double),
                ("sigma_split", C.c_double), ("C0", C.c_double), ("rule", C.c_int32),
                ("r_lo", C.c_double), ("r_hi", C.c_double)]


class rs_aopts(C.Structure):
    _fields_ = [("eps_tucker", C.c_double), ("r_max", C.c_int32),
                ("fixed_ranks", C.c_int32 * 3), ("prec", C.c_int32),
                ("oversample", C.c_int32), ("power_iters", C.c_int32),
                ("interp_order", C.c_int32), ("gram", C.c_int32), ("sketch", C.c_int32),
                ("subspace_min", C.c_int32), ("als_sweeps", C.c_int32)]


class rs_info(C.Structure):
    _fields_ = [("N", C.c_int64), ("n", C.c_int64), ("b", C.c_double), ("h", C.c_double),
                ("R", C.c_int32), ("R_l", C.c_int32), ("n_s", C.c_int32), ("prec", C.c_int32),
                ("interp_order", C.c_int32), ("ranks", C.c_int32 * 3),
                ("subspace", C.c_int32 * 3), ("sigma_first", C.c_double * 3),
                ("sigma_last_kept", C.c_double * 3), ("sigma_next", C.c_double * 3),
                ("S0", C.c_double), ("S_l0", C.c_double), ("tucker_storage", C.c_int64),
                ("device_bytes", C.c_int64), ("rank_capped", C.c_int32),
                ("stage_ms", C.c_double * 12), ("eig_phase_ms", C.c_double * 4)]


EIG_PHASES = ("eig_subspace", "eig_tridiag", "eig_values_vectors", "eig_orth_backtransform")
STAGES = ("factors", "gram", "eigen", "bins", "basis", "project", "core", "expand1",
          "expand2", "grid", "short", "core_kernel")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1606_09218_amd/build.py` "
                          "(there is no fallback implementation)")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    D = C.POINTER(C.c_double)
    sig = {
        "rs_ctx_create": ([C.c_int, C.POINTER(P)], C.c_int),
        "rs_ctx_destroy": ([P], None),
        "rs_ctx_set_timing": ([P, C.c_int], C.c_int),
        "rs_ctx_set_hbm_budget": ([P, C.c_size_t], C.c_int),
        "rs_ctx_trim": ([P], C.c_int),
        "rs_stream_release": ([P, P], C.c_int),
        "rs_build_factors": ([P, C.POINTER(rs_grid), C.POINTER(rs_fdesc), C.POINTER(P)], C.c_int),
        "rs_factors_get": ([P, D, D, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                            C.POINTER(C.c_int32)], C.c_int),
        "rs_factors_free": ([P], None),
        "rs_assemble": ([P, P, C.c_int64, P, P, C.POINTER(rs_aopts), P, C.POINTER(P), P], C.c_int),
        "rs_weighted_gram": ([P, P, C.c_int64, P, P, C.c_int32, P, P], C.c_int),
        "rs_eval_points": ([P, C.c_int64, P, P, C.c_int32, P], C.c_int),
        "rs_energy": ([P, P, P, P], C.c_int),
        "rs_forces": ([P, C.c_double, P, P], C.c_int),
        "rs_energy_forces": ([P, P, P, C.c_double, P, P], C.c_int),
        "rs_energy_forces_noalloc": ([P, P, P, C.c_double, P, P], C.c_int),
        "rs_gradient_grid": ([P, C.c_int32, P, P], C.c_int),
        "rs_tensor_grid": ([P, P, P], C.c_int),
        "rs_dot": ([P, P, P, P], C.c_int),
        "rs_rbf_matvec": ([P, P, P, P, P], C.c_int),
        "rs_eval_gradient_points": ([P, C.c_int64, P, P, P, C.c_int32, P], C.c_int),
        "rs_footprint_bytes": ([C.POINTER(rs_grid), C.POINTER(rs_fdesc), C.c_int64, C.c_int32,
                                C.c_int32, C.c_int32], C.c_size_t),
        "rs_tensor_info": ([P, C.POINTER(rs_info)], C.c_int),
        "rs_tensor_export": ([P, P, P, P, P, P], C.c_int),
        "rs_tensor_save": ([P, C.c_char_p], C.c_int),
        "rs_tensor_load": ([P, C.c_char_p, C.POINTER(P)], C.c_int),
        "rs_tensor_free": ([P], None),
        "rs_status_str": ([C.c_int], C.c_char_p),
        "rs_last_error": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()

# Handles are released explicitly (close/free) or by __del__ while the
# interpreter runs normally; once it starts to exit, __del__ makes no library
# call (the HIP runtime and the modules it would need may already be going
# away, and the process is about to release everything anyway).
_exiting = False


def _at_exit():
    global _exiting
    _exiting = True


atexit.register(_at_exit)


def _may_release() -> bool:
    return not _exiting and not sys.is_finalizing()

EXPORTED = ("rs_ctx_create", "rs_ctx_destroy", "rs_ctx_set_timing", "rs_ctx_set_hbm_budget",
            "rs_ctx_trim",
            "rs_stream_release", "rs_build_factors", "rs_factors_get",
            "rs_factors_free", "rs_assemble", "rs_weighted_gram", "rs_eval_points", "rs_energy",
            "rs_forces", "rs_energy_forces", "rs_energy_forces_noalloc", "rs_gradient_grid",
            "rs_eval_gradient_points", "rs_tensor_grid", "rs_dot", "rs_rbf_matvec",
            "rs_footprint_bytes", "rs_tensor_info", "rs_tensor_export",
            "rs_tensor_save", "rs_tensor_load", "rs_tensor_free", "rs_status_str",
            "rs_last_error")


def _check(status: int, allow_rank_cap: bool = False) -> int:
    if status == RS_OK or (allow_rank_cap and status == RS_E_RANK_CAP):
        return status
    raise RSError(status, lib.rs_last_error().decode())


# ---- marshalling helpers (torch is used for device memory and streams only) ----

def _dev_ptr(t, dtype_name: str, numel: Optional[int] = None, what: str = "tensor"):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    want = {"f64": torch.float64, "f32": torch.float32}[dtype_name]
    if t.dtype != want:
        raise TypeError(f"{what} must have dtype {want}, got {t.dtype}")
    if not t.is_cuda:
        raise TypeError(f"{what} must live in HIP device memory")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Context:
    def __init__(self, device: int = 0, hbm_budget: int = 0):
        h = C.c_void_p()
        _check(lib.rs_ctx_create(int(device), C.byref(h)))
        self.handle = h
        self.device = device
        if hbm_budget:
            self.set_hbm_budget(hbm_budget)

    def set_hbm_budget(self, nbytes: int):
        """Admission budget: later assemblies whose footprint bound exceeds
        `nbytes` are refused with RS_E_NOMEM before allocating; 0 sets no
        budget (rs_ctx_set_hbm_budget)."""
        _check(lib.rs_ctx_set_hbm_budget(self.handle, int(nbytes)))

    def set_timing(self, enable=True):
        """HIP-event timing of later assemblies: False/0 off, True/1 every
        stage, 2 the grid stage only, 3 the core kernel only (rs_ctx_set_timing)."""
        mode = int(enable) if not isinstance(enable, bool) else int(enable)
        _check(lib.rs_ctx_set_timing(self.handle, mode))

    def trim(self):
        """Return the device memory cached for reuse (rs_ctx_trim)."""
        _check(lib.rs_ctx_trim(self.handle))

    def release_stream(self, stream):
        """Synchronise a torch stream and detach cached buffers from it
        (rs_stream_release), before the caller destroys it."""
        _check(lib.rs_stream_release(self.handle, _stream_ptr(stream)))

    def close(self):
        if getattr(self, "handle", None):
            lib.rs_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        if _may_release():
            self.close()


class Factors:
    """Quadrature table and split for one grid (rs_build_factors)."""

    def __init__(self, ctx: Context, b: float, n: int, R: int, R_l: int = -1, n_s: int = -1,
                 kernel: str = "newton", lam: float = 0.5, delta_rel: float = 1e-4,
                 sigma_split: float = 0.0, C0: float = 3.0, rule: str = "literal",
                 r_lo: float = 0.0, r_hi: float = 0.0):
        self.ctx = ctx
        self.grid = rs_grid(float(b), int(n))
        self.fdesc = rs_fdesc(KERNELS[kernel], float(lam), int(R), int(R_l), int(n_s),
                              float(delta_rel), float(sigma_split), float(C0), RULES[rule],
                              float(r_lo), float(r_hi))
        h = C.c_void_p()
        _check(lib.rs_build_factors(ctx.handle, C.byref(self.grid), C.byref(self.fdesc), C.byref(h)))
        self.handle = h
        t = (C.c_double * R)()
        a = (C.c_double * R)()
        Rv, Rl, ns = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib.rs_factors_get(h, t, a, C.byref(Rv), C.byref(Rl), C.byref(ns)))
        self.t = list(t)
        self.a = list(a)
        self.R, self.R_l, self.n_s = Rv.value, Rl.value, ns.value
        self.b, self.n = float(b), int(n)

    def close(self):
        if getattr(self, "handle", None):
            lib.rs_factors_free(self.handle)
            self.handle = None

    def __del__(self):
        if _may_release():
            self.close()


def make_aopts(eps_tucker=1e-6, r_max=0, fixed_ranks: Optional[Sequence[int]] = None,
               prec="fp64", oversample=0, power_iters=-1, interp_order=0,
               gram="identity", sketch="gram", subspace_min=0, als_sweeps=0) -> rs_aopts:
    fr = (C.c_int32 * 3)(*(list(fixed_ranks) if fixed_ranks else [0, 0, 0]))
    return rs_aopts(float(eps_tucker), int(r_max), fr, PRECS[prec], int(oversample),
                    int(power_iters), int(interp_order), GRAMS[gram], SKETCHES[sketch],
                    int(subspace_min), int(als_sweeps))


class Tensor:
    """An RS-Tucker tensor handle (rs_tensor)."""

    def __init__(self, handle, ctx: Context, status: int, N: Optional[int] = None):
        self.handle = handle
        self.ctx = ctx
        self.status = status
        self._N = N

    @property
    def N(self) -> int:
        """Number of particles (known at assembly; info() waits for the
        assembly to finish when timing is on, this does not)."""
        if self._N is None:
            self._N = int(self.info().N)
        return self._N

    def info(self) -> rs_info:
        inf = rs_info()
        _check(lib.rs_tensor_info(self.handle, C.byref(inf)))
        return inf

    def stage_ms(self) -> dict:
        inf = self.info()
        out = {name: float(inf.stage_ms[i]) for i, name in enumerate(STAGES)}
        for i, name in enumerate(EIG_PHASES):
            out[name] = float(inf.eig_phase_ms[i])
        return out

    def free(self):
        if getattr(self, "handle", None):
            lib.rs_tensor_free(self.handle)
            self.handle = None

    def __del__(self):
        if _may_release():
            self.free()


def assemble(ctx: Context, f: Factors, pos, q, grid=None, opts: Optional[rs_aopts] = None,
             stream=None) -> Tensor:
    N = int(q.numel())
    p_pos = _dev_ptr(pos, "f64", 3 * N, "pos")
    p_q = _dev_ptr(q, "f64", N, "q")
    opts = opts or make_aopts()
    p_grid = None
    if grid is not None:
        want = "f64" if opts.prec == 0 else "f32"
        p_grid = _dev_ptr(grid, want, f.n ** 3, "grid")
    h = C.c_void_p()
    st = _check(lib.rs_assemble(ctx.handle, f.handle, N, p_pos, p_q, C.byref(opts), p_grid,
                                C.byref(h), _stream_ptr(stream)), allow_rank_cap=True)
    return Tensor(h, ctx, st, N)


def weighted_gram(ctx: Context, f: Factors, pos, q, G, method: str = "identity", stream=None):
    N = int(q.numel())
    _check(lib.rs_weighted_gram(ctx.handle, f.handle, N, _dev_ptr(pos, "f64", 3 * N, "pos"),
                                _dev_ptr(q, "f64", N, "q"), GRAMS[method],
                                _dev_ptr(G, "f64", 3 * f.n * f.n, "G"), _stream_ptr(stream)))


def eval_points(T: Tensor, pts, vals, part: int = 0, stream=None):
    M = int(vals.numel())
    _check(lib.rs_eval_points(T.handle, M, _dev_ptr(pts, "f64", 3 * M, "pts"),
                              _dev_ptr(vals, "f64", M, "vals"), int(part), _stream_ptr(stream)))


def energy(T: Tensor, E, dEdq=None, stream=None):
    N = T.N
    _check(lib.rs_energy(T.handle, _dev_ptr(E, "f64", 1, "E"),
                         None if dEdq is None else _dev_ptr(dEdq, "f64", N, "dEdq"),
                         _stream_ptr(stream)))


def forces(T: Tensor, F, scale: float = 1.0, stream=None):
    N = T.N
    _check(lib.rs_forces(T.handle, float(scale), _dev_ptr(F, "f64", 3 * N, "F"), _stream_ptr(stream)))


def energy_forces(T: Tensor, E, F, scale: float = 1.0, dEdq=None, stream=None):
    """Energy and forces from one evaluation pass (rs_energy_forces)."""
    N = T.N
    _check(lib.rs_energy_forces(T.handle, _dev_ptr(E, "f64", 1, "E"),
                                None if dEdq is None else _dev_ptr(dEdq, "f64", N, "dEdq"),
                                float(scale), _dev_ptr(F, "f64", 3 * N, "F"), _stream_ptr(stream)))


def energy_forces_noalloc(T: Tensor, E, F, scale: float = 1.0, dEdq=None, stream=None):
    """rs_energy_forces_noalloc: as energy_forces, with the scratch in the
    library's static device array (no device allocation)."""
    N = T.N
    _check(lib.rs_energy_forces_noalloc(T.handle, _dev_ptr(E, "f64", 1, "E"),
                                        None if dEdq is None else _dev_ptr(dEdq, "f64", N, "dEdq"),
                                        float(scale), _dev_ptr(F, "f64", 3 * N, "F"),
                                        _stream_ptr(stream)))


def eval_gradient_points(T: Tensor, pts, out, normals=None, part: int = 0, stream=None):
    """rs_eval_gradient_points: M x 3 gradients at the points, or the M
    normal derivatives when `normals` (M x 3) is given."""
    M = int(pts.numel()) // 3
    p_n = None if normals is None else _dev_ptr(normals, "f64", 3 * M, "normals")
    _check(lib.rs_eval_gradient_points(T.handle, M, _dev_ptr(pts, "f64", 3 * M, "pts"), p_n,
                                       _dev_ptr(out, "f64", M if normals is not None else 3 * M, "out"),
                                       int(part), _stream_ptr(stream)))


def rbf_matvec(ctx: Context, f: Factors, c, y, stream=None):
    """rs_rbf_matvec: y = A c with the RS form of the RBF matrix on the n^3
    grid (c, y device FP64 n^3)."""
    n3 = f.n ** 3
    _check(lib.rs_rbf_matvec(ctx.handle, f.handle, _dev_ptr(c, "f64", n3, "c"),
                             _dev_ptr(y, "f64", n3, "y"), _stream_ptr(stream)))


def dot(A: Tensor, B: Tensor, out, stream=None):
    """rs_dot: out[0] = sum_i A(i) B(i) over the common grid (device FP64)."""
    _check(lib.rs_dot(A.handle, B.handle, _dev_ptr(out, "f64", 1, "out"), _stream_ptr(stream)))


def tensor_grid(T: Tensor, grid, stream=None):
    """rs_tensor_grid: the n^3 grid of a tensor handle (FP64 grid for FP64
    tensors, FP32 otherwise)."""
    inf = T.info()
    want = "f64" if inf.prec == 0 else "f32"
    _check(lib.rs_tensor_grid(T.handle, _dev_ptr(grid, want, inf.n ** 3, "grid"), _stream_ptr(stream)))


def gradient_grid(T: Tensor, axis: int, grid, stream=None):
    """rs_gradient_grid: the finite difference of the RS tensor along `axis`
    on the whole grid (FP64 grid for FP64 tensors, FP32 otherwise)."""
    inf = T.info()
    want = "f64" if inf.prec == 0 else "f32"
    _check(lib.rs_gradient_grid(T.handle, int(axis), _dev_ptr(grid, want, inf.n ** 3, "grid"),
                                _stream_ptr(stream)))


def tensor_export(T: Tensor, V1=None, V2=None, V3=None, beta=None, stream=None):
    inf = T.info()
    n, r = inf.n, list(inf.ranks)
    args = []
    for V, rl, nm in ((V1, r[0], "V1"), (V2, r[1], "V2"), (V3, r[2], "V3")):
        args.append(None if V is None else _dev_ptr(V, "f64", n * rl, nm))
    b = None if beta is None else _dev_ptr(beta, "f64", r[0] * r[1] * r[2], "beta")
    _check(lib.rs_tensor_export(T.handle, *args, b, _stream_ptr(stream)))


def tensor_save(T: Tensor, path: str):
    _check(lib.rs_tensor_save(T.handle, path.encode()))


def tensor_load(ctx: Context, path: str) -> Tensor:
    h = C.c_void_p()
    _check(lib.rs_tensor_load(ctx.handle, path.encode(), C.byref(h)))
    return Tensor(h, ctx, RS_OK)


def footprint_bytes(f: Factors, N: int, r_max: int, prec: str = "fp64", with_grid: bool = True) -> int:
    return int(lib.rs_footprint_bytes(C.byref(f.grid), C.byref(f.fdesc), int(N), int(r_max),
                                      PRECS[prec], int(with_grid)))
