"""ctypes marshalling for libmfe.so (see include/mfe.h for the contract of each call)."""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))

STATUS = {0: "MFE_OK", -1: "MFE_EINVAL", -2: "MFE_EDIM", -3: "MFE_ENONFINITE", -4: "MFE_EDEVICE",
          -5: "MFE_ENOMEM", -6: "MFE_EUNSUPPORTED"}
KIND = {"dense_f64": 0, "dense_bf16": 1, "csr_f32": 2, "operator": 3}


class LibraryMissing(RuntimeError):
    """libmfe.so is not built; there is no fallback implementation."""


class MfeError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


# int apply(void* ctx, int trans, int32 k, const double* X, int64 ldx, double* Y, int64 ldy, void* stream)
APPLY_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p,
                       C.c_int64, C.c_void_p)


class _Matrix(C.Structure):
    _fields_ = [("kind", C.c_int32), ("m", C.c_int64), ("n", C.c_int64), ("data", C.c_void_p),
                ("ld", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("val", C.c_void_p), ("apply", APPLY_FN), ("ctx", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("alpha", C.c_double), ("beta", C.c_double), ("gamma", C.c_double), ("box_M", C.c_double),
                ("steps", C.c_int32), ("probes", C.c_int32), ("seed", C.c_uint64), ("t0", C.c_int32),
                ("batch", C.c_int32), ("u0", C.c_void_p), ("v0", C.c_void_p), ("stream", C.c_void_p)]


class _CcpInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("norm_iters", C.c_int32), ("op_norm", C.c_double), ("tau", C.c_double),
                ("sigma", C.c_double), ("objective", C.c_double)]


class _LsqrInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("stop_reason", C.c_int32), ("rel_resid", C.c_double),
                ("normal_eq", C.c_double)]


_LIB = None


def library_path() -> str:
    return os.environ.get("MFE_LIBRARY", os.path.join(_HERE, "libmfe.so"))


def _lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise LibraryMissing(f"{path} is not built; run __graft_entry__.build() or "
                             "python paper_1602_06621_amd/build.py")
    lib = C.CDLL(path)
    i32, i64, u64, dbl, vp = C.c_int32, C.c_int64, C.c_uint64, C.c_double, C.c_void_p
    sig = {
        "mfe_default_alpha_beta": [i64, i64, C.POINTER(dbl), C.POINTER(dbl)],
        "mfe_equilibrate": [C.POINTER(_Matrix), C.POINTER(_Params), vp, vp, vp, vp],
        "mfe_plan_create": [C.POINTER(_Matrix), i32, i32, vp, C.POINTER(vp)],
        "mfe_plan_equilibrate": [vp, C.POINTER(_Params), vp, vp, i32, vp, vp, vp, vp],
        "mfe_plan_last_timing": [vp, C.POINTER(dbl), C.POINTER(dbl)],
        "mfe_last_timing": [C.POINTER(dbl), C.POINTER(dbl)],
        "mfe_plan_destroy": [vp],
        "mfe_lsqr": [C.POINTER(_Matrix), vp, vp, vp, dbl, i32, i32, vp, C.POINTER(_LsqrInfo), vp],
        "mfe_plan_lsqr": [vp, vp, vp, vp, dbl, i32, i32, vp, C.POINTER(_LsqrInfo), vp],
        "mfe_residual": [C.POINTER(_Matrix), vp, vp, dbl, dbl, C.POINTER(dbl), C.POINTER(dbl),
                         C.POINTER(i64), vp],
        "mfe_draw_signs": [u64, i32, i64, i32, i64, vp, vp],
        "mfe_plan_equilibrate_trace": [vp, C.POINTER(_Params), i32, C.POINTER(dbl), vp, vp, vp, vp],
        "mfe_plan_autotune": [vp, C.POINTER(_Params), vp, vp, i32, vp, C.POINTER(dbl), C.POINTER(i32)],
        "mfe_plan_warmstart": [vp, vp, u64, i32, vp, vp, dbl, dbl, i32, vp, vp, vp],
        "mfe_plan_set_tuning": [vp, i32, i32, i32, i32, i32, i32],
        "mfe_plan_create_symmetric": [C.POINTER(_Matrix), i32, vp, C.POINTER(vp)],
        "mfe_plan_op_norm": [vp, vp, vp, i32, dbl, C.POINTER(dbl), C.POINTER(i32), vp],
        "mfe_plan_ccp_lasso": [vp, vp, vp, vp, dbl, dbl, i32, i32, vp, vp, C.POINTER(_CcpInfo), vp],
        "mfe_plan_set_targets": [vp, vp, vp, vp],
        "mfe_plan_set_blocks": [vp, vp, i64, vp, i64],
        "mfe_plan_sketch_features": [vp, u64, i32, vp, vp, dbl, dbl, vp, vp, vp, vp, vp],
        "mfe_mlp_sizes": [C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)],
        "mfe_mlp_forward": [vp, vp, i64, vp, vp],
        "mfe_mlp_loss_grad": [vp, vp, vp, i64, vp, C.POINTER(dbl), vp],
        "mfe_mlp_train": [vp, vp, vp, i32, vp, vp, i64, i64, i32, C.c_float, u64, vp, vp],
        "mfe_warmstart_apply": [i64, vp, vp, dbl, vp, vp],
        "mfe_check_targets": [i64, i64, dbl, dbl, C.POINTER(dbl)],
        "mfe_equilibrate_noalloc": [C.POINTER(_Matrix), C.POINTER(_Params), vp, vp, vp, vp],
        "mfe_probe_gather": [i64, i64, i32, i32, C.POINTER(dbl), vp],
        "mfe_probe_gather_sorted": [i64, i64, i32, i32, C.POINTER(dbl), vp],
        "mfe_probe_stream": [i64, i32, C.POINTER(dbl), vp],
        "mfe_plan_training_set": [vp, u64, i32, vp, vp, dbl, dbl, vp, vp, i64, u64, vp, vp, vp, C.POINTER(i64),
                                  vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.mfe_last_error.restype = C.c_char_p
    lib.mfe_last_error.argtypes = []
    lib.mfe_version.restype = C.c_char_p
    lib.mfe_version.argtypes = []
    _LIB = lib
    return lib


def last_error() -> str:
    return _lib().mfe_last_error().decode()


def check_targets(m: int, n: int, alpha: float, beta: float):
    """mfe_check_targets: (relative mismatch of m alpha^2 and n beta^2, warning text or "")."""
    rel = C.c_double()
    _check(_lib().mfe_check_targets(int(m), int(n), float(alpha), float(beta), C.byref(rel)))
    msg = last_error()
    return rel.value, (msg if msg.startswith("warning:") else "")


def probe_gather(table_bytes: int, gathers: int, in_flight: int = 1, reps: int = 5, stream=None) -> float:
    """Milliseconds per launch of `gathers` random 8-byte reads from a table of table_bytes,
    in_flight (1, 2, 4 or 8) independent gathers per lane at a time."""
    ms = C.c_double()
    _check(_lib().mfe_probe_gather(int(table_bytes), int(gathers), int(in_flight), int(reps), C.byref(ms),
                                   _stream(stream)))
    return ms.value


def probe_gather_sorted(table_bytes: int, gathers: int, per_row: int = 10, reps: int = 5, stream=None) -> float:
    """Milliseconds per launch of `gathers` 8-byte reads from a table of table_bytes, in
    rows of per_row (5, 10, 20 or 40) hashed indices each read in increasing order, one
    at a time per lane."""
    ms = C.c_double()
    _check(_lib().mfe_probe_gather_sorted(int(table_bytes), int(gathers), int(per_row), int(reps), C.byref(ms),
                                          _stream(stream)))
    return ms.value


def probe_stream(nbytes: int, reps: int = 5, stream=None) -> float:
    """Milliseconds per launch of one streaming read of nbytes."""
    ms = C.c_double()
    _check(_lib().mfe_probe_stream(int(nbytes), int(reps), C.byref(ms), _stream(stream)))
    return ms.value


def version() -> str:
    return _lib().mfe_version().decode()


def _check(status: int):
    if status != 0:
        raise MfeError(status, last_error())


def _ptr(t: Optional[torch.Tensor], dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor (got {t.device})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    return C.c_void_p(t.data_ptr())


def _stream(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


# --------------------------------------------------------------- matrices

@dataclass
class Csr:
    """CSR matrix in device memory: row_ptr int32 [m+1], col_idx int32 [nnz], val float32 [nnz]."""

    m: int
    n: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    val: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    @staticmethod
    def from_arrays(m, n, row_ptr, col_idx, val, device="cuda") -> "Csr":
        t = lambda a, dt: torch.as_tensor(a).to(device=device, dtype=dt).contiguous()  # noqa: E731
        return Csr(int(m), int(n), t(row_ptr, torch.int32), t(col_idx, torch.int32), t(val, torch.float32))

    def struct(self) -> _Matrix:
        s = _Matrix()
        s.kind = KIND["csr_f32"]
        s.m, s.n, s.nnz = self.m, self.n, self.nnz
        s.row_ptr = _ptr(self.row_ptr, torch.int32, "row_ptr")
        s.col_idx = _ptr(self.col_idx, torch.int32, "col_idx") if self.nnz else None
        s.val = _ptr(self.val, torch.float32, "val") if self.nnz else None
        return s


@dataclass
class Dense:
    """Dense row-major matrix in device memory: float64, or bfloat16 bit patterns (int16/uint16)."""

    data: torch.Tensor
    ld: Optional[int] = None

    @property
    def m(self) -> int:
        return int(self.data.shape[0])

    @property
    def n(self) -> int:
        return int(self.data.shape[1])

    def struct(self) -> _Matrix:
        s = _Matrix()
        if self.data.dtype == torch.float64:
            s.kind = KIND["dense_f64"]
        elif self.data.dtype in (torch.int16, torch.bfloat16) or str(self.data.dtype) == "torch.uint16":
            s.kind = KIND["dense_bf16"]
        else:
            raise TypeError("dense data must be float64 or bfloat16 bit patterns")
        s.m, s.n = self.m, self.n
        s.ld = self.ld if self.ld is not None else self.data.stride(0)
        if self.data.stride(1) != 1:
            raise ValueError("dense data must be row-major with unit column stride")
        s.data = C.c_void_p(self.data.data_ptr())
        return s


class Operator:
    """Matrix-free operator: apply(trans, k, X, ldx, Y, ldy, rows_in, rows_out, stream) fills
    the FP64 device block Y (row-major, rows_out x k) with A X (trans = 0) or A' X
    (trans = 1); X and Y are raw device addresses, work goes on `stream`."""

    def __init__(self, m: int, n: int, apply):
        self.m, self.n = int(m), int(n)
        self._apply = apply

        def cb(ctx, trans, k, X, ldx, Y, ldy, stream):
            try:
                rows_in = self.m if trans else self.n
                rows_out = self.n if trans else self.m
                self._apply(int(trans), int(k), int(X or 0), int(ldx), int(Y or 0), int(ldy), rows_in, rows_out,
                            int(stream or 0))
                return 0
            except Exception:  # errors are reported through the status code
                return 1

        self._cb = APPLY_FN(cb)

    def struct(self) -> _Matrix:
        s = _Matrix()
        s.kind = KIND["operator"]
        s.m, s.n = self.m, self.n
        s.apply = self._cb
        return s


def _params(alpha, beta, gamma, M, steps, probes, seed, t0, batch, u0, v0, stream) -> _Params:
    p = _Params()
    p.alpha, p.beta, p.gamma, p.box_M = float(alpha), float(beta), float(gamma), float(M)
    p.steps, p.probes, p.seed = int(steps), int(probes), int(seed) & ((1 << 64) - 1)
    p.t0, p.batch = int(t0), int(batch)
    p.u0 = _ptr(u0, torch.float64, "u0")
    p.v0 = _ptr(v0, torch.float64, "v0")
    p.stream = _stream(stream)
    return p


def last_timing():
    """Step-loop timing of the last equilibrate() on this thread (dense BF16 path)."""
    a, b = C.c_double(), C.c_double()
    _check(_lib().mfe_last_timing(C.byref(a), C.byref(b)))
    return dict(loop_ms=a.value, step_ms=b.value)


def default_alpha_beta(m: int, n: int):
    a, b = C.c_double(), C.c_double()
    _check(_lib().mfe_default_alpha_beta(int(m), int(n), C.byref(a), C.byref(b)))
    return a.value, b.value


def equilibrate(A, alpha=None, beta=None, gamma=0.1, M=10.0, steps=100, probes=1, seed=0, t0=0,
                batch=0, u0=None, v0=None, stream=None, device="cuda"):
    """Algorithm 1 on one matrix.  Returns dict(d, e, u_bar, v_bar) of float64 device tensors."""
    lib = _lib()
    if alpha is None or beta is None:
        alpha, beta = default_alpha_beta(A.m, A.n)
    d = torch.empty(A.m, dtype=torch.float64, device=device)
    e = torch.empty(A.n, dtype=torch.float64, device=device)
    ub = torch.empty_like(d)
    vb = torch.empty_like(e)
    s = A.struct()
    p = _params(alpha, beta, gamma, M, steps, probes, seed, t0, batch, u0, v0, stream)
    _check(lib.mfe_equilibrate(C.byref(s), C.byref(p), _ptr(d), _ptr(e), _ptr(ub), _ptr(vb)))
    return dict(d=d, e=e, u_bar=ub, v_bar=vb)


def equilibrate_noalloc(A, alpha=None, beta=None, gamma=0.1, M=10.0, steps=100, probes=1, seed=0, t0=0,
                        batch=0, u0=None, v0=None, stream=None, out=None, device="cuda"):
    """mfe_equilibrate_noalloc (dense FP64): the library allocates nothing; the outputs are
    the caller's (`out` = dict(d, e, u_bar, v_bar) of float64 device tensors, made here
    when not given)."""
    lib = _lib()
    if alpha is None or beta is None:
        alpha, beta = default_alpha_beta(A.m, A.n)
    if out is None:
        out = dict(d=torch.empty(A.m, dtype=torch.float64, device=device),
                   e=torch.empty(A.n, dtype=torch.float64, device=device),
                   u_bar=torch.empty(A.m, dtype=torch.float64, device=device),
                   v_bar=torch.empty(A.n, dtype=torch.float64, device=device))
    s = A.struct()
    p = _params(alpha, beta, gamma, M, steps, probes, seed, t0, batch, u0, v0, stream)
    _check(lib.mfe_equilibrate_noalloc(C.byref(s), C.byref(p), _ptr(out["d"], torch.float64),
                                       _ptr(out["e"], torch.float64), _ptr(out.get("u_bar"), torch.float64),
                                       _ptr(out.get("v_bar"), torch.float64)))
    return out


class Plan:
    """Preprocessed CSR matrices (one or a batch) for repeated equilibration / LSQR runs."""

    def __init__(self, mats: Sequence[Csr], max_probes: int = 16, stream=None, symmetric=False):
        lib = _lib()
        self.mats = list(mats)
        h = C.c_void_p()
        if symmetric:
            if len(self.mats) != 1:
                raise ValueError("a symmetric plan holds one matrix")
            m0 = self.mats[0].struct()
            _check(lib.mfe_plan_create_symmetric(C.byref(m0), int(max_probes), _stream(stream), C.byref(h)))
        else:
            arr = (_Matrix * len(self.mats))(*[m.struct() for m in self.mats])
            _check(lib.mfe_plan_create(arr, len(self.mats), int(max_probes), _stream(stream), C.byref(h)))
        self._h = h
        self.symmetric = bool(symmetric)
        self.M = sum(m.m for m in self.mats)
        self.N = sum(m.n for m in self.mats)
        self._blocks = (None, None)
        self._targets_dev = (None, None)

    @classmethod
    def symmetric_plan(cls, A: Csr, max_probes: int = 16, stream=None) -> "Plan":
        """Plan for Algorithm 2 (symmetric equilibration, Section 6) of a symmetric matrix."""
        return cls([A], max_probes=max_probes, stream=stream, symmetric=True)

    def set_targets(self, row_target=None, col_target=None, stream=None):
        """Squared row / column norm targets per index (Section 6, varying norms); None
        restores alpha^2 / beta^2 on that side.  Device FP64 tensors of sum m / sum n."""
        rt = None if row_target is None else row_target.to(torch.float64).contiguous()
        ct = None if col_target is None else col_target.to(torch.float64).contiguous()
        if rt is not None and rt.numel() != self.M:
            raise ValueError("row_target needs one value per row")
        if ct is not None and ct.numel() != self.N:
            raise ValueError("col_target needs one value per column")
        _check(_lib().mfe_plan_set_targets(self._h, _ptr(rt), _ptr(ct), _stream(stream)))
        self._targets_dev = (rt, ct)

    def set_blocks(self, row_ptr=None, col_ptr=None):
        """Block equilibration (Section 6): offsets of row / column blocks (host sequences
        from 0 to m / n), or None for a side without blocks."""
        def arr(ptr):
            if ptr is None:
                return None, 0
            vals = [int(x) for x in ptr]
            return (C.c_int64 * len(vals))(*vals), len(vals) - 1
        ra, rn = arr(row_ptr)
        ca, cn = arr(col_ptr)
        _check(_lib().mfe_plan_set_blocks(self._h, ra, rn, ca, cn))
        self._blocks = (rn if row_ptr is not None else None, cn if col_ptr is not None else None)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib().mfe_plan_destroy(self._h)
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

    def equilibrate(self, alpha=None, beta=None, gamma=0.1, M=10.0, steps=100, probes=1, seed=0, t0=0,
                    batch=0, u0=None, v0=None, use_graph=False, stream=None, out=None, device="cuda"):
        """alpha/beta: scalars for every matrix, per-matrix sequences, or None for the
        default (n_b/m_b)^(1/4), (m_b/n_b)^(1/4) of each matrix."""
        lib = _lib()
        cnt = len(self.mats)
        if alpha is None or beta is None:
            ab = [default_alpha_beta(mm.m, mm.n) for mm in self.mats]
            alpha = [a for a, _ in ab]
            beta = [b for _, b in ab]
        ah = bh = None
        if not isinstance(alpha, (int, float)) or not isinstance(beta, (int, float)):
            al = [float(alpha)] * cnt if isinstance(alpha, (int, float)) else [float(a) for a in alpha]
            be = [float(beta)] * cnt if isinstance(beta, (int, float)) else [float(b) for b in beta]
            ah = (C.c_double * cnt)(*al)
            bh = (C.c_double * cnt)(*be)
            a0, b0 = al[0], be[0]
        else:
            a0, b0 = alpha, beta
        if out is None:
            nu = self._blocks[0] if self._blocks[0] is not None else self.M
            nv = self._blocks[1] if self._blocks[1] is not None else self.N
            out = dict(d=torch.empty(self.M, dtype=torch.float64, device=device),
                       e=torch.empty(self.N, dtype=torch.float64, device=device),
                       u_bar=torch.empty(nu, dtype=torch.float64, device=device),
                       v_bar=torch.empty(nv, dtype=torch.float64, device=device))
        p = _params(a0, b0, gamma, M, steps, probes, seed, t0, batch, u0, v0, stream)
        _check(lib.mfe_plan_equilibrate(self._h, C.byref(p), ah, bh, int(bool(use_graph)), _ptr(out["d"]),
                                        _ptr(out["e"]), _ptr(out.get("u_bar")), _ptr(out.get("v_bar"))))
        return out

    def _targets(self, alpha, beta):
        cnt = len(self.mats)
        if alpha is None or beta is None:
            ab = [default_alpha_beta(mm.m, mm.n) for mm in self.mats]
            alpha = [a for a, _ in ab]
            beta = [b for _, b in ab]
        al = [float(alpha)] * cnt if isinstance(alpha, (int, float)) else [float(a) for a in alpha]
        be = [float(beta)] * cnt if isinstance(beta, (int, float)) else [float(b) for b in beta]
        return (C.c_double * cnt)(*al), (C.c_double * cnt)(*be), al[0], be[0]

    def autotune(self, alpha=None, beta=None, gamma=0.1, M=10.0, probes=1, seed=0, trial_steps=20, stream=None):
        """Times every launch configuration of the step kernels (results are identical under
        all of them) and keeps the fastest for this plan.  Returns the choice."""
        ah, bh, a0, b0 = self._targets(alpha, beta)
        p = _params(a0, b0, gamma, M, trial_steps, probes, seed, 0, 0, None, None, stream)
        chosen = (C.c_int32 * 6)()
        best, n = C.c_double(), C.c_int32()
        _check(_lib().mfe_plan_autotune(self._h, C.byref(p), ah, bh, int(trial_steps), chosen, C.byref(best),
                                        C.byref(n)))
        return dict(loads_in_flight=chosen[0], rows_mode=chosen[1], cols_mode=chosen[2], stream_hints=chosen[3],
                    slice_order=chosen[4], workgroup_threads=chosen[5], step_ms=best.value,
                    candidates=n.value)

    def set_tuning(self, loads_in_flight=1, rows_mode=2, cols_mode=2, stream_hints=-1, slice_order=-1,
                   workgroup_threads=0):
        """Launch configuration of the step kernels (see mfe_plan_set_tuning); the defaults
        are the library's (one load in flight, both directions in one launch, stream hints
        by the plan's size, slice order by the launch shape, 256 threads per workgroup)."""
        _check(_lib().mfe_plan_set_tuning(self._h, int(loads_in_flight), int(rows_mode), int(cols_mode),
                                          int(stream_hints), int(slice_order), int(workgroup_threads)))

    def last_timing(self):
        a, b = C.c_double(), C.c_double()
        _check(_lib().mfe_plan_last_timing(self._h, C.byref(a), C.byref(b)))
        return dict(loop_ms=a.value, step_ms=b.value)

    def equilibrate_trace(self, alpha, beta, gamma=0.1, M=10.0, steps=100, probes=1, seed=0, t0=0, u0=None,
                          v0=None, trace_every=25, stream=None, device="cuda"):
        """Single-matrix run recording the RMS equilibration error of the running average
        every trace_every steps.  Returns (outputs, numpy trace)."""
        import numpy as np

        out = dict(d=torch.empty(self.M, dtype=torch.float64, device=device),
                   e=torch.empty(self.N, dtype=torch.float64, device=device),
                   u_bar=torch.empty(self.M, dtype=torch.float64, device=device),
                   v_bar=torch.empty(self.N, dtype=torch.float64, device=device))
        n_tr = -(-int(steps) // int(trace_every)) if steps > 0 else 0
        tr = (C.c_double * max(n_tr, 1))()
        p = _params(alpha, beta, gamma, M, steps, probes, seed, t0, 0, u0, v0, stream)
        _check(_lib().mfe_plan_equilibrate_trace(self._h, C.byref(p), int(trace_every), tr, _ptr(out["d"]),
                                                  _ptr(out["e"]), _ptr(out["u_bar"]), _ptr(out["v_bar"])))
        return out, np.array(tr[:n_tr])

    def sketch_features(self, seed, probes=4, gamma=0.1, M=10.0, alpha=None, beta=None, stream=None, device="cuda"):
        """Sketch features [*, 8] (FP32) and sketch initialisations (FP64) of every row and
        column of the plan's matrices (see mfe.h)."""
        cnt = len(self.mats)
        ah = bh = None
        if alpha is not None:
            ah = (C.c_double * cnt)(*([float(alpha)] * cnt if isinstance(alpha, (int, float)) else alpha))
            bh = (C.c_double * cnt)(*([float(beta)] * cnt if isinstance(beta, (int, float)) else beta))
        fr = torch.empty(self.M, 8, dtype=torch.float32, device=device)
        fc = torch.empty(self.N, 8, dtype=torch.float32, device=device)
        us = torch.empty(self.M, dtype=torch.float64, device=device)
        vs = torch.empty(self.N, dtype=torch.float64, device=device)
        _check(_lib().mfe_plan_sketch_features(self._h, int(seed) & ((1 << 64) - 1), int(probes), ah, bh,
                                               float(gamma), float(M), _ptr(fr), _ptr(fc), _ptr(us), _ptr(vs),
                                               _stream(stream)))
        return dict(feat_rows=fr, feat_cols=fc, u_sketch=us, v_sketch=vs)

    def training_set(self, seed, u_label, v_label, per_matrix=4096, sample_seed=0, probes=4, gamma=0.1, M=10.0,
                     alpha=None, beta=None, stream=None, device="cuda"):
        """(X [count, 8] FP32, t [count] FP32, idx [count] int64): stratified samples of up
        to per_matrix rows and columns of every matrix, their sketch features and the
        targets label - sketch initialisation (see mfe_plan_training_set)."""
        ah = bh = None
        if alpha is not None:
            ah, bh, _, _ = self._targets(alpha, beta)
        lib = _lib()
        u_label = u_label.to(torch.float64).contiguous()
        v_label = v_label.to(torch.float64).contiguous()
        if u_label.numel() != self.M or v_label.numel() != self.N:
            raise ValueError("labels need sum m row values and sum n column values")
        cnt = C.c_int64()
        args = (self._h, int(seed) & ((1 << 64) - 1), int(probes), ah, bh, float(gamma), float(M), _ptr(u_label),
                _ptr(v_label), int(per_matrix), int(sample_seed) & ((1 << 64) - 1))
        _check(lib.mfe_plan_training_set(*args, None, None, None, C.byref(cnt), _stream(stream)))
        X = torch.empty(cnt.value, 8, dtype=torch.float32, device=device)
        t = torch.empty(cnt.value, dtype=torch.float32, device=device)
        idx = torch.empty(cnt.value, dtype=torch.int64, device=device)
        _check(lib.mfe_plan_training_set(*args, _ptr(X), _ptr(t), _ptr(idx), C.byref(cnt), _stream(stream)))
        return X, t, idx

    def warm_start(self, params, seed, probes=4, gamma=0.1, M=10.0, learned=True, alpha=None, beta=None,
                   stream=None, device="cuda"):
        """(u0, v0) for every matrix of the plan in one call: sketch, network, clip (see mfe.h)."""
        ah = bh = None
        if alpha is not None:
            ah, bh, _, _ = self._targets(alpha, beta)
        u0 = torch.empty(self.M, dtype=torch.float64, device=device)
        v0 = torch.empty(self.N, dtype=torch.float64, device=device)
        _check(_lib().mfe_plan_warmstart(self._h, _ptr(params, torch.float32, "params") if learned else None,
                                         int(seed) & ((1 << 64) - 1), int(probes), ah, bh, float(gamma), float(M),
                                         int(bool(learned)), _ptr(u0), _ptr(v0), _stream(stream)))
        return u0, v0

    def op_norm(self, d=None, e=None, max_iter=1000, tol=1e-10, stream=None):
        """||D A E||_2 by Golub-Kahan bidiagonalisation (see mfe_plan_op_norm).  Returns
        (norm, steps)."""
        nrm, it = C.c_double(), C.c_int32()
        _check(_lib().mfe_plan_op_norm(self._h, _ptr(d, torch.float64), _ptr(e, torch.float64), int(max_iter),
                                       float(tol), C.byref(nrm), C.byref(it), _stream(stream)))
        return nrm.value, it.value

    def ccp_lasso(self, b, lam, d=None, e=None, iters=1000, op_norm=0.0, trace_every=0, stream=None,
                  device="cuda"):
        """CCP on the Lasso of Section 5.2 (see mfe_plan_ccp_lasso).  Returns (x, info, trace)."""
        import numpy as np

        x = torch.empty(self.N, dtype=torch.float64, device=device)
        n_tr = int(iters) // int(trace_every) if trace_every > 0 else 0
        tr = (C.c_double * max(n_tr, 1))() if trace_every > 0 else None
        info = _CcpInfo()
        _check(_lib().mfe_plan_ccp_lasso(self._h, _ptr(b, torch.float64), _ptr(d, torch.float64),
                                         _ptr(e, torch.float64), float(lam), float(op_norm), int(iters),
                                         int(trace_every), tr, _ptr(x), C.byref(info), _stream(stream)))
        inf = dict(iters=info.iters, norm_iters=info.norm_iters, op_norm=info.op_norm, tau=info.tau,
                   sigma=info.sigma, objective=info.objective)
        return x, inf, (np.array(tr[:n_tr]) if tr is not None else np.zeros(0))

    def lsqr(self, b, d=None, e=None, tol=1e-6, max_iter=1000, check_every=10, stream=None, device="cuda"):
        x = torch.empty(self.N, dtype=torch.float64, device=device)
        info = _LsqrInfo()
        _check(_lib().mfe_plan_lsqr(self._h, _ptr(b, torch.float64, "b"), _ptr(d, torch.float64, "d"),
                                    _ptr(e, torch.float64, "e"), float(tol), int(max_iter), int(check_every),
                                    _ptr(x), C.byref(info), _stream(stream)))
        return x, _info(info)


def _info(info: _LsqrInfo):
    return dict(iters=info.iters, stop_reason=info.stop_reason, rel_resid=info.rel_resid,
                normal_eq=info.normal_eq)


def lsqr(A, b, d=None, e=None, tol=1e-6, max_iter=1000, check_every=10, stream=None, device="cuda"):
    """LSQR on (DAE) xbar = D b, x = E xbar (Section 5.1).  Returns (x, info)."""
    x = torch.empty(A.n, dtype=torch.float64, device=device)
    info = _LsqrInfo()
    s = A.struct()
    _check(_lib().mfe_lsqr(C.byref(s), _ptr(b, torch.float64, "b"), _ptr(d, torch.float64, "d"),
                           _ptr(e, torch.float64, "e"), float(tol), int(max_iter), int(check_every), _ptr(x),
                           C.byref(info), _stream(stream)))
    return x, _info(info)


def residual(A, d=None, e=None, alpha=None, beta=None, stream=None):
    """RMS equilibration error of DAE (Section 4).  Returns (rms, rms_nonempty, n_empty)."""
    if alpha is None or beta is None:
        alpha, beta = default_alpha_beta(A.m, A.n)
    r, rn, ne = C.c_double(), C.c_double(), C.c_int64()
    s = A.struct()
    _check(_lib().mfe_residual(C.byref(s), _ptr(d, torch.float64, "d"), _ptr(e, torch.float64, "e"),
                               float(alpha), float(beta), C.byref(r), C.byref(rn), C.byref(ne), _stream(stream)))
    return r.value, rn.value, ne.value


def mlp_sizes():
    a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
    _check(_lib().mfe_mlp_sizes(C.byref(a), C.byref(b), C.byref(c)))
    return dict(params=a.value, features=b.value, width=c.value)


def mlp_forward(params, X, stream=None):
    y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _check(_lib().mfe_mlp_forward(_ptr(params, torch.float32, "params"), _ptr(X, torch.float32, "X"),
                                  int(X.shape[0]), _ptr(y), _stream(stream)))
    return y


def mlp_loss_grad(params, X, t, stream=None):
    g = torch.empty_like(params)
    loss = C.c_double()
    _check(_lib().mfe_mlp_loss_grad(_ptr(params, torch.float32, "params"), _ptr(X, torch.float32, "X"),
                                    _ptr(t, torch.float32, "t"), int(X.shape[0]), _ptr(g), C.byref(loss),
                                    _stream(stream)))
    return loss.value, g


def mlp_train(params, adam_m, adam_v, step0, X, t, batch, iters, lr, seed, stream=None):
    """Adam on mini-batches (in place).  Returns the per-step loss trace (numpy)."""
    import numpy as np

    tr = (C.c_double * max(int(iters), 1))()
    _check(_lib().mfe_mlp_train(_ptr(params, torch.float32, "params"), _ptr(adam_m, torch.float32, "adam_m"),
                                _ptr(adam_v, torch.float32, "adam_v"), int(step0), _ptr(X, torch.float32, "X"),
                                _ptr(t, torch.float32, "t"), int(X.shape[0]), int(batch), int(iters),
                                float(lr), int(seed) & ((1 << 64) - 1), tr, _stream(stream)))
    return np.array(tr[:int(iters)])


def warmstart_apply(sketch, delta, M, stream=None):
    out = torch.empty_like(sketch)
    _check(_lib().mfe_warmstart_apply(int(sketch.numel()), _ptr(sketch, torch.float64, "sketch"),
                                      _ptr(delta, torch.float32, "delta"), float(M), _ptr(out), _stream(stream)))
    return out


def draw_signs(seed: int, batch: int, step: int, side: int, nwords: int, stream=None, device="cuda"):
    """First nwords 64-bit words of the probe sign stream, as an int64 device tensor."""
    w = torch.empty(max(int(nwords), 1), dtype=torch.int64, device=device)
    _check(_lib().mfe_draw_signs(int(seed) & ((1 << 64) - 1), int(batch), int(step), int(side), int(nwords),
                                 _ptr(w), _stream(stream)))
    return w[:nwords]
