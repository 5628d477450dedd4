"""ctypes binding of libparaexp.so (C ABI declared in include/paraexp.h).

Argument marshalling only: every numerical step runs in the HIP library.  PyTorch
(ROCm) provides device memory and the current stream.  Matrices that the ABI takes
column-major (n x k, leading dimension n) are held as contiguous torch tensors of shape
(k, n): row i of the tensor is column i of the matrix.

The library must be built (``python -m paper_1509_04567_amd.build``); importing a
missing or unloadable library raises immediately -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libparaexp.so")

PE_OK = 0
PE_ERR_ARG = -1
PE_ERR_NONFINITE = -2
PE_ERR_DEVICE = -3
PE_ERR_OOM = -4
PE_ERR_UNSUPPORTED = -5
PE_FP64 = 0
PE_MIXED = 1
PE_KRYLOV_POLY = 0
PE_KRYLOV_SAI = 1
PE_FIT_CHEBYSHEV = 0
PE_FIT_SPLINE = 1
FLAG_NOT_CONVERGED = 1
FLAG_BREAKDOWN = 2
FLAG_RANK_CAPPED = 4
FLAG_FIT_CAPPED = 8

EXPORTED = ["pe_create", "pe_destroy", "pe_last_error", "pe_version", "pe_stencil_apply", "pe_compress",
            "pe_compress_noalloc",
            "pe_expaction_batch", "pe_solve_batch", "pe_workspace_query", "pe_superpose", "pe_wr_burgers",
            "pe_profile_enable", "pe_profile_read", "pe_autotune", "pe_autotune_table",
            # host-only decision rules (include/paraexp_policy.h)
            "pe_policy_step", "pe_policy_step_growth", "pe_policy_reorth_skip"]
PE_STEP_ACCEPT = 0
PE_STEP_REJECT = 1
PE_STEP_STOP = 2


class PeStencil(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("per_point", ctypes.c_int32), ("coeffs", ctypes.c_void_p)]


class PeProblem(ctypes.Structure):
    _fields_ = [
        ("op", PeStencil),
        ("u0", ctypes.c_void_p),
        ("t0", ctypes.c_double),
        ("t1", ctypes.c_double),
        ("t_samples", ctypes.c_void_p),
        ("s", ctypes.c_int32),
        ("G", ctypes.c_void_p),
        ("ldG", ctypes.c_int64),
        ("shift", ctypes.c_int32),
        ("t_out", ctypes.c_void_p),
        ("n_out", ctypes.c_int32),
        ("out", ctypes.c_void_p),
        ("ldOut", ctypes.c_int64),
        ("krylov_steps", ctypes.c_int32),
        ("rank_max", ctypes.c_int32),
        ("q_max", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("svd_tol", ctypes.c_double),
        ("fit_tol", ctypes.c_double),
        ("prec", ctypes.c_int32),
        ("krylov", ctypes.c_int32),
        ("sai_shift", ctypes.c_double),
        ("source_fit", ctypes.c_int32),
    ]


class PeReport(ctypes.Structure):
    _fields_ = [
        ("rank", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("cycles", ctypes.c_int32),
        ("rejected", ctypes.c_int32),
        ("block_steps", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("resid_est", ctypes.c_double),
        ("fit_resid", ctypes.c_double),
        ("svd_tail", ctypes.c_double),
        ("sigma1", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PeWrProblem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("nu", ctypes.c_double),
        ("T", ctypes.c_double),
        ("P", ctypes.c_int32),
        ("s", ctypes.c_int32),
        ("K", ctypes.c_int32),
        ("jacobian", ctypes.c_int32),
        ("u0", ctypes.c_void_p),
        ("u_init", ctypes.c_void_p),
        ("u_final", ctypes.c_void_p),
        ("krylov_steps", ctypes.c_int32),
        ("rank_max", ctypes.c_int32),
        ("q_max", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("svd_tol", ctypes.c_double),
        ("fit_tol", ctypes.c_double),
        ("prec", ctypes.c_int32),
        ("krylov", ctypes.c_int32),
        ("sai_shift", ctypes.c_double),
        ("forcing", ctypes.c_void_p),
        ("source_fit", ctypes.c_int32),
    ]


class PeStepTrial(ctypes.Structure):
    _fields_ = [("nsq", ctypes.c_int32), ("est", ctypes.c_void_p), ("alpha", ctypes.c_double),
                ("tol", ctypes.c_double), ("ref", ctypes.c_double), ("tspan", ctypes.c_double),
                ("dmin", ctypes.c_double), ("krylov_steps", ctypes.c_int32), ("pexp", ctypes.c_double)]


class PeStepDecision(ctypes.Structure):
    _fields_ = [("action", ctypes.c_int32), ("level", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("step", ctypes.c_double), ("rho", ctypes.c_double), ("pexp", ctypes.c_double),
                ("err", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"paraexp status {status}: {msg}")
        self.status = status


_LIB = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libparaexp.so and declare the C signatures (raises if it is missing)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_1509_04567_amd.build`")
    # torch (ROCm) ships its own HIP runtime; loading it first makes the library bind to
    # that same runtime (same soname), so torch's memory and streams are valid here.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.pe_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.pe_destroy.argtypes = [vp]
    lib.pe_last_error.argtypes = [vp]
    lib.pe_last_error.restype = ctypes.c_char_p
    lib.pe_version.restype = ctypes.c_char_p
    lib.pe_stencil_apply.argtypes = [vp, ctypes.POINTER(PeStencil), vp, i64, vp, i64, i32, vp]
    lib.pe_compress.argtypes = [vp, ctypes.POINTER(PeProblem), vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(PeReport), vp]
    lib.pe_compress_noalloc.argtypes = lib.pe_compress.argtypes
    lib.pe_expaction_batch.argtypes = [vp, ctypes.POINTER(PeProblem), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                       ctypes.POINTER(i32), ctypes.POINTER(i32), i32, ctypes.POINTER(PeReport), vp]
    lib.pe_solve_batch.argtypes = [vp, ctypes.POINTER(PeProblem), i32, ctypes.POINTER(PeReport), vp]
    lib.pe_workspace_query.argtypes = [vp, ctypes.POINTER(PeProblem), i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.pe_superpose.argtypes = [vp, vp, ctypes.POINTER(vp), i32, i64, i32, i64, vp, i64, vp]
    lib.pe_wr_burgers.argtypes = [vp, ctypes.POINTER(PeWrProblem), ctypes.POINTER(PeReport),
                                  ctypes.POINTER(ctypes.c_double), vp]
    lib.pe_profile_enable.argtypes = [vp, ctypes.c_char_p]
    lib.pe_autotune.argtypes = [vp, ctypes.POINTER(PeProblem), i32, ctypes.c_char_p, ctypes.POINTER(i32), vp]
    lib.pe_autotune_table.argtypes = [vp, ctypes.POINTER(i32), i32]
    lib.pe_autotune_table.restype = i32
    lib.pe_profile_read.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.pe_policy_step.argtypes = [ctypes.POINTER(PeStepTrial), ctypes.POINTER(PeStepDecision)]
    lib.pe_policy_step.restype = None
    lib.pe_policy_step_growth.argtypes = [ctypes.c_double, ctypes.c_double, i32]
    lib.pe_policy_step_growth.restype = ctypes.c_double
    lib.pe_policy_reorth_skip.argtypes = [vp, vp, i32, ctypes.c_double]
    lib.pe_policy_reorth_skip.restype = i32
    for name in ["pe_create", "pe_destroy", "pe_stencil_apply", "pe_compress", "pe_compress_noalloc",
                 "pe_expaction_batch",
                 "pe_solve_batch", "pe_superpose", "pe_wr_burgers", "pe_profile_enable", "pe_profile_read",
                 "pe_autotune"]:
        getattr(lib, name).restype = ctypes.c_int
    _LIB = lib
    return lib


def policy_step(est, alpha, tol, ref, tspan, dmin, krylov_steps, pexp=0.0):
    """pe_policy_step (host only): the library's decision on one step-size trial.
    est: per squaring level k = 0..nsq the pair (error estimate, |y_k|)."""
    lib = load_library()
    arr, ptr = _host_doubles(np.asarray(est, dtype=np.float64).reshape(-1))
    t = PeStepTrial(nsq=arr.size // 2 - 1, est=ptr, alpha=alpha, tol=tol, ref=ref, tspan=tspan, dmin=dmin,
                    krylov_steps=krylov_steps, pexp=pexp)
    out = PeStepDecision()
    lib.pe_policy_step(ctypes.byref(t), ctypes.byref(out))
    return out.as_dict()


def policy_step_growth(rho, pexp, krylov_steps):
    return float(load_library().pe_policy_step_growth(rho, pexp, krylov_steps))


def policy_reorth_skip(R, Rn, kappa=0.3):
    """pe_policy_reorth_skip (host only): R (bw x bw upper triangular), Rn (bw,)."""
    lib = load_library()
    Ra, Rp = _host_doubles(R)
    na, npp = _host_doubles(Rn)
    return bool(lib.pe_policy_reorth_skip(Rp, npp, int(Ra.shape[0]), float(kappa)))


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(x, device):
    """float64 contiguous device tensor (copies host arrays)."""
    torch = _torch()
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device=device)


def _host_doubles(a):
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return arr, arr.ctypes.data_as(ctypes.c_void_p)


@dataclasses.dataclass
class DeviceProblem:
    """Device-side buffers of one window subproblem plus the host arrays the ABI reads.
    `src` is any object with the fields of the ABI's pe_problem (numpy or torch arrays)."""

    struct: PeProblem
    out: "object"               # torch (n_out, n): row k = solution at t_out[k]
    keep: list


def make_problem(src, device, precision: int = PE_FP64, out=None) -> DeviceProblem:
    torch = _torch()
    n = int(src.n)
    keep = []
    coeffs = np.asarray(src.coeffs, dtype=np.float64) if not isinstance(src.coeffs, torch.Tensor) else src.coeffs
    per_point = 1 if np.ndim(coeffs) == 2 else 0
    if per_point:
        c_dev = _dev(coeffs, device).reshape(3, n)
        keep.append(c_dev)
        cptr = ctypes.c_void_p(c_dev.data_ptr())
    else:
        c_host, cptr = _host_doubles(coeffs)
        keep.append(c_host)
    u0 = _dev(src.u0, device).reshape(n)
    keep.append(u0)
    G = getattr(src, "G", None)
    ts = getattr(src, "t_samples", None)
    if G is not None:
        Gt = _dev(np.asarray(G).T if not isinstance(G, torch.Tensor) else G.T, device)  # (s, n)
        keep.append(Gt)
        s = int(Gt.shape[0])
        ts_host, ts_ptr = _host_doubles(ts)
        keep.append(ts_host)
        gptr = ctypes.c_void_p(Gt.data_ptr())
    else:
        s, ts_ptr, gptr = 0, None, None
    to_host, to_ptr = _host_doubles(src.t_out)
    keep.append(to_host)
    n_out = int(to_host.shape[0])
    if out is None:
        out = torch.empty((max(n_out, 1), n), dtype=torch.float64, device=device)
    keep.append(out)
    st = PeProblem()
    st.op = PeStencil(n, per_point, cptr)
    st.u0 = u0.data_ptr()
    st.t0 = float(src.t0)
    st.t1 = float(src.t1)
    st.t_samples = ts_ptr
    st.s = s
    st.G = gptr
    st.ldG = n
    st.shift = 1 if bool(getattr(src, "shift", True)) else 0
    st.t_out = to_ptr
    st.n_out = n_out
    st.out = out.data_ptr()
    st.ldOut = n
    st.krylov_steps = int(src.krylov_steps)
    st.rank_max = int(src.rank_max)
    st.q_max = int(src.q_max)
    st.tol = float(src.tol)
    st.svd_tol = float(getattr(src, "svd_tol", 1e-13))
    st.fit_tol = float(getattr(src, "fit_tol", 1e-13))
    st.prec = int(precision)
    st.krylov = int(getattr(src, "krylov", PE_KRYLOV_POLY))
    st.sai_shift = float(getattr(src, "sai_shift", 0.0))
    st.source_fit = int(getattr(src, "source_fit", PE_FIT_CHEBYSHEV))
    return DeviceProblem(struct=st, out=out[:n_out], keep=keep)


def workspace_query(problems: Sequence, precision: int = PE_FP64, ctx=None) -> int:
    """pe_workspace_query: bytes of device memory pe_solve_batch may need for these
    problems.  Only sizes are read; host arithmetic, so no GPU is needed."""
    lib = load_library()
    arr = (PeProblem * max(1, len(problems)))()
    for i, p in enumerate(problems):
        st = arr[i]
        st.op = PeStencil(int(p.n), 0, None)
        ts = getattr(p, "t_samples", None)
        st.s = int(len(ts)) if ts is not None else int(getattr(p, "s", 0))
        st.krylov_steps = int(p.krylov_steps)
        st.rank_max = int(p.rank_max)
        st.q_max = int(p.q_max)
        st.prec = int(precision)
    out = ctypes.c_size_t(0)
    h = ctx.h if ctx is not None else None
    status = lib.pe_workspace_query(h, arr, len(problems), ctypes.byref(out))
    if status != PE_OK:
        msg = lib.pe_last_error(h).decode() if h is not None else "pe_workspace_query failed"
        raise PeError(status, msg)
    return int(out.value)


class Context:
    """One library context on a HIP device (workspace is cached across calls)."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        self.device_index = device
        torch = _torch()
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        st = self.lib.pe_create(ctypes.byref(h), device)
        if st != PE_OK:
            raise PeError(st, "pe_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.pe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != PE_OK:
            raise PeError(st, self.lib.pe_last_error(self.h).decode())

    # -- S0
    def stencil_apply(self, coeffs, X):
        """Y = L X for X a torch (k, n) device tensor (k columns of length n)."""
        torch = _torch()
        X = _dev(X, self.device)
        k, n = X.shape
        Y = torch.empty_like(X)
        keep = []
        if np.ndim(coeffs) == 2:
            cd = _dev(coeffs, self.device)
            keep.append(cd)
            op = PeStencil(n, 1, ctypes.c_void_p(cd.data_ptr()))
        else:
            ch, cp = _host_doubles(coeffs)
            keep.append(ch)
            op = PeStencil(n, 0, cp)
        self._check(self.lib.pe_stencil_apply(self.h, ctypes.byref(op), ctypes.c_void_p(X.data_ptr()), n,
                                              ctypes.c_void_p(Y.data_ptr()), n, k, _stream_ptr()))
        return Y

    # -- S1-S4
    def compress(self, src, precision: int = PE_FP64, noalloc: bool = False):
        """Compression of one problem; noalloc=True calls pe_compress_noalloc (the
        library's fixed device scratch instead of its growable workspace)."""
        torch = _torch()
        dp = make_problem(src, self.device, precision)
        n, rmax, qmax = int(src.n), int(src.rank_max), int(src.q_max)
        spline = int(getattr(src, "source_fit", PE_FIT_CHEBYSHEV)) == PE_FIT_SPLINE
        npc = max(int(dp.struct.s) - 1, 1)
        U = torch.zeros((max(rmax, 1), n), dtype=torch.float64, device=self.device)
        Pi = torch.zeros((4 * npc if spline else qmax, max(rmax, 1)), dtype=torch.float64, device=self.device)
        m, q = ctypes.c_int32(), ctypes.c_int32()
        sig = (ctypes.c_double * max(dp.struct.s, 1))()
        rep = PeReport()
        fn = self.lib.pe_compress_noalloc if noalloc else self.lib.pe_compress
        self._check(fn(self.h, ctypes.byref(dp.struct), ctypes.c_void_p(U.data_ptr()),
                       ctypes.c_void_p(Pi.data_ptr()), ctypes.byref(m), ctypes.byref(q), sig,
                       ctypes.byref(rep), _stream_ptr()))
        mm, qq = m.value, q.value
        if spline:  # piece coefficients: Pw[(i 4 + k) m + a] -> (pieces, 4, m)
            flat = Pi.reshape(-1)[:4 * npc * mm]
            return dict(U=U[:mm], Pw=flat.reshape(npc, 4, mm), m=mm, q=qq,
                        sigma=np.array(sig[:dp.struct.s]), report=rep.as_dict())
        # U rows 0..m-1 are the retained columns; Pi is (rank_max x q_max) column-major
        return dict(U=U[:mm], Pi=Pi[:qq, :mm].T.contiguous() if mm else Pi[:0, :0], m=mm, q=qq,
                    sigma=np.array(sig[:dp.struct.s]), report=rep.as_dict())

    # -- S1-S8
    def solve_batch(self, problems: Sequence, precision: int = PE_FP64):
        dps = [make_problem(p, self.device, precision) for p in problems]
        arr = (PeProblem * len(dps))(*[d.struct for d in dps])
        reps = (PeReport * len(dps))()
        self._check(self.lib.pe_solve_batch(self.h, arr, len(dps), reps, _stream_ptr()))
        return [d.out for d in dps], [r.as_dict() for r in reps]

    def workspace_query(self, problems: Sequence, precision: int = PE_FP64) -> int:
        return workspace_query(problems, precision, self)

    def prepare(self, problems: Sequence, precision: int = PE_FP64):
        """Stage a batch on the device once (for repeated solves, e.g. benchmarking)."""
        dps = [make_problem(p, self.device, precision) for p in problems]
        arr = (PeProblem * len(dps))(*[d.struct for d in dps])
        return dict(dps=dps, arr=arr, reps=(PeReport * len(dps))())

    def solve_prepared(self, staged, stream=None):
        """pe_solve_batch on a staged batch; outputs land in staged['dps'][i].out."""
        self._check(self.lib.pe_solve_batch(self.h, staged["arr"], len(staged["dps"]), staged["reps"],
                                            _stream_ptr(stream)))
        return [d.out for d in staged["dps"]], [r.as_dict() for r in staged["reps"]]

    # -- S5-S8 with a given compressed source
    def expaction_batch(self, problems: Sequence, Us: Sequence, Pis: Sequence, precision: int = PE_FP64):
        """Us[i]: torch (m, n) rows = columns of U; Pis[i]: (m, q) numpy/torch Chebyshev coefficients."""
        torch = _torch()
        dps = [make_problem(p, self.device, precision) for p in problems]
        keep = []
        Uptr = (ctypes.c_void_p * len(dps))()
        Pptr = (ctypes.c_void_p * len(dps))()
        ms = (ctypes.c_int32 * len(dps))()
        qs = (ctypes.c_int32 * len(dps))()
        for i, (U, Pi) in enumerate(zip(Us, Pis)):
            U = _dev(U, self.device)
            Pi = _dev(Pi, self.device)
            m = int(U.shape[0]) if U.numel() else 0
            q = int(Pi.shape[1]) if m else 0
            Pcm = Pi.T.contiguous() if m else Pi   # column-major m x q == torch (q, m)
            keep += [U, Pcm]
            Uptr[i] = U.data_ptr() if m else None
            Pptr[i] = Pcm.data_ptr() if m else None
            ms[i], qs[i] = m, q
        arr = (PeProblem * len(dps))(*[d.struct for d in dps])
        reps = (PeReport * len(dps))()
        self._check(self.lib.pe_expaction_batch(self.h, arr, Uptr, Pptr, ms, qs, len(dps), reps, _stream_ptr()))
        return [d.out for d in dps], [r.as_dict() for r in reps]

    # -- tile autotuning
    def autotune(self, shapes, cache_path: Optional[str] = None) -> int:
        """pe_autotune on (n, rank_max, precision) triples; returns the number of keys timed."""
        shapes = list(shapes)
        arr = (PeProblem * max(1, len(shapes)))()
        for i, (n, rank_max, prec) in enumerate(shapes):
            arr[i].op.n = int(n)
            arr[i].rank_max = int(rank_max)
            arr[i].prec = int(prec)
        tuned = ctypes.c_int32()
        self._check(self.lib.pe_autotune(self.h, arr, len(shapes), cache_path.encode() if cache_path else None,
                                         ctypes.byref(tuned), _stream_ptr()))
        return tuned.value

    def autotune_table(self):
        """The context's tiling choices: {(log2n, width, mixed): (rows_u, rows_p)}."""
        k = self.lib.pe_autotune_table(self.h, None, 0)
        rows = (ctypes.c_int32 * (5 * max(1, k)))()
        self.lib.pe_autotune_table(self.h, rows, k)
        return {(rows[5 * i], rows[5 * i + 1], rows[5 * i + 2]): (rows[5 * i + 3], rows[5 * i + 4]) for i in range(k)}

    # -- kernel timing
    def profile_enable(self, family: Optional[str]):
        self._check(self.lib.pe_profile_enable(self.h, family.encode() if family else None))

    def profile_read(self):
        n = ctypes.c_int64()
        ms, by, fl = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.pe_profile_read(self.h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by),
                                             ctypes.byref(fl)))
        return dict(launches=n.value, ms=ms.value, bytes=by.value, flops=fl.value)

    # -- S10
    def wr_burgers(self, bp, precision: int = PE_FP64, u_init=None):
        """Waveform relaxation for Burgers (fields of a BurgersProblem-like object).

        Returns (U, reports, increments): U is a torch (P*s, n) tensor of the final
        iterate at every window sample (window-major), reports the P window solves of
        the last iteration, increments the K relative iterate changes."""
        torch = _torch()
        n, P, s, K = int(bp.n), int(bp.P), int(bp.s), int(bp.K)
        u0 = _dev(bp.u0, self.device)
        out = torch.empty((P * s, n), dtype=torch.float64, device=self.device)
        ui = _dev(u_init, self.device) if u_init is not None else None
        fo = getattr(bp, "forcing", None)
        # (n, P*s) samples, window-major columns -> device (P*s, n) rows, i.e. ld n
        fd = _dev(np.ascontiguousarray(np.asarray(fo, dtype=np.float64).T), self.device) if fo is not None else None
        wp = PeWrProblem(n=n, nu=float(bp.nu), T=float(bp.T), P=P, s=s, K=K, jacobian=int(bool(bp.jacobian)),
                         u0=u0.data_ptr(), u_init=ui.data_ptr() if ui is not None else None,
                         u_final=out.data_ptr(), krylov_steps=int(bp.krylov_steps), rank_max=int(bp.rank_max),
                         q_max=int(bp.q_max), tol=float(bp.tol), svd_tol=float(bp.svd_tol),
                         fit_tol=float(bp.fit_tol), prec=int(precision),
                         krylov=int(getattr(bp, "krylov", PE_KRYLOV_POLY)),
                         sai_shift=float(getattr(bp, "sai_shift", 0.0)),
                         forcing=fd.data_ptr() if fd is not None else None,
                         source_fit=int(getattr(bp, "source_fit", PE_FIT_CHEBYSHEV)))
        reps = (PeReport * P)()
        inc = (ctypes.c_double * max(K, 1))()
        self._check(self.lib.pe_wr_burgers(self.h, ctypes.byref(wp), reps, inc, _stream_ptr()))
        return out, [r.as_dict() for r in reps], list(inc[:K])

    # -- S8
    def superpose(self, u0, vs: Sequence):
        """u(t_k) = u0 + sum_j v_j(t_k); vs are torch (n_out, n) tensors."""
        torch = _torch()
        u0 = _dev(u0, self.device)
        n = int(u0.shape[0])
        n_out = int(vs[0].shape[0]) if vs else 0
        vs = [_dev(v, self.device) for v in vs]
        ptrs = (ctypes.c_void_p * max(len(vs), 1))(*[v.data_ptr() for v in vs])
        u = torch.empty((max(n_out, 1), n), dtype=torch.float64, device=self.device)
        self._check(self.lib.pe_superpose(self.h, ctypes.c_void_p(u0.data_ptr()), ptrs, len(vs), n, n_out, n,
                                          ctypes.c_void_p(u.data_ptr()), n, _stream_ptr()))
        return u[:n_out]
