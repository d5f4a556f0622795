"""ctypes binding of libnrto.so (argument marshalling only; every step of the
solve runs in the HIP library).  Names follow include/nrto.h.

Device buffers and streams come from PyTorch; host arrays are numpy float64.
Loading fails loudly if the library has not been built (python -m
paper_2603_02642_amd.build): there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnrto.so")

NRTO_OK, NRTO_MAXITER, NRTO_INFEASIBLE, NRTO_FALLBACK_COLD = 0, 1, 2, 3
NRTO_DR, NRTO_FULLADMM = 0, 1
NRTO_FP64, NRTO_FP32 = 0, 1
NRTO_WS_NO_GAINS = 2

_dp = C.POINTER(C.c_double)


class Problem(C.Structure):
    _fields_ = [("dyn", C.c_int32), ("nx", C.c_int32), ("nu", C.c_int32), ("T", C.c_int32),
                ("dt", C.c_double), ("radius", C.c_double), ("mass", C.c_double),
                ("inertia", _dp), ("links", _dp), ("x0", _dp), ("xg", _dp), ("Q", _dp),
                ("Ru", _dp), ("RK", _dp), ("n_obs", C.c_int32), ("obs", _dp),
                ("u_lo", _dp), ("u_hi", _dp), ("x_lo", _dp), ("x_hi", _dp), ("u_init", _dp)]


class Options(C.Structure):
    _fields_ = [("method", C.c_int32), ("precision", C.c_int32), ("max_admm", C.c_int32),
                ("max_inner", C.c_int32), ("check_every", C.c_int32), ("block_threads", C.c_int32),
                ("rho", C.c_double), ("alpha", C.c_double), ("sigma_chi", C.c_double),
                ("sigma_s", C.c_double), ("eps_dr_abs", C.c_double), ("eps_dr_rel", C.c_double),
                ("eps_kkt", C.c_double), ("r_trust", C.c_double), ("cold_init", C.c_int32),
                ("rho_adapt", C.c_int32), ("rho_mu", C.c_double), ("rho_tau", C.c_double),
                ("rho_min", C.c_double), ("rho_max", C.c_double), ("sigma_adapt", C.c_int32),
                ("sigma_every", C.c_int32), ("sigma_thr", C.c_double), ("sigma_min", C.c_double),
                ("sigma_max", C.c_double), ("infeas_window", C.c_int32), ("admm_chunk", C.c_int32)]


class SolveReport(C.Structure):
    _fields_ = [("status", C.c_int32), ("admm_iters", C.c_int32), ("inner_iters", C.c_int32),
                ("qp_newton", C.c_int32), ("kkt", C.c_double), ("r_p", C.c_double),
                ("r_d", C.c_double), ("mu", C.c_double), ("rho", C.c_double),
                ("t_dr_us", C.c_double), ("t_qp_us", C.c_double), ("t_kkt_us", C.c_double),
                ("t_total_us", C.c_double), ("sigma_s", C.c_double), ("sigma_updates", C.c_int32),
                ("nan_flag", C.c_int32)]


class SocpDev(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("A", "B", "xhat", "uhat", "g0", "w", "bhat", "bvec")]


class StateDev(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("st", "kt", "ptt", "du", "K", "p", "pt", "lam", "pi")]


class StepReport(C.Structure):
    _fields_ = [("accepted", C.c_int32), ("status", C.c_int32), ("merit_old", C.c_double),
                ("merit_new", C.c_double), ("predicted", C.c_double), ("r_trust", C.c_double),
                ("kkt", C.c_double), ("admm_iters", C.c_int32), ("inner_iters", C.c_int32)]


_lib = None


class NrtoError(RuntimeError):
    pass


def load() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise NrtoError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_02642_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    P = C.POINTER
    sig = {
        "nrto_default_options": (None, [P(Options)]),
        "nrto_project_soc": (i32, [vp, vp, vp, i64, i64, i32, i32, vp]),
        "nrto_project_soc_noalloc": (i32, [vp, vp, vp, i64, i64, i32, vp]),
        "nrto_setup": (i32, [P(Problem), i32, P(Options), vp, P(vp)]),
        "nrto_destroy": (None, [vp]),
        "nrto_last_error": (C.c_char_p, [vp]),
        "nrto_set_options": (i32, [vp, P(Options)]),
        "nrto_instance_sizes": (i32, [vp, i32, P(C.c_int64)]),
        "nrto_linearize": (i32, [vp]),
        "nrto_upload_socp": (i32, [vp, i32] + [_dp] * 8),
        "nrto_download_socp": (i32, [vp, i32] + [_dp] * 8),
        "nrto_solve_socp": (i32, [vp, i32, P(SolveReport)]),
        "nrto_solve_socp_dev": (i32, [vp, P(SocpDev), P(StateDev), i32, P(SolveReport)]),
        "nrto_get_solution": (i32, [vp, i32] + [_dp] * 7),
        "nrto_get_state": (i32, [vp, i32] + [_dp] * 4),
        "nrto_set_state": (i32, [vp, i32] + [_dp] * 9),
        "nrto_scp_step": (i32, [vp, P(StepReport)]),
        "nrto_scp_accept": (i32, [vp, P(StepReport)]),
        "nrto_get_reports": (i32, [vp, P(SolveReport)]),
        "nrto_capture_step": (i32, [vp, i32, i32]),
        "nrto_launch_step": (i32, [vp]),
        "nrto_get_nominal": (i32, [vp, i32, _dp, _dp]),
        "nrto_warm_start": (i32, [vp, vp, i64, i32, P(C.c_int32), _dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(st: int, ctx=None):
    if st < 0:
        msg = load().nrto_last_error(ctx)
        raise NrtoError(f"nrto status {st}: {msg.decode() if msg else ''}")
    return st


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def default_options(**kw) -> Options:
    o = Options()
    load().nrto_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def project_soc(x, seg_off, out=None, validate: bool = False, stream=None):
    """Projection of concatenated cones (torch tensors on the GPU; float64 or
    float32 values, int64 offsets of length n_cones + 1)."""
    import torch
    if out is None:
        out = torch.empty_like(x)
    dtype = 0 if x.dtype == torch.float64 else 1 if x.dtype == torch.float32 else -1
    if dtype < 0:
        raise TypeError("float64 or float32 values required")
    if not (x.is_cuda and seg_off.is_cuda and out.is_cuda):
        raise TypeError("device tensors required")
    if seg_off.dtype != torch.int64:
        raise TypeError("int64 offsets required")
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(load().nrto_project_soc(C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
                                   C.c_void_p(seg_off.data_ptr()), seg_off.numel() - 1, x.numel(),
                                   dtype, 1 if validate else 0, C.c_void_p(s)))
    return out


def project_soc_noalloc(x, seg_off, out=None, stream=None):
    """nrto_project_soc_noalloc: the validated projection without any device
    allocation inside the call (torch tensors on the GPU, as project_soc)."""
    import torch
    if out is None:
        out = torch.empty_like(x)
    dtype = 0 if x.dtype == torch.float64 else 1 if x.dtype == torch.float32 else -1
    if dtype < 0:
        raise TypeError("float64 or float32 values required")
    if not (x.is_cuda and seg_off.is_cuda and out.is_cuda):
        raise TypeError("device tensors required")
    if seg_off.dtype != torch.int64:
        raise TypeError("int64 offsets required")
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(load().nrto_project_soc_noalloc(C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
                                           C.c_void_p(seg_off.data_ptr()), seg_off.numel() - 1, x.numel(),
                                           dtype, C.c_void_p(s)))
    return out


class _ProblemHolder:
    """Keeps the numpy arrays behind one ctypes Problem alive."""

    def __init__(self, p):
        f = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        self.arrays = dict(x0=f(p.x0), xg=f(p.xg), Q=f(p.Q), Ru=f(p.Ru), RK=f(p.RK),
                           obs=f(p.obstacles.ravel()) if p.n_obs else None,
                           u_lo=f(p.u_lo), u_hi=f(p.u_hi), x_lo=f(p.x_lo), x_hi=f(p.x_hi),
                           u_init=f(p.u_init.ravel()), inertia=f(p.inertia), links=f(p.links))
        s = Problem()
        s.dyn, s.nx, s.nu, s.T = p.dyn, p.nx, p.nu, p.T
        s.dt, s.radius, s.mass = p.dt, p.radius, p.mass
        s.n_obs = p.n_obs
        for k, a in self.arrays.items():
            setattr(s, k, _ptr(a))
        self.struct = s


class Context:
    """A batch of problems on one stream."""

    def __init__(self, problems: Sequence, options: Optional[Options] = None, stream=None):
        import torch
        lib = load()
        self.problems = list(problems)
        self._holders = [_ProblemHolder(p) for p in self.problems]
        arr = (Problem * len(self._holders))(*[h.struct for h in self._holders])
        self._arr = arr
        self.options = options if options is not None else default_options()
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = C.c_void_p()
        _check(lib.nrto_setup(arr, len(self._holders), C.byref(self.options), C.c_void_p(stream), C.byref(h)))
        self.h = h
        self.n = len(self._holders)

    def close(self):
        if self.h:
            load().nrto_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_options(self, options: Options):
        self.options = options
        _check(load().nrto_set_options(self.h, C.byref(options)), self.h)

    def sizes(self, i: int) -> dict:
        out = (C.c_int64 * 7)()
        _check(load().nrto_instance_sizes(self.h, i, out), self.h)
        keys = ["ng", "nent", "nblk", "nstate", "T", "nx", "nu"]
        return {k: int(v) for k, v in zip(keys, out)}

    def linearize(self):
        _check(load().nrto_linearize(self.h), self.h)

    def upload_socp(self, i, A, B, xhat, uhat, g0, w, bhat, bvec):
        f = lambda a: np.ascontiguousarray(a, dtype=np.float64).ravel()
        arrs = [f(a) for a in (A, B, xhat, uhat, g0, w, bhat, bvec)]
        _check(load().nrto_upload_socp(self.h, i, *[_ptr(a) for a in arrs]), self.h)

    def download_socp(self, i) -> dict:
        s = self.sizes(i)
        T, nx, nu, ng = s["T"], s["nx"], s["nu"], s["ng"]
        out = dict(A=np.zeros(T * nx * nx), B=np.zeros(T * nx * nu), xhat=np.zeros((T + 1) * nx),
                   uhat=np.zeros(T * nu), g0=np.zeros(ng), w=np.zeros(ng * nx),
                   bhat=np.zeros(s["nent"]), bvec=np.zeros(s["nblk"] * nu))
        _check(load().nrto_download_socp(self.h, i, *[_ptr(out[k]) for k in
                                                       ("A", "B", "xhat", "uhat", "g0", "w", "bhat", "bvec")]), self.h)
        return out

    def solve(self, warm: bool = False) -> List[SolveReport]:
        rep = (SolveReport * self.n)()
        _check(load().nrto_solve_socp(self.h, 1 if warm else 0, rep), self.h)
        return list(rep)

    def solve_dev(self, socp: dict, state: dict, warm: bool = False, report: bool = True):
        """nrto_solve_socp_dev on caller-owned device tensors (float64, the
        concatenated per-instance layout): socp keys A, B, xhat, uhat, g0, w,
        bhat, bvec; state keys st, kt, ptt, du, K, p, pt, lam, pi."""
        sd = SocpDev(*[C.c_void_p(socp[k].data_ptr()) for k, _ in SocpDev._fields_])
        st = StateDev(*[C.c_void_p(state[k].data_ptr()) for k, _ in StateDev._fields_])
        rep = (SolveReport * self.n)() if report else None
        _check(load().nrto_solve_socp_dev(self.h, C.byref(sd), C.byref(st), 1 if warm else 0, rep), self.h)
        return list(rep) if report else None

    def solve_async(self, warm: bool = False):
        _check(load().nrto_solve_socp(self.h, 1 if warm else 0, None), self.h)

    def solution(self, i) -> dict:
        s = self.sizes(i)
        T, nx, nu, ng = s["T"], s["nx"], s["nu"], s["ng"]
        out = dict(du=np.zeros(T * nu), K=np.zeros(T * nu * nx), p=np.zeros(ng), pt=np.zeros(ng),
                   pi=np.zeros(ng), lam=np.zeros(ng), mu=np.zeros(1))
        _check(load().nrto_get_solution(self.h, i, *[_ptr(out[k]) for k in
                                                     ("du", "K", "p", "pt", "pi", "lam", "mu")]), self.h)
        out["K"] = out["K"].reshape(T, nu, nx)
        out["mu"] = float(out["mu"][0])
        return out

    def state(self, i) -> dict:
        s = self.sizes(i)
        T, nx, nu, ng = s["T"], s["nx"], s["nu"], s["ng"]
        out = dict(st=np.zeros(s["nent"]), nu=np.zeros(s["nent"]), kt=np.zeros(T * nu * nx), ptt=np.zeros(ng))
        _check(load().nrto_get_state(self.h, i, *[_ptr(out[k]) for k in ("st", "nu", "kt", "ptt")]), self.h)
        out["kt"] = out["kt"].reshape(T, nu, nx)
        return out

    def set_state(self, i, st=None, nu=None, kt=None, ptt=None, du=None, K=None, p=None, pt=None, lam=None):
        f = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64).ravel()
        arrs = [f(a) for a in (st, nu, kt, ptt, du, K, p, pt, lam)]
        _check(load().nrto_set_state(self.h, i, *[_ptr(a) for a in arrs]), self.h)

    def warm_start(self, pred, ld=None, fallback_test=True, gains=True):
        """Set the NRTO-DR state from prediction rows (torch float32 tensor on the GPU);
        gains=False: rows hold du, p~, pi only."""
        acc = np.zeros(self.n, dtype=np.int32)
        res = np.zeros(2 * self.n)
        ld = pred.shape[1] if ld is None else ld
        flags = (1 if fallback_test else 0) | (0 if gains else NRTO_WS_NO_GAINS)
        _check(load().nrto_warm_start(self.h, C.c_void_p(pred.data_ptr()), ld, flags,
                                      acc.ctypes.data_as(C.POINTER(C.c_int32)), _ptr(res)), self.h)
        return acc, res.reshape(self.n, 2)

    def scp_step(self) -> List[StepReport]:
        rep = (StepReport * self.n)()
        _check(load().nrto_scp_step(self.h, rep), self.h)
        return list(rep)

    def capture_step(self, warm: bool = False, with_linearize: bool = True):
        """Capture (linearise +) solve into a HIP graph (non-default stream only)."""
        _check(load().nrto_capture_step(self.h, 1 if warm else 0, 1 if with_linearize else 0), self.h)

    def launch_step(self):
        _check(load().nrto_launch_step(self.h), self.h)

    def reports(self) -> List[SolveReport]:
        rep = (SolveReport * self.n)()
        _check(load().nrto_get_reports(self.h, rep), self.h)
        return list(rep)

    def scp_accept(self) -> List[StepReport]:
        rep = (StepReport * self.n)()
        _check(load().nrto_scp_accept(self.h, rep), self.h)
        return list(rep)

    def nominal(self, i):
        s = self.sizes(i)
        T, nx, nu = s["T"], s["nx"], s["nu"]
        u = np.zeros(T * nu)
        K = np.zeros(T * nu * nx)
        _check(load().nrto_get_nominal(self.h, i, _ptr(u), _ptr(K)), self.h)
        return u.reshape(T, nu), K.reshape(T, nu, nx)


def _ws_sigs(lib):
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    fp = C.POINTER(C.c_float)
    sig = {
        "nrto_ws_create": (i32, [C.POINTER(C.c_int32), i32, i32, C.c_uint64, vp, C.POINTER(vp)]),
        "nrto_ws_destroy": (None, [vp]),
        "nrto_ws_set_norm": (i32, [vp, fp, fp, fp, fp]),
        "nrto_ws_infer": (i32, [vp, vp, i32, vp]),
        "nrto_ws_train_step": (i32, [vp, vp, vp, i32, C.c_float, fp]),
        "nrto_ws_gradients": (i32, [vp, vp, vp, i32, fp, fp]),
        "nrto_ws_params": (i32, [vp, fp, fp]),
        "nrto_ws_gemm_bf16": (i32, [vp, i64, i64, vp, i64, i64, i32, i32, i32, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args


def _fptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_float))


class WarmStartNet:
    """GELU MLP on the matrix cores (nrto_ws_*).  Tensors are torch float32 on the GPU."""

    def __init__(self, widths, max_batch, seed=0, stream=None):
        import torch
        lib = load()
        _ws_sigs(lib)
        self.widths = [int(w) for w in widths]
        self.max_batch = int(max_batch)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        arr = (C.c_int32 * len(self.widths))(*self.widths)
        h = C.c_void_p()
        _check(lib.nrto_ws_create(arr, len(self.widths), self.max_batch, seed, C.c_void_p(stream), C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            load().nrto_ws_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_norm(self, xmean, xstd, ymean, ystd):
        f = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float32)
        a = [f(x) for x in (xmean, xstd, ymean, ystd)]
        _check(load().nrto_ws_set_norm(self.h, *[_fptr(x) for x in a]))

    def infer(self, X, out=None):
        import torch
        if out is None:
            out = torch.empty((X.shape[0], self.widths[-1]), dtype=torch.float32, device=X.device)
        _check(load().nrto_ws_infer(self.h, C.c_void_p(X.data_ptr()), X.shape[0], C.c_void_p(out.data_ptr())))
        return out

    def train_step(self, X, T, lr=1e-3, want_loss=True):
        loss = np.zeros(1, dtype=np.float32)
        _check(load().nrto_ws_train_step(self.h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()), X.shape[0],
                                         float(lr), _fptr(loss) if want_loss else None))
        return float(loss[0])

    def _nparams(self):
        return sum(self.widths[l] * self.widths[l + 1] + self.widths[l + 1] for l in range(len(self.widths) - 1))

    def _split(self, flat):
        out, off = [], 0
        for l in range(len(self.widths) - 1):
            fi, fo = self.widths[l], self.widths[l + 1]
            W = flat[off:off + fi * fo].reshape(fo, fi)
            off += fi * fo
            b = flat[off:off + fo]
            off += fo
            out.append([W.copy(), b.copy()])
        return out

    def gradients(self, X, T):
        g = np.zeros(self._nparams(), dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        _check(load().nrto_ws_gradients(self.h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()), X.shape[0],
                                        _fptr(g), _fptr(loss)))
        return self._split(g), float(loss[0])

    def get_params(self):
        p = np.zeros(self._nparams(), dtype=np.float32)
        _check(load().nrto_ws_params(self.h, _fptr(p), None))
        return self._split(p)

    def set_params(self, params):
        flat = np.concatenate([np.concatenate([np.asarray(W, np.float32).ravel(), np.asarray(b, np.float32).ravel()])
                               for W, b in params]).astype(np.float32)
        _check(load().nrto_ws_params(self.h, None, _fptr(flat)))


def gemm_bf16(A_bits, sam, sak, B_bits, sbk, sbn, M, N, K, C_out, stream=None):
    """C_out (M x N float32) = A B on the matrix cores; A_bits, B_bits are int16 tensors of bf16 patterns."""
    import torch
    lib = load()
    _ws_sigs(lib)
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(lib.nrto_ws_gemm_bf16(C.c_void_p(A_bits.data_ptr()), sam, sak, C.c_void_p(B_bits.data_ptr()), sbk, sbn,
                                 M, N, K, C.c_void_p(C_out.data_ptr()), C.c_void_p(s)))
    return C_out
