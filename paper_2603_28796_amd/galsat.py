"""Python binding of libgalsat (ctypes; argument marshalling only).

Every step of the computation runs in the HIP library: this module passes
torch tensors' device pointers and the current HIP stream to the C ABI of
``include/galsat.h`` and raises on any non-OK status.  When the shared
library is missing it raises instead of computing anything on the CPU.

Shapes: a state ``x`` is a float32 CUDA tensor ``[n, ld]`` (``ld >= R``,
row stride ``ld``, unit column stride) whose first R columns are the
restarts; per-(formula, restart) outputs are ``[F, R]``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgalsat.so")

OPT = {"sgd": 0, "sgd_clamp": 0, "adam": 1}
PARTIALS = {"auto": 0, "store": 1, "recompute": 2}
SCHEDULE = {"auto": 0, "general": 1, "lds": 2, "plain": 3}
SCHEDULE_NAME = {v: k for k, v in SCHEDULE.items()}

_P = ctypes.c_void_p
_I32 = ctypes.c_int32


class _Problem(ctypes.Structure):
    _fields_ = [
        ("num_formulas", _I32),
        ("formula_var_begin", _P),
        ("formula_clause_begin", _P),
        ("n_vars", _I32),
        ("n_clauses", _I32),
        ("n_lits", _I32),
        ("clause_ptr", _P),
        ("clause_lits", _P),
        ("var_ptr", _P),
        ("var_occ", _P),
        ("restarts", _I32),
        ("inputs_on_device", _I32),
    ]


class _Options(ctypes.Structure):
    _fields_ = [
        ("optimizer", _I32),
        ("lr", ctypes.c_float),
        ("beta1", ctypes.c_float),
        ("beta2", ctypes.c_float),
        ("eps", ctypes.c_float),
        ("partials", _I32),
        ("recompute_max_len", _I32),
        ("workspace_budget_bytes", ctypes.c_size_t),
        ("validate", _I32),
        ("schedule", _I32),
        ("use_graph", _I32),
        ("plan_override", ctypes.c_char_p),
    ]


class _Info(ctypes.Structure):
    _fields_ = [
        ("num_formulas", _I32), ("n_vars", _I32), ("n_clauses", _I32), ("n_lits", _I32),
        ("restarts", _I32), ("max_clause_len", _I32), ("recompute_max_len", _I32),
        ("stored_lits", ctypes.c_int64), ("schedule", _I32), ("lanes_per_item", _I32),
        ("restarts_per_lane", _I32), ("var_chunks", _I32), ("clause_chunks", _I32),
        ("two_phase", _I32), ("xseq_chunks", _I32), ("device_bytes", ctypes.c_size_t), ("adam_step", _I32),
        ("lds_restarts_per_group", _I32), ("lds_staged", _I32), ("flat", _I32),
        ("clause_rows", _I32),
    ]


# every symbol include/galsat.h declares
EXPORTS = ("galsat_default_options", "galsat_create", "galsat_destroy", "galsat_init_state",
           "galsat_loss_grad", "galsat_step", "galsat_step_prepare", "galsat_gumbel_step",
           "galsat_gumbel_noise", "galsat_candidates", "galsat_confidence",
           "galsat_select_vars", "galsat_round_check", "galsat_round_check_static",
           "galsat_set_adam_step",
           "galsat_autotune", "galsat_get_info", "galsat_profile", "galsat_kernel_times",
           "galsat_tseitin",
           "galsat_status_string", "galsat_last_error")

KERNEL_KINDS = ("var_pass", "clause_pass", "finalize", "copy", "pack", "count", "select",
                "occ_pass", "var_sum", "seg_pass", "heavy")


class _KernelTimes(ctypes.Structure):
    _fields_ = [("launches", _I32 * len(KERNEL_KINDS)),
                ("total_ms", ctypes.c_double * len(KERNEL_KINDS))]

_lib = None


class GalsatError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def load_library(path: Optional[str] = None):
    """Load libgalsat.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libgalsat.so not found at {p}: build it first "
                           "(python -c 'import __graft_entry__; __graft_entry__.build()')")
    lib = ctypes.CDLL(p)
    lib.galsat_default_options.argtypes = [ctypes.POINTER(_Options)]
    lib.galsat_default_options.restype = None
    lib.galsat_create.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(_Options), _P,
                                  ctypes.POINTER(_P)]
    lib.galsat_destroy.argtypes = [_P]
    lib.galsat_init_state.argtypes = [_P, _P, _I32, ctypes.c_uint64, _P]
    lib.galsat_loss_grad.argtypes = [_P, _P, _I32, _P, _P, _P, _P]
    lib.galsat_step.argtypes = [_P, _P, _I32, _P, _I32, _P, _P, _P]
    lib.galsat_step_prepare.argtypes = [_P, _P, _I32, _P, _I32, _P, _P]
    lib.galsat_gumbel_step.argtypes = [_P, _P, _I32, _P, ctypes.c_uint64, _I32, _I32,
                                       ctypes.c_float, _P, _P, _P, _P]
    lib.galsat_gumbel_noise.argtypes = [_P, ctypes.c_uint64, _I32, _P, _I32, _P]
    lib.galsat_candidates.argtypes = [_P, _P, _I32, _P, _I32, ctypes.c_uint64, ctypes.c_float, _P,
                                      _P, _P]
    lib.galsat_confidence.argtypes = [_P, _P, _I32, _P, ctypes.c_float, _P, _P]
    lib.galsat_select_vars.argtypes = [_P, _P, _I32, _I32, ctypes.c_float, _I32, _P, _P, _P]
    lib.galsat_round_check.argtypes = [_P, _P, _I32, _P, _P, _P, _P]
    lib.galsat_round_check_static.argtypes = [_P, _P, _I32, _P, _P, _P, _P]
    lib.galsat_set_adam_step.argtypes = [_P, _I32]
    lib.galsat_get_info.argtypes = [_P, ctypes.POINTER(_Info)]
    lib.galsat_profile.argtypes = [_P, _I32]
    lib.galsat_kernel_times.argtypes = [_P, ctypes.POINTER(_KernelTimes)]
    lib.galsat_tseitin.argtypes = [_I32, _I32, _I32, _P, _P, _P, _P, _P, _P, _P]
    lib.galsat_autotune.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(_Options), _P, _I32,
                                    _I32, _P, ctypes.c_char_p, _I32, ctypes.POINTER(ctypes.c_double)]
    lib.galsat_autotune.restype = ctypes.c_int
    lib.galsat_tseitin.restype = ctypes.c_int
    lib.galsat_status_string.argtypes = [ctypes.c_int]
    lib.galsat_status_string.restype = ctypes.c_char_p
    lib.galsat_last_error.argtypes = [_P]
    lib.galsat_last_error.restype = ctypes.c_char_p
    for fn in ("galsat_create", "galsat_destroy", "galsat_init_state", "galsat_loss_grad",
               "galsat_step", "galsat_step_prepare", "galsat_gumbel_step", "galsat_gumbel_noise",
               "galsat_candidates", "galsat_confidence", "galsat_select_vars",
               "galsat_round_check", "galsat_set_adam_step",
               "galsat_get_info",
               "galsat_profile", "galsat_kernel_times"):
        getattr(lib, fn).restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _state_ld(x: torch.Tensor, n: int, R: int, name: str = "x") -> int:
    if not (x.is_cuda and x.dtype == torch.float32 and x.dim() == 2):
        raise ValueError(f"{name} must be a float32 CUDA tensor [n, ld]")
    if x.shape[0] != n or x.shape[1] < R or x.stride(1) != 1 or (n > 1 and x.stride(0) < R):
        raise ValueError(f"{name} must be [n={n}, ld>={R}] with unit column stride")
    return int(x.stride(0)) if n > 1 else int(max(x.shape[1], R))


def _structs(cnf, restarts, optimizer="sgd", lr=0.1, beta1=0.9, beta2=0.999, eps=1e-8,
             partials="auto", recompute_max_len=0, workspace_budget_bytes=0, validate=True,
             schedule="auto", use_graph=False, plan_override=None):
    """(problem struct, options struct, arrays kept alive)."""
    lib = load_library()
    keep = [np.ascontiguousarray(a, dtype=np.int32) for a in
            (cnf.formula_var_begin, cnf.formula_clause_begin, cnf.clause_ptr, cnf.clause_lits,
             cnf.var_ptr, cnf.var_occ)]
    fvb, fcb, cp, cl, vp, vo = keep
    prob = _Problem(cnf.F, fvb.ctypes.data, fcb.ctypes.data, cnf.n, cnf.m, cnf.L,
                    cp.ctypes.data, cl.ctypes.data, vp.ctypes.data, vo.ctypes.data, int(restarts), 0)
    opt = _Options()
    lib.galsat_default_options(ctypes.byref(opt))
    opt.optimizer = OPT[optimizer]
    opt.lr, opt.beta1, opt.beta2, opt.eps = lr, beta1, beta2, eps
    opt.partials = PARTIALS[partials]
    opt.recompute_max_len = recompute_max_len
    opt.workspace_budget_bytes = workspace_budget_bytes
    opt.validate = 1 if validate else 0
    opt.schedule = SCHEDULE[schedule]
    opt.use_graph = 1 if use_graph else 0
    ov = plan_override.encode() if plan_override else None
    keep.append(ov)
    opt.plan_override = ov
    return prob, opt, keep


def autotune(cnf, restarts: int, x0: torch.Tensor, steps: int = 5, **options):
    """Time the candidate plans on `steps` real steps from x0; returns
    (plan string, ms per step)."""
    lib = load_library()
    prob, opt, keep = _structs(cnf, restarts, **options)
    ld = _state_ld(x0, cnf.n, int(restarts), "x0")
    buf = ctypes.create_string_buffer(256)
    best = ctypes.c_double()
    st = lib.galsat_autotune(ctypes.byref(prob), ctypes.byref(opt), _ptr(x0), ld, int(steps),
                             _stream(), buf, 256, ctypes.byref(best))
    if st != 0:
        raise GalsatError(st, "galsat_autotune", lib.galsat_last_error(None).decode())
    return buf.value.decode(), best.value


class Problem:
    """A handle on one batch of formulas with R restarts each."""

    def __init__(self, cnf, restarts: int, *, optimizer: str = "sgd", lr: float = 0.1,
                 beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                 partials: str = "auto", recompute_max_len: int = 0,
                 workspace_budget_bytes: int = 0, validate: bool = True, schedule: str = "auto",
                 use_graph: bool = False, plan_override: Optional[str] = None):
        self._lib = load_library()
        self._h = None
        self.n, self.m, self.L, self.F, self.R = cnf.n, cnf.m, cnf.L, cnf.F, int(restarts)
        keep = [np.ascontiguousarray(a, dtype=np.int32) for a in
                (cnf.formula_var_begin, cnf.formula_clause_begin, cnf.clause_ptr,
                 cnf.clause_lits, cnf.var_ptr, cnf.var_occ)]
        fvb, fcb, cp, cl, vp, vo = keep
        prob = _Problem(self.F, fvb.ctypes.data, fcb.ctypes.data, self.n, self.m, self.L,
                        cp.ctypes.data, cl.ctypes.data, vp.ctypes.data, vo.ctypes.data,
                        self.R, 0)
        opt = _Options()
        self._lib.galsat_default_options(ctypes.byref(opt))
        opt.optimizer = OPT[optimizer]
        opt.lr, opt.beta1, opt.beta2, opt.eps = lr, beta1, beta2, eps
        opt.partials = PARTIALS[partials]
        opt.recompute_max_len = recompute_max_len
        opt.workspace_budget_bytes = workspace_budget_bytes
        opt.validate = 1 if validate else 0
        opt.schedule = SCHEDULE[schedule]
        opt.use_graph = 1 if use_graph else 0
        self._override = plan_override.encode() if plan_override else None
        opt.plan_override = self._override
        self.optimizer = optimizer
        self.lr = float(np.float32(lr))
        h = ctypes.c_void_p()
        st = self._lib.galsat_create(ctypes.byref(prob), ctypes.byref(opt), _stream(), ctypes.byref(h))
        if st != 0:
            raise GalsatError(st, "galsat_create", self._lib.galsat_last_error(None).decode())
        self._h = h

    # -- lifetime
    def close(self):
        if self._h is not None:
            self._lib.galsat_destroy(self._h)
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

    def _check(self, st: int, where: str):
        if st != 0:
            raise GalsatError(st, where, self._lib.galsat_last_error(self._h).decode())

    # -- calls
    def new_state(self, ld: Optional[int] = None) -> torch.Tensor:
        ld = ld or self.R
        return torch.empty((self.n, ld), dtype=torch.float32, device="cuda")

    def init_state(self, seed: int, x: Optional[torch.Tensor] = None) -> torch.Tensor:
        if x is None:
            x = self.new_state()
        ld = _state_ld(x, self.n, self.R)
        self._check(self._lib.galsat_init_state(self._h, _ptr(x), ld, ctypes.c_uint64(seed), _stream()),
                    "galsat_init_state")
        return x

    def loss_grad(self, x: torch.Tensor, upstream: Optional[torch.Tensor] = None,
                  want_grad: bool = True, grad: Optional[torch.Tensor] = None):
        """Returns (loss [F, R], grad [n, ld] or None)."""
        ld = _state_ld(x, self.n, self.R)
        loss = torch.empty((self.F, self.R), dtype=torch.float32, device=x.device)
        if want_grad and grad is None:
            # same strides as x (a column slice of a wider tensor keeps its
            # row stride); columns past R are never written by the kernels,
            # so they start at zero rather than uninitialised
            grad = torch.empty_strided(x.size(), x.stride(), dtype=torch.float32, device=x.device)
            if x.shape[1] > self.R:
                grad[:, self.R:].zero_()
        if grad is not None:
            gl = _state_ld(grad, self.n, self.R, "grad")
            if gl != ld:
                raise ValueError("grad must have the same row stride as x")
        if upstream is not None:
            upstream = upstream.to(device=x.device, dtype=torch.float32).contiguous()
            if upstream.numel() != self.F * self.R:
                raise ValueError("upstream must have F*R elements")
        self._check(self._lib.galsat_loss_grad(self._h, _ptr(x), ld, _ptr(upstream), _ptr(loss),
                                               _ptr(grad if want_grad else None), _stream()),
                    "galsat_loss_grad")
        return loss, (grad if want_grad else None)

    def loss(self, x: torch.Tensor) -> torch.Tensor:
        return self.loss_grad(x, want_grad=False)[0]

    def new_opt_state(self, x: torch.Tensor) -> torch.Tensor:
        return torch.zeros((2,) + tuple(x.shape), dtype=torch.float32, device=x.device)

    def step(self, x: torch.Tensor, steps: int = 1, opt_state: Optional[torch.Tensor] = None,
             trace: bool = False, loss_trace: Optional[torch.Tensor] = None,
             unsat_trace: Optional[torch.Tensor] = None):
        """Runs `steps` fused iterations in place on x.  With trace=True
        returns (loss_trace [steps, F, R], unsat_trace [steps, F, R])."""
        ld = _state_ld(x, self.n, self.R)
        if self.optimizer == "adam":
            if opt_state is None:
                raise ValueError("Adam needs opt_state (see new_opt_state)")
            if opt_state.shape != (2,) + tuple(x.shape) or not opt_state.is_contiguous() or \
                    x.stride(0) != x.shape[1]:
                raise ValueError("opt_state must be a contiguous [2, n, ld] tensor matching x")
        if trace:
            if loss_trace is None:
                loss_trace = torch.empty((steps, self.F, self.R), dtype=torch.float32, device=x.device)
            if unsat_trace is None:
                unsat_trace = torch.empty((steps, self.F, self.R), dtype=torch.int32, device=x.device)
        self._check(self._lib.galsat_step(self._h, _ptr(x), ld, _ptr(opt_state), int(steps),
                                          _ptr(loss_trace), _ptr(unsat_trace), _stream()),
                    "galsat_step")
        return (loss_trace, unsat_trace) if trace else None

    def gumbel_step(self, d: torch.Tensor, steps: int = 1, opt_state: Optional[torch.Tensor] = None,
                    seed: int = 0, step0: int = 0, tau: float = 1.0,
                    noise: Optional[torch.Tensor] = None, trace: bool = False):
        """Straight-through Gumbel steps on the logit differences d [n, ld]
        (in place).  With trace=True returns (loss_trace, unsat_trace)."""
        ld = _state_ld(d, self.n, self.R, "d")
        if self.optimizer == "adam" and opt_state is None:
            raise ValueError("Adam needs opt_state (see new_opt_state)")
        if noise is not None:
            if noise.shape[-2:] != d.shape or not noise.is_contiguous() or d.stride(0) != d.shape[1]:
                raise ValueError("noise must be a contiguous [steps, n, ld] tensor matching d")
        lt = ut = None
        if trace:
            lt = torch.empty((steps, self.F, self.R), dtype=torch.float32, device=d.device)
            ut = torch.empty((steps, self.F, self.R), dtype=torch.int32, device=d.device)
        self._check(self._lib.galsat_gumbel_step(self._h, _ptr(d), ld, _ptr(opt_state),
                                                 ctypes.c_uint64(seed), int(step0), int(steps),
                                                 float(tau), _ptr(noise), _ptr(lt), _ptr(ut),
                                                 _stream()), "galsat_gumbel_step")
        return (lt, ut) if trace else None

    def gumbel_noise(self, seed: int, step: int, ld: Optional[int] = None) -> torch.Tensor:
        out = torch.zeros((self.n, ld or self.R), dtype=torch.float32, device="cuda")
        self._check(self._lib.galsat_gumbel_noise(self._h, ctypes.c_uint64(seed), int(step),
                                                  _ptr(out), out.shape[1], _stream()),
                    "galsat_gumbel_noise")
        return out

    def candidates(self, d: torch.Tensor, best: torch.Tensor, num: int = 100, seed: int = 0,
                   tau: float = 1.0):
        """Candidate pool (Eq. 8): (assign [num, n] uint8, conf [num, n])."""
        ld = _state_ld(d, self.n, self.R, "d")
        best = best.to(device=d.device, dtype=torch.int32).contiguous()
        assign = torch.empty((num, self.n), dtype=torch.uint8, device=d.device)
        conf = torch.empty((num, self.n), dtype=torch.float32, device=d.device)
        self._check(self._lib.galsat_candidates(self._h, _ptr(d), ld, _ptr(best), int(num),
                                                ctypes.c_uint64(seed), float(tau), _ptr(assign),
                                                _ptr(conf), _stream()), "galsat_candidates")
        return assign, conf

    def confidence(self, d: torch.Tensor, best: torch.Tensor, tau: float = 1.0) -> torch.Tensor:
        ld = _state_ld(d, self.n, self.R, "d")
        best = best.to(device=d.device, dtype=torch.int32).contiguous()
        conf = torch.empty((1, self.n), dtype=torch.float32, device=d.device)
        self._check(self._lib.galsat_confidence(self._h, _ptr(d), ld, _ptr(best), float(tau),
                                                _ptr(conf), _stream()), "galsat_confidence")
        return conf

    def select_vars(self, conf: torch.Tensor, highest: bool = True, frac: float = 0.0005,
                    min_count: int = 1):
        """Returns (offsets [F+1] numpy, ids [num, offsets[-1]] int32 tensor)."""
        conf = conf.to(dtype=torch.float32).contiguous()
        num = conf.shape[0]
        off = np.zeros(self.F + 1, dtype=np.int32)
        self._check(self._lib.galsat_select_vars(self._h, None, num, 1 if highest else 0,
                                                 float(frac), int(min_count), off.ctypes.data, None,
                                                 _stream()), "galsat_select_vars")
        out = torch.empty((num, max(int(off[-1]), 1)), dtype=torch.int32, device=conf.device)
        self._check(self._lib.galsat_select_vars(self._h, _ptr(conf), num, 1 if highest else 0,
                                                 float(frac), int(min_count), off.ctypes.data,
                                                 _ptr(out), _stream()), "galsat_select_vars")
        return off, out[:, :int(off[-1])]

    def prepare(self, x: torch.Tensor, steps: int, loss_trace: Optional[torch.Tensor] = None,
                unsat_trace: Optional[torch.Tensor] = None):
        """Capture the graph of step(x, steps, ...) without running it."""
        ld = _state_ld(x, self.n, self.R)
        self._check(self._lib.galsat_step_prepare(self._h, _ptr(x), ld, None, int(steps),
                                                  _ptr(loss_trace), _ptr(unsat_trace)),
                    "galsat_step_prepare")

    def round_check(self, x: torch.Tensor, want_assign: bool = True):
        """Returns (unsat [F, R] int32, best_restart [F] int32, assignment [n] uint8)."""
        ld = _state_ld(x, self.n, self.R)
        unsat = torch.empty((self.F, self.R), dtype=torch.int32, device=x.device)
        best = torch.empty(self.F, dtype=torch.int32, device=x.device)
        assign = torch.empty(self.n, dtype=torch.uint8, device=x.device) if want_assign else None
        self._check(self._lib.galsat_round_check(self._h, _ptr(x), ld, _ptr(unsat), _ptr(best),
                                                 _ptr(assign), _stream()), "galsat_round_check")
        return unsat, best, assign

    def round_check_static(self, x: torch.Tensor, unsat: torch.Tensor, best: Optional[torch.Tensor] = None,
                           assign: Optional[torch.Tensor] = None):
        """galsat_round_check_static into caller-provided buffers (unsat [F, R]
        int32, best [F] int32 or None, assign [n] uint8 or None): the library
        allocates nothing during the call."""
        ld = _state_ld(x, self.n, self.R)
        if unsat.dtype != torch.int32 or unsat.numel() != self.F * self.R or not unsat.is_contiguous():
            raise ValueError("unsat must be a contiguous int32 tensor of F*R elements")
        if best is not None and (best.dtype != torch.int32 or best.numel() != self.F):
            raise ValueError("best must be an int32 tensor of F elements")
        if assign is not None and (assign.dtype != torch.uint8 or assign.numel() != self.n):
            raise ValueError("assign must be a uint8 tensor of n elements")
        self._check(self._lib.galsat_round_check_static(self._h, _ptr(x), ld, _ptr(unsat), _ptr(best),
                                                        _ptr(assign), _stream()),
                    "galsat_round_check_static")

    def set_adam_step(self, t: int):
        self._check(self._lib.galsat_set_adam_step(self._h, int(t)), "galsat_set_adam_step")

    def profile(self, enable: bool = True):
        """Start (clearing the record) or stop per-kernel event timing."""
        self._check(self._lib.galsat_profile(self._h, 1 if enable else 0), "galsat_profile")

    def kernel_times(self) -> dict:
        """{kind: (launches, total_ms)} of the launches recorded while profiling."""
        kt = _KernelTimes()
        self._check(self._lib.galsat_kernel_times(self._h, ctypes.byref(kt)), "galsat_kernel_times")
        return {k: (int(kt.launches[i]), float(kt.total_ms[i])) for i, k in enumerate(KERNEL_KINDS)
                if kt.launches[i]}

    def info(self) -> dict:
        inf = _Info()
        self._check(self._lib.galsat_get_info(self._h, ctypes.byref(inf)), "galsat_get_info")
        d = {k: getattr(inf, k) for k, _ in _Info._fields_}
        d["schedule"] = SCHEDULE_NAME.get(d["schedule"], d["schedule"])
        return d


def tseitin(cnf, width: int = 3):
    """Fixed-width chain normalization of a single formula (galsat_tseitin,
    host code).  Returns a CNF with the auxiliary variables appended after
    the original ones."""
    from . import inputs as I

    if cnf.F != 1:
        raise ValueError("normalize one formula at a time (CNF.sub)")
    lib = load_library()
    cp = np.ascontiguousarray(cnf.clause_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(cnf.clause_lits, dtype=np.int32)
    nv, nm, nl = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    args = (int(width), cnf.n, cnf.m, cp.ctypes.data, cl.ctypes.data if cl.size else None,
            ctypes.byref(nv), ctypes.byref(nm), ctypes.byref(nl))
    st = lib.galsat_tseitin(*args, None, None)
    if st != 0:
        raise GalsatError(st, "galsat_tseitin", lib.galsat_status_string(st).decode())
    ocp = np.empty(nm.value + 1, dtype=np.int32)
    ocl = np.empty(max(nl.value, 1), dtype=np.int32)
    st = lib.galsat_tseitin(*args, ocp.ctypes.data, ocl.ctypes.data)
    if st != 0:
        raise GalsatError(st, "galsat_tseitin", lib.galsat_status_string(st).decode())
    return I.csr_from_clause_major(nv.value, ocp, ocl[:nl.value], name=f"{cnf.name}/w{width}")


class GalsatLoss(torch.autograd.Function):
    """loss'[F, R] of x as an autograd node.

    Forward evaluates the clause polynomial only (nothing but x is saved);
    backward recomputes the clause products inside the library and scales
    each restart's gradient by the incoming gradient of its loss entry.
    """

    @staticmethod
    def forward(ctx, x: torch.Tensor, problem: Problem):
        ctx.problem = problem
        ctx.save_for_backward(x)
        return problem.loss(x)

    @staticmethod
    def backward(ctx, gloss: torch.Tensor):
        (x,) = ctx.saved_tensors
        _, grad = ctx.problem.loss_grad(x, upstream=gloss.contiguous())
        return grad, None


def galsat_loss(x: torch.Tensor, problem: Problem) -> torch.Tensor:
    return GalsatLoss.apply(x, problem)
