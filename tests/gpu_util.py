"""Shared helpers of the GPU parity tests: layout conversion and the
tolerances of the parity contract.

Tolerances (FP32 kernels against the FP64 oracle at the same state):
  loss      |l - l_ref| <= 1e-5 * l_ref + 1e-30 * m_f   (a sum of
            non-negative terms, so relative; the absolute floor covers
            products below FP32's range)
  gradient  |g - g_ref| <= 1e-5 * (|g_ref| + A) + 1e-30 where A is the sum of
            the magnitudes of the summed contributions (the signed sum can
            cancel, so the bound is relative to what was summed)
  update    |x1 - x1_ref| <= 1e-5 * |x1_ref - x0| + 2^-24   (relative on the
            step, plus FP32's spacing near 1)
  counts    exact equality
"""
import sys

import numpy as np
import torch

import oracle

LOSS_RTOL = 1e-5
GRAD_RTOL = 1e-5
TINY = 1e-30
X_ULP = 2.0 ** -24


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def to_oracle(x: torch.Tensor, R: int) -> np.ndarray:
    """GPU state [n, ld] float32 -> oracle layout [R, n] float64 (exact)."""
    return x[:, :R].detach().to("cpu", torch.float64).t().contiguous().numpy()


def from_oracle(xr: np.ndarray, ld: int = None) -> torch.Tensor:
    R, n = xr.shape
    ld = ld or R
    out = torch.zeros((n, ld), dtype=torch.float32)
    out[:, :R] = torch.from_numpy(np.ascontiguousarray(xr.T)).float()
    return out.cuda()


def clause_counts(cnf) -> np.ndarray:
    return np.diff(cnf.formula_clause_begin).astype(np.float64)


def check_loss(loss_gpu: torch.Tensor, loss_ref: np.ndarray, cnf, what=""):
    got = loss_gpu.detach().cpu().numpy().astype(np.float64)
    tol = LOSS_RTOL * np.abs(loss_ref) + TINY * clause_counts(cnf)[:, None]
    bad = np.abs(got - loss_ref) > tol
    assert not bad.any(), (f"loss mismatch {what}: {bad.sum()} entries, worst "
                           f"{np.max(np.abs(got - loss_ref) / np.maximum(tol, 1e-300)):.3g} x tol")


def check_grad(grad_gpu: torch.Tensor, g_ref: np.ndarray, A: np.ndarray, R: int, what="",
               rows=None):
    got = to_oracle(grad_gpu, R)
    if rows is not None:
        got = got[rows]
    tol = GRAD_RTOL * (np.abs(g_ref) + A) + TINY
    err = np.abs(got - g_ref)
    bad = err > tol
    assert not bad.any(), (f"gradient mismatch {what}: {bad.sum()} of {bad.size}, worst "
                           f"{np.max(err / tol):.3g} x tol")
    if err.size == 0:  # no variables
        return 0.0
    return float(np.max(err / np.maximum(np.abs(g_ref) + A, 1e-300)))


def check_update(x1_gpu: torch.Tensor, x1_ref: np.ndarray, x0: np.ndarray, R: int, what=""):
    got = to_oracle(x1_gpu, R)
    tol = LOSS_RTOL * np.abs(x1_ref - x0) + X_ULP
    err = np.abs(got - x1_ref)
    bad = err > tol
    assert not bad.any(), f"update mismatch {what}: {bad.sum()} entries, worst {np.max(err / tol):.3g} x tol"


def check_update_oracle(x1_gpu: torch.Tensor, x0: np.ndarray, g_ref: np.ndarray, A: np.ndarray,
                        lr: float, R: int, what="", rows=None):
    """x_{k+1} of the fused step against the oracle's projected SGD step from
    the same x_k with the oracle's own gradient.  The gradient tolerance
    carries through the step (the clamp is a contraction): |x1 - x1_ref| <=
    lr * 1e-5 * (|g_ref| + A) + 1e-5 * |x1_ref - x0| + 2^-24."""
    got = to_oracle(x1_gpu, R)
    if rows is not None:
        got = got[rows]
    x1_ref = oracle.step_sgd(x0, g_ref, lr)
    tol = lr * GRAD_RTOL * (np.abs(g_ref) + A) + LOSS_RTOL * np.abs(x1_ref - x0) + X_ULP
    err = np.abs(got - x1_ref)
    bad = err > tol
    assert not bad.any(), (f"update mismatch {what}: {bad.sum()} of {bad.size}, worst "
                           f"{np.max(err / tol):.3g} x tol")


def check_counts(unsat_gpu: torch.Tensor, unsat_ref: np.ndarray, what=""):
    got = unsat_gpu.detach().cpu().numpy()
    assert np.array_equal(got, unsat_ref), f"unsat counts differ {what}: {(got != unsat_ref).sum()} entries"


def parity_at(prob, cnf, x: torch.Tensor, what="", upstream=None):
    """loss, gradient and rounded counts of the GPU at x against the oracle at x."""
    R = prob.R
    xr = to_oracle(x, R)
    lo_ref, g_ref, A = oracle.grad(cnf, xr, with_abs=True)
    up = None
    if upstream is not None:
        up = upstream.detach().cpu().numpy().astype(np.float64)  # [F, R]
        fov = cnf.formula_of_var()
        w = up[fov, :].T  # [R, n]
        g_ref = g_ref * w
        A = A * np.abs(w)
    loss, grad = prob.loss_grad(x, upstream=upstream)
    loss_only = prob.loss(x)
    unsat, best, assign = prob.round_check(x)
    torch.cuda.synchronize()
    check_loss(loss, lo_ref, cnf, what + " (loss_grad)")
    check_loss(loss_only, lo_ref, cnf, what + " (loss only)")
    rel = check_grad(grad, g_ref, A, R, what)
    us_ref = oracle.unsat(cnf, xr)
    check_counts(unsat, us_ref, what)
    best_ref = oracle.best(us_ref)
    assert np.array_equal(best.cpu().numpy(), best_ref), f"best restart differs {what}"
    a = assign.cpu().numpy()
    fov = cnf.formula_of_var()
    want = (xr[best_ref[fov], np.arange(cnf.n)] > 0.5).astype(np.uint8) if cnf.n else a
    assert np.array_equal(a, want), f"best assignment differs {what}"
    return rel
