"""Helpers of the GPU parity tests (imported by test modules; not collected).

Tolerances (values compared element by element with the FP64 oracle):
  FP64 results      : |V - V*| <= 1e-9
  FP32 results      : |V - V*| <= 1e-5 * max(1, ||V*||_inf)
  BF16 one backup   : |V - V*| <= 1e-3 * max(1, ||V*||_inf)
Policies: equal wherever the oracle's best action beats the runner-up by
more than twice the value tolerance; at the remaining (near-)ties the GPU's
action must be within twice the tolerance of the oracle's maximum (several
policies are then correct).
"""
import sys

import numpy as np

TOL_FP64 = 1e-9
TOL_FP32_REL = 1e-5
TOL_BF16_REL = 1e-3


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def tol_for(precision, vref):
    scale = max(1.0, float(np.max(np.abs(vref))))
    return {0: TOL_FP64, 1: TOL_FP32_REL * scale, 2: TOL_BF16_REL * scale}[precision]


def compare_policy(pi_gpu, Q, tol, exact_ties=False):
    """pi_gpu vs the oracle Q-values [A, S] (see module docstring).  Returns
    (number of clearly decided states, number of near-tie states)."""
    A, S = Q.shape
    pi_gpu = np.asarray(pi_gpu, np.int64)
    assert pi_gpu.shape == (S,)
    assert np.all((pi_gpu >= 0) & (pi_gpu < A))
    best = Q.max(axis=0)
    srt = np.sort(Q, axis=0)
    gap = srt[-1] - srt[-2] if A > 1 else np.full(S, np.inf)
    clear = gap > 2 * tol
    oracle_pi = np.argmax(Q, axis=0)
    bad = np.nonzero(clear & (pi_gpu != oracle_pi))[0]
    assert bad.size == 0, f"{bad.size} clear states differ, e.g. {bad[:5]}"
    chosen = Q[pi_gpu, np.arange(S)]
    assert np.all(best - chosen <= 2 * tol + 1e-15), float(np.max(best - chosen))
    return int(clear.sum()), int((~clear).sum())


def assert_close(got, ref, tol, what=""):
    err = float(np.max(np.abs(np.asarray(got, np.float64) - ref))) if ref.size else 0.0
    assert err <= tol, f"{what}: max error {err:.3e} > {tol:.3e}"
    return err
