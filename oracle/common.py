"""Greedy-policy rules shared by the oracle tiers (test infrastructure).

Eq. 1 of the paper takes a max over actions; it does not say which action to
report when several attain it.  The oracle's reading: report the lowest action
index among those within a tolerance tol = 1e-12 * max(1, ||V||_inf) of the
maximum, and during policy improvement keep the incumbent action unless it is
beaten by more than tol (Sec. 2.1: policy iteration ends when improvement
leaves the policy unchanged).
"""
import numpy as np

TIE_REL = 1e-12


def tie_tolerance(V) -> float:
    V = np.asarray(V, np.float64)
    return TIE_REL * max(1.0, float(np.max(np.abs(V))) if V.size else 1.0)


def greedy(Q: np.ndarray, V) -> np.ndarray:
    """Lowest action index a with Q[a, s] >= max_b Q[b, s] - tol."""
    tol = tie_tolerance(V)
    best = Q.max(axis=0)
    ok = Q >= best[None, :] - tol
    return np.argmax(ok, axis=0).astype(np.int32)


def improve(Q: np.ndarray, V, pi_old: np.ndarray) -> np.ndarray:
    """Greedy improvement that keeps the incumbent unless beaten by > tol."""
    tol = tie_tolerance(V)
    best = Q.max(axis=0)
    pi_new = greedy(Q, V)
    S = Q.shape[1]
    keep = Q[pi_old, np.arange(S)] >= best - tol
    return np.where(keep, pi_old, pi_new).astype(np.int32)


# Obstacles (Sec. 3.2: states the agent has no access to).  The paper does not
# say what a move towards an obstacle does; the oracle's reading: the agent
# stays where it is (as at the grid edge), and an obstacle state itself is
# outside the problem, with value 0 (no reward, no continuation).

def obstacle_mask(inst) -> np.ndarray:
    """bool [S]: obstacle states (all False when the instance has none)."""
    obs = getattr(inst, "obstacle", None)
    if obs is None:
        return np.zeros(inst.n_states, bool)
    return np.asarray(obs).astype(bool)


def rewards_of(inst) -> np.ndarray:
    """R(s), with 0 at obstacle states."""
    return np.where(obstacle_mask(inst), 0.0, inst.rewards)


def ended(inst) -> np.ndarray:
    """bool [S]: states with no continuation (terminal or obstacle)."""
    return (inst.terminal != 0) | obstacle_mask(inst)


def coords_of(sizes, s: int):
    """Multi-index of flat state s under the row-major order of Def. 2."""
    out = []
    for m in reversed([int(x) for x in sizes]):
        out.append(s % m)
        s //= m
    return tuple(reversed(out))
