"""O1: tabular FP64 oracle over the explicitly reconstructed dense P_a
(test infrastructure; tiny state spaces only).

P_a is expanded as a sum of Kronecker products of the per-dimension factors,
P_a = sum_r lambda_{a,r} kron(T^(1), kron(T^(2), ...)) -- the CP form, a sum of
rank-one terms (Sec. 2.2), in the row-major state order of Def. 2 (np.kron
makes its first operand the slowest index).  Terminal rows have no
continuation (Sec. 3.2).  With obstacles, the probability of every move into
an obstacle is moved onto the source state itself (the agent stays put), and
an obstacle state has value 0 (see ``common``).  The backup is Eq. 1:
    V(s) = R(s) + gamma * max_a sum_s' P(s'|s,a) V(s').
"""
import itertools

import numpy as np

from .common import ended, greedy, improve, obstacle_mask, rewards_of

MAX_DENSE_STATES = 8192


def transition_matrices(inst) -> np.ndarray:
    """[A, S, S] FP64 with P[a, s, s'] = P(s' | s, a)."""
    S, A = inst.n_states, inst.n_actions
    if S > MAX_DENSE_STATES:
        raise ValueError(f"dense oracle limited to {MAX_DENSE_STATES} states")
    P = np.zeros((A, S, S))
    for a in range(A):
        for r, t in enumerate(inst.terms_of(a)):
            K = np.ones((1, 1))
            for k in range(inst.n_dims):
                K = np.kron(K, inst.factor(t, k))
            P[a] += inst.lambdas[t] * K
    obs = obstacle_mask(inst)
    if obs.any():
        # a move into an obstacle leaves the agent at s: column o's mass
        # joins the diagonal, column o becomes zero
        blocked = P[:, :, obs].sum(axis=2)               # [A, S]
        P[:, :, obs] = 0.0
        P[:, np.arange(S), np.arange(S)] += blocked
    return P


def continuation(inst) -> np.ndarray:
    """gamma per state, 0 at terminal and obstacle states."""
    return inst.gamma * (1.0 - ended(inst).astype(np.float64))


def q_values(inst, P, V) -> np.ndarray:
    """Q[a, s] = R(s) + gamma (1 - tau(s)) (P_a V)(s)."""
    c = continuation(inst)
    return rewards_of(inst)[None, :] + c[None, :] * np.einsum("ast,t->as", P, V)


def value_iteration(inst, eps=1e-13, max_iter=100000, V0=None, P=None):
    """Sweeps V <- max_a Q_a(V) until ||V' - V||_inf <= eps (Sec. 2.1).
    Returns (V, pi, sweeps, residual) with residual = ||B V - V||_inf of the
    returned V and pi greedy with respect to it."""
    if P is None:
        P = transition_matrices(inst)
    V = np.zeros(inst.n_states) if V0 is None else np.array(V0, np.float64)
    sweeps = 0
    while sweeps < max_iter:
        Vn = q_values(inst, P, V).max(axis=0)
        sweeps += 1
        res = np.max(np.abs(Vn - V))
        V = Vn
        if res <= eps:
            break
    Q = q_values(inst, P, V)
    res = float(np.max(np.abs(Q.max(axis=0) - V)))
    return V, greedy(Q, V), sweeps, res


def evaluate(inst, P, pi) -> np.ndarray:
    """Exact V_pi: solve (I - gamma (1-tau) P_pi) V = R."""
    S = inst.n_states
    P_pi = P[pi, np.arange(S), :]
    M = np.eye(S) - continuation(inst)[:, None] * P_pi
    return np.linalg.solve(M, rewards_of(inst))


def policy_iteration(inst, pi0=None, max_outer=10000, P=None):
    """Exact evaluation + greedy improvement until the policy is unchanged
    (Sec. 2.1).  Returns (V, pi, outer_iterations)."""
    if P is None:
        P = transition_matrices(inst)
    pi = np.zeros(inst.n_states, np.int32) if pi0 is None else \
        np.array(pi0, np.int32)
    for it in range(1, max_outer + 1):
        V = evaluate(inst, P, pi)
        pi_new = improve(q_values(inst, P, V), V, pi)
        if np.array_equal(pi_new, pi):
            return V, pi, it
        pi = pi_new
    return V, pi, max_outer


def brute_force(inst, P=None):
    """Enumerate every deterministic policy (A^S of them), evaluate each
    exactly and take the elementwise maximum.  Returns (V*, optimal) where
    optimal[s] is the set of actions that some optimal policy takes at s.
    Tiny instances only."""
    S, A = inst.n_states, inst.n_actions
    if A ** S > 200000:
        raise ValueError("too many policies to enumerate")
    if P is None:
        P = transition_matrices(inst)
    values, pols = [], []
    for pol in itertools.product(range(A), repeat=S):
        pi = np.asarray(pol, np.int32)
        values.append(evaluate(inst, P, pi))
        pols.append(pi)
    values = np.asarray(values)
    vstar = values.max(axis=0)
    optimal = [set() for _ in range(S)]
    for V, pi in zip(values, pols):
        if np.all(V >= vstar - 1e-10):
            for s in range(S):
                optimal[s].add(int(pi[s]))
    return vstar, optimal
