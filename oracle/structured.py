"""O3: FP64 oracle that applies each rank term as a chain of mode products
(test infrastructure).

For the CP form P_a = sum_r lambda_{a,r} kron_k T^(k)_{a,r} (a sum of rank-one
terms, Sec. 2.2), applying P_a to the value vector reshaped as an n-way tensor
(row-major order, Def. 2) is, term by term, the mode-k product of V with every
factor: U[.., i_k, ..] = sum_j T^(k)[i_k, j] V[.., j, ..].  The Q-values are
those of Eq. 1: Q_a = R + gamma (1 - tau) sum_r lambda_{a,r} U_{a,r}.  Each mode
product is one numpy tensordot; nothing is blocked or fused.  Works for dense
factors too; the cost per backup is 2 * sum_a R_a * sum_k m_k flops per state.
Obstacles break the Kronecker form, so instances with obstacles are refused
here (the dense and successor-list oracles handle them).
"""
import numpy as np

from .common import greedy, improve, obstacle_mask


def _refuse_obstacles(inst):
    if obstacle_mask(inst).any():
        raise ValueError("mode-product chains cannot express obstacles")


def mode_product(X: np.ndarray, T: np.ndarray, k: int) -> np.ndarray:
    """(X x_k T)[.., i, ..] = sum_j T[i, j] X[.., j, ..]."""
    Y = np.tensordot(T, X, axes=([1], [k]))   # new axis 0 = i
    return np.moveaxis(Y, 0, k)


def apply_term(inst, t: int, Vt: np.ndarray) -> np.ndarray:
    U = Vt
    for k in range(inst.n_dims):
        U = mode_product(U, inst.factor(t, k), k)
    return U


def apply_action(inst, a: int, V: np.ndarray) -> np.ndarray:
    """(P_a V) as a flat vector, by mode-product chains."""
    _refuse_obstacles(inst)
    shape = tuple(int(m) for m in inst.sizes)
    Vt = np.asarray(V, np.float64).reshape(shape)
    acc = np.zeros(shape)
    for t in inst.terms_of(a):
        acc += inst.lambdas[t] * apply_term(inst, t, Vt)
    return acc.ravel()


def q_values(inst, V) -> np.ndarray:
    c = inst.gamma * (1.0 - inst.terminal.astype(np.float64))
    Q = np.empty((inst.n_actions, inst.n_states))
    for a in range(inst.n_actions):
        Q[a] = inst.rewards + c * apply_action(inst, a, V)
    return Q


def backup(inst, V):
    """One Bellman backup: (max_a Q_a, greedy pi, Q)."""
    Q = q_values(inst, V)
    return Q.max(axis=0), greedy(Q, V), Q


def policy_apply(inst, V, pi) -> np.ndarray:
    """(P_pi V)(s) = (P_{pi(s)} V)(s), evaluated for every action then
    selected per state."""
    out = np.zeros(inst.n_states)
    for a in range(inst.n_actions):
        sel = pi == a
        if np.any(sel):
            out[sel] = apply_action(inst, a, V)[sel]
    return out


def value_iteration(inst, eps=1e-13, max_iter=100000, V0=None):
    V = np.zeros(inst.n_states) if V0 is None else np.array(V0, np.float64)
    sweeps = 0
    while sweeps < max_iter:
        Vn = q_values(inst, V).max(axis=0)
        sweeps += 1
        res = float(np.max(np.abs(Vn - V)))
        V = Vn
        if res <= eps:
            break
    Q = q_values(inst, V)
    res = float(np.max(np.abs(Q.max(axis=0) - V)))
    return V, greedy(Q, V), sweeps, res


def evaluate(inst, pi, V0=None, eps=1e-13, max_iter=1000000):
    c = inst.gamma * (1.0 - inst.terminal.astype(np.float64))
    V = np.zeros(inst.n_states) if V0 is None else np.array(V0, np.float64)
    for _ in range(max_iter):
        Vn = inst.rewards + c * policy_apply(inst, V, pi)
        res = float(np.max(np.abs(Vn - V)))
        V = Vn
        if res <= eps:
            break
    return V


def policy_iteration(inst, pi0=None, eps=1e-13, max_outer=10000):
    pi = np.zeros(inst.n_states, np.int32) if pi0 is None else \
        np.array(pi0, np.int32)
    V = None
    for it in range(1, max_outer + 1):
        V = evaluate(inst, pi, V0=V, eps=eps)
        pi_new = improve(q_values(inst, V), V, pi)
        if np.array_equal(pi_new, pi):
            return V, pi, it
        pi = pi_new
    return V, pi, max_outer


def q_at_states(inst, V, states):
    """Q[a, i] for the listed states only, straight from the definition
    (P_a V)(s) = sum_r lambda_{a,r} sum_j prod_k T^(k)_{a,r}[i_k, j_k] V[j]:
    V is contracted with row i_k of every factor, one dimension at a time.
    For spot checks of instances too large for a full oracle backup."""
    _refuse_obstacles(inst)
    shape = tuple(int(m) for m in inst.sizes)
    Vt = np.asarray(V, np.float64).reshape(shape)
    states = np.asarray(states, np.int64)
    Q = np.empty((inst.n_actions, states.size))
    for col, s in enumerate(states):
        coords = np.unravel_index(int(s), shape)   # row-major, Def. 2
        cont = inst.gamma * (1.0 - float(inst.terminal[s]))
        for a in range(inst.n_actions):
            tot = 0.0
            for t in inst.terms_of(a):
                U = Vt
                for k in range(inst.n_dims):
                    U = np.tensordot(inst.factor(t, k)[coords[k]], U, axes=([0], [0]))
                tot += inst.lambdas[t] * float(U)
            Q[a, col] = inst.rewards[s] + cont * tot
    return Q


def q_on_slab(inst, V, fixed):
    """Q[a, j] for every state whose coordinate k equals fixed[k] (for each k
    in the dict `fixed`), and those states' indices (row-major order of the
    free coordinates, Def. 2).  Straight from the definition
    (P_a V)(s) = sum_r lambda_{a,r} sum_j prod_k T^(k)_{a,r}[i_k, j_k] V[j]:
    per term, V is contracted with row fixed[k] of the factor of every fixed
    coordinate k, and the remaining factors are applied as mode products,
    which gives the term on all states of the slab at once.  For checks of
    whole rows or columns of instances too large for a full oracle backup."""
    _refuse_obstacles(inst)
    shape = tuple(int(m) for m in inst.sizes)
    fdims = sorted(int(k) for k in fixed)
    free = [k for k in range(inst.n_dims) if k not in fixed]
    # fixed coordinates first (one copy), so each contraction is over axis 0
    Vt = np.ascontiguousarray(np.moveaxis(np.asarray(V, np.float64).reshape(shape),
                                          fdims, list(range(len(fdims)))))
    grid = np.indices([shape[k] for k in free]).reshape(len(free), -1) if free \
        else np.zeros((0, 1), np.int64)
    coords = np.empty((inst.n_dims, grid.shape[1]), np.int64)
    for k in fdims:
        coords[k] = int(fixed[k])
    for pos, k in enumerate(free):
        coords[k] = grid[pos]
    states = np.ravel_multi_index(tuple(coords), shape) if inst.n_dims else np.zeros(1, np.int64)
    cont = inst.gamma * (1.0 - inst.terminal[states].astype(np.float64))
    Q = np.empty((inst.n_actions, states.size))
    for a in range(inst.n_actions):
        tot = np.zeros([shape[k] for k in free])
        for t in inst.terms_of(a):
            U = Vt
            for k in fdims:
                U = np.tensordot(inst.factor(t, k)[int(fixed[k])], U, axes=([0], [0]))
            for pos, k in enumerate(free):
                U = mode_product(U, inst.factor(t, k), pos)
            tot = tot + inst.lambdas[t] * U
        Q[a] = inst.rewards[states] + cont * np.ravel(tot)
    return Q, states

