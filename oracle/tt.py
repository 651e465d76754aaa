"""O4: FP64 oracle for Tensor-Train and Tucker transition models (test
infrastructure; the GPU library never calls it).

Sec. 5 of the paper names Tensor-Train and Tucker decompositions as transition
models beyond the CP form of Sec. 2.2.  The oracle writes both out from their
definitions, over the row-major state order of Def. 2:

  * Tensor-Train (matrix-product operator): for action a with cores
    G_k of shape [b_k, m_k, m_k, b_{k+1}] (b_0 = b_n = 1),
        P_a[s, s'] = G_0[:, s_0, s'_0, :] G_1[:, s_1, s'_1, :] ... G_{n-1}[:, s_{n-1}, s'_{n-1}, :],
    a product of small matrices whose bond indices are summed;
  * Tucker: P_a = sum_{r_0..r_{n-1}} C_a[r_0, .., r_{n-1}] kron_k U^{(k)}_{a, r_k}.

The dense matrices go to the tabular oracle O1 (``dense.q_values``,
``dense.value_iteration`` ... with ``P=``), which applies Eq. 1 unchanged.
"""
import itertools

import numpy as np

from .dense import MAX_DENSE_STATES


def _check_size(inst):
    if inst.n_states > MAX_DENSE_STATES:
        raise ValueError(f"dense oracle limited to {MAX_DENSE_STATES} states")


def tt_matrix(inst, a: int) -> np.ndarray:
    """[S, S] FP64: the Tensor-Train operator of action a.  M holds, for the
    leading k dims, the partial products P[(s_0..s_{k-1}), (s'_0..s'_{k-1}), b]
    with the open bond b; each new core multiplies into the bond and appends
    its row and column coordinates (slowest first, as Def. 2 orders them)."""
    M = np.ones((1, 1, 1))
    for k in range(inst.n_dims):
        G = inst.core(a, k)                             # [l, i, j, r]
        X = np.einsum("ucl,lijr->uicjr", M, G)          # rows (u, i), cols (c, j)
        u, i, c, j, r = X.shape
        M = X.reshape(u * i, c * j, r)
    return M[:, :, 0]


def tt_transition_matrices(inst) -> np.ndarray:
    """[A, S, S] FP64 with P[a, s, s'] = P(s' | s, a) for a TTInstance."""
    _check_size(inst)
    return np.stack([tt_matrix(inst, a) for a in range(inst.n_actions)])


def tt_entry(inst, a: int, s: int, t: int) -> float:
    """One entry P_a[s, t], as the product of the matrices G_k[:, s_k, t_k, :]."""
    from .common import coords_of
    cs, ct = coords_of(inst.sizes, s), coords_of(inst.sizes, t)
    v = np.ones((1, 1))
    for k in range(inst.n_dims):
        v = v @ inst.core(a, k)[:, cs[k], ct[k], :]
    return float(v[0, 0])


def tt_row(inst, a: int, s: int) -> np.ndarray:
    """Row P_a[s, :] (length S) for one state, built from the cores with the
    row coordinates fixed: W[(s'_0..s'_k), b] = W[(..), l] G_k[l, s_k, s'_k, b]."""
    from .common import coords_of
    cs = coords_of(inst.sizes, s)
    W = np.ones((1, 1))
    for k in range(inst.n_dims):
        G = inst.core(a, k)[:, cs[k], :, :]             # [l, j, r]
        X = np.einsum("ul,ljr->ujr", W, G)
        u, j, r = X.shape
        W = X.reshape(u * j, r)
    return W[:, 0]


def tt_q_at_states(inst, V, states) -> np.ndarray:
    """Q[a, i] = R(s) + gamma (1 - tau(s)) P_a[s, :] V at s = states[i]
    (Eq. 1), one row at a time; for state spaces too large for O1."""
    V = np.asarray(V, np.float64)
    states = [int(s) for s in states]
    Q = np.empty((inst.n_actions, len(states)))
    for i, s in enumerate(states):
        c = 0.0 if inst.terminal[s] else inst.gamma
        for a in range(inst.n_actions):
            Q[a, i] = inst.rewards[s] + c * float(tt_row(inst, a, s) @ V)
    return Q


def tucker_matrix(inst, a: int) -> np.ndarray:
    """[S, S] FP64: sum over every core index of C_a[r] kron_k U^{(k)}_{a, r_k}."""
    C = inst.core(a)
    S = inst.n_states
    P = np.zeros((S, S))
    for r in itertools.product(*[range(int(x)) for x in inst.core_ranks[a]]):
        K = np.ones((1, 1))
        for k in range(inst.n_dims):
            K = np.kron(K, inst.factor(a, k, r[k]))
        P += C[r] * K
    return P


def tucker_transition_matrices(inst) -> np.ndarray:
    """[A, S, S] FP64 with P[a, s, s'] = P(s' | s, a) for a TuckerInstance."""
    _check_size(inst)
    return np.stack([tucker_matrix(inst, a) for a in range(inst.n_actions)])


def tucker_entry(inst, a: int, s: int, t: int) -> float:
    """One entry: sum_r C_a[r] prod_k U^{(k)}_{a, r_k}[s_k, t_k]."""
    from .common import coords_of
    cs, ct = coords_of(inst.sizes, s), coords_of(inst.sizes, t)
    C = inst.core(a)
    tot = 0.0
    for r in itertools.product(*[range(int(x)) for x in inst.core_ranks[a]]):
        p = C[r]
        for k in range(inst.n_dims):
            p *= inst.factor(a, k, r[k])[cs[k], ct[k]]
        tot += p
    return tot
