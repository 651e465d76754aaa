"""O2: FP64 oracle over the per-state successor lists of Def. 3 (test
infrastructure).

Def. 3 represents the model of each state s as the list of its tensor
components (s, s', P(s'|s,a)) with P(s'|s,a) > 0.  Here the lists are built by
enumerating the non-zeros of every rank term's Kronecker product (the product
of the per-dimension factor entries, times lambda), merging repeated
successors, and dropping the rows of terminal states (the interaction ends
there, Sec. 3.2).  A successor that is an obstacle is replaced by the state
itself (the agent stays put) and obstacle rows are dropped too (value 0, see
``common``).  They are stored as one CSR matrix per action.  Value
iteration and policy iteration then run by plain sweeps of Eq. 1.

Reach: factors with few non-zeros per row (identity and shift factors);
a dense m x m factor multiplies the list length by m per dimension.
"""
import numpy as np
import scipy.sparse as sp

from .common import ended, greedy, improve, obstacle_mask, rewards_of

MAX_TRIPLES = 400_000_000


def component_lists(inst, a: int):
    """Def. 3 triples of action a as arrays (s, s', p), before merging."""
    S_list, Sp_list, p_list = [], [], []
    for t in inst.terms_of(a):
        s = np.zeros(1, np.int64)
        sp_ = np.zeros(1, np.int64)
        p = np.array([inst.lambdas[t]])
        count = 1
        for k in range(inst.n_dims):
            T = inst.factor(t, k)
            m = T.shape[0]
            i_k, j_k = np.nonzero(T)
            v_k = T[i_k, j_k]
            count *= len(v_k)
            if count > MAX_TRIPLES:
                raise ValueError("successor lists too long for the sparse oracle")
            s = (s[:, None] * m + i_k[None, :]).ravel()
            sp_ = (sp_[:, None] * m + j_k[None, :]).ravel()
            p = (p[:, None] * v_k[None, :]).ravel()
        S_list.append(s)
        Sp_list.append(sp_)
        p_list.append(p)
    return np.concatenate(S_list), np.concatenate(Sp_list), np.concatenate(p_list)


def transition_csr(inst):
    """List of A CSR matrices, row s = the merged Def. 3 list of state s;
    terminal and obstacle rows are empty."""
    S = inst.n_states
    live = ~ended(inst)
    obs = obstacle_mask(inst)
    mats = []
    for a in range(inst.n_actions):
        s, s2, p = component_lists(inst, a)
        s2 = np.where(obs[s2], s, s2)          # blocked move: stay at s
        keep = live[s] & (p > 0)
        M = sp.coo_matrix((p[keep], (s[keep], s2[keep])), shape=(S, S)).tocsr()
        M.sum_duplicates()
        mats.append(M)
    return mats


def lists_csr(mdp):
    """A CSR matrices of an MDP given directly as Def. 3 lists (action-major
    rows a * S + s, see ``instances.ListsMDP``); terminal rows are empty.
    The other functions of this module take the result as ``mats`` together
    with the MDP (which carries rewards, gamma and the terminal mask)."""
    S, A = mdp.n_states, mdp.n_actions
    live = mdp.terminal == 0
    mats = []
    for a in range(A):
        lo, hi = mdp.row_ptr[a * S], mdp.row_ptr[(a + 1) * S]
        counts = np.diff(mdp.row_ptr[a * S:(a + 1) * S + 1])
        rows = np.repeat(np.arange(S), counts)
        p = mdp.prob[lo:hi]
        keep = live[rows]
        M = sp.coo_matrix((p[keep], (rows[keep], mdp.succ[lo:hi][keep])), shape=(S, S)).tocsr()
        M.sum_duplicates()
        mats.append(M)
    return mats


def q_values(inst, mats, V) -> np.ndarray:
    """Q[a, s] = R(s) + gamma * (P_a V)(s); terminal and obstacle rows are
    empty so their continuation is zero."""
    Q = np.empty((len(mats), inst.n_states))
    R = rewards_of(inst)
    for a, M in enumerate(mats):
        Q[a] = R + inst.gamma * (M @ V)
    return Q


def backup(inst, V, mats=None):
    """One Bellman backup: (max_a Q_a, greedy pi, Q)."""
    if mats is None:
        mats = transition_csr(inst)
    Q = q_values(inst, mats, np.asarray(V, np.float64))
    return Q.max(axis=0), greedy(Q, V), Q


def value_iteration(inst, eps=1e-13, max_iter=100000, V0=None, mats=None,
                    callback=None):
    """Sweeps until ||V' - V||_inf <= eps.  Returns (V, pi, sweeps, residual)
    as the dense oracle does."""
    if mats is None:
        mats = transition_csr(inst)
    V = np.zeros(inst.n_states) if V0 is None else np.array(V0, np.float64)
    sweeps = 0
    while sweeps < max_iter:
        Vn = q_values(inst, mats, V).max(axis=0)
        sweeps += 1
        res = float(np.max(np.abs(Vn - V)))
        V = Vn
        if callback is not None:
            callback(sweeps, res)
        if res <= eps:
            break
    Q = q_values(inst, mats, V)
    res = float(np.max(np.abs(Q.max(axis=0) - V)))
    return V, greedy(Q, V), sweeps, res


def policy_matrix(inst, mats, pi):
    """CSR P_pi whose row s is row s of P_{pi(s)}."""
    S = inst.n_states
    out = None
    for a, M in enumerate(mats):
        sel = sp.diags((pi == a).astype(np.float64), shape=(S, S), format="csr")
        part = sel @ M
        out = part if out is None else out + part
    return out.tocsr()


def evaluate(inst, mats, pi, V0=None, eps=1e-13, max_iter=1000000):
    """V_pi by sweeps V <- R + gamma P_pi V until the change is <= eps."""
    P_pi = policy_matrix(inst, mats, pi)
    R = rewards_of(inst)
    V = np.zeros(inst.n_states) if V0 is None else np.array(V0, np.float64)
    for _ in range(max_iter):
        Vn = R + inst.gamma * (P_pi @ V)
        res = float(np.max(np.abs(Vn - V)))
        V = Vn
        if res <= eps:
            break
    return V


def policy_iteration(inst, pi0=None, eps=1e-13, max_outer=10000, mats=None):
    """Evaluation by sweeps + greedy improvement with the incumbent rule, until
    the policy is unchanged.  Returns (V, pi, outer_iterations)."""
    if mats is None:
        mats = transition_csr(inst)
    pi = np.zeros(inst.n_states, np.int32) if pi0 is None else \
        np.array(pi0, np.int32)
    V = None
    for it in range(1, max_outer + 1):
        V = evaluate(inst, mats, pi, V0=V, eps=eps)
        pi_new = improve(q_values(inst, mats, V), V, pi)
        if np.array_equal(pi_new, pi):
            return V, pi, it
        pi = pi_new
    return V, pi, max_outer


def q_at_states(inst, V, states):
    """Q[a, i] for the listed states only, from their own Def. 3 lists: for
    state s with coordinates i, term t of action a reaches s' with
    probability lambda_t prod_k T_k[i_k, j_k] for every combination of
    non-zero entries of the rows T_k[i_k, :]; Q_a(s) = R(s) + gamma (1 -
    tau(s)) sum over those successors of probability times V(s'), where a
    successor that is an obstacle counts as s itself.  For spot checks of
    instances too large for whole-matrix oracles."""
    sizes = [int(m) for m in inst.sizes]
    V = np.asarray(V, np.float64)
    states = np.asarray(states, np.int64)
    obs = obstacle_mask(inst)
    stop = ended(inst)
    R = rewards_of(inst)
    Q = np.empty((inst.n_actions, states.size))
    for col, s in enumerate(states):
        coords = np.unravel_index(int(s), sizes)      # row-major, Def. 2
        cont = inst.gamma * (1.0 - float(stop[s]))
        for a in range(inst.n_actions):
            tot = 0.0
            for t in inst.terms_of(a):
                succ = np.zeros(1, np.int64)
                prob = np.array([inst.lambdas[t]])
                for k in range(inst.n_dims):
                    row = inst.factor(t, k)[coords[k]]
                    j = np.nonzero(row)[0]
                    succ = (succ[:, None] * sizes[k] + j[None, :]).ravel()
                    prob = (prob[:, None] * row[j][None, :]).ravel()
                succ = np.where(obs[succ], s, succ)
                tot += float(prob @ V[succ])
            Q[a, col] = R[s] + cont * tot
    return Q
