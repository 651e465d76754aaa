"""Seeded synthetic MDP instances: the one module that both the CPU oracle and
the GPU path read.

It builds inputs only -- sizes, transition factors, mixture weights, rewards,
terminal masks and discount factors as FP64 host arrays -- and performs none
of the solver's arithmetic (no backup, no mode product, no max).

Problem statement followed (Kuinchtner, Sales & Meneguzzi, CP-MDP):
  * the MDP tuple <S, A, P, R, gamma> of Sec. 2.1;
  * dimensions d_1..d_D each with its own number of states (Def. 1) and the
    state space as their Cartesian product, enumerated with the LAST
    dimension varying fastest (Def. 2), i.e. row-major:
    s = sum_k i_k * prod_{j>k} m_j;
  * GridWorld with two actions per axis, |A| = 2|D| (Sec. 3.2), and terminal
    states that end the interaction (Sec. 3.2).

The transition model of action a is a rank-R_a Kronecker/CP sum over the
dimensions, P_a = sum_r lambda_{a,r} kron_k T^{(k)}_{a,r}, each factor an
m_k x m_k row-stochastic matrix with T[i, j] = P(next coordinate j | current
coordinate i).  The paper does not state a slip model, reward noise, goal
placement or seeds; the readings used here are:
  * action index a = 2k + (0 for a +1 move along dim k, 1 for a -1 move);
  * an action moves as intended with probability 1 - slip, and the slip mass
    is split evenly over the 2(n-1) perpendicular unit moves, giving rank
    2n - 1; a move off the grid stays put (clamped shift);
  * terminal states take V(s) = R(s) and no continuation;
  * rewards are per state, i.i.d. normal with the stated standard deviation,
    with the goal corner (m-1, ..., m-1) set to +1 and made terminal.

Flat factor layout (shared with the C ABI): for term t = 0..sum_a R_a - 1
(action-major: all terms of action 0, then action 1, ...), for dim k, one
m_k x m_k row-major block.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

# Seeds of the named workloads.
SEED_GRID4 = 20210002        # 32^4 GridWorld
SEED_GRID4_LARGE = 20210012  # 96^4 GridWorld (HBM-resident supplement)
SEED_DENSE6 = 20210003       # 16^6 dense-factor grid
SEED_DENSE6_SMALL = 20210013  # 12^6 dense-factor grid (parity instance)
SEED_BATCH = 20210004        # 512 mixed GridWorlds
SEED_WARM = 20210005         # 64^3 warm-start instances
SEED_PAPER2D = 20210006      # 1000 x 1000 GridWorld of Table 1 (22 terminals, 800 obstacles)


@dataclass
class Instance:
    """One MDP, all arrays FP64 / integer host arrays."""

    sizes: np.ndarray            # int64 [n]
    ranks: np.ndarray            # int32 [A]
    factors: np.ndarray          # float64 flat, layout described above
    lambdas: np.ndarray          # float64 [sum R]
    rewards: np.ndarray          # float64 [S], row-major state order
    gamma: float
    terminal: np.ndarray         # uint8 [S], 1 = terminal
    name: str = ""
    meta: Dict[str, float] = field(default_factory=dict)
    obstacle: Optional[np.ndarray] = None   # uint8 [S], 1 = obstacle (or None)

    @property
    def n_dims(self) -> int:
        return int(self.sizes.shape[0])

    @property
    def n_states(self) -> int:
        return int(np.prod(self.sizes))

    @property
    def n_actions(self) -> int:
        return int(self.ranks.shape[0])

    @property
    def n_terms(self) -> int:
        return int(self.ranks.sum())

    @property
    def term_stride(self) -> int:
        return int(sum(int(m) * int(m) for m in self.sizes))

    def term_index(self, a: int, r: int) -> int:
        return int(self.ranks[:a].sum()) + r

    def factor(self, t: int, k: int) -> np.ndarray:
        """View of T^{(k)} of flat term t as an m_k x m_k matrix."""
        off = t * self.term_stride + sum(int(m) * int(m) for m in self.sizes[:k])
        m = int(self.sizes[k])
        return self.factors[off:off + m * m].reshape(m, m)

    def terms_of(self, a: int) -> List[int]:
        start = int(self.ranks[:a].sum())
        return list(range(start, start + int(self.ranks[a])))


def _pack(sizes: Sequence[int], per_action: List[List[tuple]]) -> tuple:
    """per_action[a] = list of (lambda, [T_0, ..., T_{n-1}]) -> flat arrays."""
    blocks, lams, ranks = [], [], []
    for terms in per_action:
        ranks.append(len(terms))
        for lam, mats in terms:
            lams.append(float(lam))
            for k, T in enumerate(mats):
                assert T.shape == (sizes[k], sizes[k])
                blocks.append(np.ascontiguousarray(T, dtype=np.float64).ravel())
    return (np.concatenate(blocks), np.asarray(lams, np.float64),
            np.asarray(ranks, np.int32))


def shift_matrix(m: int, step: int) -> np.ndarray:
    """Clamped unit move along one axis: row i has a single 1 at i+step,
    clamped to [0, m-1] (a move off the grid stays put)."""
    T = np.zeros((m, m))
    for i in range(m):
        T[i, min(max(i + step, 0), m - 1)] = 1.0
    return T


def gridworld_terms(sizes: Sequence[int], slip: float) -> List[List[tuple]]:
    """Per-action CP terms of the slip GridWorld: 2n actions, rank 2n-1
    (n >= 2) or 1 (n == 1).  Term order inside an action: the intended move,
    then for every other dim j in ascending order the +1 and the -1 slip."""
    n = len(sizes)
    eye = [np.eye(m) for m in sizes]
    per_action = []
    for k in range(n):
        for step in (+1, -1):
            mats = list(eye)
            mats[k] = shift_matrix(sizes[k], step)
            if n == 1:
                terms = [(1.0, mats)]
            else:
                terms = [(1.0 - slip, mats)]
                w = slip / (2 * (n - 1))
                for j in range(n):
                    if j == k:
                        continue
                    for s2 in (+1, -1):
                        mj = list(eye)
                        mj[j] = shift_matrix(sizes[j], s2)
                        terms.append((w, mj))
            per_action.append(terms)
    return per_action


def flat_index(sizes: Sequence[int], coords: Sequence[int]) -> int:
    """Row-major (last dimension fastest) state index of Def. 2."""
    s = 0
    for m, i in zip(sizes, coords):
        s = s * int(m) + int(i)
    return s


def make_gridworld(sizes, slip, rewards, gamma, terminals=(), name="",
                   meta=None) -> Instance:
    sizes = [int(m) for m in sizes]
    S = int(np.prod(sizes))
    factors, lams, ranks = _pack(sizes, gridworld_terms(sizes, slip))
    rewards = np.asarray(rewards, np.float64).reshape(S).copy()
    term = np.zeros(S, np.uint8)
    for coords, rv in terminals:
        s = flat_index(sizes, coords)
        rewards[s] = rv
        term[s] = 1
    m = {"slip": float(slip)}
    if meta:
        m.update(meta)
    return Instance(np.asarray(sizes, np.int64), ranks, factors, lams, rewards,
                    float(gamma), term, name, m)


# ---------------------------------------------------------------- workloads

def grid2d_16() -> Instance:
    """16x16 GridWorld, 4 actions, rank 3 (0.8 / 0.1 / 0.1), step reward
    -0.04, terminal goal +1 at (15,15) and terminal pit -1 at (8,8),
    gamma = 0.95."""
    sizes = [16, 16]
    return make_gridworld(sizes, 0.2, np.full(256, -0.04), 0.95,
                          terminals=[((15, 15), 1.0), ((8, 8), -1.0)],
                          name="grid2d_16x16")


def _noisy_goal_grid(sizes, slip, gamma, rng, name, meta=None) -> Instance:
    S = int(np.prod(sizes))
    R = rng.normal(0.0, 0.1, S)
    goal = tuple(int(m) - 1 for m in sizes)
    return make_gridworld(sizes, slip, R, gamma, terminals=[(goal, 1.0)],
                          name=name, meta=meta)


def grid4d(m: int = 32, seed: int = SEED_GRID4) -> Instance:
    """m^4 GridWorld, 8 actions, slip 0.1 over the 6 perpendicular moves
    (rank 7), rewards N(0, 0.1) per state, +1 terminal goal corner,
    gamma = 0.99."""
    rng = np.random.default_rng(seed)
    return _noisy_goal_grid([m] * 4, 0.1, 0.99, rng, f"grid4d_{m}^4")


def grid_small(sizes, slip=0.1, gamma=0.99, seed=0) -> Instance:
    """Same generator as grid4d at arbitrary sizes (tests)."""
    rng = np.random.default_rng(seed)
    return _noisy_goal_grid(list(sizes), slip, gamma, rng,
                            "grid_" + "x".join(map(str, sizes)))


def dense_grid(m: int = 16, n: int = 6, n_actions: int = 12, rank: int = 8,
               seed: int = SEED_DENSE6, gamma: float = 0.95,
               alpha: float = 0.5) -> Instance:
    """n-D grid with dense factors: lambda_a ~ Dirichlet(1), each factor row
    ~ Dirichlet(alpha), rewards N(0, 0.1), no terminals."""
    rng = np.random.default_rng(seed)
    sizes = [m] * n
    per_action = []
    for _a in range(n_actions):
        lam = rng.dirichlet(np.ones(rank))
        lam = lam / lam.sum()
        terms = []
        for r in range(rank):
            mats = []
            for k in range(n):
                T = rng.dirichlet(alpha * np.ones(sizes[k]), size=sizes[k])
                T = T / T.sum(axis=1, keepdims=True)
                mats.append(T)
            terms.append((lam[r], mats))
        per_action.append(terms)
    factors, lams, ranks = _pack(sizes, per_action)
    S = int(np.prod(sizes))
    R = rng.normal(0.0, 0.1, S)
    return Instance(np.asarray(sizes, np.int64), ranks, factors, lams, R,
                    float(gamma), np.zeros(S, np.uint8),
                    f"dense_{m}^{n}", {"alpha": alpha})


def batch_instance(i: int, base: int = SEED_BATCH) -> Instance:
    """Instance i of the 512-instance mixed batch: n ~ U{2,3,4},
    m ~ U{8..48}, slip ~ U[0.05, 0.3], gamma ~ U[0.9, 0.99], rewards
    N(0, 0.1) plus a +1 terminal goal corner."""
    rng = np.random.default_rng(np.random.SeedSequence([base, i]))
    n = int(rng.integers(2, 5))
    m = int(rng.integers(8, 49))
    slip = float(rng.uniform(0.05, 0.3))
    gamma = float(rng.uniform(0.9, 0.99))
    return _noisy_goal_grid([m] * n, slip, gamma, rng, f"batch{i}_{m}^{n}",
                            meta={"index": i})


def batch_shapes(count: int = 512, base: int = SEED_BATCH):
    """(n, m) of each batch instance without building the arrays."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(np.random.SeedSequence([base, i]))
        out.append((int(rng.integers(2, 5)), int(rng.integers(8, 49))))
    return out


def warm_instance(split: int, i: int, m: int = 64,
                  base: int = SEED_WARM) -> Instance:
    """64^3 instance for the learned warm start; split 0 = train,
    1 = validation, 2 = test.  Slip and gamma drawn as in the batch."""
    rng = np.random.default_rng(np.random.SeedSequence([base, split, i]))
    slip = float(rng.uniform(0.05, 0.3))
    gamma = float(rng.uniform(0.9, 0.99))
    return _noisy_goal_grid([m] * 3, slip, gamma, rng,
                            f"warm{split}_{i}_{m}^3",
                            meta={"split": split, "index": i})


# ------------------------------------------------------- small test builders

def random_dense(sizes, n_actions, rank, seed, gamma=0.9, alpha=1.0,
                 n_terminal=0, reward_scale=1.0) -> Instance:
    """Tiny random instance with dense factors (and optional terminals)."""
    rng = np.random.default_rng(seed)
    sizes = [int(m) for m in sizes]
    S = int(np.prod(sizes))
    ranks = np.atleast_1d(rank)
    if ranks.size == 1:
        ranks = np.full(n_actions, int(ranks[0]))
    per_action = []
    for a in range(n_actions):
        lam = rng.dirichlet(np.ones(int(ranks[a])))
        terms = []
        for r in range(int(ranks[a])):
            mats = [rng.dirichlet(alpha * np.ones(m), size=m) for m in sizes]
            mats = [T / T.sum(axis=1, keepdims=True) for T in mats]
            terms.append((lam[r] / lam.sum(), mats))
        per_action.append(terms)
    factors, lams, rk = _pack(sizes, per_action)
    R = rng.normal(0.0, reward_scale, S)
    term = np.zeros(S, np.uint8)
    if n_terminal:
        term[rng.choice(S, n_terminal, replace=False)] = 1
    return Instance(np.asarray(sizes, np.int64), rk, factors, lams, R,
                    float(gamma), term, "random_dense")


def chain_1d(m: int, step_reward: float, goal_reward: float,
             gamma: float) -> Instance:
    """Deterministic 1-D chain (slip 0), goal at i = m-1, terminal."""
    R = np.full(m, step_reward)
    return make_gridworld([m], 0.0, R, gamma,
                          terminals=[((m - 1,), goal_reward)], name="chain")


def with_rewards(inst: Instance, rewards, terminal=None) -> Instance:
    """Copy of inst with other rewards (and optionally another mask)."""
    S = inst.n_states
    term = inst.terminal.copy() if terminal is None else \
        np.asarray(terminal, np.uint8).reshape(S)
    return Instance(inst.sizes.copy(), inst.ranks.copy(), inst.factors.copy(),
                    inst.lambdas.copy(),
                    np.asarray(rewards, np.float64).reshape(S).copy(),
                    inst.gamma, term, inst.name, dict(inst.meta),
                    None if inst.obstacle is None else inst.obstacle.copy())


def with_obstacles(inst: Instance, cells) -> Instance:
    """Copy of inst with obstacles at the given flat state indices (an
    obstacle must not be terminal)."""
    obs = np.zeros(inst.n_states, np.uint8)
    obs[np.asarray(list(cells), np.int64)] = 1
    if np.any(obs & inst.terminal):
        raise ValueError("a state cannot be both terminal and an obstacle")
    out = with_rewards(inst, inst.rewards)
    out.obstacle = obs
    return out


def paper_gridworld(sizes, n_terminal: int, n_obstacle: int, seed: int,
                    slip: float = 0.2, gamma: float = 0.9,
                    step_reward: float = -3.0) -> Instance:
    """GridWorld of the paper's experiments (Sec. 4, Table 1): 2|D| actions,
    step reward -3, randomly placed terminal states (+100 for the first half,
    -100 for the rest) and obstacles, gamma = 0.9.  The paper does not give
    the slip model or the placement seeds: moves go as intended with
    probability 1 - slip and slip is spread over the perpendicular moves, as
    in the other GridWorlds here."""
    sizes = [int(m) for m in sizes]
    S = int(np.prod(sizes))
    rng = np.random.default_rng(seed)
    cells = rng.choice(S, n_terminal + n_obstacle, replace=False)
    terms = []
    for j, s in enumerate(cells[:n_terminal]):
        coords = np.unravel_index(int(s), sizes)
        terms.append((tuple(int(c) for c in coords), 100.0 if j < (n_terminal + 1) // 2
                      else -100.0))
    inst = make_gridworld(sizes, slip, np.full(S, step_reward), gamma, terminals=terms,
                          name="paper_grid_" + "x".join(map(str, sizes)),
                          meta={"n_terminal": n_terminal, "n_obstacle": n_obstacle})
    return with_obstacles(inst, cells[n_terminal:])


# ------------------------------------------- Def. 3 successor lists (no CP form)

@dataclass
class ListsMDP:
    """An MDP given directly by the per-state successor lists of Def. 3: for
    each action a and state s, the successors s' with P(s'|s,a) > 0.  Stored
    as one CSR matrix per action, stacked: row a * S + s holds
    succ[row_ptr[r]:row_ptr[r+1]] and prob[...] (the C ABI's layout)."""

    n_states: int
    n_actions: int
    row_ptr: np.ndarray          # int64 [A*S + 1]
    succ: np.ndarray             # int64 [nnz]
    prob: np.ndarray             # float64 [nnz]
    rewards: np.ndarray          # float64 [S]
    gamma: float
    terminal: np.ndarray         # uint8 [S]
    name: str = ""
    obstacle: Optional[np.ndarray] = None   # always None: lists encode any blocking


def _lists_from_rows(S, A, rows, rewards, gamma, terminal, name) -> ListsMDP:
    """rows[a][s] = dict successor -> probability."""
    ptr, succ, prob = [0], [], []
    for a in range(A):
        for s in range(S):
            items = sorted(rows[a][s].items())
            succ += [k for k, _ in items]
            prob += [v for _, v in items]
            ptr.append(len(succ))
    return ListsMDP(S, A, np.asarray(ptr, np.int64), np.asarray(succ, np.int64),
                    np.asarray(prob, np.float64), np.asarray(rewards, np.float64).copy(),
                    float(gamma), np.asarray(terminal, np.uint8).copy(), name)


def gridworld_lists(sizes, slip, rewards, gamma, terminal=None, obstacle=None,
                    name="") -> ListsMDP:
    """The slip GridWorld written directly as Def. 3 lists by moving an agent
    (no Kronecker factors): action a = 2k + d moves along dim k (d = 0: +1,
    d = 1: -1) with probability 1 - slip, or one step along another dim with
    slip / (2(n-1)) each; a move that leaves the grid or lands on an obstacle
    keeps the agent in place.  Obstacle states get reward 0 and are made
    terminal (their value is 0)."""
    sizes = [int(m) for m in sizes]
    n = len(sizes)
    S = int(np.prod(sizes))
    term = np.zeros(S, np.uint8) if terminal is None else np.asarray(terminal, np.uint8).copy()
    obs = np.zeros(S, bool) if obstacle is None else np.asarray(obstacle).astype(bool)
    R = np.asarray(rewards, np.float64).reshape(S).copy()
    R[obs] = 0.0
    term[obs] = 1
    strides = [int(np.prod(sizes[k + 1:])) for k in range(n)]
    coords = np.stack(np.unravel_index(np.arange(S), sizes), axis=1)
    src = np.arange(S, dtype=np.int64)
    ptr, succ, prob = [np.zeros(1, np.int64)], [], []
    base = 0
    for a in range(2 * n):
        k, step = a // 2, (1 if a % 2 == 0 else -1)
        moves = [(k, step, 1.0 if n == 1 else 1.0 - slip)]
        if n > 1:
            for j in range(n):
                if j != k:
                    w = slip / (2 * (n - 1))
                    moves += [(j, +1, w), (j, -1, w)]
        ss, tt, pp = [], [], []
        for dim, st, p in moves:
            if p == 0.0:
                continue
            c = coords[:, dim] + st
            ok = (c >= 0) & (c < sizes[dim])
            tgt = np.where(ok, src + st * strides[dim], src)
            tgt = np.where(obs[tgt], src, tgt)
            ss.append(src)
            tt.append(tgt)
            pp.append(np.full(S, p))
        ss, tt, pp = np.concatenate(ss), np.concatenate(tt), np.concatenate(pp)
        # merge moves that reach the same successor, rows in state order,
        # successors ascending inside a row
        key, inv = np.unique(ss * S + tt, return_inverse=True)
        merged = np.zeros(key.size)
        np.add.at(merged, inv, pp)
        counts = np.bincount(key // S, minlength=S)
        ptr.append(base + np.cumsum(counts))
        base += key.size
        succ.append(key % S)
        prob.append(merged)
    return ListsMDP(S, 2 * n, np.concatenate(ptr), np.concatenate(succ), np.concatenate(prob),
                    R, float(gamma), term, name or "lists_grid")


def random_lists(S: int, A: int, k_max: int, seed: int, gamma: float = 0.9,
                 n_terminal: int = 0, locality: int = 0) -> ListsMDP:
    """A random MDP with no structure: each (s, a) has 1..k_max distinct
    successors (near s when locality > 0, else anywhere) with Dirichlet(1)
    probabilities; rewards N(0, 1)."""
    rng = np.random.default_rng(seed)
    rows = []
    for a in range(A):
        per_state = []
        for s in range(S):
            k = int(rng.integers(1, k_max + 1))
            if locality > 0:
                cand = np.arange(max(0, s - locality), min(S, s + locality + 1))
            else:
                cand = np.arange(S)
            k = min(k, cand.size)
            tg = rng.choice(cand, k, replace=False)
            p = rng.dirichlet(np.ones(k))
            per_state.append({int(t): float(v) for t, v in zip(tg, p)})
        rows.append(per_state)
    term = np.zeros(S, np.uint8)
    if n_terminal:
        term[rng.choice(S, n_terminal, replace=False)] = 1
    return _lists_from_rows(S, A, rows, rng.normal(0.0, 1.0, S), gamma, term, "random_lists")


def paper_gridworld_lists(inst: Instance) -> ListsMDP:
    """The Table 1 GridWorld instance (CP form, with obstacles) rewritten as
    Def. 3 lists by move simulation, for the same problem on both paths."""
    return gridworld_lists([int(m) for m in inst.sizes], float(inst.meta["slip"]),
                           inst.rewards, inst.gamma, inst.terminal, inst.obstacle,
                           name=inst.name + "_lists")


def seeded_values(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """A seeded FP64 value vector (e.g. the common V fed to one backup)."""
    return np.random.default_rng(seed).normal(0.0, scale, n)


def named(name: str) -> Instance:
    """Workloads by name."""
    table = {
        "grid2d_16x16": grid2d_16,
        "grid4d_32": lambda: grid4d(32, SEED_GRID4),
        "grid4d_96": lambda: grid4d(96, SEED_GRID4_LARGE),
        "dense6_16": lambda: dense_grid(16, seed=SEED_DENSE6),
        "dense6_12": lambda: dense_grid(12, seed=SEED_DENSE6_SMALL),
        "paper2d_1000": lambda: paper_gridworld([1000, 1000], 22, 800, SEED_PAPER2D),
    }
    return table[name]()


# ------------------------------- Tensor-Train and Tucker transition models

SEED_TT6 = 20210007          # 16^6 grid with Tensor-Train transitions


@dataclass
class TTInstance:
    """An MDP whose transition operator of each action is a Tensor-Train
    (matrix-product) operator over the dimensions:
        P_a[s, s'] = G_0[:, s_0, s'_0, :] G_1[:, s_1, s'_1, :] ... G_{n-1}[...]
    a product of b_k x b_{k+1} matrices with b_0 = b_n = 1 (the Tensor-Train
    form that Sec. 5 names as a future transition model; a CP term is the
    special case of diagonal bonds).  Flat core layout (the C ABI's):
    action-major, then k = 0..n-1, one block [b_k][m_k][m_k][b_{k+1}]
    row-major."""

    sizes: np.ndarray            # int64 [n]
    bonds: np.ndarray            # int32 [A, n + 1]
    cores: np.ndarray            # float64 flat
    rewards: np.ndarray          # float64 [S]
    gamma: float
    terminal: np.ndarray         # uint8 [S]
    name: str = ""
    meta: Dict[str, float] = field(default_factory=dict)
    obstacle: Optional[np.ndarray] = None   # always None

    @property
    def n_dims(self) -> int:
        return int(self.sizes.shape[0])

    @property
    def n_states(self) -> int:
        return int(np.prod(self.sizes))

    @property
    def n_actions(self) -> int:
        return int(self.bonds.shape[0])

    def core_offset(self, a: int, k: int) -> int:
        off = 0
        for b in range(self.n_actions):
            for j in range(self.n_dims):
                if b == a and j == k:
                    return off
                m = int(self.sizes[j])
                off += int(self.bonds[b, j]) * m * m * int(self.bonds[b, j + 1])
        raise IndexError((a, k))

    def core(self, a: int, k: int) -> np.ndarray:
        """View of G_k of action a as [b_k, m_k, m_k, b_{k+1}]."""
        m = int(self.sizes[k])
        bl, br = int(self.bonds[a, k]), int(self.bonds[a, k + 1])
        off = self.core_offset(a, k)
        return self.cores[off:off + bl * m * m * br].reshape(bl, m, m, br)


def random_tt(sizes, n_actions: int, bond: int, seed: int, gamma: float = 0.9,
              alpha: float = 1.0, n_terminal: int = 0, reward_scale: float = 1.0,
              name: str = "random_tt") -> TTInstance:
    """Row-stochastic Tensor-Train operators: core k is
    G[l, i, j, r] = w[l, i, r] * T[l, r, i, j] with w[l, i, :] ~ Dirichlet(1)
    over the right bond and T[l, r, i, :] ~ Dirichlet(alpha) over the next
    coordinate.  Then sum_{j, r} G[l, i, j, r] = 1 for every (l, i), so the
    bond matrices sum_j G[:, i, j, :] are row-stochastic and so is every
    P_a (a hidden chain over the bond index moving along the dimensions).
    Internal bonds are all `bond` (clipped to 1 at both ends)."""
    rng = np.random.default_rng(seed)
    sizes = [int(m) for m in sizes]
    n = len(sizes)
    S = int(np.prod(sizes))
    bonds = np.full((n_actions, n + 1), int(bond), np.int32)
    bonds[:, 0] = 1
    bonds[:, n] = 1
    blocks = []
    for a in range(n_actions):
        for k in range(n):
            m, bl, br = sizes[k], int(bonds[a, k]), int(bonds[a, k + 1])
            w = rng.dirichlet(np.ones(br), size=(bl, m))                  # [l, i, r]
            T = rng.dirichlet(alpha * np.ones(m), size=(bl, br, m))       # [l, r, i, j]
            T = T / T.sum(axis=-1, keepdims=True)
            G = w[:, :, None, :] * np.transpose(T, (0, 2, 3, 1))           # [l, i, j, r]
            blocks.append(np.ascontiguousarray(G).ravel())
    R = rng.normal(0.0, reward_scale, S)
    term = np.zeros(S, np.uint8)
    if n_terminal:
        term[rng.choice(S, n_terminal, replace=False)] = 1
    return TTInstance(np.asarray(sizes, np.int64), bonds, np.concatenate(blocks), R,
                      float(gamma), term, name, {"alpha": alpha, "bond": bond})


def tt_grid(m: int = 16, n: int = 6, n_actions: int = 12, bond: int = 4,
            seed: int = SEED_TT6, gamma: float = 0.95, alpha: float = 0.5) -> TTInstance:
    """The dense-factor grid's shape (m^n states, 12 actions, Dirichlet(alpha)
    coordinate rows, rewards N(0, 0.1), no terminals) with Tensor-Train
    transitions of internal bond `bond`."""
    return random_tt([m] * n, n_actions, bond, seed, gamma=gamma, alpha=alpha,
                     reward_scale=0.1, name=f"tt_{m}^{n}_b{bond}")


@dataclass
class TuckerInstance:
    """An MDP whose transition operator of each action is in Tucker form over
    the dimensions (Sec. 5 names Tucker as a future transition model):
        P_a = sum_{r_0..r_{n-1}} C_a[r_0, .., r_{n-1}] kron_k U^{(k)}_{a, r_k}
    with a core C_a of shape R_{a,0} x .. x R_{a,n-1} and R_{a,k} row-stochastic
    m_k x m_k factors per dimension.  The CP form is the special case of a
    diagonal core.  Flat layouts (the C ABI's): cores action-major, each
    row-major; factors action-major, then k, then r_k, one m_k x m_k
    row-major block each."""

    sizes: np.ndarray            # int64 [n]
    core_ranks: np.ndarray       # int32 [A, n]
    cores: np.ndarray            # float64 flat
    factors: np.ndarray          # float64 flat
    rewards: np.ndarray          # float64 [S]
    gamma: float
    terminal: np.ndarray         # uint8 [S]
    name: str = ""
    meta: Dict[str, float] = field(default_factory=dict)
    obstacle: Optional[np.ndarray] = None   # always None

    @property
    def n_dims(self) -> int:
        return int(self.sizes.shape[0])

    @property
    def n_states(self) -> int:
        return int(np.prod(self.sizes))

    @property
    def n_actions(self) -> int:
        return int(self.core_ranks.shape[0])

    def core(self, a: int) -> np.ndarray:
        off = sum(int(np.prod(self.core_ranks[b])) for b in range(a))
        shape = tuple(int(r) for r in self.core_ranks[a])
        return self.cores[off:off + int(np.prod(shape))].reshape(shape)

    def factor(self, a: int, k: int, r: int) -> np.ndarray:
        off = 0
        for b in range(self.n_actions):
            for j in range(self.n_dims):
                m = int(self.sizes[j])
                for q in range(int(self.core_ranks[b, j])):
                    if (b, j, q) == (a, k, r):
                        return self.factors[off:off + m * m].reshape(m, m)
                    off += m * m
        raise IndexError((a, k, r))


def random_tucker(sizes, n_actions: int, core_ranks, seed: int, gamma: float = 0.9,
                  alpha: float = 1.0, n_terminal: int = 0,
                  name: str = "random_tucker") -> TuckerInstance:
    """Tucker operators with a Dirichlet(1) core over all its entries (a
    probability mixture) and Dirichlet(alpha) factor rows: every P_a is
    row-stochastic.  core_ranks: one rank per dimension (all actions) or an
    [A, n] array."""
    rng = np.random.default_rng(seed)
    sizes = [int(m) for m in sizes]
    n = len(sizes)
    S = int(np.prod(sizes))
    cr = np.asarray(core_ranks, np.int32)
    if cr.ndim == 1:
        cr = np.tile(cr, (n_actions, 1))
    cores, facs = [], []
    for a in range(n_actions):
        cores.append(rng.dirichlet(np.ones(int(np.prod(cr[a])))))
        for k in range(n):
            for _r in range(int(cr[a, k])):
                U = rng.dirichlet(alpha * np.ones(sizes[k]), size=sizes[k])
                facs.append((U / U.sum(axis=1, keepdims=True)).ravel())
    term = np.zeros(S, np.uint8)
    if n_terminal:
        term[rng.choice(S, n_terminal, replace=False)] = 1
    return TuckerInstance(np.asarray(sizes, np.int64), cr, np.concatenate(cores),
                          np.concatenate(facs), rng.normal(0.0, 1.0, S), float(gamma), term,
                          name)


# ------------------------------------------------------- CP fitting inputs

def transition_coo(inst: Instance, a: int):
    """The transition matrix P_a of a shift/identity (GridWorld) instance as
    COO triples (s, s', P(s'|s,a)), one per successor, rows in state order:
    the tabular input that CP fitting starts from.  Built by moving an agent
    (no Kronecker product is formed)."""
    sizes = [int(m) for m in inst.sizes]
    n = len(sizes)
    S = inst.n_states
    strides = [int(np.prod(sizes[k + 1:])) for k in range(n)]
    coords = np.stack(np.unravel_index(np.arange(S), sizes), axis=1)
    src = np.arange(S, dtype=np.int64)
    rows, cols, vals = [], [], []
    for t in inst.terms_of(a):
        tgt = src.copy()
        for k in range(n):
            T = inst.factor(t, k)
            m = sizes[k]
            if np.array_equal(T, np.eye(m)):
                continue
            step = +1 if np.array_equal(T, shift_matrix(m, 1)) else -1
            assert np.array_equal(T, shift_matrix(m, step)), "shift/identity factors only"
            c = np.clip(coords[:, k] + step, 0, m - 1)
            tgt = tgt + (c - coords[:, k]) * strides[k]
        rows.append(src)
        cols.append(tgt)
        vals.append(np.full(S, float(inst.lambdas[t])))
    rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    key, inv = np.unique(rows * S + cols, return_inverse=True)
    merged = np.zeros(key.size)
    np.add.at(merged, inv, vals)
    return key // S, key % S, merged


def random_sparse_coo(sizes, nnz_per_row: int, seed: int):
    """A random row-stochastic sparse S x S matrix (nnz_per_row distinct
    successors per state, Dirichlet(1) weights) as COO triples."""
    rng = np.random.default_rng(seed)
    S = int(np.prod([int(m) for m in sizes]))
    k = min(nnz_per_row, S)
    rows = np.repeat(np.arange(S, dtype=np.int64), k)
    cols = np.concatenate([np.sort(rng.choice(S, k, replace=False)) for _ in range(S)])
    vals = rng.dirichlet(np.ones(k), size=S).ravel()
    return rows, cols, vals


def cp_fit_init(sizes, rank: int, seed: int) -> np.ndarray:
    """Seeded starting factors for CP fitting, in the flat term layout of
    cpmdp_create (term r, dim k, one m_k x m_k block): entries U(0.1, 1)."""
    rng = np.random.default_rng(seed)
    stride = sum(int(m) * int(m) for m in sizes)
    return rng.uniform(0.1, 1.0, rank * stride)
