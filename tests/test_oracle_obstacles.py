"""Pins of the oracle's obstacle reading (Sec. 3.2: obstacles are states the
agent has no access to; a move towards one leaves the agent where it is, and
an obstacle state holds value 0).  The checks come from outside the oracle:
the GridWorld's moves simulated cell by cell, a corridor's closed form,
brute-force policy enumeration and the per-state successor enumeration.
CPU only."""
import itertools

import numpy as np
import pytest

from oracle import dense, sparse, structured
from paper_2103_00331_amd import instances as I


def _simulated_P(sizes, slip, obstacle):
    """P[a, s, s'] of the slip GridWorld built by moving an agent: action
    a = 2k + d moves along dim k (d = 0: +1, d = 1: -1) with probability
    1 - slip, or one step along another dim with slip / (2(n-1)) each; a move
    that leaves the grid or lands on an obstacle keeps the agent at s."""
    n = len(sizes)
    S = int(np.prod(sizes))
    P = np.zeros((2 * n, S, S))
    for s, coords in enumerate(itertools.product(*[range(m) for m in sizes])):
        for a in range(2 * n):
            k, step = a // 2, (1 if a % 2 == 0 else -1)
            moves = [(k, step, 1.0 if n == 1 else 1.0 - slip)]
            if n > 1:
                for j in range(n):
                    if j != k:
                        moves += [(j, +1, slip / (2 * (n - 1))), (j, -1, slip / (2 * (n - 1)))]
            for dim, st, p in moves:
                c = list(coords)
                c[dim] += st
                target = s
                if 0 <= c[dim] < sizes[dim]:
                    t = I.flat_index(sizes, c)
                    if not obstacle[t]:
                        target = t
                P[a, s, target] += p
    return P


def _grid_with_walls():
    g = I.grid_small([4, 5], slip=0.2, gamma=0.9, seed=3)
    return I.with_obstacles(g, [I.flat_index([4, 5], c) for c in [(1, 1), (1, 2), (2, 3), (0, 4)]])


def test_obstacle_transitions_match_move_simulation():
    inst = _grid_with_walls()
    live = (inst.terminal == 0) & (inst.obstacle == 0)
    ref = _simulated_P([4, 5], 0.2, inst.obstacle)
    P = dense.transition_matrices(inst)
    np.testing.assert_allclose(P[:, live, :], ref[:, live, :], atol=1e-15)
    mats = sparse.transition_csr(inst)
    for a, M in enumerate(mats):
        np.testing.assert_allclose(M.toarray()[live], ref[a, live], atol=1e-15)
        assert M.toarray()[~live].sum() == 0.0       # terminal / obstacle rows end
    # invariants: rows stay stochastic, nothing flows into an obstacle
    np.testing.assert_allclose(P.sum(axis=2), 1.0, atol=1e-14)
    assert np.all(P[:, live][:, :, inst.obstacle == 1] == 0.0)


@pytest.mark.parametrize("tier", ["dense", "sparse"])
def test_obstacle_corridor_closed_form(tier):
    """1-D corridor of 7 cells, goal G (terminal) at 6, obstacle at 2, step
    reward c, no slip.  Right of the obstacle: V(i) = c (1 - g^d)/(1 - g) +
    g^d G with d = 6 - i and move +1; the obstacle holds 0; left of it the
    agent is walled in: V = c / (1 - g), and both actions tie (lowest index
    reported)."""
    m, c, G, g = 7, -0.1, 1.0, 0.9
    inst = I.with_obstacles(I.chain_1d(m, c, G, g), [2])
    mod = {"dense": dense, "sparse": sparse}[tier]
    V, pi, _, res = mod.value_iteration(inst)
    assert res <= 1e-12
    d = 6 - np.arange(m)
    expect = c * (1 - g ** d) / (1 - g) + g ** d * G
    expect[2] = 0.0
    expect[:2] = c / (1 - g)
    np.testing.assert_allclose(V, expect, atol=1e-11)
    assert list(pi[3:6]) == [0, 0, 0]
    assert list(pi[:2]) == [0, 0]
    if tier == "dense":
        Vp, pip, _ = dense.policy_iteration(inst)
        np.testing.assert_allclose(Vp, expect, atol=1e-11)


@pytest.mark.parametrize("cells", [[1], [2, 5]])
def test_obstacle_brute_force_enumeration(cells):
    """V* over all A^S policies (obstacle rows have no continuation, so any
    action there is optimal); VI and PI of both tiers reach it."""
    base = I.make_gridworld([2, 4], 0.2, [-0.04] * 8, 0.9,
                            terminals=[((1, 3), 1.0)])
    inst = I.with_obstacles(base, cells)
    vstar, optimal = dense.brute_force(inst)
    assert np.all(vstar[cells] == 0.0)
    for mod in (dense, sparse):
        V, pi, _, _ = mod.value_iteration(inst)
        np.testing.assert_allclose(V, vstar, atol=1e-10)
        for s in range(inst.n_states):
            assert int(pi[s]) in optimal[s]
    Vp, _, _ = dense.policy_iteration(inst)
    np.testing.assert_allclose(Vp, vstar, atol=1e-10)
    Vs, _, _ = sparse.policy_iteration(inst)
    np.testing.assert_allclose(Vs, vstar, atol=1e-10)


def test_obstacle_per_state_q_matches_dense():
    inst = _grid_with_walls()
    V = I.seeded_values(inst.n_states, 11)
    Q = dense.q_values(inst, dense.transition_matrices(inst), V)
    states = np.arange(inst.n_states)
    np.testing.assert_allclose(sparse.q_at_states(inst, V, states), Q, atol=1e-13)


def test_paper_gridworld_generator():
    g = I.paper_gridworld([30, 40], 6, 50, seed=1)
    assert g.terminal.sum() == 6 and g.obstacle.sum() == 50
    assert not np.any(g.terminal & g.obstacle)
    assert sorted(set(g.rewards[g.terminal == 1])) == [-100.0, 100.0]
    assert np.all(g.rewards[(g.terminal == 0)] == -3.0)


def test_structured_refuses_obstacles():
    with pytest.raises(ValueError):
        structured.value_iteration(_grid_with_walls())


def test_pins_catch_unredirected_obstacle_moves(monkeypatch):
    """Leaving the probability on the obstacle column (instead of moving it
    to the source state) must fail the move simulation."""
    def no_fold(inst):
        P = np.zeros((inst.n_actions, inst.n_states, inst.n_states))
        for a in range(inst.n_actions):
            for t in inst.terms_of(a):
                K = np.ones((1, 1))
                for k in range(inst.n_dims):
                    K = np.kron(K, inst.factor(t, k))
                P[a] += inst.lambdas[t] * K
        return P
    monkeypatch.setattr(dense, "transition_matrices", no_fold)
    with pytest.raises(AssertionError):
        test_obstacle_transitions_match_move_simulation()


def test_pins_catch_obstacle_reward(monkeypatch):
    """Giving an obstacle its own reward must fail the corridor closed form."""
    import oracle.dense as od
    monkeypatch.setattr(od, "rewards_of", lambda inst: inst.rewards)
    monkeypatch.setattr(od, "continuation", lambda inst: inst.gamma * (1.0 - inst.terminal))
    with pytest.raises(AssertionError):
        test_obstacle_corridor_closed_form("dense")


# ------------------------------------------------ Def. 3 lists given directly

@pytest.mark.parametrize("case", ["plain", "walls"])
def test_lists_by_move_simulation_equal_cp_successor_lists(case):
    """The GridWorld written as Def. 3 lists by moving an agent equals the
    successor lists that O2 enumerates from the Kronecker factors (two
    independent constructions of the same operator)."""
    inst = I.grid_small([5, 4, 6], slip=0.2, gamma=0.95, seed=8)
    if case == "walls":
        inst = I.with_obstacles(inst, [3, 17, 40, 41, 42, 77])
    lists = I.gridworld_lists([5, 4, 6], 0.2, inst.rewards, inst.gamma, inst.terminal,
                              inst.obstacle)
    A = sparse.lists_csr(lists)
    Bm = sparse.transition_csr(inst)
    for a in range(inst.n_actions):
        assert abs(A[a] - Bm[a]).max() <= 1e-15
    V1, pi1, _, _ = sparse.value_iteration(lists, mats=A)
    V2, pi2, _, _ = sparse.value_iteration(inst, mats=Bm)
    np.testing.assert_allclose(V1, V2, atol=1e-12)
    assert np.array_equal(pi1, pi2)


def test_lists_random_mdp_brute_force():
    """A random MDP with no structure, as lists: VI and PI of O2 reach the
    elementwise maximum over all A^S deterministic policies (each evaluated
    by an exact linear solve)."""
    mdp = I.random_lists(7, 3, 3, seed=9, gamma=0.85, n_terminal=1)
    mats = sparse.lists_csr(mdp)
    P = np.stack([M.toarray() for M in mats])
    S = mdp.n_states
    live = mdp.terminal == 0
    np.testing.assert_allclose(P[:, live].sum(axis=2), 1.0, atol=1e-14)
    best = np.full(S, -np.inf)
    for pol in itertools.product(range(mdp.n_actions), repeat=S):
        P_pi = P[np.asarray(pol), np.arange(S), :]
        V = np.linalg.solve(np.eye(S) - mdp.gamma * P_pi, mdp.rewards)
        best = np.maximum(best, V)
    V, _, _, res = sparse.value_iteration(mdp, mats=mats)
    assert res <= 1e-12
    np.testing.assert_allclose(V, best, atol=1e-10)
    Vp, _, _ = sparse.policy_iteration(mdp, mats=mats)
    np.testing.assert_allclose(Vp, best, atol=1e-10)
