"""Pins of the Tensor-Train / Tucker oracle (O4) against facts it does not
compute itself: the CP special cases (pinned separately), an agent's moves
simulated state by state, single entries as explicit matrix products, and the
row-stochastic invariant the generators guarantee.  Two planted mistakes
(a transposed core, swapped bond axes) must fail these pins."""
import numpy as np
import pytest

import oracle
from oracle import tt as O4
from paper_2103_00331_amd import instances as I
from tests.tt_helpers import cp_as_tt, cp_as_tucker, mixture_move_tt


def test_tt_bond_one_is_kronecker_product():
    """Bonds of 1 make P_a the Kronecker product of the cores: a rank-1 CP
    term, expanded by O1."""
    cp = I.random_dense([3, 4, 2], 2, 1, seed=70)
    tt = cp_as_tt(cp)
    assert np.all(tt.bonds == 1)
    np.testing.assert_allclose(O4.tt_transition_matrices(tt),
                               oracle.dense.transition_matrices(cp), rtol=0, atol=1e-15)


@pytest.mark.parametrize("sizes,rank", [([3, 4, 2], 3), ([5, 3], 2), ([2, 3, 2, 2], 4), ([7], 3)])
def test_tt_diagonal_bonds_equal_cp(sizes, rank):
    cp = I.random_dense(sizes, 3, rank, seed=71, n_terminal=1)
    tt = cp_as_tt(cp)
    np.testing.assert_allclose(O4.tt_transition_matrices(tt),
                               oracle.dense.transition_matrices(cp), rtol=0, atol=1e-14)


def test_tt_mixture_of_moves_matches_simulation():
    """A bond of 2 encodes 'with probability p move +1 along dim 0, else +1
    along dim 1'; P built by moving an agent from every state."""
    m0, m1, p = 5, 4, 0.3
    tt = mixture_move_tt((m0, m1), p)
    P = np.zeros((m0 * m1, m0 * m1))
    for x in range(m0):
        for y in range(m1):
            s = x * m1 + y
            P[s, min(x + 1, m0 - 1) * m1 + y] += p
            P[s, x * m1 + min(y + 1, m1 - 1)] += 1 - p
    np.testing.assert_allclose(O4.tt_transition_matrices(tt)[0], P, rtol=0, atol=1e-15)


@pytest.mark.parametrize("bond", [1, 2, 3])
def test_tt_rows_stochastic(bond):
    tt = I.random_tt([3, 2, 4, 2], 3, bond, seed=72)
    P = O4.tt_transition_matrices(tt)
    assert P.min() >= 0.0
    np.testing.assert_allclose(P.sum(axis=2), 1.0, rtol=0, atol=1e-13)


def test_tt_entries_by_explicit_products():
    tt = I.random_tt([3, 4, 2], 2, 3, seed=73)
    P = O4.tt_transition_matrices(tt)
    rng = np.random.default_rng(0)
    for _ in range(40):
        a, s, t = int(rng.integers(2)), int(rng.integers(24)), int(rng.integers(24))
        assert abs(P[a, s, t] - O4.tt_entry(tt, a, s, t)) <= 1e-15


def test_tt_rows_and_q_at_states():
    tt = I.random_tt([4, 3, 5], 3, 2, seed=74, n_terminal=3)
    P = O4.tt_transition_matrices(tt)
    V = I.seeded_values(tt.n_states, 75)
    Q = oracle.dense.q_values(tt, P, V)
    states = [0, 7, 31, 59] + list(np.flatnonzero(tt.terminal))
    np.testing.assert_allclose(O4.tt_q_at_states(tt, V, states), Q[:, states], rtol=0, atol=1e-13)
    for s in states:
        np.testing.assert_allclose(O4.tt_row(tt, 1, s), P[1, s], rtol=0, atol=1e-15)


def test_tucker_superdiagonal_core_equals_cp():
    cp = I.random_dense([3, 4, 2], 2, 3, seed=76)
    tk = cp_as_tucker(cp)
    np.testing.assert_allclose(O4.tucker_transition_matrices(tk),
                               oracle.dense.transition_matrices(cp), rtol=0, atol=1e-14)


def test_tucker_rank_one_is_kronecker_product():
    tk = I.random_tucker([3, 2, 4], 2, [1, 1, 1], seed=77)
    for a in range(2):
        K = np.ones((1, 1))
        for k in range(3):
            K = np.kron(K, tk.factor(a, k, 0))
        # a rank-1 core is the single weight 1, so P_a is the Kronecker product
        assert tk.core(a).reshape(-1)[0] == pytest.approx(1.0, abs=1e-15)
        np.testing.assert_allclose(O4.tucker_matrix(tk, a), K, rtol=0, atol=1e-15)


def test_tucker_rows_stochastic_and_entries():
    tk = I.random_tucker([3, 2, 4], 2, [2, 3, 2], seed=78)
    P = O4.tucker_transition_matrices(tk)
    assert P.min() >= 0.0
    np.testing.assert_allclose(P.sum(axis=2), 1.0, rtol=0, atol=1e-13)
    rng = np.random.default_rng(1)
    for _ in range(30):
        a, s, t = int(rng.integers(2)), int(rng.integers(24)), int(rng.integers(24))
        assert abs(P[a, s, t] - O4.tucker_entry(tk, a, s, t)) <= 1e-15


def test_tt_value_iteration_matches_cp_policy_enumeration():
    """VI through the TT operator reaches the optimum that brute-force policy
    enumeration finds on the same operator written in CP form."""
    cp = I.random_dense([2, 3], 2, 2, seed=79, gamma=0.8)
    tt = cp_as_tt(cp)
    P = O4.tt_transition_matrices(tt)
    V, pi, _, res = oracle.dense.value_iteration(tt, eps=1e-13, P=P)
    vstar, optimal = oracle.dense.brute_force(cp)
    np.testing.assert_allclose(V, vstar, rtol=0, atol=1e-10)
    assert all(int(pi[s]) in optimal[s] for s in range(cp.n_states))


# ---------------------------------------------------------- planted mistakes

class _TransposedCores:
    """A TT instance whose cores come back with row and column coordinates
    swapped (a transposed operand)."""

    def __init__(self, inst):
        self._i = inst

    def __getattr__(self, k):
        return getattr(self._i, k)

    def core(self, a, k):
        return np.transpose(self._i.core(a, k), (0, 2, 1, 3))


class _SwappedBonds(_TransposedCores):
    def core(self, a, k):
        G = self._i.core(a, k)
        return np.transpose(G, (3, 1, 2, 0)) if G.shape[0] == G.shape[3] else G


@pytest.mark.parametrize("planted", [_TransposedCores, _SwappedBonds])
def test_planted_mistakes_fail_the_pins(planted):
    tt = I.random_tt([3, 2, 4], 2, 3, seed=80)
    bad = planted(tt)
    P = O4.tt_transition_matrices(bad)
    assert np.abs(P.sum(axis=2) - 1.0).max() > 1e-3
    if planted is _TransposedCores:
        mv = planted(mixture_move_tt((5, 4), 0.3))
        assert np.abs(O4.tt_transition_matrices(mv)[0].sum(axis=1) - 1.0).max() > 0.1
