"""Pins of the CP-fitting oracle (O5): the tensor and CP conventions against a
GridWorld built by move simulation, the matricised-tensor-times-Khatri-Rao
product against brute-force loops, every ALS update against an explicit
least-squares solve, and closed-form ALS behaviour (one-iteration recovery of
a rank-one tensor, a fixed point at an exact CP model, monotone error).  Two
planted mistakes must fail."""
import itertools

import numpy as np
import pytest

from oracle import cpfit as O5
from paper_2103_00331_amd import instances as I


def _true_factors(inst, a):
    """The instance's own CP form of action a as (A^(k), lambda)."""
    terms = inst.terms_of(a)
    A = [np.stack([inst.factor(t, k).ravel() for t in terms], axis=1) for k in range(inst.n_dims)]
    return A, np.array([inst.lambdas[t] for t in terms])


@pytest.mark.parametrize("sizes", [[4, 3], [3, 2, 4], [5]])
def test_gridworld_tensor_is_its_cp_form(sizes):
    """P_a from move simulation, as the paired-coordinate tensor, equals the
    sum of outer products of the instance's vectorised factors (Sec. 2.2)."""
    g = I.grid_small(sizes, slip=0.2, seed=3)
    for a in range(g.n_actions):
        X = O5.dense_tensor(sizes, *I.transition_coo(g, a))
        A, lam = _true_factors(g, a)
        np.testing.assert_allclose(O5.reconstruct(A, lam), X, rtol=0, atol=1e-15)


def test_mttkrp_brute_force():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(3, 4, 2))
    A = [rng.normal(size=(d, 3)) for d in X.shape]
    for k in range(3):
        M = np.zeros((X.shape[k], 3))
        for idx in itertools.product(*[range(d) for d in X.shape]):
            for r in range(3):
                p = X[idx]
                for l in range(3):
                    if l != k:
                        p *= A[l][idx[l], r]
                M[idx[k], r] += p
        np.testing.assert_allclose(O5.mttkrp(X, A, k), M, rtol=1e-13, atol=1e-13)


def test_mttkrp_sparse_matches_dense():
    sizes = [3, 4, 2]
    coo = I.random_sparse_coo(sizes, 5, seed=1)
    X = O5.dense_tensor(sizes, *coo)
    rng = np.random.default_rng(2)
    A = [rng.uniform(size=(m * m, 4)) for m in sizes]
    for k in range(3):
        np.testing.assert_allclose(O5.mttkrp_sparse(sizes, *coo, A, k), O5.mttkrp(X, A, k),
                                   rtol=1e-13, atol=1e-14)


def _unfold(X, k):
    return np.moveaxis(X, k, 0).reshape(X.shape[k], -1)


def _khatri_rao_others(A, k):
    """Rows over the other modes in increasing order, last fastest (the
    column order of _unfold)."""
    R = A[0].shape[1]
    others = [A[l] for l in range(len(A)) if l != k]
    K = np.ones((1, R))
    for B in others:
        K = (K[:, None, :] * B[None, :, :]).reshape(-1, R)
    return K


def test_each_update_solves_its_least_squares_problem():
    sizes = [3, 2, 3]
    X = O5.dense_tensor(sizes, *I.random_sparse_coo(sizes, 4, seed=4))
    rng = np.random.default_rng(5)
    A = [rng.uniform(0.1, 1, size=(m * m, 3)) for m in sizes]
    for k in range(3):
        V = np.ones((3, 3))
        for l in range(3):
            if l != k:
                V *= A[l].T @ A[l]
        upd = O5.mttkrp(X, A, k) @ np.linalg.pinv(V)
        sol = np.linalg.lstsq(_khatri_rao_others(A, k), _unfold(X, k).T, rcond=None)[0].T
        np.testing.assert_allclose(upd, sol, rtol=1e-10, atol=1e-12)


def test_error_never_increases():
    sizes = [3, 3, 2]
    X = O5.dense_tensor(sizes, *I.random_sparse_coo(sizes, 6, seed=6))
    A0 = O5.factors_from_flat(sizes, 4, I.cp_fit_init(sizes, 4, seed=7))
    _, _, errs = O5.als(X, A0, 25)
    assert np.all(np.diff(errs) <= 1e-12), errs
    assert errs[-1] < errs[0]


def test_rank_one_recovered_in_one_iteration():
    rng = np.random.default_rng(8)
    a, b, c = rng.uniform(0.2, 1, 9), rng.uniform(0.2, 1, 4), rng.uniform(0.2, 1, 16)
    X = 0.7 * np.multiply.outer(np.multiply.outer(a, b), c)
    A0 = [rng.uniform(0.1, 1, (d, 1)) for d in X.shape]
    A, lam, errs = O5.als(X, A0, 1)
    assert errs[0] < 1e-13


def test_exact_cp_model_is_a_fixed_point():
    g = I.grid_small([4, 3], slip=0.2, seed=9)
    X = O5.dense_tensor([4, 3], *I.transition_coo(g, 1))
    A, lam = _true_factors(g, 1)
    A = [Ak / np.linalg.norm(Ak, axis=0) for Ak in A]
    A2, lam2, errs = O5.als(X, A, 3)
    assert errs.max() < 1e-13
    np.testing.assert_allclose(O5.reconstruct(A2, lam2), X, rtol=0, atol=1e-14)


def test_planted_rank_two_recovered_from_a_nearby_start():
    rng = np.random.default_rng(10)
    sizes = [3, 2, 3]
    At = [rng.normal(size=(m * m, 2)) for m in sizes]      # well-separated columns
    X = O5.reconstruct(At, np.array([0.6, 0.4]))
    A0 = [Ak * (1 + 0.05 * rng.normal(size=Ak.shape)) for Ak in At]
    _, _, errs = O5.als(X, A0, 40)
    assert errs[-1] < 1e-8


def test_flat_layout_round_trip():
    sizes = [3, 2]
    flat = I.cp_fit_init(sizes, 3, seed=11)
    A = O5.factors_from_flat(sizes, 3, flat)
    assert A[0].shape == (9, 3) and A[1].shape == (4, 3)
    np.testing.assert_array_equal(O5.factors_to_flat(A), flat)


# ---------------------------------------------------------- planted mistakes

def test_planted_mistakes_fail_the_pins(monkeypatch):
    sizes = [3, 2, 3]
    X = O5.dense_tensor(sizes, *I.random_sparse_coo(sizes, 4, seed=12))
    rng = np.random.default_rng(13)
    A = [rng.uniform(0.1, 1, size=(m * m, 3)) for m in sizes]

    good = O5.mttkrp

    def wrong_mode(X, A, k):        # contracts the other modes with shifted factors
        return good(X, [A[(l + 1) % len(A)] if l != k and A[(l + 1) % len(A)].shape == A[l].shape
                        else Ak for l, Ak in enumerate(A)], k)

    def transposed(X, A, k):        # pairs (j, i) instead of (i, j) in mode k
        m = int(round(np.sqrt(X.shape[k])))
        M = good(X, A, k)
        return M.reshape(m, m, -1).transpose(1, 0, 2).reshape(m * m, -1)

    for bad in (wrong_mode, transposed):
        monkeypatch.setattr(O5, "mttkrp", bad)
        caught = False
        for k in range(3):
            V = np.ones((3, 3))
            for l in range(3):
                if l != k:
                    V *= A[l].T @ A[l]
            upd = O5.mttkrp(X, A, k) @ np.linalg.pinv(V)
            sol = np.linalg.lstsq(_khatri_rao_others(A, k), _unfold(X, k).T, rcond=None)[0].T
            caught |= not np.allclose(upd, sol, rtol=1e-8, atol=1e-10)
        assert caught, bad.__name__
    monkeypatch.setattr(O5, "mttkrp", good)


def test_sparse_als_matches_dense_als():
    sizes = [3, 2, 3]
    coo = I.random_sparse_coo(sizes, 4, seed=14)
    X = O5.dense_tensor(sizes, *coo)
    A0 = O5.factors_from_flat(sizes, 3, I.cp_fit_init(sizes, 3, seed=15))
    Ad, ld, ed = O5.als(X, A0, 6)
    As, ls, es = O5.als_sparse(sizes, *coo, A0, 6)
    for a, b in zip(Ad, As):
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(ls, ld, rtol=1e-10)
    np.testing.assert_allclose(es, ed, rtol=0, atol=1e-8)
