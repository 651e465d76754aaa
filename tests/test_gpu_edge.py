"""GPU parity at the degenerate ends of the problem statement, through the C
ABI: no discount, every state terminal, the maximum number of dimensions,
dimensions of size 1 (on both kernel paths) and successor lists with
repeated successors."""
import numpy as np
import pytest

import oracle
from paper_2103_00331_amd import instances as I
from tests.parity import assert_close, compare_policy, log, tol_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    from paper_2103_00331_amd import binding
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return binding


def _vi(B, inst, prec, eps):
    model = B.Model(inst)
    V = torch.zeros(inst.n_states, dtype=torch.float64, device="cuda")
    pi = torch.zeros(inst.n_states, dtype=torch.int32, device="cuda")
    code, sweeps, res = B.cpmdp_value_iteration(model.h, V, pi, eps, 200000, prec)
    torch.cuda.synchronize()
    model.close()
    return V.cpu().numpy(), pi.cpu().numpy(), code, sweeps, res


def _backup(B, inst, V, prec):
    model = B.Model(inst)
    dt = torch.float64 if prec == 0 else torch.float32
    Vin = torch.as_tensor(V, dtype=dt, device="cuda")
    Vout = torch.empty_like(Vin)
    pi = torch.full((inst.n_states,), -1, dtype=torch.int32, device="cuda")
    B.cpmdp_backup(model.h, Vin, Vout, pi, residual=False, precision=prec)
    torch.cuda.synchronize()
    model.close()
    return Vout.cpu().numpy().astype(np.float64), pi.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
def test_no_discount(B, prec):
    """gamma = 0: every action gives Q_a = R, so V* = R and every state
    reports action 0 (exact ties, lowest index)."""
    inst = I.grid_small([6, 8, 4], slip=0.2, gamma=0.0, seed=61)
    log(f"[edge] gamma = 0, prec={prec}")
    V, pi, code, sweeps, res = _vi(B, inst, prec, 1e-12)
    assert code == B.CPMDP_OK and res <= 1e-12
    np.testing.assert_array_equal(V, inst.rewards)
    assert np.all(pi == 0)


def test_every_state_terminal(B):
    """All states terminal: V* = R after one sweep, action 0 everywhere."""
    g = I.grid_small([5, 7], slip=0.1, gamma=0.95, seed=62)
    inst = I.with_rewards(g, g.rewards, terminal=np.ones(g.n_states, np.uint8))
    log("[edge] every state terminal")
    V, pi, code, sweeps, res = _vi(B, inst, 0, 1e-12)
    assert code == B.CPMDP_OK and res == 0.0
    np.testing.assert_array_equal(V, inst.rewards)
    assert np.all(pi == 0)


@pytest.mark.parametrize("prec", [0, 1])
def test_eight_dimensions(B, prec):
    """n = 8 (the most the library takes): 16 actions of rank 15."""
    inst = I.grid_small([2, 2, 3, 2, 2, 3, 2, 2], slip=0.2, gamma=0.9, seed=63)
    log(f"[edge] 8 dimensions, prec={prec}")
    P = oracle.dense.transition_matrices(inst)
    V0 = I.seeded_values(inst.n_states, 64, scale=2.0)
    if prec == 1:
        V0 = V0.astype(np.float32).astype(np.float64)
    Q = oracle.dense.q_values(inst, P, V0)
    Vg, pig = _backup(B, inst, V0, prec)
    tol = 4e-13 * max(1.0, np.abs(V0).max()) if prec == 0 else tol_for(1, Q.max(0))
    assert_close(Vg, Q.max(0), tol, "V'")
    compare_policy(pig, Q, tol)
    Vs, _, _, _ = oracle.dense.value_iteration(inst, P=P)
    eps = 0.5 * tol_for(prec, Vs) * (1 - inst.gamma)
    V, pi, code, sweeps, res = _vi(B, inst, prec, eps)
    assert code == B.CPMDP_OK and res <= eps
    assert_close(V, Vs, tol_for(prec, Vs), "V*")
    compare_policy(pi, oracle.dense.q_values(inst, P, Vs), eps / (1 - inst.gamma) + 1e-12)


UNIT = {
    # shift/identity factors with size-1 dims (a move along them stays put);
    # last side 8: four states per lane
    "stencil_5x1x8": lambda: I.grid_small([5, 1, 8], slip=0.2, gamma=0.9, seed=65),
    # last side 1: one state per lane
    "stencil_4x6x1": lambda: I.grid_small([4, 6, 1], slip=0.1, gamma=0.95, seed=66),
    # dense factors with a size-1 mode (the mode product is a scalar multiply)
    "dense_3x1x4": lambda: I.random_dense([3, 1, 4], 3, 2, seed=67, gamma=0.9),
}


@pytest.mark.parametrize("name", list(UNIT))
@pytest.mark.parametrize("prec", [0, 1])
def test_size_one_dimensions(B, name, prec):
    inst = UNIT[name]()
    log(f"[edge] size-1 dims {name} prec={prec}")
    P = oracle.dense.transition_matrices(inst)
    Vs, _, _, _ = oracle.dense.value_iteration(inst, P=P)
    eps = 0.5 * tol_for(prec, Vs) * (1 - inst.gamma)
    V, pi, code, sweeps, res = _vi(B, inst, prec, eps)
    assert code == B.CPMDP_OK and res <= eps
    assert_close(V, Vs, tol_for(prec, Vs), "V*")
    compare_policy(pi, oracle.dense.q_values(inst, P, Vs), eps / (1 - inst.gamma) + 1e-12)


def test_lists_with_repeated_successors(B):
    """Def. 3 lists where a successor appears several times in one list (its
    probabilities add up), against the oracle built from the same lists."""
    base = I.random_lists(300, 3, 4, seed=68, gamma=0.9, n_terminal=2, locality=20)
    # split every entry in two halves with the same successor
    S, A = base.n_states, base.n_actions
    counts = np.diff(base.row_ptr)
    ptr = np.concatenate([[0], np.cumsum(2 * counts)])
    succ = np.repeat(base.succ, 2)
    prob = np.repeat(base.prob / 2.0, 2)
    dup = I.ListsMDP(S, A, ptr.astype(np.int64), succ, prob, base.rewards.copy(), base.gamma,
                     base.terminal.copy(), "dup_lists")
    log("[edge] repeated successors in lists")
    mats = oracle.sparse.lists_csr(dup)
    Vs, _, _, _ = oracle.sparse.value_iteration(dup, mats=mats)
    V, pi, code, sweeps, res = _vi(B, dup, 0, 1e-11)
    assert code == B.CPMDP_OK and res <= 1e-11
    assert_close(V, Vs, 1e-9, "V*")
    compare_policy(pi, oracle.sparse.q_values(dup, mats, Vs), 1e-9)


# ------------------------------------------- Tensor-Train / Tucker, CP fitting

def _tt_vi(B, inst, prec, eps):
    return _vi(B, inst, prec, eps)


@pytest.mark.parametrize("prec", [0, 1])
def test_tt_no_discount_and_all_terminal(B, prec):
    """Tensor-Train operators at the degenerate ends: gamma = 0 gives V* = R
    with action 0 everywhere; every state terminal gives the same after one
    sweep."""
    from oracle import tt as O4  # noqa: F401  (operators are irrelevant here)
    t0 = I.random_tt([16, 16, 3], 3, 2, seed=71, gamma=0.0)
    log(f"[edge] tt gamma = 0, prec={prec}")
    V, pi, code, sweeps, res = _tt_vi(B, t0, prec, 1e-12)
    assert code == B.CPMDP_OK and res <= 1e-12
    np.testing.assert_array_equal(V, t0.rewards)
    assert np.all(pi == 0)
    t1 = I.random_tt([5, 4], 2, 3, seed=72, gamma=0.9)
    t1.terminal[:] = 1
    V, pi, code, sweeps, res = _tt_vi(B, t1, prec, 1e-12)
    assert code == B.CPMDP_OK and res == 0.0
    np.testing.assert_array_equal(V, t1.rewards)


@pytest.mark.parametrize("prec", [0, 1])
def test_tt_eight_dimensions(B, prec):
    """n = 8 (the most the library takes) with bond 2 and mixed sizes."""
    from oracle import tt as O4
    t = I.random_tt([2, 3, 2, 2, 3, 2, 2, 2], 2, 2, seed=73, gamma=0.9, n_terminal=3)
    log(f"[edge] tt 8 dimensions, prec={prec}")
    P = O4.tt_transition_matrices(t)
    Vs, _, _, _ = oracle.dense.value_iteration(t, P=P)
    eps = 0.5 * tol_for(prec, Vs) * (1 - t.gamma)
    V, pi, code, sweeps, res = _tt_vi(B, t, prec, eps)
    assert code == B.CPMDP_OK and res <= eps
    assert_close(V, Vs, tol_for(prec, Vs), "V*")
    compare_policy(pi, oracle.dense.q_values(t, P, Vs), eps / (1 - t.gamma) + 1e-12)


def _cp_dev(coo):
    r, c, v = coo
    return (torch.as_tensor(np.asarray(r, np.int32), device="cuda"),
            torch.as_tensor(np.asarray(c, np.int32), device="cuda"),
            torch.as_tensor(np.asarray(v, np.float64), device="cuda"))


def test_cp_fit_rank_one_eight_dims_and_entry_order(B):
    """CP fitting at rank 1 and on an 8-dimensional grid against the oracle
    from the same start; repeated or unsorted entries are rejected (the
    reported error needs distinct entries)."""
    from oracle import cpfit as O5
    sizes = [3, 4, 2]
    r, c, v = I.random_sparse_coo(sizes, 4, seed=74)
    log("[edge] cp fit: rank 1, 8 dims, entry order")
    for bad in ((np.repeat(r, 2), np.repeat(c, 2), np.repeat(v / 2.0, 2)),
                (r[::-1].copy(), c[::-1].copy(), v[::-1].copy())):
        with pytest.raises(B.CpmdpError) as e:
            B.cpmdp_cp_fit(sizes, *_cp_dev(bad), 2, I.cp_fit_init(sizes, 2, seed=76), max_iter=2)
        assert e.value.code == B.CPMDP_E_ARG
    for coo, R, sz in (((r, c, v), 1, sizes),
                       (I.random_sparse_coo([2] * 8, 3, seed=75), 2, [2] * 8)):
        init = I.cp_fit_init(sz, R, seed=76)
        fac, lam, errs, it = B.cpmdp_cp_fit(sz, *_cp_dev(coo), R, init, max_iter=5)
        A_ref, l_ref, e_ref = O5.als(O5.dense_tensor(sz, *coo), O5.factors_from_flat(sz, R, init), it)
        A = O5.factors_from_flat(sz, R, fac)
        for a, b in zip(A, A_ref):
            assert np.abs(a - b).max() <= 1e-9
        assert np.abs(lam - l_ref).max() <= 1e-9 * max(1.0, l_ref.max())
        assert np.abs(errs - e_ref).max() <= 1e-7
