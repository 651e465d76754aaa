"""GPU parity of the Def. 3 successor-list path (cpmdp_create_lists) against
the FP64 successor-list oracle (O2 built from the same lists), through the
C ABI."""
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


def _dt(prec):
    return torch.float64 if prec == 0 else torch.float32


CASES = {
    # successors near the state, S a multiple of 64
    "random_local_1024": lambda: I.random_lists(1024, 3, 5, seed=51, gamma=0.9, n_terminal=7,
                                                locality=40),
    # successors anywhere, ragged last slice (777 = 12 x 64 + 9), long lists
    "random_global_777": lambda: I.random_lists(777, 5, 9, seed=52, gamma=0.95, n_terminal=3),
    # one action, one state
    "single_state": lambda: I.random_lists(1, 1, 1, seed=53, gamma=0.5),
    # a GridWorld with walls written as lists (blocked moves stay put)
    "grid_walls_lists": lambda: I.paper_gridworld_lists(I.paper_gridworld([20, 30], 4, 40,
                                                                          seed=54)),
}


def _backup(B, model, V, prec, pi_in=None):
    Vin = torch.as_tensor(np.asarray(V), dtype=_dt(prec), device="cuda")
    Vout = torch.empty_like(Vin)
    if pi_in is None:
        pi = torch.full((model.S,), -7, dtype=torch.int32, device="cuda")
        r = B.cpmdp_backup(model.h, Vin, Vout, pi, residual=True, precision=prec)
    else:
        pi = torch.as_tensor(pi_in, device="cuda")
        r = B.cpmdp_policy_backup(model.h, Vin, Vout, pi, residual=False, precision=prec)
    torch.cuda.synchronize()
    return Vout.cpu().numpy().astype(np.float64), pi.cpu().numpy(), r


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", [0, 1])
def test_lists_backup_matches_oracle(B, name, prec):
    mdp = CASES[name]()
    log(f"[lists backup] {name} prec={prec}")
    model = B.Model(mdp)
    assert model.path == B.CPMDP_PATH_LISTS
    V = I.seeded_values(mdp.n_states, 5, scale=2.0)
    if prec == 1:
        V = V.astype(np.float32).astype(np.float64)
    mats = oracle.sparse.lists_csr(mdp)
    Q = oracle.sparse.q_values(mdp, mats, V)
    Vg, pig, r = _backup(B, model, V, prec)
    tol = 1e-13 * max(1, np.abs(V).max()) * 4 if prec == 0 else tol_for(1, Q.max(0))
    assert_close(Vg, Q.max(0), tol, "V'")
    assert abs(r - np.max(np.abs(Q.max(0) - V))) <= 2 * tol
    compare_policy(pig, Q, tol)
    pi = np.random.default_rng(7).integers(0, mdp.n_actions, mdp.n_states).astype(np.int32)
    ref = Q[pi, np.arange(mdp.n_states)]
    Eg, _, _ = _backup(B, model, V, prec, pi_in=pi)
    assert_close(Eg, ref, tol, "P_pi V")
    model.close()


def _solve(B, model, method, prec, eps, max_iter=200000):
    V = torch.zeros(model.S, dtype=torch.float64, device="cuda")
    pi = torch.zeros(model.S, dtype=torch.int32, device="cuda")
    if method == "vi":
        code, sweeps, res = B.cpmdp_value_iteration(model.h, V, pi, eps, max_iter, prec)
    else:
        code, _, sweeps, res = B.cpmdp_policy_iteration(model.h, V, pi, eps, max_iter, prec)
        code = B.CPMDP_OK if code == B.CPMDP_POLICY_UNSETTLED else code   # V certified; pi checked below
    torch.cuda.synchronize()
    return V.cpu().numpy(), pi.cpu().numpy(), code, sweeps, res


@pytest.mark.parametrize("name", ["random_local_1024", "grid_walls_lists"])
@pytest.mark.parametrize("method", ["vi", "pi"])
@pytest.mark.parametrize("prec", [0, 1])
def test_lists_solve_matches_oracle(B, name, method, prec):
    mdp = CASES[name]()
    log(f"[lists solve] {name} {method} prec={prec}")
    mats = oracle.sparse.lists_csr(mdp)
    Vs, _, _, _ = oracle.sparse.value_iteration(mdp, mats=mats)
    model = B.Model(mdp)
    eps = 0.5 * tol_for(prec, Vs) * (1 - mdp.gamma)
    V, pi, code, sweeps, res = _solve(B, model, method, prec, eps)
    assert code == B.CPMDP_OK and res <= eps
    assert_close(V, Vs, tol_for(prec, Vs), "V*")
    compare_policy(pi, oracle.sparse.q_values(mdp, mats, Vs), eps / (1 - mdp.gamma) + 1e-12)
    model.close()


def test_lists_reject_bf16(B):
    model = B.Model(CASES["random_local_1024"]())
    V = torch.zeros(model.S, dtype=torch.float64, device="cuda")
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_value_iteration(model.h, V, None, 1e-6, 100, B.CPMDP_BF16)
    assert e.value.code == B.CPMDP_E_UNSUPPORTED
    model.close()


def test_paper2d_lists_and_stencil_agree(B):
    """The 1000 x 1000 Table 1 GridWorld solved twice to eps = 1e-6 (FP32
    sweeps + FP64 certificate): once from its Kronecker factors (stencil
    path), once from its Def. 3 lists.  Both are certified, so both values
    lie within res / (1 - gamma) of V*; the policies agree wherever the
    greedy choice is decided by more than that."""
    inst = I.named("paper2d_1000")
    lists = I.paper_gridworld_lists(inst)
    log("[lists] paper 1000x1000: lists vs stencil")
    out = []
    for mdp in (inst, lists):
        model = B.Model(mdp)
        V, pi, code, sweeps, res = _solve(B, model, "vi", 1, 1e-6)
        assert code == B.CPMDP_OK and res <= 1e-6
        out.append((V, pi, res))
        model.close()
    (V1, pi1, r1), (V2, pi2, r2) = out
    bound = (r1 + r2) / (1 - inst.gamma)
    assert np.max(np.abs(V1 - V2)) <= bound + 1e-9
    rng = np.random.default_rng(55)
    states = np.unique(np.concatenate([rng.integers(0, inst.n_states, 2000),
                                       np.nonzero(inst.obstacle)[0][:100] + 1]))
    states = states[states < inst.n_states]
    Q = oracle.sparse.q_at_states(inst, V1, states)
    compare_policy(pi2[states], Q, bound + 1e-9)
