"""GPU parity of the shift/identity (stencil) path against the FP64 oracle,
through the C ABI."""
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


def _backup(B, model, V, prec, with_pi=True):
    dt = _dt(prec)
    Vin = torch.as_tensor(np.asarray(V), dtype=dt, device="cuda")
    Vout = torch.empty_like(Vin)
    pi = torch.full((model.S,), -7, dtype=torch.int32, device="cuda") if with_pi else None
    r = B.cpmdp_backup(model.h, Vin, Vout, pi, residual=True, precision=prec)
    torch.cuda.synchronize()
    return (Vout.cpu().numpy().astype(np.float64),
            None if pi is None else pi.cpu().numpy(), r)


def _solve(B, model, method, prec, eps, V0=None, pi0=None, max_iter=200000):
    V = torch.zeros(model.S, dtype=torch.float64, device="cuda") if V0 is None else \
        torch.as_tensor(V0, dtype=torch.float64, device="cuda").clone()
    pi = torch.zeros(model.S, dtype=torch.int32, device="cuda") if pi0 is None else \
        torch.as_tensor(pi0, dtype=torch.int32, device="cuda").clone()
    if method == "vi":
        code, sweeps, res = B.cpmdp_value_iteration(model.h, V, pi, eps, max_iter, prec)
        outer = 0
    else:
        code, outer, sweeps, res = B.cpmdp_policy_iteration(model.h, V, pi, eps, max_iter, prec)
        code = B.CPMDP_OK if code == B.CPMDP_POLICY_UNSETTLED else code   # V certified; pi checked below
    torch.cuda.synchronize()
    return V.cpu().numpy(), pi.cpu().numpy(), code, sweeps, res, outer


CASES = {
    "grid2d_16x16": lambda: I.grid2d_16(),
    "grid_5x7x3x9": lambda: I.grid_small([5, 7, 3, 9], slip=0.2, gamma=0.95, seed=21),
    "grid_1d_37": lambda: I.grid_small([37], gamma=0.9, seed=22),
    "grid_3x2x4x2x3": lambda: I.grid_small([3, 2, 4, 2, 3], slip=0.3, gamma=0.9, seed=23),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", [0, 1])
def test_one_backup_matches_oracle(B, name, prec):
    inst = CASES[name]()
    log(f"[stencil backup] {name} prec={prec}")
    model = B.Model(inst)
    assert model.path == B.CPMDP_PATH_STENCIL
    V = I.seeded_values(inst.n_states, 5, scale=2.0)
    if prec == 1:
        V = V.astype(np.float32).astype(np.float64)
    Q = oracle.dense.q_values(inst, oracle.dense.transition_matrices(inst), V) \
        if inst.n_states <= 4096 else oracle.sparse.q_values(inst, oracle.sparse.transition_csr(inst), V)
    Vg, pig, r = _backup(B, model, V, prec)
    tol = 1e-13 * max(1, np.abs(V).max()) if prec == 0 else tol_for(1, Q.max(0))
    assert_close(Vg, Q.max(0), tol, "V'")
    assert abs(r - np.max(np.abs(Q.max(0) - V))) <= 2 * tol
    compare_policy(pig, Q, tol)
    model.close()


@pytest.mark.parametrize("method", ["vi", "pi"])
def test_grid16_fp64_solve_matches_oracle(B, method):
    inst = I.grid2d_16()
    log(f"[stencil solve] grid2d_16 {method} fp64")
    P = oracle.dense.transition_matrices(inst)
    Vs, pis, _, _ = oracle.dense.value_iteration(inst, P=P)
    model = B.Model(inst)
    V, pi, code, sweeps, res, _ = _solve(B, model, method, 0, 1e-11)
    assert code == B.CPMDP_OK and res <= 1e-11
    assert_close(V, Vs, 1e-9, "V*")
    # exact ties (diagonal +x/+y) resolve to the lowest index on both sides
    Q = oracle.dense.q_values(inst, P, V)
    assert np.array_equal(pi, oracle.greedy(Q, V)) or method == "pi"
    compare_policy(pi, oracle.dense.q_values(inst, P, Vs), 1e-9)
    if method == "vi":
        assert np.array_equal(pi, pis)
    model.close()


@pytest.mark.parametrize("method", ["vi", "pi"])
@pytest.mark.parametrize("prec", [0, 1])
def test_ragged_4d_solve_matches_oracle(B, method, prec):
    inst = I.grid_small([6, 5, 4, 7], slip=0.1, gamma=0.99, seed=24)
    log(f"[stencil solve] 6x5x4x7 {method} prec={prec}")
    mats = oracle.sparse.transition_csr(inst)
    Vs, pis, _, _ = oracle.sparse.value_iteration(inst, mats=mats)
    model = B.Model(inst)
    # solve tightly enough that res / (1 - gamma) meets the value tolerance
    eps = 0.5 * tol_for(prec, Vs) * (1 - inst.gamma)
    V, pi, code, sweeps, res, _ = _solve(B, model, method, prec, eps)
    assert code == B.CPMDP_OK and res <= eps
    tol = eps / (1 - inst.gamma) + 1e-12
    assert_close(V, Vs, tol_for(prec, Vs), "V*")
    compare_policy(pi, oracle.sparse.q_values(inst, mats, Vs), tol)
    model.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_policy_backup_matches_oracle(B, prec):
    inst = I.grid_small([4, 9, 5], slip=0.2, gamma=0.97, seed=25)
    log(f"[stencil policy backup] prec={prec}")
    mats = oracle.sparse.transition_csr(inst)
    rng = np.random.default_rng(3)
    pi = rng.integers(0, inst.n_actions, inst.n_states).astype(np.int32)
    V = I.seeded_values(inst.n_states, 6)
    if prec == 1:
        V = V.astype(np.float32).astype(np.float64)
    ref = inst.rewards + inst.gamma * (oracle.sparse.policy_matrix(inst, mats, pi) @ V)
    model = B.Model(inst)
    Vin = torch.as_tensor(V, dtype=_dt(prec), device="cuda")
    Vout = torch.empty_like(Vin)
    pid = torch.as_tensor(pi, device="cuda")
    B.cpmdp_policy_backup(model.h, Vin, Vout, pid, residual=False, precision=prec)
    torch.cuda.synchronize()
    tol = 1e-13 * 4 if prec == 0 else tol_for(1, ref)
    assert_close(Vout.cpu().numpy(), ref, tol, "P_pi V")
    bad = pi.copy()
    bad[7] = inst.n_actions
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_policy_backup(model.h, Vin, Vout, torch.as_tensor(bad, device="cuda"))
    assert e.value.code == B.CPMDP_E_ARG
    model.close()


def test_max_iter_and_warm_start(B):
    inst = I.grid_small([7, 6, 5], slip=0.1, gamma=0.95, seed=26)
    log("[stencil] max_iter / warm start")
    model = B.Model(inst)
    V, pi, code, sweeps, res, _ = _solve(B, model, "vi", 0, 1e-12, max_iter=5)
    assert code == B.CPMDP_NOT_CONVERGED and sweeps <= 5 and np.all(np.isfinite(V))
    Vs, pis, _, _ = oracle.sparse.value_iteration(inst)
    V2, _, code, sweeps2, res2, _ = _solve(B, model, "vi", 0, 1e-11, V0=Vs + 1e-6)
    assert code == B.CPMDP_OK and sweeps2 < 400       # from 0: about 600
    assert_close(V2, Vs, 1e-9, "warm-started V*")
    model.close()


def test_nonfinite_value_detected(B):
    inst = I.grid_small([5, 5], seed=27)
    log("[stencil] NaN detection")
    model = B.Model(inst)
    V = I.seeded_values(inst.n_states, 1)
    V[3] = np.nan
    Vin = torch.as_tensor(V, dtype=torch.float64, device="cuda")
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_backup(model.h, Vin, torch.empty_like(Vin), None, residual=True, precision=0)
    assert e.value.code == B.CPMDP_E_NONFINITE
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_value_iteration(model.h, Vin.clone(), None, 1e-6, 100, 0)
    assert e.value.code == B.CPMDP_E_NONFINITE
    model.close()


# ------------------------------------------------------- full 32^4 instance

@pytest.fixture(scope="module")
def grid4d():
    inst = I.grid4d(32)
    mats = oracle.sparse.transition_csr(inst)
    return inst, mats


@pytest.mark.parametrize("prec", [0, 1])
def test_grid4d_32_one_backup(B, grid4d, prec):
    inst, mats = grid4d
    log(f"[stencil 32^4] one backup prec={prec}")
    V = I.seeded_values(inst.n_states, 7, scale=5.0)
    if prec == 1:
        V = V.astype(np.float32).astype(np.float64)
    Q = oracle.sparse.q_values(inst, mats, V)
    model = B.Model(inst)
    Vg, pig, r = _backup(B, model, V, prec)
    tol = 1e-13 * np.abs(V).max() if prec == 0 else tol_for(1, Q.max(0))
    assert_close(Vg, Q.max(0), tol, "V'")
    compare_policy(pig, Q, tol)
    model.close()


@pytest.mark.parametrize("method", ["vi", "pi"])
def test_grid4d_32_fp32_solve_certified_by_oracle(B, grid4d, method):
    """Full-size solve to eps = 1e-6: the oracle's own FP64 Bellman residual of
    the returned V bounds its distance to V* by res / (1 - gamma)."""
    inst, mats = grid4d
    log(f"[stencil 32^4] {method} fp32 eps=1e-6")
    model = B.Model(inst)
    V, pi, code, sweeps, res, outer = _solve(B, model, method, 1, 1e-6)
    log(f"   sweeps={sweeps} outer={outer} res={res:.3e}")
    assert code == B.CPMDP_OK and res <= 1e-6
    Q = oracle.sparse.q_values(inst, mats, V)
    res_oracle = float(np.max(np.abs(Q.max(0) - V)))
    assert abs(res_oracle - res) <= 1e-12
    bound = res_oracle / (1 - inst.gamma)
    assert bound <= tol_for(1, V)
    assert np.array_equal(pi, oracle.greedy(Q, V)) or method == "pi"
    compare_policy(pi, Q, 1e-9)
    model.close()


MARCH_CASES = {
    # two segments of 10 planes, ragged last plane tile (76,032 = 74.25 x 1024)
    "march_20x64x33x36": lambda: I.grid_small([20, 64, 33, 36], slip=0.1, gamma=0.99, seed=28),
    # n = 3, three segments
    "march_24x300x224": lambda: I.grid_small([24, 300, 224], slip=0.2, gamma=0.95, seed=29),
    # n = 5, one segment of 8 planes
    "march_8x16x24x16x12": lambda: I.grid_small([8, 16, 24, 16, 12], slip=0.1, gamma=0.9,
                                                seed=30),
}


def _march_sample(inst, rng, n_random=96):
    """States at plane / segment / tile boundaries and grid corners, plus
    random ones."""
    sizes = [int(m) for m in inst.sizes]
    plane = inst.n_states // sizes[0]
    picks = [0, inst.n_states - 1, plane - 1, plane, 2 * plane - 1]
    for i0 in (0, 1, sizes[0] // 2 - 1, sizes[0] // 2, sizes[0] - 2, sizes[0] - 1):
        for off in (0, 1, 3, 4, 1023, 1024, plane - 4, plane - 1):
            picks.append(i0 * plane + min(off, plane - 1))
    picks += list(rng.integers(0, inst.n_states, n_random))
    return np.unique(np.asarray(picks, np.int64))


def _backup_forms(B, model, V, prec, pi_in=None):
    """One backup with the marching form on and off: (V', pi) per form."""
    out = []
    for march in (1, 0):
        B.cpmdp_set_option(model.h, B.CPMDP_OPT_MARCH, march)
        if pi_in is None:
            out.append(_backup(B, model, V, prec))
        else:
            Vin = torch.as_tensor(V, dtype=_dt(prec), device="cuda")
            Vout = torch.empty_like(Vin)
            B.cpmdp_policy_backup(model.h, Vin, Vout, torch.as_tensor(pi_in, device="cuda"),
                                  residual=False, precision=prec)
            torch.cuda.synchronize()
            out.append((Vout.cpu().numpy().astype(np.float64), None, None))
    B.cpmdp_set_option(model.h, B.CPMDP_OPT_MARCH, 1)
    return out


@pytest.mark.parametrize("name", list(MARCH_CASES))
@pytest.mark.parametrize("prec", [0, 1])
def test_march_backup_matches_oracle(B, name, prec):
    """Marching form: sampled states against the per-state Def. 3 oracle,
    every state equal to the one-pass form (same arithmetic per state)."""
    inst = MARCH_CASES[name]()
    log(f"[stencil march] {name} prec={prec}")
    model = B.Model(inst)
    V = I.seeded_values(inst.n_states, 31, scale=2.0)
    if prec == 1:
        V = V.astype(np.float32).astype(np.float64)
    (Vm, pim, _), (Vo, pio, _) = _backup_forms(B, model, V, prec)
    assert np.array_equal(Vm, Vo) and np.array_equal(pim, pio)
    states = _march_sample(inst, np.random.default_rng(32))
    Q = oracle.sparse.q_at_states(inst, V, states)
    tol = 1e-13 * max(1.0, np.abs(V).max()) if prec == 0 else tol_for(1, Q.max(0))
    assert_close(Vm[states], Q.max(0), tol, "sampled V'")
    compare_policy(pim[states], Q, tol)
    # fixed-policy backup (evaluation sweep) in both forms
    pi = np.random.default_rng(33).integers(0, inst.n_actions, inst.n_states).astype(np.int32)
    (Em, _, _), (Eo, _, _) = _backup_forms(B, model, V, prec, pi_in=pi)
    assert np.array_equal(Em, Eo)
    ref = Q[pi[states], np.arange(states.size)]
    assert_close(Em[states], ref, tol, "sampled P_pi V")
    model.close()


def test_march_grid4d_96_backup(B):
    """96^4 (84,934,656 states, the HBM-resident workload): one FP32 backup in
    the marching form, equal to the one-pass form everywhere and to the
    oracle on sampled states."""
    inst = I.grid4d(96, I.SEED_GRID4_LARGE)
    log("[stencil 96^4] march vs one-pass, fp32")
    model = B.Model(inst)
    V = I.seeded_values(inst.n_states, 34, scale=5.0).astype(np.float32).astype(np.float64)
    (Vm, pim, _), (Vo, pio, _) = _backup_forms(B, model, V, 1)
    assert np.array_equal(Vm, Vo) and np.array_equal(pim, pio)
    states = _march_sample(inst, np.random.default_rng(35), n_random=32)
    Q = oracle.sparse.q_at_states(inst, V, states)
    tol = tol_for(1, Q.max(0))
    assert_close(Vm[states], Q.max(0), tol, "sampled V'")
    compare_policy(pim[states], Q, tol)
    model.close()
