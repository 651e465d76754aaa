"""GPU parity of the Tensor-Train / Tucker path (cpmdp_create_tt,
cpmdp_create_tucker) against the FP64 oracle O4 (operators expanded from
their definitions, then Eq. 1 by O1), through the C ABI.  The cases cover
both step kernels (matrix cores for m_k = 16, in the row, wide and
last-dimension layouts, and the fused launch of the last two dimensions in
FP32; vector ALUs otherwise), bonds 1..8, ragged mode sizes, one dimension,
terminals, and the 16^6 workload at sampled states."""
import numpy as np
import pytest

import oracle
from oracle import tt as O4
from paper_2103_00331_amd import instances as I
from tests.parity import assert_close, compare_policy, log, tol_for
from tests.tt_helpers import cp_as_tt

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
    # m = 16 everywhere: dims 0 and 1 on the matrix cores (bond 3 pads to 4)
    "tt_16x16x16_b3": lambda: I.random_tt([16, 16, 16], 2, 3, seed=91, n_terminal=5),
    # two dims of 16: in FP32 both products run in the fused launch, which
    # writes P_a V itself
    "tt_16x16_b3": lambda: I.random_tt([16, 16], 3, 3, seed=89, n_terminal=4),
    # bond 4: the first dimension (4 -> 1) through the LDS-shared tile kernel
    "tt_16x16x16_b4": lambda: I.random_tt([16, 16, 16], 2, 4, seed=88, n_terminal=2),
    # bond 8: the wide layout with 8 input channels (fewer outputs per block)
    "tt_16x16x16_b8": lambda: I.random_tt([16, 16, 16], 2, 8, seed=90),
    # bond 5 (matrix-core kernel with 8 input channels, FP64 in pairs of outputs)
    "tt_16x16_b5": lambda: I.random_tt([16, 16], 3, 5, seed=92, gamma=0.95),
    # bond 8, mixed sizes: m = 8 and ragged 5, 3, 7 on the vector kernel
    "tt_8x5x3x7_b8": lambda: I.random_tt([8, 5, 3, 7], 2, 8, seed=93, n_terminal=2),
    # bonds of 1 (Kronecker products) and of 2; one dimension
    "tt_6x9_b1": lambda: I.random_tt([6, 9], 4, 1, seed=94),
    "tt_4x16x16_b2": lambda: I.random_tt([4, 16, 16], 3, 2, seed=95, alpha=0.3),
    "tt_13_b1": lambda: I.random_tt([13], 3, 1, seed=96, gamma=0.8),
    # Tucker cores, rewritten as Tensor-Trains by the library
    "tucker_3x4x2": lambda: I.random_tucker([3, 4, 2], 3, [2, 3, 2], seed=97, n_terminal=2),
    "tucker_16x16x4": lambda: I.random_tucker([16, 16, 4], 2, [2, 2, 2], seed=98),
}


def _P(inst):
    if hasattr(inst, "bonds"):
        return O4.tt_transition_matrices(inst)
    return O4.tucker_transition_matrices(inst)


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
def test_tt_backup_matches_oracle(B, name, prec):
    inst = CASES[name]()
    log(f"[tt backup] {name} prec={prec}")
    model = B.Model(inst)
    assert model.path == B.CPMDP_PATH_TT
    V = I.seeded_values(inst.n_states, 9, scale=2.0)
    if prec == 1:
        V = V.astype(np.float32).astype(np.float64)
    P = _P(inst)
    Q = oracle.dense.q_values(inst, P, V)
    Vg, pig, r = _backup(B, model, V, prec)
    tol = 1e-13 * max(1, np.abs(V).max()) * 4 if prec == 0 else tol_for(1, Q.max(0))
    assert_close(Vg, Q.max(0), tol, "V'")
    assert abs(r - np.max(np.abs(Q.max(0) - V))) <= 2 * tol
    compare_policy(pig, Q, tol)
    pi = np.random.default_rng(8).integers(0, inst.n_actions, inst.n_states).astype(np.int32)
    Eg, _, _ = _backup(B, model, V, prec, pi_in=pi)
    assert_close(Eg, Q[pi, np.arange(inst.n_states)], tol, "P_pi V")
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


@pytest.mark.parametrize("name", ["tt_16x16x16_b3", "tt_8x5x3x7_b8", "tucker_3x4x2"])
@pytest.mark.parametrize("method", ["vi", "pi"])
@pytest.mark.parametrize("prec", [0, 1])
def test_tt_solve_matches_oracle(B, name, method, prec):
    inst = CASES[name]()
    log(f"[tt solve] {name} {method} prec={prec}")
    P = _P(inst)
    Vs, _, _, _ = oracle.dense.value_iteration(inst, P=P)
    model = B.Model(inst)
    eps = 0.5 * tol_for(prec, Vs) * (1 - inst.gamma)
    V, pi, code, sweeps, res = _solve(B, model, method, prec, eps)
    assert code == B.CPMDP_OK and res <= eps
    assert_close(V, Vs, tol_for(prec, Vs), "V*")
    compare_policy(pi, oracle.dense.q_values(inst, P, Vs), eps / (1 - inst.gamma) + 1e-12)
    model.close()


def test_cp_written_as_tt_matches_cp_path(B):
    """One CP instance solved on the dense-chain path and, rewritten with
    diagonal bonds, on the Tensor-Train path: both certified against O1."""
    cp = I.random_dense([16, 8, 16], 3, 3, seed=99, gamma=0.9, n_terminal=4)
    tt = cp_as_tt(cp)
    log("[tt] CP instance on both paths")
    P = oracle.dense.transition_matrices(cp)
    Vs, _, _, _ = oracle.dense.value_iteration(cp, P=P)
    eps = 1e-10
    out = []
    for inst in (cp, tt):
        model = B.Model(inst)
        V, pi, code, _, res = _solve(B, model, "vi", 0, eps)
        assert code == B.CPMDP_OK and res <= eps
        assert_close(V, Vs, 1e-9, "V*")
        out.append(pi)
        model.close()
    compare_policy(out[1], oracle.dense.q_values(cp, P, Vs), 1e-9)


def test_tt_rejects_bf16(B):
    model = B.Model(CASES["tt_6x9_b1"]())
    V = torch.zeros(model.S, dtype=torch.float64, device="cuda")
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_value_iteration(model.h, V, None, 1e-6, 100, B.CPMDP_BF16)
    assert e.value.code == B.CPMDP_E_UNSUPPORTED
    model.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_tt_full_size_sampled(B, prec):
    """The 16^6 workload (12 actions, bond 4), in the launch configuration
    the benchmark times: one backup from a seeded V, checked at sampled
    states (corners, interior, the last state) against O4 row by row."""
    inst = I.tt_grid()
    log(f"[tt] 16^6 bond 4 sampled, prec={prec}")
    model = B.Model(inst)
    V = I.seeded_values(inst.n_states, 10, scale=1.0)
    if prec == 1:
        V = V.astype(np.float32).astype(np.float64)
    Vg, pig, _ = _backup(B, model, V, prec)
    model.close()
    rng = np.random.default_rng(11)
    states = [0, inst.n_states - 1, 15, 16 ** 5 * 7 + 3] + list(rng.integers(0, inst.n_states, 2))
    Q = O4.tt_q_at_states(inst, V, states)
    tol = 1e-12 if prec == 0 else tol_for(1, Q.max(0))
    assert_close(Vg[states], Q.max(0), tol, "V' at samples")
    compare_policy(pig[states], Q, tol)
