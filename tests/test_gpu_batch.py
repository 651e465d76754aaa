"""GPU parity of the batched solver: every instance of a batch against the
FP64 oracle and against its own single-instance solve, through the C ABI."""
import os
import tempfile

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


def _small_batch(count=14, seed=7):
    """Instances of the batch generator at small sizes: n in {1..4}, odd and
    even side lengths (both thread layouts), several terminals."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(1, 5))
        sizes = [int(rng.integers(3, 13 if n > 2 else 40)) for _ in range(n)]
        out.append(I.grid_small(sizes, slip=float(rng.uniform(0.05, 0.3)),
                                gamma=float(rng.uniform(0.9, 0.99)), seed=100 + i))
    return out


def _solve_batch(B, insts, prec, eps, tune=False, max_iter=200000, V0=None, method=0,
                 sched=None):
    bm = B.BatchModel(insts)
    if tune:
        B.cpmdp_batch_autotune(bm.b, True, None)
    if sched is not None:
        B.cpmdp_batch_set_schedule(bm.b, *sched)
    Vs = [torch.zeros(x.n_states, dtype=torch.float64, device="cuda") if V0 is None else
          torch.as_tensor(V0[i], dtype=torch.float64, device="cuda").clone()
          for i, x in enumerate(insts)]
    pis = [torch.zeros(x.n_states, dtype=torch.int32, device="cuda") for x in insts]
    code, sweeps, res = B.cpmdp_batch_solve(bm.b, Vs, pis, eps, max_iter, prec, method)
    torch.cuda.synchronize()
    if method == 1 and code == B.CPMDP_POLICY_UNSETTLED:
        log("   policy iteration: some policies unsettled at near-ties (V certified)")
        code = B.CPMDP_OK          # the policies are checked state by state by the callers
    out = [(V.cpu().numpy(), p.cpu().numpy()) for V, p in zip(Vs, pis)]
    bm.close()
    return code, out, sweeps, res


@pytest.mark.parametrize("prec", [0, 1])
def test_small_batch_matches_oracle(B, prec):
    insts = _small_batch()
    log(f"[batch] small batch prec={prec}")
    refs = []
    for x in insts:
        mats = oracle.sparse.transition_csr(x)
        Vs, _, _, _ = oracle.sparse.value_iteration(x, mats=mats)
        refs.append((mats, Vs))
    eps = min(0.5 * tol_for(prec, Vs) * (1 - x.gamma) for x, (_, Vs) in zip(insts, refs))
    code, out, sweeps, res = _solve_batch(B, insts, prec, eps)
    assert code == B.CPMDP_OK
    assert np.all(res <= eps)
    for x, (mats, Vs), (V, pi) in zip(insts, refs, out):
        assert_close(V, Vs, tol_for(prec, Vs), x.name)
        compare_policy(pi, oracle.sparse.q_values(x, mats, Vs), eps / (1 - x.gamma) + 1e-12)


def test_small_batch_policy_iteration_matches_oracle(B):
    """Batched policy iteration (FP32 correction sweeps, FP64 residual and
    improvement) from pi = 0: every instance against the oracle's V* and
    policy, and certified like value iteration."""
    insts = _small_batch(count=12, seed=9)
    log("[batch] policy iteration, small batch")
    refs = []
    for x in insts:
        mats = oracle.sparse.transition_csr(x)
        Vs, _, _, _ = oracle.sparse.value_iteration(x, mats=mats)
        refs.append((mats, Vs))
    eps = min(0.5 * tol_for(1, Vs) * (1 - x.gamma) for x, (_, Vs) in zip(insts, refs))
    code, out, sweeps, res = _solve_batch(B, insts, 1, eps, tune=True, method=1)
    log(f"   sweeps {list(sweeps)}")
    assert code == B.CPMDP_OK and np.all(res <= eps)
    for x, (mats, Vs), (V, pi) in zip(insts, refs, out):
        assert_close(V, Vs, tol_for(1, Vs), x.name)
        compare_policy(pi, oracle.sparse.q_values(x, mats, Vs), eps / (1 - x.gamma) + 1e-12)


def test_batch_time_sweeps_then_solve(B):
    """The timing helper runs whole-batch sweeps on internal buffers; a solve
    afterwards still starts from the caller's V and matches the oracle."""
    insts = _small_batch(count=4, seed=21)
    bm = B.BatchModel(insts)
    ms = B.cpmdp_batch_time_sweeps(bm.b, 5)
    assert ms > 0
    Vs = [torch.zeros(x.n_states, dtype=torch.float64, device="cuda") for x in insts]
    pis = [torch.zeros(x.n_states, dtype=torch.int32, device="cuda") for x in insts]
    code, sweeps, res = B.cpmdp_batch_solve(bm.b, Vs, pis, 1e-9, 200000, 1, 0)
    assert code == B.CPMDP_OK
    for x, V in zip(insts, Vs):
        Vo, _, _, _ = oracle.sparse.value_iteration(x)
        assert_close(V.cpu().numpy(), Vo, 1e-9 / (1 - x.gamma) + tol_for(0, Vo), x.name)
    bm.close()


def test_batch_policy_iteration_rejects_bad_policy(B):
    insts = _small_batch(count=2, seed=19)
    bm = B.BatchModel(insts)
    Vs = [torch.zeros(x.n_states, dtype=torch.float64, device="cuda") for x in insts]
    pis = [torch.zeros(x.n_states, dtype=torch.int32, device="cuda") for x in insts]
    pis[1][3] = insts[1].n_actions
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_batch_solve(bm.b, Vs, pis, 1e-6, 1000, 1, 1)
    assert e.value.code == B.CPMDP_E_ARG
    bm.close()


@pytest.fixture(scope="module")
def march_batch():
    insts = [I.grid_small([8, 20, 24, 36], slip=0.15, gamma=0.9, seed=41),
             I.grid_small([10, 16, 32, 32], slip=0.1, gamma=0.92, seed=42),
             I.grid_small([9, 40, 44], slip=0.2, gamma=0.9, seed=43),
             I.grid_small([6, 7, 5], slip=0.1, gamma=0.95, seed=44),
             # last side not a multiple of 4: one state per lane, one-pass tiles
             I.grid_small([8, 21, 25, 35], slip=0.1, gamma=0.9, seed=45),
             I.grid_small([9, 130, 131], slip=0.2, gamma=0.9, seed=46),
             # 16 planes of 17,280 states: with few tiles in the batch, four
             # marching segments of 4 planes
             I.grid_small([16, 18, 30, 32], slip=0.12, gamma=0.9, seed=47)]
    log("[batch] oracle for the marching batch")
    refs = []
    for x in insts:
        mats = oracle.sparse.transition_csr(x)
        Vs, _, _, _ = oracle.sparse.value_iteration(x, mats=mats, eps=1e-12)
        refs.append((mats, Vs))
    return insts, refs


# (tile states, grid, march, sched): marching tiles with either schedule,
# one-pass tiles only with the interleaved schedule, and small tiles and grid
@pytest.mark.parametrize("sched", [(4096, 2048, 1, 0), (4096, 2048, 1, 1), (8192, 1024, 0, 1),
                                   (1024, 64, 1, 1)])
@pytest.mark.parametrize("method", [0, 1])
def test_batch_marching_tiles_match_oracle(B, march_batch, method, sched):
    """Instances whose planes of fixed i_0 hold >= 16384 states get marching
    tiles (1024 plane offsets per tile; a batch this small cuts each dim-0
    column into segments of at least 4 planes) next to one-pass tiles of
    small instances; rows whose last side is not a multiple of 4 are padded
    in the batch's layout.  Every tile schedule: VI and PI against the
    oracle."""
    insts, refs = march_batch
    log(f"[batch] marching tiles, method {method}, schedule {sched}")
    eps = 1e-7
    code, out, sweeps, res = _solve_batch(B, insts, 1, eps, method=method, sched=sched)
    assert code == B.CPMDP_OK and np.all(res <= eps)
    for x, (mats, Vs), (V, pi) in zip(insts, refs, out):
        assert_close(V, Vs, eps / (1 - x.gamma) + 1e-10, x.name)
        compare_policy(pi, oracle.sparse.q_values(x, mats, Vs), eps / (1 - x.gamma) + 1e-10)


def test_repeated_solves_on_one_batch(B, march_batch):
    """One bound batch solved again and again with other methods and
    precisions, a timing run in between: the tile tables and descriptors the
    batch keeps on the device between calls (and re-copies only when they
    change) must follow each call's own stages and tile sets."""
    insts, refs = march_batch
    log("[batch] repeated solves on one bound batch")
    eps = 1e-7
    bm = B.BatchModel(insts)
    Vs = [torch.zeros(x.n_states, dtype=torch.float64, device="cuda") for x in insts]
    pis = [torch.zeros(x.n_states, dtype=torch.int32, device="cuda") for x in insts]

    def check(tag, prec, method, reset=True):
        if reset:
            for V, p in zip(Vs, pis):
                V.zero_()
                p.zero_()
        code, sweeps, res = B.cpmdp_batch_solve(bm.b, Vs, pis, eps, 200000, prec, method)
        torch.cuda.synchronize()
        assert code in (B.CPMDP_OK, B.CPMDP_POLICY_UNSETTLED), (tag, code)
        assert np.all(res <= eps), (tag, res)
        for x, (mats, Vr), V, p in zip(insts, refs, Vs, pis):
            assert_close(V.cpu().numpy(), Vr, eps / (1 - x.gamma) + 1e-10, f"{tag} {x.name}")
            compare_policy(p.cpu().numpy(), oracle.sparse.q_values(x, mats, Vr),
                           eps / (1 - x.gamma) + 1e-10)
        return sweeps

    first = check("vi fp32", 1, 0)
    B.cpmdp_batch_time_sweeps(bm.b, 3)          # stages and tables of a timing run
    assert np.array_equal(check("vi fp32 again", 1, 0), first)
    check("pi", 1, 1)
    check("vi fp64", 0, 0)
    # from the converged values: far fewer sweeps than from V0 = 0 (the FP32
    # stage rounds V, which a few FP64 sweeps take back below eps)
    warm = check("vi fp32 warm", 1, 0, reset=False)
    assert np.all(warm < 0.5 * first), (warm, first)
    bm.close()


@pytest.mark.parametrize("sizes", [[3], [5], [17]])
def test_batch_of_one_tiny_instance(B, sizes):
    """The degenerate batch: a single 1-D instance of a few states (one tile,
    one row, padded to a multiple of 4 in the batch's layout), value and
    policy iteration against the oracle."""
    inst = I.grid_small(sizes, slip=0.1, gamma=0.95, seed=3)
    mats = oracle.sparse.transition_csr(inst)
    Vs, _, _, _ = oracle.sparse.value_iteration(inst, mats=mats, eps=1e-12)
    eps = 1e-9
    for method in (0, 1):
        log(f"[batch] one instance of sizes {sizes}, method {method}")
        code, out, sweeps, res = _solve_batch(B, [inst], 1, eps, method=method)
        assert code == B.CPMDP_OK and np.all(res <= eps), (code, res)
        V, pi = out[0]
        assert_close(V, Vs, eps / (1 - inst.gamma) + 1e-10, f"{sizes} method {method}")
        compare_policy(pi, oracle.sparse.q_values(inst, mats, Vs), eps / (1 - inst.gamma) + 1e-10)


def test_batch_equals_single_solves_and_autotune(B):
    insts = _small_batch(count=9, seed=11)
    log("[batch] vs single-instance solves, autotuned")
    eps = 1e-9
    code, out, sweeps, res = _solve_batch(B, insts, 1, eps, tune=True)
    assert code == B.CPMDP_OK
    for x, (V, pi) in zip(insts, out):
        m = B.Model(x)
        Vs = torch.zeros(x.n_states, dtype=torch.float64, device="cuda")
        ps = torch.zeros(x.n_states, dtype=torch.int32, device="cuda")
        c, sw, r = B.cpmdp_value_iteration(m.h, Vs, ps, eps, 200000, 1)
        assert c == B.CPMDP_OK
        assert_close(V, Vs.cpu().numpy(), 2 * eps / (1 - x.gamma), x.name)
        m.close()


def test_autotune_cache_roundtrip(B):
    insts = _small_batch(count=5, seed=13)
    log("[batch] autotune cache")
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.txt")
        bm = B.BatchModel(insts)
        B.cpmdp_batch_autotune(bm.b, True, path)
        cfg = B.cpmdp_batch_config(bm.b)
        sched = B.cpmdp_batch_schedule(bm.b)
        bm.close()
        assert os.path.exists(path)
        bm2 = B.BatchModel(insts)
        B.cpmdp_batch_autotune(bm2.b, False, path)
        assert B.cpmdp_batch_config(bm2.b) == cfg
        assert B.cpmdp_batch_schedule(bm2.b) == sched
        bm2.close()


def test_batch_max_iter_and_rejects_dense(B):
    insts = _small_batch(count=3, seed=17)
    code, out, sweeps, res = _solve_batch(B, insts, 1, 1e-12, max_iter=10)
    assert code == B.CPMDP_NOT_CONVERGED and np.all(sweeps <= 12)
    d = I.random_dense([3, 4], 2, 2, seed=1)
    h = B.cpmdp_create(d.sizes, d.ranks, d.factors, d.lambdas, d.rewards, d.gamma)
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_batch_create([h])
    assert e.value.code == B.CPMDP_E_UNSUPPORTED
    B.cpmdp_destroy(h)


@pytest.fixture(scope="module")
def batch512():
    return [I.batch_instance(i) for i in range(512)]


@pytest.mark.parametrize("method", [0, 1])
def test_batch512_full_certified(B, batch512, method):
    """The 512-instance mixed batch (sum of states ~2.2e8), value iteration
    and policy iteration (FP32 correction sweeps, FP64 residual and
    improvement): every instance certified to eps = 1e-6 in FP64; on a
    sample the oracle recomputes the residual of the returned V and checks
    the policy (equal to the oracle's greedy action wherever the best action
    wins by more than the tolerance, within it elsewhere)."""
    insts = batch512
    log(f"[batch512] method {method}, total states {sum(x.n_states for x in insts)}")
    code, out, sweeps, res = _solve_batch(B, insts, 1, 1e-6, tune=True, method=method)
    assert code == B.CPMDP_OK and np.all(res <= 1e-6)
    log(f"   sweeps: total {int(np.sum(sweeps))}, max {int(np.max(sweeps))}")
    order = np.argsort([x.n_states for x in insts])
    big = [int(i) for i in order if insts[i].n_states <= 1_500_000][-1]
    for i in list(order[:4]) + [int(order[len(order) // 2]), big]:
        x = insts[i]
        V, pi = out[i]
        mats = oracle.sparse.transition_csr(x)
        Q = oracle.sparse.q_values(x, mats, V)
        r_or = float(np.max(np.abs(Q.max(0) - V)))
        assert abs(r_or - res[i]) <= 1e-12
        assert r_or / (1 - x.gamma) <= tol_for(1, V)
        compare_policy(pi, Q, 1e-9)


def test_batch_orders_after_callers_stream(B):
    """V0 written on the caller's (default) stream right before the call must
    be what the batch starts from: repeated solves from a fresh V0 = 0 run
    the same number of sweeps for every instance."""
    insts = _small_batch(count=6, seed=19)
    bm = B.BatchModel(insts)
    Vs = [torch.zeros(x.n_states, dtype=torch.float64, device="cuda") for x in insts]
    runs = []
    for _ in range(3):
        for V in Vs:
            V.zero_()
        code, sweeps, res = B.cpmdp_batch_solve(bm.b, Vs, None, 1e-9, 200000, 1, 0)
        assert code == B.CPMDP_OK
        runs.append(list(sweeps))
    bm.close()
    assert runs[0] == runs[1] == runs[2], runs
