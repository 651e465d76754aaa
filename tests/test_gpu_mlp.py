"""GPU parity of the warm-start MLP kernels against the FP64 oracle, and the
warm-start A/B test: value iteration from the trained network's V0 needs
fewer sweeps than from V0 = 0 and reaches the same certified solution."""
import numpy as np
import pytest

from oracle import mlp as OM
from paper_2103_00331_amd import instances as I
from tests.parity import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    from paper_2103_00331_amd import binding
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return binding


def _params(B, seed=3):
    p = torch.empty(B.cpmdp_mlp_param_count(), dtype=torch.float32, device="cuda")
    B.cpmdp_mlp_init(p, seed)
    torch.cuda.synchronize()
    return p


def _ws(B, n):
    return torch.empty(B.cpmdp_mlp_workspace_bytes(n), dtype=torch.uint8, device="cuda")


def test_init_statistics(B):
    p = _params(B).cpu().numpy().astype(np.float64)
    q = OM.unpack(p)
    assert np.all(q["b1"] == 0) and np.all(q["b2"] == 0) and q["b3"][0] == 0
    assert np.all(q["w3"] == 0)
    assert abs(q["W1"].std() - np.sqrt(2 / 130)) < 0.01 * np.sqrt(2 / 130) * 10
    assert abs(q["W2"].std() - np.sqrt(2 / 256)) < 0.05 * np.sqrt(2 / 256)
    assert abs(q["W2"].mean()) < 1e-3


@pytest.mark.parametrize("m", [1, 4, 9])
def test_features_match_oracle(B, m):
    inst = I.warm_instance(1, 0, m=m)
    log(f"[mlp] features m={m}")
    R = torch.as_tensor(inst.rewards, dtype=torch.float32, device="cuda")
    S = inst.n_states
    X = torch.empty(S, 130, dtype=torch.float32, device="cuda")
    B.cpmdp_mlp_features(R, m, inst.gamma, inst.meta["slip"], 0, S, X)
    torch.cuda.synchronize()
    Rf = inst.rewards.astype(np.float32).astype(np.float64)
    ref = OM.features(Rf, m, np.float32(inst.gamma), np.float32(inst.meta["slip"]), np.arange(S))
    np.testing.assert_allclose(X.cpu().numpy(), ref, rtol=2e-6, atol=2e-6)


# 1 row: every product on the vector tile kernel (fewer than 64 rows);
# 64 rows: one whole 64 x 64 matrix-core tile; 700 rows: 64 x 64 tiles with
# a ragged tail; 4,099 rows: weight gradients split over K with a ragged
# last slice; 32,845 rows: the 128 x 128 tiles (from 32,768 rows) with a
# ragged tail
@pytest.mark.parametrize("n", [1, 64, 700, 4099, 32845])
def test_forward_and_gradient_match_oracle(B, n):
    log(f"[mlp] forward + gradient rows={n}")
    rng = np.random.default_rng(4)
    X = rng.normal(0, 1, (n, 130)).astype(np.float32)
    t = rng.normal(0, 1, n).astype(np.float32)
    p = _params(B, 5)
    p += 0.05 * torch.randn(p.numel(), device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    pd = p.cpu().numpy().astype(np.float64)
    Xd, td = torch.as_tensor(X, device="cuda"), torch.as_tensor(t, device="cuda")
    ws = _ws(B, n)
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    B.cpmdp_mlp_forward(p, Xd, n, y, ws)
    g = torch.empty_like(p)
    loss = B.cpmdp_mlp_loss_grad(p, Xd, td, n, g, ws)
    torch.cuda.synchronize()
    y_ref, _ = OM.forward(pd, X.astype(np.float64))
    np.testing.assert_allclose(y.cpu().numpy(), y_ref, rtol=1e-4, atol=1e-4 * np.abs(y_ref).max())
    L_ref, g_ref = OM.loss_grad(pd, X.astype(np.float64), t.astype(np.float64))
    assert abs(loss - L_ref) <= 1e-4 * L_ref
    gg = g.cpu().numpy().astype(np.float64)
    for name, sl in _slices().items():
        ref = g_ref[sl]
        np.testing.assert_allclose(gg[sl], ref, rtol=0, atol=2e-4 * np.abs(ref).max() + 1e-7,
                                   err_msg=name)


def _slices():
    out, off = {}, 0
    for name, shape in OM.SIZES:
        k = int(np.prod(shape))
        out[name] = slice(off, off + k)
        off += k
    return out


def _bf16(a):
    """Round float32 values to the nearest BF16 (ties to even), as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# The BF16 forward pass against the oracle's forward pass on BF16-rounded
# operands (features, W1, W2 and the hidden activations H1): what remains is
# FP32 accumulation and the rare H1 value whose FP32 sum rounds to the other
# BF16 neighbour, far below the BF16 rounding itself.
@pytest.mark.parametrize("n", [1, 700, 32845])
def test_forward_bf16_matches_rounded_oracle(B, n):
    log(f"[mlp] bf16 forward rows={n}")
    rng = np.random.default_rng(6)
    X = rng.normal(0, 1, (n, 130)).astype(np.float32)
    p = _params(B, 7)
    p += 0.05 * torch.randn(p.numel(), device="cuda", generator=torch.Generator("cuda").manual_seed(2))
    q = OM.unpack(p.cpu().numpy().astype(np.float64))
    ws = _ws(B, n)
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    B.cpmdp_mlp_forward(p, torch.as_tensor(X, device="cuda"), n, y, ws, precision=B.CPMDP_BF16)
    y32 = torch.empty_like(y)
    B.cpmdp_mlp_forward(p, torch.as_tensor(X, device="cuda"), n, y32, ws)
    torch.cuda.synchronize()
    f32 = lambda a: a.astype(np.float32)
    H1 = np.maximum(_bf16(X) @ _bf16(f32(q["W1"])) + q["b1"], 0.0)
    H2 = np.maximum(_bf16(f32(H1)) @ _bf16(f32(q["W2"])) + q["b2"], 0.0)
    y_ref = H2 @ q["w3"] + q["b3"][0]
    scale = np.abs(y_ref).max()
    np.testing.assert_allclose(y.cpu().numpy(), y_ref, rtol=0, atol=2e-3 * scale)
    # and it is a BF16 result: farther from the FP32 pass than FP32 rounding
    assert np.abs(y.cpu().numpy() - y32.cpu().numpy()).max() > 1e-5 * scale


def test_train_step_matches_oracle(B):
    """One training step (SplitMix64 sampling, features, forward, backward,
    Adam) against the oracle reproducing the same samples."""
    m, n_inst, batch, seed, lr = 6, 3, 256, 99, 1e-3
    insts = [I.warm_instance(1, i, m=m) for i in range(n_inst)]
    rng = np.random.default_rng(5)
    Vs = [rng.normal(0, 3, x.n_states) for x in insts]
    R = [torch.as_tensor(x.rewards, dtype=torch.float32, device="cuda") for x in insts]
    V = [torch.as_tensor(v, dtype=torch.float64, device="cuda") for v in Vs]
    Rp = torch.tensor([r.data_ptr() for r in R], dtype=torch.int64, device="cuda")
    Vp = torch.tensor([v.data_ptr() for v in V], dtype=torch.int64, device="cuda")
    gam = torch.tensor([x.gamma for x in insts], dtype=torch.float64, device="cuda")
    slp = torch.tensor([x.meta["slip"] for x in insts], dtype=torch.float64, device="cuda")
    p = _params(B, 6)
    p += 0.05 * torch.randn(p.numel(), device="cuda", generator=torch.Generator("cuda").manual_seed(2))
    p0 = p.cpu().numpy().astype(np.float64)
    mm, vv, gg = torch.zeros_like(p), torch.zeros_like(p), torch.zeros_like(p)
    loss = B.cpmdp_mlp_train_step(p, mm, vv, gg, 1, Rp, Vp, gam, slp, n_inst, m, batch, seed, lr,
                                  _ws(B, batch), want_loss=True)
    torch.cuda.synchronize()
    X = np.empty((batch, 130))
    t = np.empty(batch)
    for i in range(batch):
        a, s = OM.sample(seed, 1, i, n_inst, m ** 3)
        x = insts[a]
        X[i] = OM.features(x.rewards.astype(np.float32).astype(np.float64), m,
                           np.float32(x.gamma), np.float32(x.meta["slip"]), [s])[0]
        t[i] = np.float32(OM.target(Vs[a][s], x.gamma))
    L_ref, g_ref = OM.loss_grad(p0, X, t)
    assert abs(loss - L_ref) <= 1e-4 * L_ref
    p1_ref, _, _ = OM.adam(p0, np.zeros_like(p0), np.zeros_like(p0), g_ref, 1, lr)
    p1 = p.cpu().numpy().astype(np.float64)
    # first Adam step moves each weight by ~lr * sign(g); compare where |g| is
    # not tiny (elsewhere the step's sign depends on rounding of g ~ 0)
    big = np.abs(g_ref) > 1e-3 * np.abs(g_ref).max()
    np.testing.assert_allclose(p1[big], p1_ref[big], rtol=0, atol=2e-6)


def test_train_step_without_loss_matches_with_loss(B):
    """A training step that does not report its loss computes the loss
    gradient inside the output layer; from the same state it must update the
    parameters as the step that reports the loss (same samples, same
    kernels otherwise)."""
    m, n_inst, batch, seed, lr = 7, 3, 1000, 5, 1e-3
    insts = [I.warm_instance(1, i, m=m) for i in range(n_inst)]
    rng = np.random.default_rng(8)
    R = [torch.as_tensor(x.rewards, dtype=torch.float32, device="cuda") for x in insts]
    V = [torch.as_tensor(rng.normal(0, 3, x.n_states), dtype=torch.float64, device="cuda")
         for x in insts]
    Rp = torch.tensor([r.data_ptr() for r in R], dtype=torch.int64, device="cuda")
    Vp = torch.tensor([v.data_ptr() for v in V], dtype=torch.int64, device="cuda")
    gam = torch.tensor([x.gamma for x in insts], dtype=torch.float64, device="cuda")
    slp = torch.tensor([x.meta["slip"] for x in insts], dtype=torch.float64, device="cuda")
    p0 = _params(B, 9)
    p0 += 0.05 * torch.randn(p0.numel(), device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    out = []
    for want in (True, False):
        p = p0.clone()
        mm, vv, gg = torch.zeros_like(p), torch.zeros_like(p), torch.zeros_like(p)
        B.cpmdp_mlp_train_step(p, mm, vv, gg, 1, Rp, Vp, gam, slp, n_inst, m, batch, seed, lr,
                               _ws(B, batch), want_loss=want)
        torch.cuda.synchronize()
        out.append((p.cpu().numpy(), gg.cpu().numpy()))
    (pa, ga), (pb, gb) = out
    np.testing.assert_allclose(gb, ga, rtol=1e-5, atol=1e-6 * np.abs(ga).max())
    # Adam moves a weight by about lr * sign(g): where g is within rounding of
    # 0 the sign (and so the update) follows the rounding; compare elsewhere
    big = np.abs(ga) > 1e-3 * np.abs(ga).max()
    np.testing.assert_allclose(pb[big], pa[big], rtol=0, atol=1e-6)


def _ab_sweeps(B, w, x, kinds=("cold", "shift", "warm", "warm+shift")):
    """FP64 value iteration of instance x from several starts: cold (V0 = 0),
    shift (V0 = 0, one backup and the McQueen bound shift: the method without
    the network), warm (the network's value level), warm+shift.  Returns
    {kind: (V, sweeps incl. the shift's backup, certificate)}."""
    model = B.Model(x)
    runs = {}
    for kind in kinds:
        V = w.predict(x) if kind.startswith("warm") else \
            torch.zeros(x.n_states, dtype=torch.float64, device="cuda")
        extra = 0
        if kind.endswith("shift"):
            B.cpmdp_bound_shift(model.h, V)
            extra = 1
        c, sw, r = B.cpmdp_value_iteration(model.h, V, None, 1e-6, 100000, B.CPMDP_FP64)
        assert c == B.CPMDP_OK and r <= 1e-6
        runs[kind] = (V, sw + extra, r)
    model.close()
    for kind in kinds[1:]:
        diff = float((runs[kinds[0]][0] - runs[kind][0]).abs().max())
        assert diff <= 2e-6 / (1 - x.gamma)
    return runs


@pytest.mark.parametrize("m,chunk", [(9, None), (9, 100), (20, None)])
def test_predict_level_is_mean_of_sampled_states(B, m, chunk):
    """Level mode: every state holds the mean of the network's predictions at
    the n = min(S, chunk, 4096) states floor(j S / n); the same network's
    per-state predictions at those states give the same mean."""
    from paper_2103_00331_amd.warmstart import WarmStart
    w = WarmStart(m=m, batch=256, seed=3)
    w.params += 0.05 * torch.randn(w.params.numel(), device="cuda",
                                   generator=torch.Generator("cuda").manual_seed(4))
    x = I.warm_instance(2, 1, m=m)
    S = x.n_states
    per = w.predict(x, level=False)
    lev = w.predict(x, chunk=chunk)
    again = w.predict(x, chunk=chunk)
    torch.cuda.synchronize()
    n = min(S, chunk or S, 4096)
    idx = (np.arange(n, dtype=np.int64) * S) // n
    mean = float(per.cpu().numpy()[idx].mean())
    assert float((lev - mean).abs().max()) <= 1e-5 * max(1.0, abs(mean))
    assert torch.equal(lev, again)                     # fixed summation order
    assert float(lev.max() - lev.min()) == 0.0


@pytest.mark.parametrize("m", [9, 20])
@pytest.mark.parametrize("bf16", [False, True])
def test_predict_levels_match_single_predictions(B, m, bf16):
    """The batched level prediction (one forward pass over every instance's
    spread states) gives each instance the level of its own level-mode
    prediction (to FP32 rounding: the forward pass may group its sums
    differently for more rows), the same bits on a repeat, and rejects
    mismatched argument lists."""
    from paper_2103_00331_amd.warmstart import WarmStart
    w = WarmStart(m=m, batch=256, seed=5)
    w.params += 0.05 * torch.randn(w.params.numel(), device="cuda",
                                   generator=torch.Generator("cuda").manual_seed(6))
    insts = [I.warm_instance(2, i, m=m) for i in range(9)]
    single = [w.predict(x, bf16=bf16) for x in insts]
    lev = w.predict_levels(insts, bf16=bf16)
    again = w.predict_levels(insts, bf16=bf16)
    torch.cuda.synchronize()
    for x, a, b, c in zip(insts, single, lev, again):
        ref = float(a[0])
        assert float(a.max() - a.min()) == 0.0
        assert float(b.max() - b.min()) == 0.0
        assert abs(float(b[0]) - ref) <= 1e-5 * max(1.0, abs(ref)), (x.gamma, float(b[0]), ref)
        assert torch.equal(b, c)
    # the levels differ between instances (the call does not mix them up)
    assert len({round(float(v[0]), 9) for v in lev}) == len(insts)
    with pytest.raises(ValueError):
        B.cpmdp_mlp_predict_levels(w.params, [torch.zeros(m ** 3, device="cuda")], [0.9, 0.9], [0.1],
                                   m, [lev[0]], w.infer_ws)


def test_warm_start_reduces_sweeps(B):
    """Train on solved instances of the generator (small grids), then solve
    held-out instances from V0 = 0, from V0 = 0 with the bound shift (the
    method without the network) and from the network's value level."""
    from paper_2103_00331_amd.warmstart import WarmStart, training_instances
    m = 12
    log("[mlp] warm start: building training set")
    w = WarmStart(m=m, batch=2048, seed=7)
    w.add_instances(training_instances(96, m=m, split=0))
    losses = w.train(800, lr=1e-3, lr_final=1e-4, log_every=100)
    log(f"   losses {losses}")
    assert losses[-1][1] < 0.6 * losses[0][1]
    sweeps = {k: [] for k in ("cold", "shift", "warm", "warm+shift")}
    for i in range(6):
        runs = _ab_sweeps(B, w, I.warm_instance(2, i, m=m))
        for k in sweeps:
            sweeps[k].append(runs[k][1])
    log(f"   sweeps {sweeps}")
    # the network's own gain: fewer sweeps than the method without it
    assert np.mean(sweeps["warm"]) < np.mean(sweeps["shift"])
    assert np.mean(sweeps["warm"]) < np.mean(sweeps["cold"])


def test_warm_start_64_held_out(B):
    """The learned warm start at the workload's size (64^3, 262,144 states):
    trained on solver-generated instances, then held-out instances solved
    from the network's V0.  Each solve is certified; the oracle recomputes
    the Bellman residual of the returned V and checks the returned policy;
    and the network saves sweeps over the method without it."""
    import oracle
    from paper_2103_00331_amd.warmstart import WarmStart, training_instances
    from tests.parity import compare_policy
    m = 64
    log("[mlp] 64^3 warm start: training set")
    w = WarmStart(m=m, batch=4096, seed=11)
    w.add_instances(training_instances(128, m=m, split=0))
    losses = w.train(1500, lr=1e-3, lr_final=1e-4, log_every=500)
    log(f"   losses {losses}")
    cold_shift, warm = [], []
    for i in range(3):
        x = I.warm_instance(2, i, m=m)
        runs = _ab_sweeps(B, w, x, kinds=("warm", "shift"))
        cold_shift.append(runs["shift"][1])
        warm.append(runs["warm"][1])
        if i == 0:
            # greedy policy of the warm-started solve, then the oracle's check
            model = B.Model(x)
            V = w.predict(x)
            pi = torch.zeros(x.n_states, dtype=torch.int32, device="cuda")
            c, sw, r = B.cpmdp_value_iteration(model.h, V, pi, 1e-6, 100000, B.CPMDP_FP64)
            model.close()
            assert c == B.CPMDP_OK and r <= 1e-6
            Vh = V.cpu().numpy()
            mats = oracle.sparse.transition_csr(x)
            Q = oracle.sparse.q_values(x, mats, Vh)
            r_or = float(np.max(np.abs(Q.max(0) - Vh)))
            assert abs(r_or - r) <= 1e-12
            compare_policy(pi.cpu().numpy(), Q, 1e-9)
    log(f"   sweeps cold+shift {cold_shift} warm {warm}")
    assert np.mean(warm) < np.mean(cold_shift)
