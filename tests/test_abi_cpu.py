"""CPU-side checks of the C ABI: the library loads, exports every function
that include/cpmdp.h declares, and rejects invalid problems in cpmdp_create
(host-only validation, no device work)."""
import os
import re

import numpy as np
import pytest

from paper_2103_00331_amd import binding as B
from paper_2103_00331_amd import instances as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(cpmdp_[a-z0-9_]+)\s*\(", txt))
    return names


def test_exports_every_declared_symbol():
    declared = _declared()
    assert "cpmdp_create" in declared and "cpmdp_value_iteration" in declared
    for name in sorted(declared):
        assert hasattr(B.lib, name), name
    assert declared <= set(B.EXPORTED)


def test_binding_shares_torch_hip_runtime():
    # Importing the binding on its own (no torch import before it) must leave
    # one HIP runtime in the process, the one torch uses.
    import ast
    import subprocess
    import sys
    code = ("from paper_2103_00331_amd import binding\n"
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps')\n"
            "              if 'libamdhip64' in l}))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True,
                         text=True, timeout=300, check=True).stdout.strip().splitlines()[-1]
    libs = ast.literal_eval(out)
    assert len(libs) == 1, libs


def _args(inst):
    return (inst.sizes, inst.ranks, inst.factors, inst.lambdas, inst.rewards, inst.gamma)


def test_create_valid_and_path_classification():
    g = I.grid2d_16()
    h = B.cpmdp_create(*_args(g))
    assert B.cpmdp_get_path(h) == B.CPMDP_PATH_STENCIL
    assert B.cpmdp_workspace_bytes(h) > 0
    B.cpmdp_set_terminal(h, g.terminal)
    B.cpmdp_destroy(h)
    d = I.random_dense([3, 4], 2, 2, seed=1)
    h = B.cpmdp_create(*_args(d))
    assert B.cpmdp_get_path(h) == B.CPMDP_PATH_DENSE
    B.cpmdp_destroy(h)


def _expect(code, **changes):
    g = I.grid_small([3, 4], seed=0)
    a = dict(sizes=g.sizes.copy(), ranks=g.ranks.copy(), factors=g.factors.copy(),
             lambdas=g.lambdas.copy(), rewards=g.rewards.copy(), gamma=g.gamma)
    for k, v in changes.items():
        a[k] = v(a[k]) if callable(v) else v
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_create(a["sizes"], a["ranks"], a["factors"], a["lambdas"], a["rewards"],
                       a["gamma"])
    assert e.value.code == code, str(e.value)


def _bump(i, by):
    def f(x):
        x = x.copy()
        x[i] += by
        return x
    return f


def test_create_rejects_invalid():
    _expect(B.CPMDP_E_ARG, gamma=1.0)
    _expect(B.CPMDP_E_ARG, gamma=-0.1)
    _expect(B.CPMDP_E_NONFINITE, gamma=float("nan"))
    _expect(B.CPMDP_E_NONFINITE, rewards=_bump(3, float("nan")))
    _expect(B.CPMDP_E_NONFINITE, factors=_bump(0, float("inf")))
    _expect(B.CPMDP_E_NOT_STOCHASTIC, factors=_bump(0, 1e-9))       # row sum off
    _expect(B.CPMDP_E_NOT_STOCHASTIC, lambdas=_bump(0, 1e-9))       # lambda sum off
    _expect(B.CPMDP_E_ARG, sizes=np.array([3, 0]))                   # size 0
    _expect(B.CPMDP_E_ARG, ranks=lambda r: np.where(np.arange(r.size) == 0, 0, r))


def test_negative_probability_rejected():
    g = I.grid_small([3, 4], seed=0)
    f = g.factors.copy()
    f[0:3] = [1.5, -0.5, 0.0]    # row 0 of the first factor still sums to 1
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_create(g.sizes, g.ranks, f, g.lambdas, g.rewards, g.gamma)
    assert e.value.code == B.CPMDP_E_NOT_STOCHASTIC


def test_obstacles_and_calls_before_bind():
    g = I.grid_small([3, 4], seed=0)
    h = B.cpmdp_create(*_args(g))
    mask = np.zeros(g.n_states, np.uint8)
    B.cpmdp_set_obstacles(h, mask)          # no obstacle: fine
    base = B.cpmdp_workspace_bytes(h)
    mask[5] = 1
    B.cpmdp_set_obstacles(h, mask)          # shift/identity factors: accepted
    assert B.cpmdp_workspace_bytes(h) >= base + 2 * g.n_states
    code = B.lib.cpmdp_value_iteration(h, None, None, 1e-6, 10, 0, None, None)
    assert code == B.CPMDP_E_STATE          # not bound to a workspace yet
    B.cpmdp_destroy(h)
    d = I.random_dense([3, 4], 2, 2, seed=1)
    h = B.cpmdp_create(*_args(d))
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_set_obstacles(h, mask)      # dense factors: not a sparse fix-up
    assert e.value.code == B.CPMDP_E_UNSUPPORTED
    B.cpmdp_destroy(h)


def test_batch_rejects_obstacles():
    g = I.grid_small([4, 8], seed=0)
    h = B.cpmdp_create(*_args(g))
    mask = np.zeros(g.n_states, np.uint8)
    mask[3] = 1
    B.cpmdp_set_obstacles(h, mask)
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_batch_create([h])
    assert e.value.code == B.CPMDP_E_UNSUPPORTED
    B.cpmdp_destroy(h)


def test_batch_rejects_empty_and_null_handles():
    """A batch needs at least one created handle: an empty list and a NULL
    handle are argument errors, before any device work."""
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_batch_create([])
    assert e.value.code == B.CPMDP_E_ARG
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_batch_create([None])
    assert e.value.code == B.CPMDP_E_ARG


def test_batch_schedule_setter_validates():
    """Host-only: the schedule setter takes the documented values and refuses
    others before any device work."""
    g = I.grid_small([4, 8], seed=0)
    h = B.cpmdp_create(*_args(g))
    b = B.cpmdp_batch_create([h])
    B.cpmdp_batch_set_schedule(b, 2048, 1024, 0, 1)
    assert B.cpmdp_batch_config(b)[0] == 2048
    assert B.cpmdp_batch_schedule(b) == (1024, 0, 1)
    for bad in [(1000, 1024, 1, 0), (2048, 1020, 1, 0), (2048, 4096, 1, 0), (2048, 1024, 2, 0),
                (2048, 1024, 1, 3), (1 << 17, 1024, 1, 0)]:
        with pytest.raises(B.CpmdpError) as e:
            B.cpmdp_batch_set_schedule(b, *bad)
        assert e.value.code == B.CPMDP_E_ARG
    assert B.cpmdp_batch_schedule(b) == (1024, 0, 1)
    B.cpmdp_batch_destroy(b)
    B.cpmdp_destroy(h)


def test_dense_factor_size_limit():
    d = I.random_dense([40, 2], 1, 1, seed=3)
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_create(*_args(d))
    assert e.value.code == B.CPMDP_E_UNSUPPORTED


def _lists_args(m):
    return (m.n_states, m.n_actions, m.row_ptr, m.succ, m.prob, m.rewards, m.gamma)


def test_create_lists_valid_and_rejects_invalid():
    m = I.random_lists(100, 3, 4, seed=2, gamma=0.9)
    h = B.cpmdp_create_lists(*_lists_args(m))
    assert B.cpmdp_get_path(h) == B.CPMDP_PATH_LISTS
    assert B.cpmdp_workspace_bytes(h) > 0
    mask = np.zeros(m.n_states, np.uint8)
    mask[3] = 1
    B.cpmdp_set_terminal(h, mask)
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_set_obstacles(h, mask)        # lists express blocked moves themselves
    assert e.value.code == B.CPMDP_E_UNSUPPORTED
    B.cpmdp_destroy(h)

    def expect(code, **kw):
        a = dict(zip(["S", "A", "row_ptr", "succ", "prob", "rewards", "gamma"],
                     [x.copy() if isinstance(x, np.ndarray) else x for x in _lists_args(m)]))
        a.update(kw)
        with pytest.raises(B.CpmdpError) as e:
            B.cpmdp_create_lists(a["S"], a["A"], a["row_ptr"], a["succ"], a["prob"],
                                 a["rewards"], a["gamma"])
        assert e.value.code == code, str(e.value)

    p = m.prob.copy()
    p[0] += 1e-6
    expect(B.CPMDP_E_NOT_STOCHASTIC, prob=p)                   # list sum off
    p = m.prob.copy()
    i = int(np.nonzero(np.diff(m.row_ptr) >= 2)[0][0])
    lo = m.row_ptr[i]
    p[lo], p[lo + 1] = p[lo] + p[lo + 1] + 0.5, -0.5
    expect(B.CPMDP_E_NOT_STOCHASTIC, prob=p)                   # negative entry
    s = m.succ.copy()
    s[5] = m.n_states
    expect(B.CPMDP_E_ARG, succ=s)                              # successor out of range
    r = m.row_ptr.copy()
    r[10], r[11] = r[11], r[10]
    if r[10] != r[11]:
        expect(B.CPMDP_E_ARG, row_ptr=r)                       # decreasing offsets
    expect(B.CPMDP_E_ARG, gamma=1.0)
    expect(B.CPMDP_E_ARG, A=0)
    rw = m.rewards.copy()
    rw[1] = np.inf
    expect(B.CPMDP_E_NONFINITE, rewards=rw)


def test_create_tt_valid_and_rejects_invalid():
    t = I.random_tt([3, 4, 2], 2, 3, seed=3)
    h = B.cpmdp_create_tt(t.sizes, t.bonds, t.cores, t.rewards, t.gamma)
    assert B.cpmdp_get_path(h) == B.CPMDP_PATH_TT
    assert B.cpmdp_workspace_bytes(h) > 0
    mask = np.zeros(t.n_states, np.uint8)
    mask[2] = 1
    B.cpmdp_set_terminal(h, mask)
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_set_obstacles(h, mask)
    assert e.value.code == B.CPMDP_E_UNSUPPORTED
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_batch_create([h])
    assert e.value.code == B.CPMDP_E_UNSUPPORTED
    B.cpmdp_destroy(h)

    def expect(code, sizes=t.sizes, bonds=t.bonds, cores=t.cores, rewards=t.rewards,
               gamma=t.gamma):
        with pytest.raises(B.CpmdpError) as e:
            B.cpmdp_create_tt(sizes, bonds, cores, rewards, gamma)
        assert e.value.code == code, str(e.value)

    c = t.cores.copy()
    c[5] *= 1.001
    expect(B.CPMDP_E_NOT_STOCHASTIC, cores=c)                  # a row of P off by ~1e-4
    c = t.cores.copy()
    c[0] = -c[0]
    expect(B.CPMDP_E_NOT_STOCHASTIC, cores=c)                  # negative entry
    c = t.cores.copy()
    c[7] = np.nan
    expect(B.CPMDP_E_NONFINITE, cores=c)
    b = t.bonds.copy()
    b[0, 0] = 2
    expect(B.CPMDP_E_ARG, bonds=b)                             # end bonds must be 1
    big = I.random_tt([2, 2], 1, 9, seed=4)
    expect(B.CPMDP_E_UNSUPPORTED, sizes=big.sizes, bonds=big.bonds, cores=big.cores,
           rewards=big.rewards)                                # bond 9 > 8
    wide = I.random_tt([17, 2], 1, 2, seed=5)
    expect(B.CPMDP_E_UNSUPPORTED, sizes=wide.sizes, bonds=wide.bonds, cores=wide.cores,
           rewards=wide.rewards)                               # m_k = 17 > 16
    expect(B.CPMDP_E_ARG, gamma=1.0)


def test_create_tucker_valid_and_rejects_invalid():
    u = I.random_tucker([3, 2, 4], 2, [2, 3, 2], seed=6)
    args = dict(sizes=u.sizes, core_ranks=u.core_ranks, cores=u.cores, factors=u.factors,
                rewards=u.rewards, gamma=u.gamma)
    h = B.cpmdp_create_tucker(**args)
    assert B.cpmdp_get_path(h) == B.CPMDP_PATH_TT
    B.cpmdp_destroy(h)

    def expect(code, **kw):
        a = dict(args)
        a.update(kw)
        with pytest.raises(B.CpmdpError) as e:
            B.cpmdp_create_tucker(**a)
        assert e.value.code == code, str(e.value)

    c = u.cores.copy()
    c[0] += 1e-6
    expect(B.CPMDP_E_NOT_STOCHASTIC, cores=c)                  # core sum off
    f = u.factors.copy()
    f[3] = -0.1
    expect(B.CPMDP_E_NOT_STOCHASTIC, factors=f)
    f = u.factors.copy()
    f[0] += 1e-3
    expect(B.CPMDP_E_NOT_STOCHASTIC, factors=f)                # factor row sum off
    r = u.core_ranks.copy()
    r[0, 0] = 0
    expect(B.CPMDP_E_ARG, core_ranks=r)
    wide = I.random_tucker([2, 2, 2, 2], 1, [3, 3, 3, 3], seed=7)
    expect(B.CPMDP_E_UNSUPPORTED, sizes=wide.sizes, core_ranks=wide.core_ranks,
           cores=wide.cores, factors=wide.factors, rewards=wide.rewards)   # bond 9 > 8


def test_cp_fit_rejects_before_device_work():
    """Argument checks of cpmdp_cp_fit that run before any device call."""
    assert B.cpmdp_cp_fit_workspace_bytes([4, 3], 100, 3) > 0
    for sizes, nnz, rank, code in [([4, 3], 100, 0, B.CPMDP_E_ARG), ([4, 3], 100, 33, B.CPMDP_E_ARG),
                                   ([4, 3], 0, 3, B.CPMDP_E_ARG),
                                   ([32, 3], 100, 9, B.CPMDP_E_UNSUPPORTED),  # 32^2 * 9 > 8192
                                   ([0, 3], 100, 3, B.CPMDP_E_ARG)]:
        with pytest.raises(B.CpmdpError) as e:
            B.cpmdp_cp_fit_workspace_bytes(sizes, nnz, rank)
        assert e.value.code == code


def test_mlp_precision_rejected():
    # argument checks run before any device work: host buffers stand in
    buf = np.zeros(16, np.float32)
    p = buf.ctypes.data
    assert B.lib.cpmdp_mlp_forward(p, p, 4, p, 5, p, 64, None) == B.CPMDP_E_ARG
    assert B.lib.cpmdp_mlp_forward(p, p, 4, p, B.CPMDP_FP64, p, 64, None) == B.CPMDP_E_ARG
    assert B.lib.cpmdp_mlp_predict(p, p, 4, 0.9, 0.1, p, 64, 9, 0, p, 64, None) == B.CPMDP_E_ARG
    # level must be 0 or 1
    assert B.lib.cpmdp_mlp_predict(p, p, 4, 0.9, 0.1, p, 64, B.CPMDP_FP32, 2, p, 1 << 40,
                                   None) == B.CPMDP_E_ARG


def test_mlp_rejects_oversized_grid():
    """m^3 >= 2^31 would overflow the kernels' 32-bit state index: the entry
    points refuse it before any device work (host buffers stand in)."""
    buf = np.zeros(16, np.float32)
    p = buf.ctypes.data
    m = 1291                                     # 1291^3 > 2^31
    assert B.lib.cpmdp_mlp_predict(p, p, m, 0.9, 0.1, p, 64, B.CPMDP_FP32, 0, p, 1 << 40,
                                   None) == B.CPMDP_E_ARG
    assert B.lib.cpmdp_mlp_features(p, m, 0.9, 0.1, 0, 4, p, None) == B.CPMDP_E_ARG
    assert B.lib.cpmdp_mlp_train_step(p, p, p, p, 1, p, p, p, p, 1, m, 64, 1, 1e-3, p, 1 << 40,
                                      None, None) == B.CPMDP_E_ARG


def test_warm_start_refuses_other_grid_sizes():
    """WarmStart indexes R, V* and V0 as m^3 arrays: an instance of another
    shape is refused before any pointer reaches a kernel."""
    import types
    from paper_2103_00331_amd.warmstart import WarmStart
    w = types.SimpleNamespace(m=8)
    WarmStart._check(w, I.warm_instance(2, 0, m=8))          # the right shape passes
    for bad in (I.warm_instance(2, 0, m=6), I.grid_small([8, 8], seed=0),
                I.grid_small([8, 8, 9], seed=0)):
        with pytest.raises(ValueError):
            WarmStart._check(w, bad)
