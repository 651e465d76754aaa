#!/usr/bin/env python3
"""Benchmark of the CP-structured Bellman backup on one MI355X.

Default workload: the batch of 512 GridWorlds (n uniform in {2, 3, 4}, side
m uniform in [8, 48], slip U[0.05, 0.3], gamma U[0.9, 0.99], rewards
N(0, 0.1) plus a +1 terminal goal corner; 219,514,047 states in total), the
largest single-GPU workload.  One step = one complete solve of all 512
instances from V0 = 0 to a certified FP64 Bellman residual <= 1e-6 per
instance by the chosen form (batched FP32 value-iteration sweeps in graph
replays, FP64 tail sweeps, FP64 certificate).  The metric is state-action
backups per second over the timed steps; time-to-eps of the chosen form and
of plain FP64 value iteration of each instance on its own from V0 = 0 are
reported beside it, with the error against the FP64 oracle on sampled
instances.

Also printed (one JSON line): the roofline of the dominant kernel (the FP32
whole-batch sweep), timed live with HIP events on the library's stream, and
the FP64 CPU oracle timed on a bounded sample of the same workload on the
host's cores and on one core.

Other workloads (--workload): grid4d_32 (32^4, cache-resident), grid4d_96
(96^4, HBM-resident), dense6_16
(16^6, dense 16x16 factors, 12 actions of rank 8), batch512 (512 mixed
GridWorlds), warm64 (learned warm start on 64^3) and paper2d_1000 (the
1000 x 1000 GridWorld of Table 1 with 22 terminals and 800 obstacles) and
paper2d_lists (the same problem given as Def. 3 successor lists) and tt6_16
(16^6, 12 actions with Tensor-Train transitions of bond 4) and cpfit_grid4d_32
(CP-ALS fit at rank 7 of one action's 32^4 transition matrix, 7.3 M entries).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("state-action Bellman backups/s; time to ε=1e-6 residual, chosen vs "
          "plain GPU VI")
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


STENCIL_SRC = ["paper_2103_00331_amd/csrc/stencil.hip", "paper_2103_00331_amd/csrc/stencil_core.cuh",
               "paper_2103_00331_amd/csrc/common.cuh"]
CHAIN_SRC = ["paper_2103_00331_amd/csrc/chain.hip", "paper_2103_00331_amd/csrc/common.cuh"]
# FP32 and BF16 max sweeps of 16^6 grids run the register-resident units
CHAIN16_SRC = ["paper_2103_00331_amd/csrc/chain16.hip", "paper_2103_00331_amd/csrc/common.cuh"]
BATCH_SRC = ["paper_2103_00331_amd/csrc/batch.hip", "paper_2103_00331_amd/csrc/stencil_core.cuh",
             "paper_2103_00331_amd/csrc/common.cuh"]
LISTS_SRC = ["paper_2103_00331_amd/csrc/lists.hip", "paper_2103_00331_amd/csrc/common.cuh"]
TT_SRC = ["paper_2103_00331_amd/csrc/tt.hip", "paper_2103_00331_amd/csrc/common.cuh"]
CPFIT_SRC = ["paper_2103_00331_amd/csrc/cpfit.hip", "paper_2103_00331_amd/csrc/common.cuh"]
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp64": 78.6}


def _traffic(profile_md, src):
    """HBM bytes per launch measured by rocprofv3 counters, if the kernel
    sources still hash to what was profiled; else None."""
    path = os.path.join(ROOT, "profiles", profile_md)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_sha = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", txt)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_sha or not m_b or m_sha.group(1) != _sha(src):
        return None
    return float(m_b.group(1))


def _copy_reference(nbytes):
    """Achievable-bandwidth references measured here with torch: a 1 GiB
    copy (GB/s counting read + write) and a copy that moves nbytes (half read,
    half written) per launch, back to back (ms per launch); each the better of
    copy_ and an elementwise multiply into the destination.
    """
    import torch
    out = {}
    for key, size in (("stream_copy", 1 << 29), ("same_bytes_copy", max(int(nbytes) // 2, 4))):
        n = size // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        reps = 20 if key == "stream_copy" else 400
        best = None
        for op in (lambda: dst.copy_(src), lambda: torch.mul(src, 1.0, out=dst)):
            for _ in range(5):
                op()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                op()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            best = ms if best is None else min(best, ms)
        out[key] = (2.0 * n * 4 / (best * 1e-3) / 1e9, best)
        del src, dst
    return {"stream_copy_GBps": out["stream_copy"][0],
            "same_bytes_copy_ms": out["same_bytes_copy"][1]}


def _cpu_baseline_grid(inst, budget_s=15.0):
    """FP64 value-iteration sweeps of the Def. 3 successor-list oracle."""
    import numpy as np

    import oracle
    _log("cpu baseline: building the oracle's successor lists")
    mats = oracle.sparse.transition_csr(inst)
    V = np.zeros(inst.n_states)
    t0 = time.perf_counter()
    V = oracle.sparse.q_values(inst, mats, V).max(axis=0)
    t1 = time.perf_counter() - t0
    n = int(max(1, min(200, budget_s / max(t1, 1e-6)))) - 1
    t0 = time.perf_counter()
    for _ in range(n):
        V = oracle.sparse.q_values(inst, mats, V).max(axis=0)
    tn = time.perf_counter() - t0
    sweeps, secs = n + 1, tn + t1
    rate = sweeps * inst.n_states * inst.n_actions / secs
    return {"value": rate, "unit": "state-action backups/s", "cores": 1, "kind": "oracle",
            "sample": f"{sweeps} FP64 value-iteration sweeps of the successor-list (Def. 3) "
                      f"oracle on the same {inst.name} instance from V0 = 0, {secs:.1f} s; "
                      "successor-list construction excluded; scipy CSR matvec, one thread"}


def _host_cpu():
    """CPU model and the cores this process may use (affinity), capped at the
    16-core share of one GPU on the GPU machines."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return model, int(avail), int(min(avail, 16))


def _oracle_batch_worker(arg):
    """One process: FP64 value-iteration sweeps of the Def. 3 successor-list
    oracle on batch instance idx from V0 = 0 for about `budget` seconds
    (list construction excluded)."""
    idx, budget = arg
    import numpy as np

    import oracle
    from paper_2103_00331_amd import instances as I
    x = I.batch_instance(idx)
    mats = oracle.sparse.transition_csr(x)
    V = np.zeros(x.n_states)
    sweeps = 0
    t0 = time.perf_counter()
    while True:
        V = oracle.sparse.q_values(x, mats, V).max(axis=0)
        sweeps += 1
        el = time.perf_counter() - t0
        if el >= budget:
            break
    return idx, sweeps * x.n_states * x.n_actions, el, sweeps


def _cpu_baseline_batch(budget_s=8.0, max_states=1 << 20):
    """The oracle on a seeded sample of the batch's instances: one process per
    core (the oracle itself is single-threaded), then one core alone.  Runs
    before the GPU is touched (the pool forks)."""
    import multiprocessing as mp

    import numpy as np

    from paper_2103_00331_amd import instances as I
    model, avail, cores = _host_cpu()
    shapes = I.batch_shapes()
    pool_idx = [i for i, (n, m) in enumerate(shapes) if m ** n <= max_states]
    rng = np.random.default_rng(2021_0099)
    sample = [int(i) for i in rng.choice(pool_idx, size=cores, replace=len(pool_idx) < cores)]
    env_keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                                "MKL_NUM_THREADS")}
    for k in env_keep:
        os.environ[k] = "1"
    try:
        ctx = mp.get_context("fork")
        _log(f"cpu baseline: oracle on {cores} batch instances, {cores} processes")
        with ctx.Pool(cores) as pool:
            multi = pool.map(_oracle_batch_worker, [(i, budget_s) for i in sample])
        _log("cpu baseline: one core")
        with ctx.Pool(1) as pool:
            one = pool.map(_oracle_batch_worker, [(i, budget_s / len(sample)) for i in sample])
    finally:
        for k, v in env_keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    rate_multi = sum(b / el for _, b, el, _ in multi)
    rate_one = sum(b for _, b, _, _ in one) / sum(el for _, _, el, _ in one)
    sizes = sorted(shapes[i][1] ** shapes[i][0] for i in sample)
    return {"value": rate_multi, "unit": "state-action backups/s", "cores": cores,
            "kind": "oracle", "cpu_model": model, "host_cpus_available": avail,
            "one_core_value": rate_one,
            "sample": (f"FP64 value-iteration sweeps of the successor-list (Def. 3) oracle from "
                       f"V0 = 0, about {budget_s:.0f} s per process: {cores} seeded batch "
                       f"instances of {sizes[0]}..{sizes[-1]} states (those <= {max_states} "
                       f"states), one single-threaded process each, summed; one_core_value = "
                       f"the same instances one after another in one process; list "
                       f"construction excluded")}


def _batch_oracle_check(insts, Vs, pis, res, count=6):
    """Error of the batched result against the FP64 oracle on a seeded sample
    of instances (the oracle's own value iteration to 1e-13), and the
    certified bound max_i res_i / (1 - gamma_i) over all instances."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(2021_0098)
    small = [i for i, x in enumerate(insts) if x.n_states <= 60000]
    pick = sorted(int(i) for i in rng.choice(small, size=min(count, len(small)), replace=False))
    err, clear_bad, near = 0.0, 0, 0
    for i in pick:
        x = insts[i]
        mats = oracle.sparse.transition_csr(x)
        Vs_o, _, _, _ = oracle.sparse.value_iteration(x, mats=mats)
        V = Vs[i].cpu().numpy()
        err = max(err, float(np.max(np.abs(V - Vs_o))))
        Q = oracle.sparse.q_values(x, mats, Vs_o)
        srt = np.sort(Q, axis=0)
        gap = srt[-1] - srt[-2]
        tol = 2 * float(res[i]) / (1 - x.gamma) + 1e-12
        clear = gap > 2 * tol
        pi = pis[i].cpu().numpy()
        clear_bad += int(np.sum(clear & (pi != np.argmax(Q, axis=0))))
        near += int(np.sum(~clear))
    bound = max(float(r) / (1 - x.gamma) for r, x in zip(res, insts))
    return {"max_abs_err_sampled": err, "sampled_instances": pick,
            "policy_mismatch_clear_states": clear_bad, "near_tie_states": near,
            "certified_bound_all": bound}


def bench_grid(args, m):
    import numpy as np
    import torch

    from paper_2103_00331_amd import binding as B
    from paper_2103_00331_amd import instances as I

    if args.workload == "paper2d_1000":
        _log("building the 1000 x 1000 GridWorld (22 terminals, 800 obstacles)")
        inst = I.named("paper2d_1000")
    else:
        seed = I.SEED_GRID4 if m == 32 else I.SEED_GRID4_LARGE
        _log(f"building {m}^4 instance")
        inst = I.grid4d(m, seed)
    S, A = inst.n_states, inst.n_actions
    n = inst.n_dims
    obstacles = inst.obstacle is not None and bool(inst.obstacle.any())
    model = B.Model(inst)
    if args.one_pass:
        B.cpmdp_set_option(model.h, B.CPMDP_OPT_MARCH, 0)
    eps = 1e-6
    V = torch.zeros(S, dtype=torch.float64, device="cuda")
    pi = torch.zeros(S, dtype=torch.int32, device="cuda")
    prec = {"fp32": B.CPMDP_FP32, "fp64": B.CPMDP_FP64}[args.precision]

    def solve():
        V.zero_()
        pi.zero_()
        if args.method == "vi":
            code, sweeps, res = B.cpmdp_value_iteration(model.h, V, pi, eps, 100000, prec)
            backups = sweeps * S * A
        else:
            code, outer, sweeps, res = B.cpmdp_policy_iteration(model.h, V, pi, eps, 100000,
                                                                prec)
            backups = sweeps * S          # evaluation sweeps dominate; counted as 1 action
        assert code == B.CPMDP_OK and res <= eps, (code, res)
        return sweeps, backups, res

    for i in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot_sweeps = tot_backups = 0
    res = None
    for i in range(args.steps):
        sw, bk, res = solve()
        tot_sweeps += sw
        tot_backups += bk
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    _log(f"chosen: {ms_per_step:.2f} ms/solve, {tot_sweeps / args.steps:.0f} sweeps, res {res:.2e}")

    # plain GPU VI: FP64 sweeps from V0 = 0 on the same instance (one untimed
    # run, then the mean over as many runs as the chosen form was timed)
    plain_runs = []
    for i in range(1 + max(1, args.steps)):
        V.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        code, plain_sweeps, plain_res = B.cpmdp_value_iteration(model.h, V, pi, eps, 100000,
                                                                B.CPMDP_FP64)
        torch.cuda.synchronize()
        assert code == B.CPMDP_OK and plain_res <= eps, (code, plain_res)
        if i > 0:
            plain_runs.append(time.perf_counter() - t0)
    plain_s = sum(plain_runs) / len(plain_runs)
    _log(f"plain FP64 VI: {plain_s * 1e3:.2f} ms, {plain_sweeps} sweeps")

    # dominant kernel: the FP32 stencil max sweep, timed per launch with events
    Va = torch.zeros(S, dtype=torch.float32, device="cuda")
    Vb = torch.zeros(S, dtype=torch.float32, device="cuda")
    ms = B.cpmdp_time_sweeps(model.h, Va, Vb, 400, B.CPMDP_FP32, 0)
    # V, R, V' words + terminal bit (+ the 16-bit blocked-direction mask)
    algo_bytes = S * (4 + 4 + 4) + S / 8.0 + (2 * S if obstacles else 0)
    achieved = algo_bytes / (ms * 1e-3) / 1e9
    plane = S // int(inst.sizes[0])
    march = (n >= 2 and plane >= 65536 and int(inst.sizes[0]) >= 8 and int(inst.sizes[-1]) % 4 == 0
             and not args.one_pass)
    if args.workload == "paper2d_1000":
        traffic = None
    else:
        traffic = _traffic("stencil_march_fp32_grid4d_96.md" if march
                           else f"stencil_fp32_grid4d_{m}.md", STENCIL_SRC)
    vec = 4 if int(inst.sizes[-1]) % 4 == 0 else 1
    kname = (f"stencil_march_kernel<float, {n}, MODE_MAX, AXIS>" if march
             else f"stencil_kernel<float, {n}, MODE_MAX, VEC={vec}, AXIS>")
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": kname, "kernel_ms": ms, "algorithmic_bytes_per_launch": algo_bytes}
    ref = _copy_reference(algo_bytes)
    roof["stream_copy_GBps"] = ref["stream_copy_GBps"]
    roof["frac_of_stream_copy"] = achieved / ref["stream_copy_GBps"]
    roof["same_bytes_copy_ms"] = ref["same_bytes_copy_ms"]

    out = {
        "metric": METRIC,
        "value": tot_backups / elapsed,
        "unit": "state-action backups/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == B.CPMDP_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": (f"gridworld_{m}^4: {S} states, {A} actions, CP rank 7, "
                                "slip 0.1, rewards N(0,0.1) + terminal goal corner, gamma 0.99")
                   if args.workload != "paper2d_1000" else
                   (f"gridworld_1000x1000 (Table 1, 2-D): {S} states, {A} actions, CP rank 3, "
                    "slip 0.2, 22 terminals (+-100), 800 obstacles, step reward -3, "
                    "gamma 0.9"),
                   "method": f"{args.method} {args.precision} sweeps + FP64 certificate",
                   "eps": eps, "sweeps_per_solve": tot_sweeps / args.steps},
        "time_to_eps_s": ms_per_step / 1e3,
        "plain_vi_time_to_eps_s": plain_s,
        "plain_vi_sweeps": plain_sweeps,
        "speedup_vs_plain_vi": plain_s / (ms_per_step / 1e3),
        "roofline": roof,
    }
    if args.workload == "paper2d_1000":
        # context, not a target: the paper's own figure for this problem shape
        out["paper_context"] = {
            "cp_mdp_vi_runtime_s": 2140.34, "memory_gb": 1.45,
            "workload": "1,000,000 states, 2-D, 4 actions (Sec. 4, Table 1)",
            "hardware": "Intel Xeon @ 2.30 GHz, 13 GB RAM, Google Colab, Python 3",
            "note": "the paper's stopping rule (maxIter 1000, the toolbox's epsilon) differs "
                    "from the eps = 1e-6 certificate here"}
    model.close()
    return out, inst


def bench_lists(args):
    """The 1000 x 1000 Table 1 GridWorld given as Def. 3 successor lists
    (cpmdp_create_lists): the same problem as paper2d_1000 without its
    Kronecker structure."""
    import torch

    from paper_2103_00331_amd import binding as B
    from paper_2103_00331_amd import instances as I

    _log("building the 1000 x 1000 GridWorld as successor lists")
    mdp = I.paper_gridworld_lists(I.named("paper2d_1000"))
    S, A = mdp.n_states, mdp.n_actions
    nnz = int(mdp.row_ptr[-1])
    model = B.Model(mdp)
    eps = 1e-6
    V = torch.zeros(S, dtype=torch.float64, device="cuda")
    pi = torch.zeros(S, dtype=torch.int32, device="cuda")
    prec = {"fp32": B.CPMDP_FP32, "fp64": B.CPMDP_FP64}[args.precision]

    def vi(p):
        V.zero_()
        code, sweeps, res = B.cpmdp_value_iteration(model.h, V, pi, eps, 100000, p)
        assert code == B.CPMDP_OK and res <= eps, (code, res)
        return sweeps

    times = {}
    for key, p in (("chosen", prec), ("plain", B.CPMDP_FP64)):
        for _ in range(max(1, args.warmup)):
            vi(p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sw = 0
        for _ in range(args.steps):
            sw += vi(p)
        torch.cuda.synchronize()
        times[key] = ((time.perf_counter() - t0) / args.steps, sw / args.steps)
    _log(f"chosen: {times['chosen'][0] * 1e3:.2f} ms ({times['chosen'][1]:.0f} sweeps); "
         f"plain FP64 VI {times['plain'][0] * 1e3:.2f} ms")
    Va = torch.zeros(S, dtype=torch.float32, device="cuda")
    Vb = torch.zeros_like(Va)
    ms = B.cpmdp_time_sweeps(model.h, Va, Vb, 200, B.CPMDP_FP32, 0)
    # V, R, V' words + terminal bit + one (successor, probability) pair of
    # 4 + 4 bytes per list entry
    algo_bytes = S * 12.0 + S / 8.0 + nnz * 8.0
    achieved = algo_bytes / (ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": _traffic("lists_fp32_paper2d_1000.md", LISTS_SRC),
            "kernel": "lists_kernel<float, MODE_MAX>", "kernel_ms": ms,
            "algorithmic_bytes_per_launch": algo_bytes, "list_entries": nnz}
    ref = _copy_reference(algo_bytes)
    roof.update(ref)
    roof["frac_of_stream_copy"] = achieved / ref["stream_copy_GBps"]
    chosen_s, chosen_sw = times["chosen"]
    out = {
        "metric": METRIC, "value": chosen_sw * S * A / chosen_s, "unit": "state-action backups/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": chosen_s * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == B.CPMDP_FP32 else "f64", "data": "synthetic",
        "config": {"workload": f"gridworld_1000x1000 (Table 1, 2-D) as Def. 3 successor lists: "
                               f"{S} states, {A} actions, {nnz} list entries, 22 terminals, "
                               "800 obstacles, gamma 0.9",
                   "method": f"vi {args.precision} sweeps + FP64 certificate", "eps": eps,
                   "sweeps_per_solve": chosen_sw},
        "time_to_eps_s": chosen_s, "plain_vi_time_to_eps_s": times["plain"][0],
        "plain_vi_sweeps": times["plain"][1], "speedup_vs_plain_vi": times["plain"][0] / chosen_s,
        "roofline": roof,
    }
    model.close()
    return out


def bench_dense(args):
    import numpy as np
    import torch

    from paper_2103_00331_amd import binding as B
    from paper_2103_00331_amd import instances as I

    _log("building 16^6 dense instance")
    inst = I.dense_grid(16, seed=I.SEED_DENSE6)
    S, A = inst.n_states, inst.n_actions
    model = B.Model(inst)
    prec = {"fp32": B.CPMDP_FP32, "fp64": B.CPMDP_FP64, "bf16": B.CPMDP_BF16}[args.precision]
    Va = torch.zeros(S, dtype=torch.float32 if prec else torch.float64, device="cuda")
    Vb = torch.zeros_like(Va)
    ms = B.cpmdp_time_sweeps(model.h, Va, Vb, 10, prec, 0)
    flops = 2.0 * inst.n_terms * sum(int(m) for m in inst.sizes) * S
    # HBM: every term's intermediate written by pass 1 and read by pass 2
    # (BF16 values in the BF16 unit), plus V (both passes), R and V'
    word = 8 if prec == B.CPMDP_FP64 else 4
    w_bytes = (2.0 * inst.n_terms * (2 if prec == B.CPMDP_BF16 else word) + 4.0 * word) * S
    # 16^6 split 3 + 3: FP32 and BF16 max sweeps run the register-resident units
    reg16 = prec in (B.CPMDP_BF16, B.CPMDP_FP32)
    peak = PEAK_TFLOPS[args.precision]
    eps = 1e-6
    V = torch.zeros(S, dtype=torch.float64, device="cuda")
    pi = torch.zeros(S, dtype=torch.int32, device="cuda")
    for _ in range(args.warmup):
        V.zero_()
        B.cpmdp_value_iteration(model.h, V, pi, eps, 100000, prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot = 0
    for _ in range(args.steps):
        V.zero_()
        code, sweeps, res = B.cpmdp_value_iteration(model.h, V, pi, eps, 100000, prec)
        tot += sweeps
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # plain GPU VI: FP64 sweeps from V0 = 0 on the same instance
    V.zero_()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pcode, plain_sweeps, pres = B.cpmdp_value_iteration(model.h, V, pi, eps, 100000, B.CPMDP_FP64)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t1
    _log(f"chosen {args.precision}: {1e3 * el / args.steps:.1f} ms; plain FP64 VI {1e3 * plain_s:.1f} ms")
    out = {"metric": METRIC, "value": tot * S * A / el, "unit": "state-action backups/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
           "config": {"workload": f"dense_16^6: {S} states, {A} actions, CP rank 8, dense "
                                  "16x16 Dirichlet(0.5) factors, gamma 0.95",
                      "method": f"vi {args.precision} sweeps, greedy-policy refinement, FP64 "
                                "certificate",
                      "eps": eps, "sweeps_per_solve": tot / args.steps},
           "time_to_eps_s": el / args.steps, "plain_vi_time_to_eps_s": plain_s,
           "plain_vi_sweeps": plain_sweeps, "speedup_vs_plain_vi": plain_s / (el / args.steps),
           "roofline": {"bound": "mfma", "achieved": flops / (ms * 1e-3) / 1e12,
                        "peak": peak, "unit": "TFLOP/s",
                        "frac": flops / (ms * 1e-3) / 1e12 / peak,
                        "traffic": _traffic(f"chain_{args.precision}_dense6_16.md",
                                            CHAIN16_SRC if reg16 else CHAIN_SRC),
                        "kernel": {B.CPMDP_BF16: "chain16_pass1 + chain16_pass2 (one sweep)",
                                   B.CPMDP_FP32: "chain16f_pass1 + chain16f_pass2 (one sweep)"}.get(
                                       prec, "chain_pass1_rows + chain_pass2 (one sweep)"),
                        "kernel_ms": ms, "algorithmic_flops_per_launch": flops,
                        "intermediate_bytes_per_launch": w_bytes,
                        "hbm_rate_gbs": w_bytes / (ms * 1e-3) / 1e9}}
    model.close()
    return out


def tt_sweep_cost(inst, word):
    """Algorithmic flops and HBM bytes of one Tensor-Train sweep: per action
    and dim k a bonded mode product (2 S m_k b_k b_{k+1} flops; reads
    b_{k+1} S words, writes b_k S words), then the epilogue (reads A S words
    of P_a V plus V and R, writes V'; one terminal bit per state).  In FP32
    with two trailing modes of 16 and bonds <= 4 the last two products run
    in one launch and the b_{n-1} channels between them stay on chip."""
    S, A, n = inst.n_states, inst.n_actions, inst.n_dims
    flops = 0.0
    words = 0.0
    for a in range(A):
        for k in range(n):
            bl, br = int(inst.bonds[a, k]), int(inst.bonds[a, k + 1])
            flops += 2.0 * S * int(inst.sizes[k]) * bl * br
            words += (bl + br) * S
        fused = (word == 4 and n >= 2 and int(inst.sizes[n - 1]) == 16 and
                 int(inst.sizes[n - 2]) == 16 and S % 256 == 0 and
                 int(inst.bonds[a, n - 1]) <= 4 and int(inst.bonds[a, n - 2]) <= 4)
        if fused:
            words -= 2 * int(inst.bonds[a, n - 1]) * S
    words += (A + 3) * S
    return flops, words * word + S / 8.0


def _cpu_baseline_tt(inst, budget_s=12.0):
    """FP64 Q-values of the Tensor-Train oracle (O4), one state at a time
    (each row of every P_a rebuilt from the cores), over seeded states."""
    import numpy as np

    from oracle import tt as O4
    rng = np.random.default_rng(12)
    V = rng.normal(0.0, 1.0, inst.n_states)
    done, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        O4.tt_q_at_states(inst, V, [int(rng.integers(inst.n_states))])
        done += 1
    secs = time.perf_counter() - t0
    return {"value": done * inst.n_actions / secs, "unit": "state-action backups/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{done} seeded states x {inst.n_actions} actions of the same {inst.name} "
                      f"instance: each P_a row rebuilt from the cores and dotted with V, "
                      f"{secs:.1f} s, numpy, one thread"}


def bench_tt(args):
    import torch

    from paper_2103_00331_amd import binding as B
    from paper_2103_00331_amd import instances as I

    _log("building the 16^6 Tensor-Train instance")
    inst = I.tt_grid()
    S, A = inst.n_states, inst.n_actions
    model = B.Model(inst)
    prec = {"fp32": B.CPMDP_FP32, "fp64": B.CPMDP_FP64}[args.precision]
    word = 8 if prec == B.CPMDP_FP64 else 4
    Va = torch.zeros(S, dtype=torch.float32 if prec else torch.float64, device="cuda")
    Vb = torch.zeros_like(Va)
    B.cpmdp_time_sweeps(model.h, Va, Vb, 2, prec, 0)
    ms = B.cpmdp_time_sweeps(model.h, Va, Vb, 10, prec, 0)
    del Va, Vb
    flops, nbytes = tt_sweep_cost(inst, word)
    eps = 1e-6
    V = torch.zeros(S, dtype=torch.float64, device="cuda")
    pi = torch.zeros(S, dtype=torch.int32, device="cuda")
    for _ in range(args.warmup):
        V.zero_()
        B.cpmdp_value_iteration(model.h, V, pi, eps, 100000, prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot = 0
    for _ in range(args.steps):
        V.zero_()
        code, sweeps, res = B.cpmdp_value_iteration(model.h, V, pi, eps, 100000, prec)
        tot += sweeps
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    V.zero_()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pcode, plain_sweeps, pres = B.cpmdp_value_iteration(model.h, V, pi, eps, 100000, B.CPMDP_FP64)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t1
    _log(f"chosen {args.precision}: {1e3 * el / args.steps:.1f} ms; plain FP64 VI {1e3 * plain_s:.1f} ms; "
         f"sweep {ms:.3f} ms")
    out = {"metric": METRIC, "value": tot * S * A / el, "unit": "state-action backups/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
           "config": {"workload": f"tt_16^6: {S} states, {A} actions, Tensor-Train transitions "
                                  "of bond 4, Dirichlet(0.5) coordinate rows, gamma 0.95",
                      "method": f"vi {args.precision} sweeps, FP64 tail sweeps and certificate",
                      "eps": eps, "sweeps_per_solve": tot / args.steps},
           "time_to_eps_s": el / args.steps, "plain_vi_time_to_eps_s": plain_s,
           "plain_vi_sweeps": plain_sweeps, "speedup_vs_plain_vi": plain_s / (el / args.steps),
           "roofline": {"bound": "hbm", "achieved": nbytes / (ms * 1e-3) / 1e9,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "traffic": _traffic(f"tt_{args.precision}_tt6_16.md", TT_SRC),
                        "kernel": "tt_step_vec + tt_step_mfma + tt_epilogue (one sweep)",
                        "kernel_ms": ms, "algorithmic_bytes_per_launch": nbytes,
                        "algorithmic_flops_per_launch": flops,
                        "flop_rate_tflops": flops / (ms * 1e-3) / 1e12,
                        "flop_frac": flops / (ms * 1e-3) / 1e12 / PEAK_TFLOPS[args.precision]}}
    model.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _cpu_baseline_tt(inst)
    return out


def _cpfit_problem():
    """Action 0 of the 32^4 GridWorld as COO entries (moves simulated) and a
    seeded rank-7 start."""
    from paper_2103_00331_amd import instances as I
    inst = I.grid4d(32, I.SEED_GRID4)
    rows, cols, vals = I.transition_coo(inst, 0)
    sizes = [32] * 4
    return inst, sizes, (rows, cols, vals), 7, I.cp_fit_init(sizes, 7, seed=20210008)


def bench_cpfit(args):
    """CP-ALS (rank 7) on one action's transition matrix of the 32^4
    GridWorld, entries resident in device memory; one step = one ALS
    iteration (all four modes)."""
    import numpy as np
    import torch

    from paper_2103_00331_amd import binding as B

    _log("building the 32^4 action-0 transition matrix")
    inst, sizes, coo, R, init = _cpfit_problem()
    rows = torch.as_tensor(coo[0].astype(np.int32), device="cuda")
    cols = torch.as_tensor(coo[1].astype(np.int32), device="cuda")
    vals = torch.as_tensor(coo[2], device="cuda")
    nnz = vals.numel()
    ws = torch.empty(B.cpmdp_cp_fit_workspace_bytes(sizes, nnz, R), dtype=torch.uint8, device="cuda")
    for _ in range(args.warmup):
        B.cpmdp_cp_fit(sizes, rows, cols, vals, R, init, max_iter=2, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fac, lam, errs, it, mttkrp_ms = B.cpmdp_cp_fit(sizes, rows, cols, vals, R, init,
                                                    max_iter=args.steps, workspace=ws, timing=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    nbytes = nnz * (4 + 4 + 8)
    _log(f"cp-als: {1e3 * el / it:.2f} ms per iteration, MTTKRP {mttkrp_ms * 1e3:.1f} us per mode, "
         f"error {errs[-1]:.3e}")
    out = {"metric": "CP-ALS iterations/s (rank-7 CP fit of one action's tabular transition matrix)",
           "value": it / el, "unit": "iterations/s", "n_gpus": 1, "steps": it,
           "warmup": args.warmup, "ms_per_step": 1e3 * el / it, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "fp64", "data": "synthetic",
           "config": {"workload": f"cpfit_grid4d_32: action 0 of the 32^4 GridWorld, {nnz} entries "
                                  "(s, s', P), rank 7, seeded U(0.1, 1) start",
                      "final_relative_error": float(errs[-1])},
           "roofline": {"bound": "hbm", "achieved": nbytes / (mttkrp_ms * 1e-3) / 1e9,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": nbytes / (mttkrp_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "traffic": _traffic("cpfit_mttkrp_grid4d_32.md", CPFIT_SRC),
                        "kernel": "cp_mttkrp_kernel + cp_reduce_kernel (one mode)",
                        "kernel_ms": mttkrp_ms, "algorithmic_bytes_per_launch": nbytes,
                        "lds_fp64_atomics_per_launch": nnz * R}}
    if not args.no_cpu_baseline:
        from oracle import cpfit as O5
        t1 = time.perf_counter()
        O5.als_sparse(sizes, *coo, O5.factors_from_flat(sizes, R, init), 1)
        secs = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": 1.0 / secs, "unit": "iterations/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"one CP-ALS iteration of the sparse oracle (numpy, "
                                         f"{nnz} entries) on the same problem, {secs:.1f} s"}
    return out


def bench_batch(args):
    """512 mixed GridWorlds solved together (FP32 sweeps, FP64 tail and
    certificate per instance, autotuned tiles / sweeps per graph) vs plain
    FP64 value iteration of each instance on its own."""
    import numpy as np
    import torch

    from paper_2103_00331_amd import binding as B
    from paper_2103_00331_amd import instances as I

    _log("building the 512-instance batch")
    insts = [I.batch_instance(i) for i in range(512)]
    tot_states = sum(x.n_states for x in insts)
    eps = 1e-6
    bm = B.BatchModel(insts)
    t0 = time.perf_counter()
    B.cpmdp_batch_autotune(bm.b, True, None)
    tune_s = time.perf_counter() - t0
    ts, k = B.cpmdp_batch_config(bm.b)
    # dominant kernel: the FP32 sweep over the whole batch, per launch
    sweep_ms = B.cpmdp_batch_time_sweeps(bm.b, 20)
    algo_bytes = sum(12.0 * x.n_states + x.n_states / 8.0 for x in insts)
    achieved = algo_bytes / (sweep_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": _traffic("batch_sweep_fp32_batch512.md", BATCH_SRC),
            "kernel": "batch_sweep_kernel<float, MODE_MAX> (all 512 instances)",
            "kernel_ms": sweep_ms, "algorithmic_bytes_per_launch": algo_bytes}
    # one allocation per array kind, a contiguous view per instance: V0 = 0 and
    # the policies are reset with one fill each
    sizes = [x.n_states for x in insts]
    V_all = torch.zeros(tot_states, dtype=torch.float64, device="cuda")
    pi_all = torch.zeros(tot_states, dtype=torch.int32, device="cuda")
    Vs = list(torch.split(V_all, sizes))
    pis = list(torch.split(pi_all, sizes))

    method = 1 if args.method == "pi" else 0
    last = {}

    def solve():
        V_all.zero_()
        pi_all.zero_()
        code, sweeps, res = B.cpmdp_batch_solve(bm.b, Vs, pis, eps, 100000, B.CPMDP_FP32, method)
        if code not in (B.CPMDP_OK, B.CPMDP_POLICY_UNSETTLED) or not np.all(res <= eps):
            bad = np.nonzero(~(res <= eps))[0]
            raise RuntimeError(f"batched solve: code {code}, {bad.size} instances above eps, "
                               f"e.g. {[(int(i), float(res[i]), int(sweeps[i])) for i in bad[:5]]}")
        last["res"] = res
        return sweeps

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    backups = 0
    for _ in range(args.steps):
        sw = solve()
        # evaluation sweeps touch one action per state (counted as 1 for PI)
        backups += sum(int(s) * x.n_states * (x.n_actions if method == 0 else 1)
                       for s, x in zip(sw, insts))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    bm.close()
    _log(f"batched {args.method}: {1e3 * el / args.steps:.1f} ms per batch solve (tile {ts}, k {k})")
    check = _batch_oracle_check(insts, Vs, pis, last["res"])
    _log(f"oracle check: {check}")
    # plain GPU VI: each instance alone, FP64 sweeps from V0 = 0
    plain = 0.0
    plain_sweeps = 0
    for x in insts:
        m = B.Model(x)
        V = torch.zeros(x.n_states, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        code, sw, res = B.cpmdp_value_iteration(m.h, V, None, eps, 100000, B.CPMDP_FP64)
        torch.cuda.synchronize()
        plain += time.perf_counter() - t1
        plain_sweeps += sw
        m.close()
    _log(f"plain per-instance FP64 VI: {plain * 1e3:.1f} ms total")
    return {"metric": METRIC, "value": backups / el, "unit": "state-action backups/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"batch of 512 GridWorlds, n in {{2,3,4}}, m in [8,48], "
                                   f"{tot_states} states in total, slip U[0.05,0.3], "
                                   "gamma U[0.9,0.99]", "eps": eps,
                       "method": f"batched {args.method}: FP32 sweeps, FP64 residual / "
                                 "certificate per instance",
                       "tile_states": ts, "sweeps_per_graph": k, "autotune_s": tune_s},
            "time_to_eps_s": el / args.steps, "plain_vi_time_to_eps_s": plain,
            "plain_vi_sweeps": plain_sweeps,
            "speedup_vs_plain_vi": plain / (el / args.steps), "err_vs_oracle": check,
            "roofline": roof}


def _warm_leg(train_instances=512, train_steps=500, test_instances=8):
    """Short warm-start comparison for the default line: train on solver-
    generated 64^3 instances, then batched solves of held-out instances from
    the network's value level, from V0 = 0 and from V0 = 0 + bound shift."""
    import numpy as np
    import torch

    from paper_2103_00331_amd import binding as B
    from paper_2103_00331_amd import instances as I
    from paper_2103_00331_amd.warmstart import WarmStart, training_instances

    eps = 1e-6
    w = WarmStart(m=64, batch=16384, seed=11)
    w.add_instances(training_instances(train_instances, m=64, split=0), eps=eps)
    w.train(train_steps, lr=1e-3, lr_final=1e-4)
    test = [I.warm_instance(2, i) for i in range(test_instances)]
    models = [B.Model(x) for x in test]
    bm = B.BatchModel(test)
    B.cpmdp_batch_autotune(bm.b, True, None)
    Vs = [torch.empty(x.n_states, dtype=torch.float64, device="cuda") for x in test]
    # inputs resident in HBM before the clock starts, as for the solves
    Rs = [torch.as_tensor(x.rewards, dtype=torch.float32, device="cuda") for x in test]
    legs = {}
    for kind in ("warm", "cold", "cold+shift"):
        for _ in range(2):                      # the second run is timed
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if kind == "warm":
                w.predict_levels(test, Rs=Rs, outs=Vs, bf16=True)
            for x, V, m, R in zip(test, Vs, models, Rs):
                if kind != "warm":
                    V.zero_()
                    if kind == "cold+shift":
                        B.cpmdp_bound_shift(m.h, V)
            code, sw, res = B.cpmdp_batch_solve(bm.b, Vs, None, eps, 100000, B.CPMDP_FP32, 0)
            torch.cuda.synchronize()
            assert code == B.CPMDP_OK and np.all(res <= eps)
            legs[kind] = (time.perf_counter() - t1,
                          int(np.sum(sw)) + (len(test) if kind == "cold+shift" else 0))
    bm.close()
    for m in models:
        m.close()
    return {"workload": f"64^3 GridWorlds, {train_instances} training instances, {train_steps} "
                        f"Adam steps of 16384 samples, {test_instances} held-out instances, "
                        "batched FP32/FP64 solves to eps = 1e-6",
            "time_to_eps_s": {k: v[0] for k, v in legs.items()},
            "sweeps": {k: v[1] for k, v in legs.items()}}


def bench_warm(args):
    """64^3 GridWorlds: train the warm-start network on solver-generated
    instances, then on held-out instances compare, with the same solvers:
    plain FP64 VI from V0 = 0 per instance; the chosen form (the network's
    value level as V0, BF16 inference, one batched FP32/FP64 solve); and two
    controls without the network, the same batched solve from V0 = 0 and
    from V0 = 0 moved by one backup and the McQueen bound shift."""
    import numpy as np
    import torch

    from paper_2103_00331_amd import binding as B
    from paper_2103_00331_amd import instances as I
    from paper_2103_00331_amd.warmstart import WarmStart, training_instances

    eps = 1e-6
    t0 = time.perf_counter()
    w = WarmStart(m=64, batch=args.train_batch, seed=11)
    train = training_instances(args.train_instances, m=64, split=0)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    w.add_instances(train, eps=eps)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    del train
    t0 = time.perf_counter()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()          # the library runs on the current stream (see binding)
    losses = w.train(args.train_steps, lr=1e-3, lr_final=1e-4, log_every=max(1, args.train_steps // 5))
    e1.record()
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    step_ms = e0.elapsed_time(e1) / max(args.train_steps, 1)
    # forward 2 (130*256 + 256*256 + 256) flop per sample, backward the weight
    # gradients (as many) and the input gradients of the two upper layers
    step_flops = args.train_batch * (2 * 2 * (130 * 256 + 256 * 256 + 256) + 2 * (256 * 256 + 256))
    _log(f"training: {args.train_instances} instances generated {t_gen:.1f}s solved {t_solve:.1f}s, "
         f"{args.train_steps} steps {t_train:.1f}s, losses {losses}")
    test = [I.warm_instance(2, i) for i in range(args.test_instances)]
    models = [B.Model(x) for x in test]
    # per instance, FP64 value iteration: plain (V0 = 0), cold + shift, network level
    per = {"plain": [0.0, []], "shift": [0.0, []], "warm": [0.0, []]}
    for x, m in zip(test, models):
        R = torch.as_tensor(x.rewards, dtype=torch.float32, device="cuda")
        for kind in per:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            V = w.predict(x, R=R) if kind == "warm" else \
                torch.zeros(x.n_states, dtype=torch.float64, device="cuda")
            if kind == "shift":
                B.cpmdp_bound_shift(m.h, V)
            code, sw, res = B.cpmdp_value_iteration(m.h, V, None, eps, 100000, B.CPMDP_FP64)
            torch.cuda.synchronize()
            assert code == B.CPMDP_OK
            per[kind][0] += time.perf_counter() - t1
            per[kind][1].append(int(sw) + (1 if kind == "shift" else 0))
    # batched mixed-precision solves of all held-out instances from three starts
    bm = B.BatchModel(test)
    B.cpmdp_batch_autotune(bm.b, True, None)
    Vs = [torch.empty(x.n_states, dtype=torch.float64, device="cuda") for x in test]
    Rs = [torch.as_tensor(x.rewards, dtype=torch.float32, device="cuda") for x in test]
    legs = {}
    for kind in ("chosen", "cold", "cold+shift"):
        for step in range(args.warmup + 1):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if kind == "chosen":
                w.predict_levels(test, Rs=Rs, outs=Vs, bf16=True)
            for x, V, m, R in zip(test, Vs, models, Rs):
                if kind != "chosen":
                    V.zero_()
                    if kind == "cold+shift":
                        B.cpmdp_bound_shift(m.h, V)
            code, sw, res = B.cpmdp_batch_solve(bm.b, Vs, None, eps, 100000, B.CPMDP_FP32, 0)
            torch.cuda.synchronize()
            assert code == B.CPMDP_OK and np.all(res <= eps)
            legs[kind] = (time.perf_counter() - t1,
                          [int(v) + (1 if kind == "cold+shift" else 0) for v in sw])
    bm.close()
    for m in models:
        m.close()
    chosen_s, chosen_sw = legs["chosen"]
    plain_s = per["plain"][0]
    S, A = test[0].n_states, test[0].n_actions
    _log(f"held-out sweeps (FP64 per instance): plain {sum(per['plain'][1])}, cold+shift "
         f"{sum(per['shift'][1])}, network level {sum(per['warm'][1])}; batched: "
         + ", ".join(f"{k} {sum(v[1])} sweeps {1e3 * v[0]:.1f} ms" for k, v in legs.items()))
    return {"metric": METRIC, "value": float(np.sum(chosen_sw)) * S * A / chosen_s,
            "unit": "state-action backups/s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
            "ms_per_step": chosen_s * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"warm start on 64^3 GridWorlds ({S} states, {A} actions): "
                                   f"{args.train_instances} training instances (the 20,000 of "
                                   f"the workload's description scaled to the run), "
                                   f"{args.train_steps} Adam steps of {args.train_batch} samples, "
                                   f"{len(test)} held-out instances",
                       "eps": eps, "train_loss": losses[-1][1],
                       "train_seconds": {"generate": t_gen, "solve": t_solve, "train": t_train}},
            "time_to_eps_s": chosen_s, "plain_vi_time_to_eps_s": plain_s,
            "speedup_vs_plain_vi": plain_s / chosen_s,
            "network_gain": {
                "batched_time_s": {k: v[0] for k, v in legs.items()},
                "batched_sweeps": {k: sum(v[1]) for k, v in legs.items()},
                "speedup_vs_batched_cold_shift": legs["cold+shift"][0] / chosen_s,
                "fp64_sweeps": {"plain": sum(per["plain"][1]), "cold+shift": sum(per["shift"][1]),
                                "network_level": sum(per["warm"][1])},
                "fp64_time_s": {k: v[0] for k, v in per.items()}},
            "sweeps_plain": per["plain"][1], "sweeps_chosen": chosen_sw,
            "roofline": {"bound": "alu", "achieved": step_flops / (step_ms * 1e-3) / 1e12,
                         "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": step_flops / (step_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
                         "traffic": None,
                         "kernel": "one MLP train step (feature gather, 3 forward and 8 backward "
                                   f"products, loss, Adam) on {args.train_batch} sampled states, events around "
                                   "all training steps on the library's stream",
                         "kernel_ms": step_ms, "algorithmic_flops_per_launch": step_flops}}


def kernel_only(args):
    """Short run for hardware-counter passes: n sweeps of the dominant kernel
    on the workload, then one plain device copy of a known size (1 GiB) whose
    counter readings calibrate the byte counters."""
    import torch

    from paper_2103_00331_amd import binding as B
    from paper_2103_00331_amd import instances as I

    if args.workload == "cpfit_grid4d_32":
        import numpy as np
        _, sizes, coo, R, init = _cpfit_problem()
        rows = torch.as_tensor(coo[0].astype(np.int32), device="cuda")
        cols = torch.as_tensor(coo[1].astype(np.int32), device="cuda")
        vals = torch.as_tensor(coo[2], device="cuda")
        out = B.cpmdp_cp_fit(sizes, rows, cols, vals, R, init, max_iter=max(1, args.sweeps // 4),
                             timing=True)
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"kernel_only": args.workload, "iterations": out[3],
                          "kernel_ms": out[4], "copy_bytes": src.numel() * 4}), flush=True)
        return
    if args.workload == "batch512":
        insts = [I.batch_instance(i) for i in range(512)]
        bm = B.BatchModel(insts)
        B.cpmdp_batch_autotune(bm.b, True, None)
        ms = B.cpmdp_batch_time_sweeps(bm.b, args.sweeps)
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"kernel_only": args.workload, "sweeps": args.sweeps, "kernel_ms": ms,
                          "tile_states": B.cpmdp_batch_config(bm.b)[0],
                          "copy_bytes": src.numel() * 4}), flush=True)
        bm.close()
        return
    if args.workload == "dense6_16":
        inst = I.dense_grid(16, seed=I.SEED_DENSE6)
    elif args.workload == "tt6_16":
        inst = I.tt_grid()
    elif args.workload == "paper2d_1000":
        inst = I.named("paper2d_1000")
    elif args.workload == "paper2d_lists":
        inst = I.paper_gridworld_lists(I.named("paper2d_1000"))
    else:
        m = 32 if args.workload == "grid4d_32" else 96
        inst = I.grid4d(m, I.SEED_GRID4 if m == 32 else I.SEED_GRID4_LARGE)
    model = B.Model(inst)
    if args.one_pass and model.path == B.CPMDP_PATH_STENCIL:
        B.cpmdp_set_option(model.h, B.CPMDP_OPT_MARCH, 0)
    prec = {"fp32": B.CPMDP_FP32, "fp64": B.CPMDP_FP64, "bf16": B.CPMDP_BF16}[args.precision]
    dt = torch.float64 if prec == B.CPMDP_FP64 else torch.float32
    Va = torch.zeros(inst.n_states, dtype=dt, device="cuda")
    Vb = torch.zeros_like(Va)
    ms = B.cpmdp_time_sweeps(model.h, Va, Vb, args.sweeps, prec, 0)
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
    dst = torch.empty_like(src)
    torch.mul(src, 2.0, out=dst)       # plain elementwise copy: reads 1 GiB, writes 1 GiB
    torch.cuda.synchronize()
    print(json.dumps({"kernel_only": args.workload, "sweeps": args.sweeps, "kernel_ms": ms,
                      "copy_bytes": src.numel() * 4}), flush=True)
    model.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch512",
                    choices=["grid4d_32", "grid4d_96", "dense6_16", "batch512", "warm64",
                             "paper2d_1000", "paper2d_lists", "tt6_16", "cpfit_grid4d_32"])
    ap.add_argument("--method", default="vi", choices=["vi", "pi"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-warm-leg", action="store_true",
                    help="batch512: skip the short warm-start comparison")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only the dominant kernel and a 1 GiB copy (counter passes)")
    ap.add_argument("--sweeps", type=int, default=20)
    ap.add_argument("--one-pass", action="store_true",
                    help="shift/identity grids: force the one-pass stencil form (no marching)")
    ap.add_argument("--train-instances", type=int, default=2048)
    ap.add_argument("--train-steps", type=int, default=1000)
    ap.add_argument("--train-batch", type=int, default=16384)
    ap.add_argument("--test-instances", type=int, default=16)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE "
              f"{world}); this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    cpu_base = None
    if args.workload == "batch512" and not args.kernel_only and not args.no_cpu_baseline:
        cpu_base = _cpu_baseline_batch()        # forks workers: before the GPU is touched
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.kernel_only:
        kernel_only(args)
        return
    if args.workload == "dense6_16":
        out = bench_dense(args)
    elif args.workload == "batch512":
        out = bench_batch(args)
        if cpu_base is not None:
            out["cpu_baseline"] = cpu_base
        if not args.no_warm_leg:
            _log("warm-start leg")
            out["warm_start_64"] = _warm_leg()
    elif args.workload == "warm64":
        out = bench_warm(args)
    elif args.workload == "paper2d_lists":
        out = bench_lists(args)
    elif args.workload == "tt6_16":
        out = bench_tt(args)
    elif args.workload == "cpfit_grid4d_32":
        out = bench_cpfit(args)
    else:
        out, inst = bench_grid(args, 32 if args.workload == "grid4d_32" else 96)
        if args.workload in ("grid4d_32", "paper2d_1000") and not args.no_cpu_baseline:
            out["cpu_baseline"] = _cpu_baseline_grid(inst)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
