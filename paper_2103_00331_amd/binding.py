"""ctypes binding of libcpmdp.so (the C ABI declared in include/cpmdp.h).

Argument marshalling only: every step of a backup or a solve runs in the HIP
kernels of the library.  PyTorch provides device memory (workspace, V, pi)
and the stream.  The library must have been built (``build.py``); importing
this module without it raises, so no caller can silently run elsewhere.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CPMDP_LIBRARY selects another build of the library (the sanitizer build
# for host-side checks); by default the in-tree libcpmdp.so
LIB_PATH = os.environ.get("CPMDP_LIBRARY") or os.path.join(_HERE, "libcpmdp.so")

CPMDP_OK = 0
CPMDP_NOT_CONVERGED = 1
CPMDP_POLICY_UNSETTLED = 2
CPMDP_E_ARG = -1
CPMDP_E_NOT_STOCHASTIC = -2
CPMDP_E_DEVICE = -3
CPMDP_E_WORKSPACE = -4
CPMDP_E_NONFINITE = -5
CPMDP_E_UNSUPPORTED = -6
CPMDP_E_STATE = -7

CPMDP_FP64, CPMDP_FP32, CPMDP_BF16 = 0, 1, 2
CPMDP_PATH_STENCIL, CPMDP_PATH_DENSE, CPMDP_PATH_LISTS, CPMDP_PATH_TT = 0, 1, 2, 3
PRECISIONS = {"fp64": CPMDP_FP64, "fp32": CPMDP_FP32, "bf16": CPMDP_BF16}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2103_00331_amd/build.py "
                      "(or __graft_entry__.build())")
# torch must be loaded before the library.  torch ships its own libamdhip64
# with the same soname as the system one, so loading torch first makes the
# library bind to that runtime.  Loaded the other way round, the process holds
# two HIP runtimes, and the one the library uses reports no device.
import torch  # noqa: E402,F401

lib = C.CDLL(LIB_PATH)

_p = C.c_void_p
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_dp = C.POINTER(C.c_double)
_u8p = C.POINTER(C.c_uint8)
_szp = C.POINTER(C.c_size_t)

_SIGS = {
    "cpmdp_create": (C.c_int, [C.POINTER(_p), C.c_int32, _i64p, C.c_int32, _i32p, _dp, _dp,
                                _dp, C.c_double]),
    "cpmdp_create_lists": (C.c_int, [C.POINTER(_p), C.c_int64, C.c_int32, _i64p, _i64p, _dp,
                                      _dp, C.c_double]),
    "cpmdp_create_tt": (C.c_int, [C.POINTER(_p), C.c_int32, _i64p, C.c_int32, _i32p, _dp, _dp,
                                   C.c_double]),
    "cpmdp_create_tucker": (C.c_int, [C.POINTER(_p), C.c_int32, _i64p, C.c_int32, _i32p, _dp,
                                       _dp, _dp, C.c_double]),
    "cpmdp_cp_fit_workspace_bytes": (C.c_int, [C.c_int32, _i64p, C.c_int64, C.c_int32, _szp]),
    "cpmdp_cp_fit": (C.c_int, [C.c_int32, _i64p, C.c_int64, _p, _p, _p, C.c_int32, C.c_int32,
                                C.c_double, _dp, _dp, _dp, _i32p, _dp, _p, C.c_size_t, _p]),
    "cpmdp_set_terminal": (C.c_int, [_p, _u8p]),
    "cpmdp_set_obstacles": (C.c_int, [_p, _u8p]),
    "cpmdp_get_path": (C.c_int, [_p, _i32p]),
    "cpmdp_workspace_bytes": (C.c_int, [_p, _szp]),
    "cpmdp_bind": (C.c_int, [_p, _p, C.c_size_t, _p]),
    "cpmdp_set_stream": (C.c_int, [_p, _p]),
    "cpmdp_set_option": (C.c_int, [_p, C.c_int, C.c_int64]),
    "cpmdp_backup": (C.c_int, [_p, _p, _p, _p, _dp, C.c_int]),
    "cpmdp_policy_backup": (C.c_int, [_p, _p, _p, _p, _dp, C.c_int]),
    "cpmdp_value_iteration": (C.c_int, [_p, _p, _p, C.c_double, C.c_int64, C.c_int, _i64p,
                                        _dp]),
    "cpmdp_policy_iteration": (C.c_int, [_p, _p, _p, C.c_double, C.c_int64, C.c_int, _i64p,
                                         _i64p, _dp]),
    "cpmdp_time_sweeps": (C.c_int, [_p, _p, _p, C.c_int32, C.c_int, C.c_int, _p, _dp]),
    "cpmdp_bound_shift": (C.c_int, [_p, _p, _dp, _dp]),
    "cpmdp_destroy": (None, [_p]),
    "cpmdp_last_error": (C.c_char_p, [_p]),
    "cpmdp_batch_create": (C.c_int, [C.POINTER(_p), C.POINTER(_p), C.c_int32]),
    "cpmdp_batch_workspace_bytes": (C.c_int, [_p, _szp]),
    "cpmdp_batch_bind": (C.c_int, [_p, _p, C.c_size_t, _p]),
    "cpmdp_batch_solve": (C.c_int, [_p, C.POINTER(_p), C.POINTER(_p), C.c_double, C.c_int64,
                                    C.c_int, C.c_int, _i64p, _dp]),
    "cpmdp_batch_autotune": (C.c_int, [_p, C.c_int, C.c_char_p]),
    "cpmdp_batch_config": (C.c_int, [_p, _i32p, _i32p]),
    "cpmdp_batch_schedule": (C.c_int, [_p, _i32p, _i32p, _i32p]),
    "cpmdp_batch_set_schedule": (C.c_int, [_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "cpmdp_batch_time_sweeps": (C.c_int, [_p, C.c_int32, _dp]),
    "cpmdp_batch_destroy": (None, [_p]),
    "cpmdp_mlp_param_count": (C.c_int, [_i64p]),
    "cpmdp_mlp_workspace_bytes": (C.c_int, [C.c_int32, _szp]),
    "cpmdp_mlp_init": (C.c_int, [_p, C.c_uint64, _p]),
    "cpmdp_mlp_features": (C.c_int, [_p, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                     C.c_int32, _p, _p]),
    "cpmdp_mlp_forward": (C.c_int, [_p, _p, C.c_int32, _p, C.c_int32, _p, C.c_size_t, _p]),
    "cpmdp_mlp_loss_grad": (C.c_int, [_p, _p, _p, C.c_int32, _p, _dp, _p, C.c_size_t, _p]),
    "cpmdp_mlp_adam": (C.c_int, [_p, _p, _p, _p, C.c_int64, C.c_double, _p]),
    "cpmdp_mlp_train_step": (C.c_int, [_p, _p, _p, _p, C.c_int64, _p, _p, _p, _p, C.c_int32,
                                       C.c_int32, C.c_int32, C.c_uint64, C.c_double, _p,
                                       C.c_size_t, _p, _dp]),
    "cpmdp_mlp_predict": (C.c_int, [_p, _p, C.c_int32, C.c_double, C.c_double, _p, C.c_int32,
                                    C.c_int32, C.c_int32, _p, C.c_size_t, _p]),
    "cpmdp_mlp_predict_noalloc": (C.c_int, [_p, _p, C.c_int32, C.c_double, C.c_double, _p,
                                            C.c_int32, C.c_int32, C.c_int32, _p]),
    "cpmdp_mlp_predict_levels": (C.c_int, [_p, _p, _p, _p, C.c_int32, C.c_int32, _p, C.c_int32,
                                           _p, C.c_size_t, _p]),
}

EXPORTED = sorted(_SIGS)
for _name, (_res, _args) in _SIGS.items():
    fn = getattr(lib, _name)
    fn.restype = _res
    fn.argtypes = _args


class CpmdpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cpmdp error {code}: {msg}")
        self.code = code


def _check(code, handle=None):
    if code < 0:
        msg = lib.cpmdp_last_error(handle)
        raise CpmdpError(code, msg.decode() if msg else "")
    return code


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_ptr(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


# ----------------------------------------------------- C-named thin wrappers

def cpmdp_create(sizes: Sequence[int], ranks: Sequence[int], factors, lambdas, rewards,
                 gamma: float):
    sizes = np.ascontiguousarray(sizes, np.int64)
    ranks = np.ascontiguousarray(ranks, np.int32)
    factors = np.ascontiguousarray(factors, np.float64)
    lambdas = np.ascontiguousarray(lambdas, np.float64)
    rewards = np.ascontiguousarray(rewards, np.float64)
    h = _p()
    _check(lib.cpmdp_create(C.byref(h), int(sizes.size), sizes.ctypes.data_as(_i64p),
                            int(ranks.size), ranks.ctypes.data_as(_i32p),
                            factors.ctypes.data_as(_dp), lambdas.ctypes.data_as(_dp),
                            rewards.ctypes.data_as(_dp), float(gamma)))
    return h


def cpmdp_create_lists(n_states: int, n_actions: int, row_ptr, succ, prob, rewards,
                       gamma: float):
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    succ = np.ascontiguousarray(succ, np.int64)
    prob = np.ascontiguousarray(prob, np.float64)
    rewards = np.ascontiguousarray(rewards, np.float64)
    h = _p()
    _check(lib.cpmdp_create_lists(C.byref(h), int(n_states), int(n_actions),
                                  row_ptr.ctypes.data_as(_i64p), succ.ctypes.data_as(_i64p),
                                  prob.ctypes.data_as(_dp), rewards.ctypes.data_as(_dp),
                                  float(gamma)))
    return h


def cpmdp_create_tt(sizes: Sequence[int], bonds, cores, rewards, gamma: float):
    sizes = np.ascontiguousarray(sizes, np.int64)
    bonds = np.ascontiguousarray(bonds, np.int32)
    cores = np.ascontiguousarray(cores, np.float64)
    rewards = np.ascontiguousarray(rewards, np.float64)
    h = _p()
    _check(lib.cpmdp_create_tt(C.byref(h), int(sizes.size), sizes.ctypes.data_as(_i64p),
                               int(bonds.shape[0]), bonds.ctypes.data_as(_i32p),
                               cores.ctypes.data_as(_dp), rewards.ctypes.data_as(_dp),
                               float(gamma)))
    return h


def cpmdp_create_tucker(sizes: Sequence[int], core_ranks, cores, factors, rewards,
                        gamma: float):
    sizes = np.ascontiguousarray(sizes, np.int64)
    core_ranks = np.ascontiguousarray(core_ranks, np.int32)
    cores = np.ascontiguousarray(cores, np.float64)
    factors = np.ascontiguousarray(factors, np.float64)
    rewards = np.ascontiguousarray(rewards, np.float64)
    h = _p()
    _check(lib.cpmdp_create_tucker(C.byref(h), int(sizes.size), sizes.ctypes.data_as(_i64p),
                                   int(core_ranks.shape[0]), core_ranks.ctypes.data_as(_i32p),
                                   cores.ctypes.data_as(_dp), factors.ctypes.data_as(_dp),
                                   rewards.ctypes.data_as(_dp), float(gamma)))
    return h


def cpmdp_cp_fit_workspace_bytes(sizes, nnz, rank) -> int:
    sizes = np.ascontiguousarray(sizes, np.int64)
    out = C.c_size_t()
    _check(lib.cpmdp_cp_fit_workspace_bytes(int(sizes.size), sizes.ctypes.data_as(_i64p),
                                            int(nnz), int(rank), C.byref(out)))
    return out.value


def cpmdp_cp_fit(sizes, rows, cols, vals, rank, factors0, max_iter=50, tol=0.0, workspace=None,
                 stream=None, timing=False):
    """rows, cols (int32) and vals (FP64) are device tensors; factors0 a host
    array in the term layout.  Returns (factors, lambdas, errors, iters[,
    mttkrp_ms])."""
    import torch
    sizes = np.ascontiguousarray(sizes, np.int64)
    nnz = int(vals.numel())
    if workspace is None:
        nbytes = cpmdp_cp_fit_workspace_bytes(sizes, nnz, rank)
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=vals.device)
    fac = np.array(factors0, np.float64, copy=True)
    lam = np.zeros(int(rank))
    errs = np.zeros(int(max_iter))
    it = C.c_int32(0)
    ms = C.c_double(0.0)
    _check(lib.cpmdp_cp_fit(int(sizes.size), sizes.ctypes.data_as(_i64p), nnz, _ptr(rows),
                            _ptr(cols), _ptr(vals), int(rank), int(max_iter), float(tol),
                            fac.ctypes.data_as(_dp), lam.ctypes.data_as(_dp),
                            errs.ctypes.data_as(_dp), C.byref(it),
                            C.byref(ms) if timing else None, workspace.data_ptr(),
                            workspace.numel() * workspace.element_size(), _stream_ptr(stream)))
    out = (fac, lam, errs[:it.value], it.value)
    return out + (ms.value,) if timing else out


def cpmdp_set_terminal(h, mask):
    mask = np.ascontiguousarray(mask, np.uint8)
    return _check(lib.cpmdp_set_terminal(h, mask.ctypes.data_as(_u8p)), h)


def cpmdp_set_obstacles(h, mask):
    mask = np.ascontiguousarray(mask, np.uint8)
    return _check(lib.cpmdp_set_obstacles(h, mask.ctypes.data_as(_u8p)), h)


def cpmdp_get_path(h) -> int:
    out = C.c_int32()
    _check(lib.cpmdp_get_path(h, C.byref(out)), h)
    return out.value


def cpmdp_workspace_bytes(h) -> int:
    out = C.c_size_t()
    _check(lib.cpmdp_workspace_bytes(h, C.byref(out)), h)
    return out.value


def cpmdp_bind(h, workspace, stream=None):
    return _check(lib.cpmdp_bind(h, workspace.data_ptr(), workspace.numel() *
                                 workspace.element_size(), _stream_ptr(stream)), h)


def cpmdp_set_stream(h, stream=None):
    return _check(lib.cpmdp_set_stream(h, _stream_ptr(stream)), h)


CPMDP_OPT_MARCH = 1


def cpmdp_set_option(h, option, value):
    return _check(lib.cpmdp_set_option(h, int(option), int(value)), h)


def cpmdp_backup(h, V_in, V_out, pi_out=None, residual=False, precision=CPMDP_FP64):
    r = C.c_double(0.0)
    _check(lib.cpmdp_backup(h, _ptr(V_in), _ptr(V_out), _ptr(pi_out),
                            C.byref(r) if residual else None, int(precision)), h)
    return r.value if residual else None


def cpmdp_policy_backup(h, V_in, V_out, pi, residual=False, precision=CPMDP_FP64):
    r = C.c_double(0.0)
    _check(lib.cpmdp_policy_backup(h, _ptr(V_in), _ptr(V_out), _ptr(pi),
                                   C.byref(r) if residual else None, int(precision)), h)
    return r.value if residual else None


def cpmdp_value_iteration(h, V, pi_out=None, eps=1e-6, max_iter=100000,
                          precision=CPMDP_FP64):
    sw = C.c_int64(0)
    res = C.c_double(0.0)
    code = _check(lib.cpmdp_value_iteration(h, _ptr(V), _ptr(pi_out), float(eps),
                                            int(max_iter), int(precision), C.byref(sw),
                                            C.byref(res)), h)
    return code, sw.value, res.value


def cpmdp_policy_iteration(h, V, pi, eps=1e-6, max_iter=100000, precision=CPMDP_FP64):
    outer = C.c_int64(0)
    sw = C.c_int64(0)
    res = C.c_double(0.0)
    code = _check(lib.cpmdp_policy_iteration(h, _ptr(V), _ptr(pi), float(eps), int(max_iter),
                                             int(precision), C.byref(outer), C.byref(sw),
                                             C.byref(res)), h)
    return code, outer.value, sw.value, res.value


def cpmdp_time_sweeps(h, V_a, V_b, n, precision=CPMDP_FP32, mode=0, pi=None) -> float:
    ms = C.c_double(0.0)
    _check(lib.cpmdp_time_sweeps(h, _ptr(V_a), _ptr(V_b), int(n), int(precision), int(mode),
                                 _ptr(pi), C.byref(ms)), h)
    return ms.value


def cpmdp_bound_shift(h, V):
    lo = C.c_double(0.0)
    hi = C.c_double(0.0)
    _check(lib.cpmdp_bound_shift(h, _ptr(V), C.byref(lo), C.byref(hi)), h)
    return lo.value, hi.value


def cpmdp_destroy(h):
    lib.cpmdp_destroy(h)


def cpmdp_last_error(h=None) -> str:
    m = lib.cpmdp_last_error(h)
    return m.decode() if m else ""


def cpmdp_batch_create(handles):
    arr = (_p * len(handles))(*[h.value if isinstance(h, _p) else h for h in handles])
    b = _p()
    _check(lib.cpmdp_batch_create(C.byref(b), arr, len(handles)))
    return b


def cpmdp_batch_workspace_bytes(b) -> int:
    out = C.c_size_t()
    _check(lib.cpmdp_batch_workspace_bytes(b, C.byref(out)))
    return out.value


def cpmdp_batch_bind(b, workspace, stream=None):
    return _check(lib.cpmdp_batch_bind(b, workspace.data_ptr(), workspace.numel() *
                                       workspace.element_size(), _stream_ptr(stream)))


def cpmdp_batch_solve(b, Vs, pis=None, eps=1e-6, max_iter=100000, precision=CPMDP_FP32,
                      method=0):
    n = len(Vs)
    varr = (_p * n)(*[v.data_ptr() for v in Vs])
    parr = (_p * n)(*[p.data_ptr() for p in pis]) if pis is not None else None
    sweeps = np.zeros(n, np.int64)
    res = np.zeros(n, np.float64)
    code = _check(lib.cpmdp_batch_solve(b, varr, parr, float(eps), int(max_iter),
                                        int(precision), int(method),
                                        sweeps.ctypes.data_as(_i64p), res.ctypes.data_as(_dp)))
    return code, sweeps, res


def cpmdp_batch_time_sweeps(b, n):
    ms = C.c_double(0.0)
    _check(lib.cpmdp_batch_time_sweeps(b, int(n), C.byref(ms)))
    return ms.value


def cpmdp_batch_autotune(b, tune=True, cache_path=None):
    return _check(lib.cpmdp_batch_autotune(b, int(bool(tune)),
                                           cache_path.encode() if cache_path else None))


def cpmdp_batch_config(b):
    t = C.c_int32()
    k = C.c_int32()
    _check(lib.cpmdp_batch_config(b, C.byref(t), C.byref(k)))
    return t.value, k.value


def cpmdp_batch_set_schedule(b, tile_states, grid, march, sched):
    return _check(lib.cpmdp_batch_set_schedule(b, int(tile_states), int(grid), int(march),
                                               int(sched)))


def cpmdp_batch_schedule(b):
    g, m, sc = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib.cpmdp_batch_schedule(b, C.byref(g), C.byref(m), C.byref(sc)))
    return g.value, m.value, sc.value


def cpmdp_batch_destroy(b):
    lib.cpmdp_batch_destroy(b)


# ------------------------------------------------------------ convenience

class Model:
    """One MDP on the GPU: creates the handle from an instance (sizes,
    ranks, factors, lambdas, rewards, gamma, terminal and obstacle masks),
    allocates the workspace as a torch uint8 tensor and binds it with the
    current stream."""

    def __init__(self, inst, device="cuda", stream=None):
        import torch
        self.inst = inst
        if hasattr(inst, "row_ptr"):          # an MDP given as Def. 3 lists
            self.h = cpmdp_create_lists(inst.n_states, inst.n_actions, inst.row_ptr,
                                        inst.succ, inst.prob, inst.rewards, inst.gamma)
        elif hasattr(inst, "bonds"):          # Tensor-Train cores
            self.h = cpmdp_create_tt(inst.sizes, inst.bonds, inst.cores, inst.rewards,
                                     inst.gamma)
        elif hasattr(inst, "core_ranks"):     # Tucker core and factors
            self.h = cpmdp_create_tucker(inst.sizes, inst.core_ranks, inst.cores,
                                         inst.factors, inst.rewards, inst.gamma)
        else:
            self.h = cpmdp_create(inst.sizes, inst.ranks, inst.factors, inst.lambdas,
                                  inst.rewards, inst.gamma)
        if np.any(inst.terminal):
            cpmdp_set_terminal(self.h, inst.terminal)
        obstacle = getattr(inst, "obstacle", None)
        if obstacle is not None and np.any(obstacle):
            cpmdp_set_obstacles(self.h, obstacle)
        self.path = cpmdp_get_path(self.h)
        nbytes = cpmdp_workspace_bytes(self.h)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.workspace.data_ptr()) % 256
        self.ws_view = self.workspace[off:off + nbytes]
        cpmdp_bind(self.h, self.ws_view, stream)
        self.S = inst.n_states
        self.device = device

    def close(self):
        if self.h is not None:
            cpmdp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchModel:
    """Many instances solved together: creates one handle per instance (host
    data only), the batch, and its workspace (torch uint8 tensor)."""

    def __init__(self, insts, device="cuda", stream=None):
        import torch
        self.insts = list(insts)
        self.handles = []
        for inst in self.insts:
            h = cpmdp_create(inst.sizes, inst.ranks, inst.factors, inst.lambdas,
                             inst.rewards, inst.gamma)
            if np.any(inst.terminal):
                cpmdp_set_terminal(h, inst.terminal)
            obstacle = getattr(inst, "obstacle", None)
            if obstacle is not None and np.any(obstacle):
                cpmdp_set_obstacles(h, obstacle)
            self.handles.append(h)
        self.b = cpmdp_batch_create(self.handles)
        nbytes = cpmdp_batch_workspace_bytes(self.b)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.workspace.data_ptr()) % 256
        self.ws_view = self.workspace[off:off + nbytes]
        cpmdp_batch_bind(self.b, self.ws_view, stream)
        self.device = device

    def close(self):
        if self.b is not None:
            cpmdp_batch_destroy(self.b)
            self.b = None
        for h in self.handles:
            cpmdp_destroy(h)
        self.handles = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ warm-start MLP

def cpmdp_mlp_param_count() -> int:
    n = C.c_int64()
    _check(lib.cpmdp_mlp_param_count(C.byref(n)))
    return n.value


def cpmdp_mlp_workspace_bytes(batch) -> int:
    b = C.c_size_t()
    _check(lib.cpmdp_mlp_workspace_bytes(int(batch), C.byref(b)))
    return b.value


def cpmdp_mlp_init(params, seed, stream=None):
    return _check(lib.cpmdp_mlp_init(_ptr(params), int(seed), _stream_ptr(stream)))


def cpmdp_mlp_features(R, m, gamma, slip, s0, count, X, stream=None):
    return _check(lib.cpmdp_mlp_features(_ptr(R), int(m), float(gamma), float(slip), int(s0),
                                         int(count), _ptr(X), _stream_ptr(stream)))


def cpmdp_mlp_forward(params, X, count, y, ws, stream=None, precision=CPMDP_FP32):
    return _check(lib.cpmdp_mlp_forward(_ptr(params), _ptr(X), int(count), _ptr(y), int(precision),
                                        _ptr(ws), ws.numel() * ws.element_size(),
                                        _stream_ptr(stream)))


def cpmdp_mlp_loss_grad(params, X, t, count, grad, ws, stream=None):
    loss = C.c_double(0.0)
    _check(lib.cpmdp_mlp_loss_grad(_ptr(params), _ptr(X), _ptr(t), int(count), _ptr(grad),
                                   C.byref(loss), _ptr(ws), ws.numel() * ws.element_size(),
                                   _stream_ptr(stream)))
    return loss.value


def cpmdp_mlp_adam(params, m, v, grad, step, lr, stream=None):
    return _check(lib.cpmdp_mlp_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), int(step),
                                     float(lr), _stream_ptr(stream)))


def cpmdp_mlp_train_step(params, adam_m, adam_v, grad, step, R_ptrs, V_ptrs, gammas, slips,
                         n_inst, m, batch, seed, lr, ws, stream=None, want_loss=False):
    loss = C.c_double(0.0)
    _check(lib.cpmdp_mlp_train_step(_ptr(params), _ptr(adam_m), _ptr(adam_v), _ptr(grad),
                                    int(step), _ptr(R_ptrs), _ptr(V_ptrs), _ptr(gammas),
                                    _ptr(slips), int(n_inst), int(m), int(batch), int(seed),
                                    float(lr), _ptr(ws), ws.numel() * ws.element_size(),
                                    _stream_ptr(stream), C.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


def cpmdp_mlp_predict(params, R, m, gamma, slip, V0, chunk, ws, stream=None,
                      precision=CPMDP_FP32, level=False):
    S = int(m) ** 3
    if R.numel() != S or V0.numel() != S or R.dtype != torch.float32 or V0.dtype != torch.float64:
        raise ValueError(f"predict on an {m}^3 grid needs float32 R and float64 V0 of {S} elements")
    return _check(lib.cpmdp_mlp_predict(_ptr(params), _ptr(R), int(m), float(gamma), float(slip),
                                        _ptr(V0), int(chunk), int(precision), int(bool(level)),
                                        _ptr(ws),
                                        ws.numel() * ws.element_size(), _stream_ptr(stream)))


def cpmdp_mlp_predict_levels(params, Rs, gammas, slips, m, V0s, ws, stream=None,
                             precision=CPMDP_FP32):
    n = len(Rs)
    S = int(m) ** 3
    if len(V0s) != n or len(gammas) != n or len(slips) != n or n < 1:
        raise ValueError("predict_levels needs equal numbers (>= 1) of R, V0, gammas and slips")
    for R, V0 in zip(Rs, V0s):
        if R.numel() != S or V0.numel() != S or R.dtype != torch.float32 or V0.dtype != torch.float64:
            raise ValueError(f"predict_levels on {m}^3 grids needs float32 R and float64 V0 of {S} "
                             "elements")
    rarr = (_p * n)(*[R.data_ptr() for R in Rs])
    varr = (_p * n)(*[V.data_ptr() for V in V0s])
    garr = (C.c_double * n)(*[float(g) for g in gammas])
    sarr = (C.c_double * n)(*[float(x) for x in slips])
    return _check(lib.cpmdp_mlp_predict_levels(_ptr(params), rarr, garr, sarr, n, int(m), varr,
                                               int(precision), _ptr(ws),
                                               ws.numel() * ws.element_size(), _stream_ptr(stream)))


def cpmdp_mlp_predict_noalloc(params, R, m, gamma, slip, V0, chunk, stream=None,
                              precision=CPMDP_FP32, level=False):
    S = int(m) ** 3
    if R.numel() != S or V0.numel() != S or R.dtype != torch.float32 or V0.dtype != torch.float64:
        raise ValueError(f"predict on an {m}^3 grid needs float32 R and float64 V0 of {S} elements")
    return _check(lib.cpmdp_mlp_predict_noalloc(_ptr(params), _ptr(R), int(m), float(gamma),
                                                float(slip), _ptr(V0), int(chunk), int(precision),
                                                int(bool(level)), _stream_ptr(stream)))
