"""Learned warm start for value iteration on 3-D GridWorlds.

Orchestration only: every step runs in the library's kernels (batched
solver for the training targets, feature gather / forward / backward / Adam
for training, forward for prediction).  Training instances come from the
seeded generator (split 0 = train, 1 = validation, 2 = test); their solved
values V* stay on the device.  The trained network gives per-state values
MLP / (1 - gamma).  By default the warm start is their mean, the instance's
predicted value level, in every state: on these GridWorlds the error that
value iteration removes slowest from V0 = 0 is almost all a constant offset
(rewards are i.i.d. per state, so V* sits near one level set by the best
reward pairs anywhere in the grid), while the per-state part of a
prediction from a 5x5x5 reward window is noise that decays only at rate
gamma.  Value iteration from V0 keeps its FP64 certificate, and plain value
iteration from V0 = 0 remains the fallback.
"""
from __future__ import annotations

import numpy as np

from . import binding as B
from . import instances as I


class WarmStart:
    def __init__(self, m: int = 64, batch: int = 4096, seed: int = 1, device: str = "cuda"):
        import torch
        self.torch = torch
        self.m, self.batch, self.seed, self.device = m, batch, seed, device
        n = B.cpmdp_mlp_param_count()
        self.params = torch.empty(n, dtype=torch.float32, device=device)
        self.adam_m = torch.zeros(n, dtype=torch.float32, device=device)
        self.adam_v = torch.zeros(n, dtype=torch.float32, device=device)
        self.grad = torch.zeros(n, dtype=torch.float32, device=device)
        B.cpmdp_mlp_init(self.params, seed)
        self.ws = torch.empty(B.cpmdp_mlp_workspace_bytes(batch), dtype=torch.uint8, device=device)
        self.infer_ws, self.infer_chunk = None, 0     # inference workspace, sized on first use
        self.step = 0
        self.R, self.Vstar, self.gammas, self.slips = [], [], [], []
        self.solve_sweeps = []

    # ------------------------------------------------------------ data
    def _check(self, inst):
        """The kernels index R, V* and V0 up to m^3 - 1: refuse any instance
        that is not an m x m x m grid before a pointer reaches them."""
        m = self.m
        if list(inst.sizes) != [m, m, m] or inst.n_states != m ** 3 or \
                np.asarray(inst.rewards).size != m ** 3:
            raise ValueError(f"warm start for {m}^3 grids got an instance of sizes "
                             f"{list(inst.sizes)} with {np.asarray(inst.rewards).size} rewards")

    def add_instances(self, insts, eps: float = 1e-6, chunk: int = 256):
        """Solve the instances with the batched solver (FP32 sweeps, FP64
        certificate) and keep (R, V*) on the device as training data."""
        torch = self.torch
        for x in insts:
            self._check(x)
        for c0 in range(0, len(insts), chunk):
            part = insts[c0:c0 + chunk]
            bm = B.BatchModel(part)
            Vs = [torch.zeros(x.n_states, dtype=torch.float64, device=self.device) for x in part]
            code, sweeps, res = B.cpmdp_batch_solve(bm.b, Vs, None, eps, 100000, B.CPMDP_FP32, 0)
            bm.close()
            if code != B.CPMDP_OK:
                raise RuntimeError(f"training instances did not converge (code {code})")
            for x, V, sw in zip(part, Vs, sweeps):
                self.R.append(torch.as_tensor(x.rewards, dtype=torch.float32, device=self.device))
                self.Vstar.append(V)
                self.gammas.append(x.gamma)
                self.slips.append(x.meta["slip"])
                self.solve_sweeps.append(int(sw))
        self._tables()

    def _tables(self):
        torch = self.torch
        self.R_ptrs = torch.tensor([r.data_ptr() for r in self.R], dtype=torch.int64, device=self.device)
        self.V_ptrs = torch.tensor([v.data_ptr() for v in self.Vstar], dtype=torch.int64, device=self.device)
        self.g_dev = torch.tensor(self.gammas, dtype=torch.float64, device=self.device)
        self.s_dev = torch.tensor(self.slips, dtype=torch.float64, device=self.device)

    # ------------------------------------------------------------ training
    def train(self, steps: int, lr: float = 1e-3, lr_final: float = 1e-4, log_every: int = 0):
        losses = []
        for k in range(steps):
            self.step += 1
            frac = k / max(steps - 1, 1)
            lr_k = lr * (lr_final / lr) ** frac          # geometric decay
            want = bool(log_every) and (k % log_every == 0 or k == steps - 1)
            loss = B.cpmdp_mlp_train_step(self.params, self.adam_m, self.adam_v, self.grad,
                                          self.step, self.R_ptrs, self.V_ptrs, self.g_dev,
                                          self.s_dev, len(self.R), self.m, self.batch,
                                          self.seed, lr_k, self.ws, want_loss=want)
            if want:
                losses.append((self.step, loss))
        return losses

    # ------------------------------------------------------------ inference
    def predict(self, inst, chunk: int | None = None, bf16: bool = False, level: bool = True,
                R=None, out=None):
        """V0 (FP64, device) for one m^3 instance; by default all states in
        one forward pass (up to 2^18 per pass), so that the forward products
        fill the chip.  bf16: hidden layers with BF16 operands (FP32
        accumulation).  level: every state gets the mean prediction (see the
        module docstring); False: the per-state predictions.  R: the
        instance's rewards already on the device (FP32), else uploaded here;
        out: an FP64 device buffer of m^3 values to write V0 into."""
        torch = self.torch
        self._check(inst)
        chunk = chunk or min(inst.n_states, 1 << 18)
        if R is None:
            R = torch.as_tensor(inst.rewards, dtype=torch.float32, device=self.device)
        V0 = out if out is not None else \
            torch.empty(inst.n_states, dtype=torch.float64, device=self.device)
        if chunk <= self.batch:
            ws = self.ws
        else:
            if chunk > self.infer_chunk:
                self.infer_ws = torch.empty(B.cpmdp_mlp_workspace_bytes(chunk), dtype=torch.uint8,
                                            device=self.device)
                self.infer_chunk = chunk
            ws = self.infer_ws
        B.cpmdp_mlp_predict(self.params, R, self.m, inst.gamma, inst.meta["slip"], V0, chunk, ws,
                            precision=B.CPMDP_BF16 if bf16 else B.CPMDP_FP32, level=level)
        return V0

    def predict_levels(self, insts, Rs=None, outs=None, bf16: bool = False):
        """The value levels of several m^3 instances in one library call (one
        forward pass over every instance's 4096 spread states; see
        cpmdp_mlp_predict_levels): V0 (FP64, device) per instance, written
        into `outs` when given.  Rs: the instances' rewards on the device
        (FP32), else uploaded here."""
        torch = self.torch
        for x in insts:
            self._check(x)
        if Rs is None:
            Rs = [torch.as_tensor(x.rewards, dtype=torch.float32, device=self.device) for x in insts]
        if outs is None:
            outs = [torch.empty(x.n_states, dtype=torch.float64, device=self.device) for x in insts]
        rows = len(insts) * min(self.m ** 3, 4096)
        if rows > self.infer_chunk:
            self.infer_ws = torch.empty(B.cpmdp_mlp_workspace_bytes(rows), dtype=torch.uint8,
                                        device=self.device)
            self.infer_chunk = rows
        B.cpmdp_mlp_predict_levels(self.params, Rs, [x.gamma for x in insts],
                                   [x.meta["slip"] for x in insts], self.m, outs, self.infer_ws,
                                   precision=B.CPMDP_BF16 if bf16 else B.CPMDP_FP32)
        return outs

    # ------------------------------------------------------------ checkpoint
    def save(self, path):
        np.savez(path, params=self.params.cpu().numpy(), adam_m=self.adam_m.cpu().numpy(),
                 adam_v=self.adam_v.cpu().numpy(), step=self.step, m=self.m)

    def load(self, path):
        d = np.load(path)
        for name in ("params", "adam_m", "adam_v"):
            getattr(self, name).copy_(self.torch.as_tensor(d[name], device=self.device))
        self.step = int(d["step"])


def training_instances(n: int, m: int = 64, split: int = 0):
    return [I.warm_instance(split, i, m=m) for i in range(n)]
