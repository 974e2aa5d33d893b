"""Harvest, training and packing of the learned Riemann flux.

Orchestration only: every arithmetic step (the solver that produces the
training records, the network's forward and backward passes, Adam, packing,
inference) runs in the HIP library through its C ABI; this module allocates
device buffers, shuffles record indices and loops.
"""
from __future__ import annotations

import ctypes

from . import Batch, NYX_FP64, _lib, default_params, make_box
from ._lib import MLP_NPARAM, MLP_PACKED_BYTES, check, lib

RECORD = 15  # floats per harvested face


def _aligned(torch, nbytes, align=256):
    raw = torch.empty(nbytes + align, dtype=torch.uint8, device="cuda")
    off = (-raw.data_ptr()) % align
    return raw[off:off + nbytes]


def harvest(workloads, steps: int, keep_fraction: float, capacity: int, seed: int = 0,
            precision: int = NYX_FP64):
    """Run the plain step on each workload (synth.Workload) for `steps` steps
    and collect final-stage face records.  Returns a (n, 15) float32 device
    tensor."""
    import torch
    rec = torch.empty((capacity, RECORD), dtype=torch.float32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    for wi, w in enumerate(workloads):
        prm = default_params(precision=precision)
        box = make_box(w.n, 4, w.dx)
        _, one = Batch.workspace_bytes(prm, [box])
        ws = _aligned(torch, one)
        plan = Batch(prm, [box], ws)
        check("nyx_batch_set_harvest", lib().nyx_batch_set_harvest(
            plan.handle, rec.data_ptr(), cnt.data_ptr(), capacity, keep_fraction,
            (seed * 1000003 + wi) & 0xFFFFFFFFFFFFFFFF))
        gdt = torch.float64 if precision == NYX_FP64 else torch.float32
        U = torch.from_numpy(w.state).cuda()
        V = torch.empty_like(U)
        G = torch.from_numpy(w.grav).to(gdt).cuda()
        dts = torch.zeros(2, dtype=torch.float64, device="cuda")
        plan.estimate_dt(U, w.a0, 0.5, dts[0:1])
        for k in range(steps):
            a0, a1 = w.a_at(k), w.a_at(k + 1)
            plan.step(U, G, dts[k % 2:k % 2 + 1], a0, a1, V, dt_next=dts[(k + 1) % 2:(k + 1) % 2 + 1])
            plan.fill_ghosts(V)
            U, V = V, U
        torch.cuda.synchronize()
        plan.close()
        del ws, U, V, G
    n = min(int(cnt.item()), capacity)
    return rec[:n]


class LearnedFlux:
    """FP32 master parameters, Adam moments and the packed BF16 weights."""

    def __init__(self, seed: int = 0):
        import torch
        self.torch = torch
        self.params = torch.empty(MLP_NPARAM, dtype=torch.float32, device="cuda")
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.packed = _aligned(torch, MLP_PACKED_BYTES)
        self.t = 0
        check("nyx_mlp_init", lib().nyx_mlp_init(self.params.data_ptr(), seed, None))

    def loss_grad(self, records, gamma=5.0 / 3.0):
        """Loss and gradient of one batch (device tensors, not synchronised)."""
        self.grad.zero_()
        self.loss.zero_()
        n = records.shape[0]
        check("nyx_mlp_loss_grad", lib().nyx_mlp_loss_grad(
            self.params.data_ptr(), records.data_ptr(), n, gamma, 1.0 / n, self.grad.data_ptr(),
            self.loss.data_ptr(), None))
        return self.loss, self.grad

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        check("nyx_mlp_adam", lib().nyx_mlp_adam(
            self.params.data_ptr(), self.m.data_ptr(), self.v.data_ptr(), self.grad.data_ptr(),
            self.t, lr, beta1, beta2, eps, None))

    def train(self, records, epochs: int, batch: int = 16384, lr: float = 2e-3,
              lr_final: float = 1e-4, seed: int = 0, log=None):
        """Adam over shuffled mini-batches with an exponentially decaying rate;
        returns the mean loss of each epoch."""
        torch = self.torch
        n = records.shape[0]
        nb = max(n // batch, 1)
        total = epochs * nb
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        hist = []
        step = 0
        for ep in range(epochs):
            perm = torch.randperm(n, device="cuda", generator=gen)
            shuf = records[perm].contiguous()
            acc = torch.zeros(1, dtype=torch.float32, device="cuda")
            for b in range(nb):
                chunk = shuf[b * batch:(b + 1) * batch]
                self.loss_grad(chunk)
                acc += self.loss
                rate = lr * (lr_final / lr) ** (step / max(total - 1, 1))
                self.adam(lr=rate)
                step += 1
            hist.append(float(acc.item()) / nb)
            if log:
                log("epoch %d loss %.4e" % (ep, hist[-1]))
        return hist

    def pack(self):
        check("nyx_mlp_pack", lib().nyx_mlp_pack(self.params.data_ptr(), self.packed.data_ptr(),
                                                 None))
        return self.packed

    def predict(self, records, gamma=5.0 / 3.0):
        out = self.torch.empty((records.shape[0], 5), dtype=self.torch.float32, device="cuda")
        check("nyx_mlp_predict", lib().nyx_mlp_predict(
            self.packed.data_ptr(), records.data_ptr(), records.shape[0], gamma, out.data_ptr(), None))
        return out


def learned_params(flux: LearnedFlux, tol: float = 1e-3, stages: int = 7, **kw):
    """Step parameters of the FP32-mixed form with the learned flux."""
    from . import NYX_MIXED, NYX_RIEMANN_LEARNED
    p = default_params(precision=NYX_MIXED, riemann=NYX_RIEMANN_LEARNED, mlp_resid_tol=tol,
                       learned_stages_mask=stages, **kw)
    p.mlp_weights = ctypes.c_void_p(flux.packed.data_ptr())
    return p


__all__ = ["harvest", "LearnedFlux", "learned_params", "RECORD", "_lib"]
