"""The variational Monte Carlo self-learning loop [Sec. 3.2] on one GPU,
driven through the C ABI: per iteration

  1. Metropolis steps of every chain (nqs_mcmc),
  2. local energies and their statistics (nqs_local_energy, nqs_energy_stats),
  3. per-sample log-derivatives (nqs_log_deriv),
  4. the SR direction by matrix-free CG (nqs_sr_solve),
  5. theta <- theta - lr * delta on the device (nqs_update_weights rebuilds
     every kernel family's packing there).

Steps 1-5 are device work only (`enqueue`), so one iteration can be captured
in a HIP graph and replayed.  The random numbers of step 1 are inputs (seeded,
drawn on the host by inputs.mcmc_randoms and staged into fixed device buffers
before the iteration), so the loop is reproducible and can be replayed
against a reference.  The chains persist from one iteration to the next.
"""
from __future__ import annotations

import numpy as np
import torch

from . import inputs
from .nqs import Context, NqsError


class VMC:
    def __init__(self, ctx: Context, spins: torch.Tensor, *, steps: int = 16, lr: float = 0.05,
                 diag_shift: float = 1e-3, cg_iters: int = 100, seed: int = 0,
                 o_dtype: str = "fp64", mode: str = "auto"):
        self.ctx = ctx
        self.spins = spins
        self.B = spins.shape[0]
        self.steps, self.lr, self.lam, self.cg_iters = steps, lr, diag_shift, cg_iters
        self.seed, self.o_dtype, self.mode = seed, o_dtype, mode
        self.it = 0
        dev = spins.device
        odt = torch.float32 if o_dtype == "fp32" else torch.float64
        self.rb = torch.zeros(steps, self.B, dtype=torch.int32, device=dev)
        self.ru = torch.zeros(steps, self.B, dtype=torch.float64, device=dev)
        self.e = torch.empty(self.B, dtype=torch.float64, device=dev)
        self.st2 = torch.empty(2, dtype=torch.float64, device=dev)
        self.O = torch.empty(self.B, ctx.P, dtype=odt, device=dev)
        self.x = torch.empty(ctx.P, dtype=torch.float64, device=dev)
        self.st4 = torch.empty(4, dtype=torch.float64, device=dev)
        self.acc = torch.zeros(self.B, dtype=torch.int32, device=dev)

    def stage(self, iteration: int | None = None):
        """Copy the random numbers of an iteration into the device buffers."""
        it = self.it if iteration is None else iteration
        rb, ru = inputs.mcmc_randoms(self.seed, it, self.steps, self.B)
        self.rb.copy_(torch.as_tensor(rb.astype(np.int32)))
        self.ru.copy_(torch.as_tensor(ru))

    def enqueue(self):
        """One iteration's device work on the current stream (capturable)."""
        ctx = self.ctx
        self.acc.zero_()
        ctx.mcmc(self.spins, self.rb, self.ru, accepted=self.acc, mode=self.mode)
        ctx.local_energy(self.spins, mode=self.mode, out=self.e)
        ctx.energy_stats(self.e, out=self.st2)
        ctx.log_deriv(self.spins, dtype=self.o_dtype, out=self.O)
        ctx.sr_solve(self.O, self.e, self.lam, self.cg_iters, out=self.x, stats=self.st4)
        ctx.update_weights(self.x, -self.lr)

    def stats(self) -> dict:
        """The iteration's energy statistics; raises NqsError when the device
        flagged an error (a non-finite local energy, say a diverged update)."""
        code = self.ctx.get_error()
        if code:
            raise NqsError(code, "VMC iteration")
        st2, st4 = self.st2.cpu().numpy(), self.st4.cpu().numpy()
        return {"energy": float(st2[0]), "variance": float(st2[1]),
                "acceptance": float(self.acc.sum().item()) / (self.B * max(self.steps, 1)),
                "sr_rel_residual": float(st4[2]), "sr_iterations": int(st4[3])}

    def step(self) -> dict:
        self.stage()
        self.enqueue()
        self.it += 1
        return self.stats()

    @property
    def weights(self) -> np.ndarray:
        return self.ctx.get_weights()
