"""One-patch method-of-lines driver over the C ABI.

A ``PatchRun`` owns the device buffers of one patch and issues, per RK4 stage,
the sequence (ghost fill) -> con2prim -> rhs -> rk_stage, all stream-ordered on
one HIP stream with no host synchronisation inside a step.
"""
import torch

from . import inputs as I
from . import mhd


class PatchRun:
    def __init__(self, ipatch, U0, eos_cfg, par_cfg, periodic=False, device="cuda", stream=None):
        self.ip = ipatch
        self.patch = mhd.patch_of(ipatch)
        self.eos = mhd.make_eos(eos_cfg)
        self.par = mhd.make_params(par_cfg)
        self.periodic = periodic
        self.dev = device
        self.stream = stream
        t = lambda a: torch.as_tensor(a, dtype=torch.float64).to(device).contiguous()
        self.Un = t(U0)
        self.Us = self.Un.clone()
        self.k = torch.zeros_like(self.Un)
        self.acc = torch.zeros_like(self.Un)
        self.P = torch.zeros((I.NP,) + tuple(ipatch.shape), dtype=torch.float64, device=device)
        self.flags = torch.zeros(tuple(ipatch.shape), dtype=torch.uint8, device=device)
        self.ws = mhd.workspace_for(self.patch, device)
        self.vmax = torch.zeros(1, dtype=torch.float64, device=device)
        self.stats = torch.zeros(mhd.MHD_NSTAT, dtype=torch.int64, device=device)

    def rhs_eval(self, U):
        """con2prim on the padded patch, then L(U) into self.k."""
        if self.periodic:
            mhd.fill_ghosts_periodic(self.patch, U, I.NU, self.stream)
        mhd.con2prim(self.patch, self.eos, U, self.P, self.flags, None, self.stats, self.stream)
        mhd.rhs(self.patch, self.par, self.eos, U, self.P, self.k, self.vmax, self.ws, self.stream)

    def step(self, dt):
        """One RK4 step (Table I).  Stage 0 evaluates L at Un itself (so
        con2prim corrections of Un persist); stages 1-3 at the stage state Us,
        whose ghost values are refilled (periodic) or kept frozen."""
        for s in range(4):
            self.rhs_eval(self.Un if s == 0 else self.Us)
            nxt = self.Us if s < 3 else self.Un
            mhd.rk_stage(self.patch, I.NU, s, dt, self.Un, self.k, self.acc, nxt, self.stream)
        if self.periodic:
            mhd.fill_ghosts_periodic(self.patch, self.Un, I.NU, self.stream)
