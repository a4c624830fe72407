"""One-patch method-of-lines driver over the C ABI.

A ``PatchRun`` owns the device buffers of one patch and issues, per RK4 stage,
the sequence (ghost fill) -> con2prim -> rhs -> rk_stage, all stream-ordered on
one HIP stream with no host synchronisation inside a step.
"""
import math

import torch

from . import inputs as I
from . import mhd


# names of the seven volume integrals of mhd_constraints, in order
MONITORS = ("H2", "M2", "baryon_mass", "Theta2", "Z2", "phi2", "B2")


def monitors(patch, ipatch, U, stream=None):
    """The constraint monitors of one patch (mhd_constraints): a dict of the
    seven volume integrals (H^2, M_i M_i, Dbar, Theta^2, Z_i Z^i, phi^2,
    gamma_ij B^i B^j), read back to the host."""
    C5 = torch.empty((5,) + tuple(ipatch.shape), dtype=torch.float64, device=U.device)
    sums = torch.zeros(7 * (ipatch.n[2] + 1), dtype=torch.float64, device=U.device)
    mhd.constraints(patch, U, C5, sums, stream)
    vals = sums[:7].cpu().tolist()
    return dict(zip(MONITORS, vals))


class PatchRun:
    def __init__(self, ipatch, U0, eos_cfg, par_cfg, periodic=False, device="cuda", stream=None, aux=None):
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
        self.m1 = bool(par_cfg.get("evolve_m1", 0))
        self.nd = self.m1 and bool(par_cfg.get("evolve_m1n", 0))
        self.nfields = I.NU_M1N if self.nd else (I.NU_M1 if self.m1 else I.NU)
        self.aux = None if aux is None else t(aux)
        self.ws = mhd.workspace_for(self.patch, device, m1=self.m1, m1n=self.nd)
        self.vmax = torch.zeros(1, dtype=torch.float64, device=device)
        self.stats = torch.zeros(mhd.MHD_NSTAT, dtype=torch.int64, device=device)
        self.mlp = None
        self.lws = None

    def use_learned(self, mlp):
        """con2prim with the learned guess (mlp: device parameter block), or the
        bracketed solver (None)."""
        self.mlp = mlp
        if mlp is not None and self.lws is None:
            n = mhd.con2prim_learned_workspace_size(self.patch)
            self.lws = torch.empty((n + 7) // 8, dtype=torch.float64, device=self.dev)

    def rhs_eval(self, U):
        """con2prim on the padded patch, then L(U) into self.k."""
        if self.periodic:
            mhd.fill_ghosts_periodic(self.patch, U, self.nfields, self.stream)
        if self.mlp is not None:
            mhd.con2prim_learned(self.patch, self.eos, self.mlp, U, self.P, self.lws, self.flags, None, self.stats,
                                 self.stream)
        else:
            mhd.con2prim(self.patch, self.eos, U, self.P, self.flags, None, self.stats, self.stream)
        mhd.rhs(self.patch, self.par, self.eos, U, self.P, self.k, self.vmax, self.ws, self.stream, aux=self.aux)

    def step(self, dt):
        """One RK4 step (Table I).  Stage 0 evaluates L at Un itself (so
        con2prim corrections of Un persist); stages 1-3 at the stage state Us,
        whose ghost values are refilled (periodic) or kept frozen."""
        for s in range(4):
            self.rhs_eval(self.Un if s == 0 else self.Us)
            nxt = self.Us if s < 3 else self.Un
            mhd.rk_stage(self.patch, self.nfields, s, dt, self.Un, self.k, self.acc, nxt, self.stream)
        if self.periodic:
            mhd.fill_ghosts_periodic(self.patch, self.Un, self.nfields, self.stream)


    def monitors(self):
        """Constraint monitors of the current state Un."""
        return monitors(self.patch, self.ip, self.Un, self.stream)

    def step_ssprk3(self, dt):
        """One SSP-RK(3,3) step (Sec. 3.1), stage structure as in step()."""
        for s in range(3):
            self.rhs_eval(self.Un if s == 0 else self.Us)
            nxt = self.Us if s < 2 else self.Un
            mhd.ssprk3_stage(self.patch, self.nfields, s, dt, self.Un, self.k, self.acc, nxt, self.stream)
        if self.periodic:
            mhd.fill_ghosts_periodic(self.patch, self.Un, self.nfields, self.stream)


class LevelRun:
    """Device buffers of a list of boxes and their batched level (mhd_level_*).
    Us starts as a copy of U so the stage states carry the (frozen) ghosts."""

    def __init__(self, ipatches, states, eos_cfg, par_cfg, device="cuda", flags=True, auxs=None, imex=False):
        self.eos = mhd.make_eos(eos_cfg)
        self.par = mhd.make_params(par_cfg)
        self.m1 = bool(par_cfg.get("evolve_m1", 0))
        self.nd = self.m1 and bool(par_cfg.get("evolve_m1n", 0))
        self.nfields = I.NU_M1N if self.nd else (I.NU_M1 if self.m1 else I.NU)
        self.boxes = []
        for b, (ip, U0) in enumerate(zip(ipatches, states)):
            pt = mhd.patch_of(ip)
            U = torch.as_tensor(U0, dtype=torch.float64).to(device).contiguous()
            d = dict(patch=pt, ip=ip, U=U, Us=U.clone(), k=torch.zeros_like(U), acc=torch.zeros_like(U),
                     P=torch.zeros((I.NP,) + tuple(ip.shape), dtype=torch.float64, device=device),
                     ws=mhd.workspace_for(pt, device, m1=self.m1, m1n=self.nd))
            if flags:
                d["flags"] = torch.zeros(tuple(ip.shape), dtype=torch.uint8, device=device)
            if auxs is not None and auxs[b] is not None:
                d["aux"] = torch.as_tensor(auxs[b], dtype=torch.float64).to(device).contiguous()
            if imex:
                shp = tuple(ip.shape)
                d["F"] = [torch.zeros_like(U) for _ in range(4)]
                d["R"] = [torch.zeros((self.nfields - I.NU,) + shp, dtype=torch.float64, device=device)
                          for _ in range(4)]
            self.boxes.append(d)
        self.level = mhd.Level(self.boxes, self.par, self.eos)
        if imex:
            self.level.set_imex([(b["F"], b["R"]) for b in self.boxes])

    def monitors(self):
        """Constraint monitors of every box, in box order (boxes of one level do
        not overlap, so the integrals of the level are the boxes' sums)."""
        return [monitors(b["patch"], b["ip"], b["U"]) for b in self.boxes]

    @property
    def ninterior(self):
        return sum(b["ip"].ninterior for b in self.boxes)

    @property
    def npts(self):
        return sum(b["ip"].npts for b in self.boxes)

    @property
    def nhalo1(self):
        return sum(b["ip"].nhalo1 for b in self.boxes)


# implicit diagonals: Table I's I42L, and the I32L paired with SSP-RK(3,3)
# (gamma = 1 - 1/sqrt(2), as the library's tableau evaluates it)
IMEX_AII = {mhd.IMEX_442: (0.0, 0.25, 1.0 / 3.0, 1.0 / 6.0),
            mhd.IMEX_332: (0.0, 1.0 - math.sqrt(0.5), 1.0 - math.sqrt(0.5))}


class ImexRun:
    """One patch with three M1 species stepped by IMEX(4,4,2) (Table I): the
    radiation's collision terms implicit (mhd_m1_implicit), everything else
    explicit.  Per stage: combine -> (ghost fill) -> con2prim -> implicit solve
    -> (ghost fill) -> split RHS.  With evolve_m1n in par_cfg the three number
    densities (47 fields, 15 aux) are evolved too, their collision sources
    implicit.  scheme: mhd.IMEX_442 (Table I) or mhd.IMEX_332 (SSP-RK(3,3)
    with the re-derived L-stable I32L).  With couple_exchange in par_cfg the
    fluid's share of the exchange is implicit too (its stiff slots, and the
    implicit solve moves what the radiation gains out of the fluid)."""

    def __init__(self, ipatch, U0, aux, eos_cfg, par_cfg, periodic=False, device="cuda", stream=None,
                 scheme=mhd.IMEX_442):
        self.scheme = scheme
        self.aii = IMEX_AII[scheme]
        self.ip = ipatch
        self.patch = mhd.patch_of(ipatch)
        self.eos = mhd.make_eos(eos_cfg)
        self.par = mhd.make_params(dict(par_cfg, evolve_m1=1))
        self.nd = bool(par_cfg.get("evolve_m1n", 0))
        self.nfields = I.NU_M1N if self.nd else I.NU_M1
        self.coupled = bool(par_cfg.get("couple_exchange", 0))
        self.m_b = float(par_cfg.get("m_b", 1.0))
        self.nstiff = mhd.imex_stiff_fields(self.nfields, self.coupled)
        self.periodic = periodic
        self.stream = stream
        t = lambda a: torch.as_tensor(a, dtype=torch.float64).to(device).contiguous()
        self.Un = t(U0)
        assert self.Un.shape[0] == self.nfields
        self.Ust = self.Un.clone()
        self.aux = t(aux)
        shp = tuple(ipatch.shape)
        self.F = [torch.zeros_like(self.Un) for _ in range(4)]
        self.R = [torch.zeros((self.nstiff,) + shp, dtype=torch.float64, device=device) for _ in range(4)]
        self.P = torch.zeros((I.NP,) + shp, dtype=torch.float64, device=device)
        self.flags = torch.zeros(shp, dtype=torch.uint8, device=device)
        self.ws = mhd.workspace_for(self.patch, device, m1=True, m1n=self.nd)
        self.vmax = torch.zeros(1, dtype=torch.float64, device=device)
        self.nfail = torch.zeros(1, dtype=torch.int64, device=device)

    def step(self, dt):
        s_ = self.stream
        nf = self.nfields
        ns = len(self.aii)
        for s in range(ns):
            mhd.imex_combine(self.patch, s, dt, self.Un, self.F, self.R, self.Ust, s_, nfields=nf, scheme=self.scheme,
                             coupled=self.coupled)
            if self.periodic:
                mhd.fill_ghosts_periodic(self.patch, self.Ust, nf, s_)
            mhd.con2prim(self.patch, self.eos, self.Ust, self.P, self.flags, None, None, s_)
            if self.aii[s] != 0.0:
                mhd.m1_implicit(self.patch, self.aux, self.Ust, self.P, self.aii[s] * dt, self.nfail, s_,
                                evolve_n=self.nd, coupled=self.coupled, m_b=self.m_b)
                if self.periodic:
                    mhd.fill_ghosts_periodic(self.patch, self.Ust, nf, s_)
            mhd.rhs_split(self.patch, self.par, self.eos, self.Ust, self.P, self.aux, self.F[s], self.R[s], self.vmax,
                          self.ws, s_)
        mhd.imex_combine(self.patch, ns, dt, self.Un, self.F, self.R, self.Un, s_, nfields=nf, scheme=self.scheme,
                         coupled=self.coupled)
        if self.periodic:
            mhd.fill_ghosts_periodic(self.patch, self.Un, nf, s_)
