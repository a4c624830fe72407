#!/usr/bin/env python3
"""Zone-update throughput of the MoL right-hand side on one MI355X.

Workload: one 128^3 FP64 patch (dx = 0.25, [-16,16]^3) holding the K=100,
Gamma=2, rho_c=1.28e-3 TOV star with a poloidal field (max b^2/rho = 1e-3) and
an atmosphere of rho = 1e-12; full CCZ4 + GRMHD right-hand side, con2prim on
the padded patch and the RK4 stage update.  One step = one RK4 step = four
right-hand-side evaluations; one zone update = one interior point through one
evaluation (con2prim + rhs + stage).  Inputs are synthetic and built on the
device (the prim->cons map runs in the library); the timed region starts with
everything resident in HBM.

Prints one JSON line (see the keys below); --gpus N > 1 is refused: the build
targets one GPU.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "zone-updates/s full RHS+con2prim, plain vs learned+batched, 1 MI355X, FP64"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128, help="interior points per axis")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-evals", type=int, default=4, help="oracle RHS evaluations in the CPU sample")
    ap.add_argument("--strip", type=int, default=0, help="tile-order strip height (0: library default)")
    ap.add_argument("--sweep-strip", action="store_true", help="time one RK4 step per strip height and report")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (3 times): the reference for scaling "
                         "the FETCH_SIZE / WRITE_SIZE counters to bytes")
    return ap.parse_args()


def copy_calibration():
    import torch

    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print('{"copy_calibration_bytes_read": %d, "copy_calibration_bytes_written": %d, "launches": 3}' % (n * 8, n * 8))


class CallTimer:
    """HIP events around each library call, on the stream the call is issued on."""

    def __init__(self, torch, enabled):
        self.torch = torch
        self.enabled = enabled
        self.ev = {}

    def wrap(self, name, fn, *a, **kw):
        if not self.enabled:
            return fn(*a, **kw)
        s = self.torch.cuda.Event(enable_timing=True)
        e = self.torch.cuda.Event(enable_timing=True)
        s.record()
        r = fn(*a, **kw)
        e.record()
        self.ev.setdefault(name, []).append((s, e))
        return r

    def avg_ms(self):
        return {k: sum(s.elapsed_time(e) for s, e in v) / len(v) for k, v in self.ev.items()}

    def count(self):
        return {k: len(v) for k, v in self.ev.items()}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2510_13965_amd import inputs as I
    from paper_2510_13965_amd import mhd
    from paper_2510_13965_amd.step import PatchRun

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    mhd.lib()
    ip, U, P, EM = I.c2_state(n=args.n)
    dev = "cuda"
    run = PatchRun(ip, U, I.EOS_IDEAL2, I.PARAMS, periodic=False, device=dev)
    # prim -> cons on the device
    Pd = torch.as_tensor(P).to(dev).contiguous()
    EMd = torch.as_tensor(EM).to(dev).contiguous()
    mhd.prim2con(run.patch, run.eos, run.Un, Pd, EMd, 0)
    run.Us.copy_(run.Un)
    dt = 0.25 * ip.dx[0]
    if args.strip:
        mhd.set_tuning(args.strip)

    timer = CallTimer(torch, False)

    def rhs_eval(Ux):
        timer.wrap("con2prim", mhd.con2prim, run.patch, run.eos, Ux, run.P, run.flags, None, run.stats)
        timer.wrap("rhs", mhd.rhs, run.patch, run.par, run.eos, Ux, run.P, run.k, run.vmax, run.ws)

    def step():
        for s in range(4):
            rhs_eval(run.Un if s == 0 else run.Us)
            nxt = run.Us if s < 3 else run.Un
            timer.wrap("rk_stage", mhd.rk_stage, run.patch, I.NU, s, dt, run.Un, run.k, run.acc, nxt)

    sweep = None
    if args.sweep_strip:
        sweep = {}
        for sh in (1, 2, 4, 8, 16, 32):
            mhd.set_tuning(sh)
            step()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(3):
                step()
            e1.record()
            torch.cuda.synchronize()
            sweep[sh] = e0.elapsed_time(e1) / 3
        best = min(sweep, key=sweep.get)
        mhd.set_tuning(best)
        sweep = {"ms_per_step": {k: round(v, 3) for k, v in sweep.items()}, "chosen": best}
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: whole steps only
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    t0.record()
    for _ in range(args.steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_total = t0.elapsed_time(t1)
    ms_step = ms_total / args.steps
    nint = ip.ninterior
    zu_s = nint * 4 / (ms_step * 1e-3)
    fin = bool(torch.isfinite(run.Un).all().item())

    # per-call durations in a second timed pass with events around each call
    timer.enabled = True
    for _ in range(max(2, args.steps // 4)):
        step()
    torch.cuda.synchronize()
    per = timer.avg_ms()

    # algorithmic bytes per call (minimum HBM traffic, FP64, perfect halo reuse)
    npad = ip.npts
    bytes_call = {
        "con2prim": npad * ((17 + 8) * 8 + 1),           # 17 inputs, 8 prims, 1 flag byte
        "rhs": nint * ((32 + 7 + 32) * 8),                 # U and prims in, 32 RHS out
        "rk_stage": nint * (32 * 8 * 5 * 3 + 32 * 8 * 4) / 4,   # stages 0-2: 5 arrays, stage 3: 4
    }
    dom = max(per, key=lambda k: per[k] * timer.count()[k])
    achieved = bytes_call[dom] / (per[dom] * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "note": "provisional: algorithmic bytes of the dominant library call / its event-timed duration"}

    out = {"metric": METRIC, "value": round(zu_s, 1), "unit": "zone-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "C2: TOV star K=100 Gamma=2 rho_c=1.28e-3, %d^3 interior, dx=%.4g, full CCZ4+GRMHD "
                                  "RHS + plain con2prim + RK4 stage" % (args.n, ip.dx[0]),
                      "interior_points": nint, "padded_points": npad, "rhs_evals_per_step": 4, "path": "plain"},
           "breakdown_ms_per_call": {k: round(v, 4) for k, v in per.items()},
           "wall_s": round(wall, 3), "finite": fin, "tuning": mhd.get_tuning(), "strip_sweep": sweep,
           "roofline": roof}

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ip, U, P, EM, args.cpu_evals)
    print(json.dumps(out), flush=True)


def cpu_baseline(ip, U, P, EM, nevals):
    """The FP64 oracle on the host cores, same workload, `nevals` RHS evaluations
    (con2prim + rhs + RK stage), rate in the same unit."""
    import numpy as np

    from oracle import orc
    from paper_2510_13965_amd import inputs as I

    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    e = orc.make_eos(I.EOS_IDEAL2)
    par = orc.make_par(I.PARAMS)
    U = U.copy()
    P = P.copy()
    orc.prim2con(g, e, U, P, EM, 0)
    Pr = np.zeros_like(P)
    k = np.zeros_like(U)
    acc = np.zeros_like(U)
    Us = U.copy()
    dt = 0.25 * ip.dx[0]
    t0 = time.perf_counter()
    for s in range(nevals):
        st = s % 4
        X = U if st == 0 else Us
        orc.con2prim(g, e, X, Pr, None, None)
        orc.rhs(g, par, e, X, Pr, k)
        orc.rk4_stage_interior(g, I.NU, st, dt, U, k, acc, Us if st < 3 else U)
    el = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp:
        cores = min(cores, int(omp))
    return {"value": round(ip.ninterior * nevals / el, 1), "unit": "zone-updates/s", "cores": cores,
            "kind": "oracle", "sample": "%d RHS evaluations (con2prim+rhs+stage) of the full %d^3 patch, %.1f s"
                                        % (nevals, ip.n[0], el)}


if __name__ == "__main__":
    main()
