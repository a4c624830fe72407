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

    def step():
        for s in range(4):
            Ux = run.Un if s == 0 else run.Us
            mhd.con2prim(run.patch, run.eos, Ux, run.P, run.flags, None, run.stats)
            mhd.rhs(run.patch, run.par, run.eos, Ux, run.P, run.k, run.vmax, run.ws)
            mhd.rk_stage(run.patch, I.NU, s, dt, run.Un, run.k, run.acc, run.Us if s < 3 else run.Un)

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
    mhd.profile_start()
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

    prof = mhd.profile_stop()
    kern = kernel_table(prof, ip, args.steps)
    roof = roofline(prof, ip, args.n)
    out = {"metric": METRIC, "value": round(zu_s, 1), "unit": "zone-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "TOV star K=100 Gamma=2 rho_c=1.28e-3, %d^3 interior, dx=%.4g, full CCZ4+GRMHD "
                                  "RHS + plain con2prim + RK4 stage" % (args.n, ip.dx[0]),
                      "interior_points": nint, "padded_points": ip.npts, "rhs_evals_per_step": 4, "path": "plain"},
           "kernels": kern,
           "wall_s": round(wall, 3), "finite": fin, "tuning": mhd.get_tuning(), "strip_sweep": sweep,
           "roofline": roof}

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ip, U, P, EM, args.cpu_evals)
    print(json.dumps(out), flush=True)


# Algorithmic work per unit, counted on this workload by oracle/opcount.py
# (the oracle's own evaluation with an op-counting scalar type; add/sub, mul,
# div, sqrt and pow/exp/log count one flop each).  Units: interior points for
# the RHS kernels, padded points for con2prim and the point fluxes, interior
# point-fields for the RK stage.  The MHD update counts every interface once.
FLOP_PER_UNIT = {
    "k_con2prim": 188.85,
    "k_mhd_point": 1608.0,
    "k_mhd_update": 5136.11,
    "ccz4 (4 kernels)": 10396.0,
    "k_rk4_stage": 4.75,
}
# HBM bytes per launch of the dominant kernel from rocprofv3 --pmc (FETCH_SIZE x 2
# + WRITE_SIZE x 1, the factors that make a plain 1 GiB copy read and write 1 GiB),
# valid only for the kernel sources they were taken on (sha256 of these files).
TRAFFIC = {}
TRAFFIC_SOURCES = {"k_mhd_update": ["paper_2510_13965_amd/csrc/grmhd.hip", "paper_2510_13965_amd/csrc/dev_common.hpp"]}


def sources_sha(files):
    import hashlib

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_table(prof, ip, steps):
    """Per-kernel launches and event-timed durations, with the achieved FP64
    rate of the algorithmic flops where the count exists."""
    units = {"k_con2prim": ip.npts, "k_mhd_point": ip.npts, "k_mhd_update": ip.ninterior,
             "k_rk4_stage": ip.ninterior * 32}
    tab = {}
    for k, (n, t) in prof.items():
        e = {"launches": n, "ms_per_launch": round(t / n, 4), "ms_per_step": round(t / steps, 4)}
        if k in units:
            e["fp64_tflops"] = round(FLOP_PER_UNIT[k] * units[k] / (t / n * 1e-3) / 1e12, 3)
        tab[k] = e
    cz = [k for k in prof if k.startswith("k_ccz4_")]
    if cz:
        t = sum(prof[k][1] for k in cz) / prof[cz[0]][0]
        tab["ccz4 (4 kernels)"] = {"ms_per_launch": round(t, 4),
                                   "fp64_tflops": round(FLOP_PER_UNIT["ccz4 (4 kernels)"] * ip.ninterior
                                                        / (t * 1e-3) / 1e12, 3)}
    return tab


def roofline(prof, ip, n):
    """Roofline entry of the kernel with the largest share of the step.

    The RHS kernels are FP64-vector bound (arithmetic intensity above the ridge
    of 78.6 TFLOP/s / 8 TB/s); their achieved rate is the algorithmic flops of
    one launch over its average event-timed duration."""
    nint, npad = ip.ninterior, ip.npts
    units = {"k_con2prim": npad, "k_mhd_point": npad, "k_mhd_update": nint, "k_rk4_stage": nint * 32}
    dom = max(prof, key=lambda k: prof[k][1])
    launches, tot = prof[dom]
    ms = tot / launches
    out = {"kernel": dom, "ms_per_launch": round(ms, 4)}
    if dom in units and dom != "k_rk4_stage":
        flop = FLOP_PER_UNIT[dom] * units[dom]
        ach = flop / (ms * 1e-3) / 1e12
        out.update({"bound": "alu", "achieved": round(ach, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(ach / FP64_PEAK_TFLOPS, 4), "flop_per_launch": flop})
    else:
        nbytes = nint * 32 * 8 * 4.75  # stages 0-2 move 5 arrays, stage 3 moves 4
        ach = nbytes / (ms * 1e-3) / 1e9
        out.update({"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_launch": nbytes})
    t = TRAFFIC.get(dom)
    out["traffic"] = t[0] if t and t[1] == sources_sha(TRAFFIC_SOURCES[dom]) else None
    return out


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
