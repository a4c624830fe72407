#!/usr/bin/env python3
"""Zone-update throughput of the MoL right-hand side on one MI355X.

Headline workload: a batched AMR level of 803 uneven boxes (edges from
{16,24,32,48,64} per axis, three 2:1 levels dx = 1, 1/2, 1/4, 40.9 M interior
points) sampled from the K=100, Gamma=2, rho_c=1.28e-3 TOV star with its
poloidal field, evolving CCZ4 + GRMHD + three grey M1 species (44 fields),
one RK4 step = four right-hand-side evaluations.  One zone update = one
interior point through one evaluation (con2prim on the padded boxes + right-
hand side + stage update).  `value` is the chosen form: the learned con2prim
guess with the batched, autotuned persistent launches; beside it the plain
form (per-box launches, bracketed con2prim) and the batched graph replays are
timed on the same level.  The steps are timed in blocks of HEADLINE_BLOCK, each
block starting from the initial data (restored outside the timed region): the
boxes' ghosts are frozen, and the level stays physical for ~30 steps only.  Secondary workloads (the 128^3 star patch, the
192-box level without radiation, random con2prim states, IMEX, the glue and
the monitors) follow under `paths`.  Inputs are synthetic and built on the
device (the prim->cons map runs in the library); every timed region starts
with everything resident in HBM.

Prints one JSON line; --gpus N > 1 is refused: the build targets one GPU.
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
HEADLINE_BLOCK = 4  # steps per timed block of the headline level, each from the initial data
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
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-con2prim path")
    ap.add_argument("--no-level", action="store_true", help="skip the batched AMR-level paths")
    ap.add_argument("--no-m1", action="store_true", help="skip the M1-radiation path")
    ap.add_argument("--level-boxes", type=int, default=192)
    ap.add_argument("--no-level-m1", action="store_true", help="skip the batched level with M1 radiation")
    ap.add_argument("--no-level-imex", action="store_true", help="skip the batched level stepped by IMEX(4,4,2)")
    ap.add_argument("--no-diag", action="store_true", help="skip the constraint-monitor timing")
    ap.add_argument("--no-glue", action="store_true", help="skip the prolongation/restriction/dense-output timings")
    ap.add_argument("--level-m1-boxes", type=int, default=803)
    ap.add_argument("--no-c2p-cells", action="store_true", help="skip con2prim on random states")
    ap.add_argument("--c2p-log2", type=int, default=24, help="log2 of the number of random con2prim states")
    ap.add_argument("--level-steps", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=1, help="timed steps of the headline's per-box plain form")
    ap.add_argument("--headline-only", action="store_true", help="only the headline level (for profiling)")
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


def say(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def time_steps(torch, step, steps, warmup):
    """Mean event-timed milliseconds per step on the current stream."""
    for _ in range(warmup):
        step()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def learned_path(torch, mhd, I, run, step, args, nint, prm):
    """Same patch and steps with the learned con2prim guess (the network
    trained on the star workloads' distribution)."""
    run.use_learned(prm)
    step()
    run.stats.zero_()
    ms = time_steps(torch, step, args.steps, 0)
    st = run.stats.cpu().numpy()
    run.use_learned(None)
    nev = 4 * args.steps * run.ip.npts
    say("learned path: %.3f ms/step, fallback %.4f" % (ms, st[2] / nev))
    return {"zone_updates_per_s": round(nint * 4 / (ms * 1e-3), 1), "ms_per_step": round(ms, 4),
            "fallback_rate": round(float(st[2]) / nev, 6), "root_evals_per_point": round(float(st[3]) / nev, 3)}


def m1_path(torch, mhd, I, ip, U, P, EM, args):
    """The same star with three grey M1 species (44 evolved fields): smooth
    radiation fields, per-point opacities (inputs.m1_fields)."""
    from paper_2510_13965_amd.step import PatchRun

    t0 = time.perf_counter()
    par = dict(I.PARAMS, evolve_m1=1)
    run0 = PatchRun(ip, U, I.EOS_IDEAL2, I.PARAMS)
    mhd.prim2con(run0.patch, run0.eos, run0.Un, torch.as_tensor(P).cuda(), torch.as_tensor(EM).cuda(), 0)
    U32 = run0.Un.cpu().numpy()
    del run0
    U44, aux = I.m1_fields(ip, U32, P, I.SEED0 + 70)
    run = PatchRun(ip, U44, I.EOS_IDEAL2, par, aux=aux)
    del U44, aux
    dt = 0.25 * ip.dx[0]
    say("m1 path: built in %.1f s" % (time.perf_counter() - t0))
    mhd.profile_start()
    ms = time_steps(torch, lambda: run.step(dt), args.steps, 1)
    prof = mhd.profile_stop()
    fin = bool(torch.isfinite(run.Un).all().item())
    say("m1 path: %.3f ms/step" % ms)
    return {"zone_updates_per_s": round(ip.ninterior * 4 / (ms * 1e-3), 1), "ms_per_step": round(ms, 4),
            "evolved_fields": 44, "finite": fin, "kernels": kernel_table(prof, ip, args.steps + 1, nfields=44)}


def c2p_cells_path(torch, mhd, I, args):
    """con2prim alone on 2^24 random states of the broad distribution (three-piece
    PWP + thermal part; densities 1e-12..1e-3, W 1..10, magnetisations 1e-4..10):
    the plain bracketed solver against the learned guess (trained here on 2^20
    states of its own seed).  Rates in states per second; the learned roots are
    compared with the plain ones state by state."""
    from paper_2510_13965_amd import learned

    n = 1 << args.c2p_log2
    t0 = time.perf_counter()
    X, T = learned.training_set(1 << 20, seed=I.SEED0 + 90)
    prm, hist = learned.train(X, T, seed=11, epochs=60, batch=1024)
    del X, T
    t_train = time.perf_counter() - t0
    ip, U, P, EM = I.c2p_cells(ncell=n, seed=I.SEED0 + 91)
    pt = mhd.patch_of(ip)
    eos = mhd.make_eos(I.EOS_PWP3)
    U0 = torch.as_tensor(U).cuda()
    mhd.prim2con(pt, eos, U0, torch.as_tensor(P).cuda(), torch.as_tensor(EM).cuda(), 1)
    del U, P, EM
    say("c2p cells: %d states ready, network trained in %.1f s" % (n, t_train))
    out = {"states": n, "train_s": round(t_train, 2), "train_loss_first_last": [hist[0], hist[-1]]}
    ws = torch.empty((mhd.con2prim_learned_workspace_size(pt) + 7) // 8, dtype=torch.float64, device="cuda")
    res = {}
    for mode in ("plain", "learned"):
        Ud = U0.clone()
        Pd = torch.zeros((I.NP,) + ip.shape, dtype=torch.float64, device="cuda")
        fl = torch.zeros(ip.shape, dtype=torch.uint8, device="cuda")
        mu = torch.zeros((2,) + ip.shape, dtype=torch.float64, device="cuda")
        st = torch.zeros(mhd.MHD_NSTAT, dtype=torch.int64, device="cuda")

        def once(stats=None):
            if mode == "plain":
                mhd.con2prim(pt, eos, Ud, Pd, fl, mu, stats)
            else:
                mhd.con2prim_learned(pt, eos, prm, Ud, Pd, ws, fl, mu, stats)

        once(st)  # the counted call, on the untouched states
        torch.cuda.synchronize()
        ms = time_steps(torch, once, 3, 1)
        mhd.profile_start()
        once()
        torch.cuda.synchronize()
        kern = {k: round(t / n, 4) for k, (n, t) in mhd.profile_stop().items()}
        res[mode] = (mu.clone(), fl.clone(), st.cpu().numpy())
        out[mode] = {"states_per_s": round(n / (ms * 1e-3), 1), "ms": round(ms, 3),
                     "root_evals_per_state": round(float(res[mode][2][3]) / n, 3), "kernels_ms": kern}
        say("c2p cells %s: %.3f ms" % (mode, ms))
        del Ud, Pd
    mup, flp, _ = res["plain"]
    mul, fll, stl = res["learned"]
    solved = (mup[1] > 0) & ((fll & 32) == 0)
    rel = ((mul[1] - mup[1]).abs() / mup[1].abs().clamp_min(1e-300))[solved]
    # Where the root function has more than one root in (0, mu_+] (possible once
    # the density and energy are clamped to the EoS range), Newton from the
    # learned guess and the bracketing solver may converge to different roots:
    # counted separately; the maximum difference is taken over the other states.
    # (The learned path does not solve for mu_+: only mu is compared.)
    other = rel > 1e-6
    out["learned"]["fallback_rate"] = round(float(stl[2]) / n, 6)
    out["learned"]["states_other_root"] = int(other.sum().item())
    out["learned"]["max_rel_root_difference"] = float(rel[~other].max().item())
    out["learned"]["flags_differ"] = int(((fll & ~32) != flp).sum().item())
    return out


def imex_path(torch, mhd, I, ip, U, P, EM, args):
    """The same star and radiation as the M1 path, opacities x1000 (kappa dt up
    to ~80 at the centre, far past the explicit stability limit), stepped by
    IMEX(4,4,2) with the implicit collision solve."""
    from paper_2510_13965_amd.step import ImexRun, PatchRun

    t0 = time.perf_counter()
    run0 = PatchRun(ip, U, I.EOS_IDEAL2, I.PARAMS)
    mhd.prim2con(run0.patch, run0.eos, run0.Un, torch.as_tensor(P).cuda(), torch.as_tensor(EM).cuda(), 0)
    U32 = run0.Un.cpu().numpy()
    del run0
    U44, aux = I.m1_fields(ip, U32, P, I.SEED0 + 70)
    aux[0::3] *= 1e3
    aux[1::3] *= 1e3
    aux[2::3] *= 1e3
    run = ImexRun(ip, U44, aux, I.EOS_IDEAL2, I.PARAMS)
    del U44, aux
    dt = 0.25 * ip.dx[0]
    say("imex path: built in %.1f s" % (time.perf_counter() - t0))
    mhd.profile_start()
    ms = time_steps(torch, lambda: run.step(dt), max(2, args.steps // 2), 1)
    prof = mhd.profile_stop()
    fin = bool(torch.isfinite(run.Un).all().item())
    say("imex path: %.3f ms/step" % ms)
    return {"zone_updates_per_s": round(ip.ninterior * 4 / (ms * 1e-3), 1), "ms_per_step": round(ms, 4),
            "evolved_fields": 44, "finite": fin, "implicit_solves_not_converged": int(run.nfail.item()),
            "kernels": {k: {"launches": n, "ms_per_launch": round(t / n, 4)} for k, (n, t) in prof.items()}}


def level_paths(torch, mhd, I, args, mlp):
    """The AMR-level workload: uneven boxes (edges 16..64) on three 2:1 levels of
    the star; per-box launches vs one batched level (autotuned), eager, as a
    replayed hipGraph, and with the learned con2prim."""
    from paper_2510_13965_amd.step import LevelRun

    t0 = time.perf_counter()
    boxes = I.amr_level_boxes(nboxes=args.level_boxes)
    Ab = I.star_field_amplitude()
    eos = mhd.make_eos(I.EOS_IDEAL2)
    ips, states = [], []
    for b in boxes:
        ip, U, P, EM = I.amr_box_state(b, Ab)
        Ud = torch.as_tensor(U).cuda()
        mhd.prim2con(mhd.patch_of(ip), eos, Ud, torch.as_tensor(P).cuda(), torch.as_tensor(EM).cuda(), 0)
        ips.append(ip)
        states.append(Ud)
    lr = LevelRun(ips, states, I.EOS_IDEAL2, I.PARAMS)
    del states
    torch.cuda.synchronize()
    say("level: %d boxes, %d interior points, built in %.1f s" % (len(ips), lr.ninterior, time.perf_counter() - t0))
    dt = 0.25 * min(ip.dx[0] for ip in ips)
    nzu = lr.ninterior * 4
    res = {"workload": "%d boxes, edges from {16,24,32,48,64}, 3 levels dx=1,1/2,1/4 of the TOV star; dt=%.4g"
                       % (len(ips), dt),
           "interior_points": lr.ninterior, "padded_points": lr.npts}

    def per_box_step():
        for s in range(4):
            for b in lr.boxes:
                Ux = b["U"] if s == 0 else b["Us"]
                mhd.con2prim(b["patch"], lr.eos, Ux, b["P"], b.get("flags"), None, None)
                mhd.rhs(b["patch"], lr.par, lr.eos, Ux, b["P"], b["k"], None, b["ws"])
                mhd.rk_stage(b["patch"], I.NU, s, dt, b["U"], b["k"], b["acc"], b["Us"] if s < 3 else b["U"])

    ms = time_steps(torch, per_box_step, 2, 1)
    res["per_box"] = {"zone_updates_per_s": round(nzu / (ms * 1e-3), 1), "ms_per_step": round(ms, 3)}
    say("level per-box: %.2f ms/step" % ms)
    tun = lr.level.autotune(dt)
    res["autotuned"] = tun
    ms = time_steps(torch, lambda: lr.level.rk4_step(dt), args.level_steps, 1)
    res["batched_eager"] = {"zone_updates_per_s": round(nzu / (ms * 1e-3), 1), "ms_per_step": round(ms, 3)}
    say("level batched eager (%s): %.2f ms/step" % (tun, ms))
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        ms = time_steps(torch, lambda: lr.level.rk4_step(dt, use_graph=True, stream=stream), args.level_steps, 1)
    res["batched_graph"] = {"zone_updates_per_s": round(nzu / (ms * 1e-3), 1), "ms_per_step": round(ms, 3)}
    say("level batched graph: %.2f ms/step" % ms)
    if mlp is not None:
        lr.level.set_learned(mlp)
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            ms = time_steps(torch, lambda: lr.level.rk4_step(dt, use_graph=True, stream=stream), args.level_steps, 1)
        res["batched_graph_learned"] = {"zone_updates_per_s": round(nzu / (ms * 1e-3), 1), "ms_per_step": round(ms, 3)}
        # con2prim statistics of one right-hand side on the evolved level, learned and plain
        for tag, m in (("learned", mlp), ("plain", None)):
            lr.level.set_learned(m)
            st = torch.zeros(mhd.MHD_NSTAT, dtype=torch.int64, device="cuda")
            lr.level.rhs(0, None, st)
            st = st.cpu().numpy()
            res["c2p_" + tag] = {"fallback_rate": round(float(st[2]) / lr.npts, 6),
                                 "root_evals_per_point": round(float(st[3]) / lr.npts, 3)}
        say("level batched graph + learned: %.2f ms/step, fallback %.4f" % (ms, res["c2p_learned"]["fallback_rate"]))
    fin = all(bool(torch.isfinite(b["U"]).all().item()) for b in lr.boxes)
    res["finite"] = fin
    lr.level.close()
    return res


class _Units:
    """Interior, padded and interior-plus-one-layer point counts of a set of
    boxes (for kernel_table)."""

    def __init__(self, ninterior, npts, nhalo1):
        self.ninterior, self.npts, self.nhalo1 = ninterior, npts, nhalo1


def build_level_m1(torch, mhd, I, nboxes):
    """The boxes of the level with radiation, built on the host in threads and
    moved to the device; returns (LevelRun, box list)."""
    from concurrent.futures import ThreadPoolExecutor

    from paper_2510_13965_amd.step import LevelRun

    boxes = I.amr_level_boxes(seed=I.SEED0 + 5, nboxes=nboxes)
    Ab = I.star_field_amplitude()
    eos = mhd.make_eos(I.EOS_IDEAL2)

    def host_box(b):
        # numpy releases the GIL in the array work: boxes are generated in threads
        ip, U, P, EM = I.amr_box_state(boxes[b], Ab)
        R, aux = I.m1_radiation(ip, P, I.SEED0 + 500 + b)
        return ip, U, P, EM, R, aux

    ips, states, auxs = [], [], []
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(workers) as ex:
        for ip, U, P, EM, R, aux in ex.map(host_box, range(len(boxes))):
            Ud = torch.empty((I.NU_M1,) + tuple(ip.shape), dtype=torch.float64, device="cuda")
            Ud[:I.NU].copy_(torch.as_tensor(U))
            Ud[I.NU:].copy_(torch.as_tensor(R))
            mhd.prim2con(mhd.patch_of(ip), eos, Ud, torch.as_tensor(P).cuda(), torch.as_tensor(EM).cuda(), 0)
            ips.append(ip)
            states.append(Ud)
            auxs.append(torch.as_tensor(aux).cuda())
    lr = LevelRun(ips, states, I.EOS_IDEAL2, dict(I.PARAMS, evolve_m1=1), auxs=auxs)
    del states, auxs
    torch.cuda.synchronize()
    return lr, boxes


def headline_level_m1(torch, mhd, I, args, mlp):
    """The headline: the coupled system with three grey M1 species (44 fields)
    on a batched level of ~800 uneven boxes (~40 M interior points) of the
    star.  Plain form: per-box launches with the bracketed con2prim.  Chosen
    form (`value`): the learned con2prim guess with the batched, autotuned
    persistent launches, timed over exactly `steps` steps after `warmup`
    untimed ones, with per-kernel HIP events on the launch stream, in blocks
    of HEADLINE_BLOCK steps from the initial data.  Also timed: the batched
    level with the bracketed con2prim, and both batched forms replayed as
    hipGraphs."""
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    lr, boxes = build_level_m1(torch, mhd, I, args.level_m1_boxes)
    say("headline level: %d boxes, %d interior points, built in %.1f s"
        % (len(lr.boxes), lr.ninterior, time.perf_counter() - t0))
    dt = 0.25 * min(b["ip"].dx[0] for b in lr.boxes)
    nzu = lr.ninterior * 4
    res = {"interior_points": lr.ninterior, "padded_points": lr.npts, "boxes": len(lr.boxes), "dt": dt,
           "evolved_fields": I.NU_M1, "steps_per_block": HEADLINE_BLOCK}
    # Every timed block of at most HEADLINE_BLOCK steps starts from the initial
    # data (restored untimed): the boxes' ghosts are frozen, and after ~30
    # steps (t ~ 2) the boundary mismatch drives the largest speed of the
    # finest boxes past the RK4 limit, so longer runs would time a blow-up.
    U0 = [b["U"].clone() for b in lr.boxes]

    def restore():
        for b, u in zip(lr.boxes, U0):
            b["U"].copy_(u)
        torch.cuda.synchronize()

    def timed_blocks(step, steps, warmup):
        restore()
        for _ in range(warmup):
            step()
        total, done = 0.0, 0
        while done < steps:
            restore()
            n = min(HEADLINE_BLOCK, steps - done)
            total += time_steps(torch, step, n, 0) * n
            done += n
        return total / steps

    def per_box_step():
        for s in range(4):
            for b in lr.boxes:
                Ux = b["U"] if s == 0 else b["Us"]
                mhd.con2prim(b["patch"], lr.eos, Ux, b["P"], b.get("flags"), None, None)
                mhd.rhs(b["patch"], lr.par, lr.eos, Ux, b["P"], b["k"], None, b["ws"], aux=b["aux"])
                mhd.rk_stage(b["patch"], I.NU_M1, s, dt, b["U"], b["k"], b["acc"], b["Us"] if s < 3 else b["U"])

    nplain = max(1, min(args.steps, args.plain_steps))
    ms = timed_blocks(per_box_step, nplain, 1)
    res["plain_per_box"] = {"zone_updates_per_s": round(nzu / (ms * 1e-3), 1), "ms_per_step": round(ms, 3),
                            "steps": nplain}
    say("headline plain (per box, bracketed con2prim): %.2f ms/step" % ms)
    t1 = time.perf_counter()
    lr.level.set_learned(mlp)
    res["autotuned"] = lr.level.autotune(dt)
    res["autotune_s"] = round(time.perf_counter() - t1, 2)
    # the chosen form, eager, with per-kernel events: the value
    restore()
    for _ in range(args.warmup):
        lr.level.rk4_step(dt)
    torch.cuda.synchronize()
    mhd.profile_start()
    ms_value = timed_blocks(lambda: lr.level.rk4_step(dt), args.steps, 0)
    prof = mhd.profile_stop()
    res["learned_batched"] = {"zone_updates_per_s": round(nzu / (ms_value * 1e-3), 1),
                              "ms_per_step": round(ms_value, 3), "steps": args.steps}
    say("headline learned + batched: %.2f ms/step" % ms_value)
    st = torch.zeros(mhd.MHD_NSTAT, dtype=torch.int64, device="cuda")
    restore()
    lr.level.rhs(0, None, st)
    st = st.cpu().numpy()
    res["c2p_learned"] = {"fallback_rate": round(float(st[2]) / lr.npts, 6),
                          "root_evals_per_point": round(float(st[3]) / lr.npts, 3)}
    stream = torch.cuda.Stream()
    nrep = max(2, min(args.steps, 5))
    for tag, m in (("learned_batched_graph", mlp), ("plain_batched_graph", None)):
        lr.level.set_learned(m)
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            restore()
            lr.level.rk4_step(dt, use_graph=True, stream=stream)   # capture + warm-up
            ms = timed_blocks(lambda: lr.level.rk4_step(dt, use_graph=True, stream=stream), nrep, 0)
        res[tag] = {"zone_updates_per_s": round(nzu / (ms * 1e-3), 1), "ms_per_step": round(ms, 3), "steps": nrep}
        say("headline %s: %.2f ms/step" % (tag, ms))
    st = torch.zeros(mhd.MHD_NSTAT, dtype=torch.int64, device="cuda")
    restore()
    lr.level.rhs(0, None, st)
    st = st.cpu().numpy()
    res["c2p_plain"] = {"root_evals_per_point": round(float(st[3]) / lr.npts, 3)}
    # per-kernel times of one eager step with the bracketed con2prim (the
    # con2prim phases of the two forms side by side)
    restore()
    mhd.profile_start()
    lr.level.rk4_step(dt)
    prof_plain = mhd.profile_stop()
    res["kernels_plain_one_step"] = {k: round(t / n, 4) for k, (n, t) in prof_plain.items()}
    res["finite"] = all(bool(torch.isfinite(b["U"]).all().item()) for b in lr.boxes)
    del U0
    units = _Units(lr.ninterior, lr.npts, lr.nhalo1)
    res["kernels"] = kernel_table(prof, units, args.steps, nfields=I.NU_M1, flops=FLOP_PER_UNIT_LEVEL_M1)
    res["roofline"] = roofline(prof, units, FLOP_PER_UNIT_LEVEL_M1, TRAFFIC_LEVEL_M1, nfields=I.NU_M1)
    lr.level.close()
    del lr
    torch.cuda.empty_cache()
    return ms_value, res


def level_imex_path(torch, mhd, I, args):
    """The 192-box level of the star with three grey M1 species, opacities and
    emissivities x100 (kappa dt up to ~8 at the centre, past the explicit RK4
    stability limit), stepped by IMEX(4,4,2): per-box launches (one ImexRun per
    box) against the batched level, eager and as a replayed hipGraph."""
    from paper_2510_13965_amd.step import ImexRun, LevelRun

    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    boxes = I.amr_level_boxes(nboxes=args.level_boxes)
    Ab = I.star_field_amplitude()
    eos = mhd.make_eos(I.EOS_IDEAL2)
    ips, states, auxs = [], [], []
    for b, box in enumerate(boxes):
        ip, U, P, EM = I.amr_box_state(box, Ab)
        R, aux = I.m1_radiation(ip, P, I.SEED0 + 700 + b)
        Ud = torch.empty((I.NU_M1,) + tuple(ip.shape), dtype=torch.float64, device="cuda")
        Ud[:I.NU].copy_(torch.as_tensor(U))
        Ud[I.NU:].copy_(torch.as_tensor(R))
        mhd.prim2con(mhd.patch_of(ip), eos, Ud, torch.as_tensor(P).cuda(), torch.as_tensor(EM).cuda(), 0)
        ips.append(ip)
        states.append(Ud)
        auxs.append(torch.as_tensor(aux * 1e2).cuda())
    lr = LevelRun(ips, states, I.EOS_IDEAL2, dict(I.PARAMS, evolve_m1=1), auxs=auxs, imex=True)
    torch.cuda.synchronize()
    say("level IMEX: %d boxes, %d interior points, built in %.1f s" % (len(ips), lr.ninterior, time.perf_counter() - t0))
    dt = 0.25 * min(ip.dx[0] for ip in ips)
    nzu = lr.ninterior * 4
    res = {"workload": "%d boxes of the star (as the batched level) + 3 grey M1 species, opacities x100, "
                       "IMEX(4,4,2); dt=%.4g" % (len(ips), dt), "interior_points": lr.ninterior}
    runs = [ImexRun(ip, U.clone(), aux, I.EOS_IDEAL2, I.PARAMS) for ip, U, aux in zip(ips, states, auxs)]
    del states, auxs
    ms = time_steps(torch, lambda: [r.step(dt) for r in runs], 1, 1)
    res["per_box"] = {"zone_updates_per_s": round(nzu / (ms * 1e-3), 1), "ms_per_step": round(ms, 3)}
    say("level IMEX per-box: %.2f ms/step" % ms)
    del runs
    res["autotuned"] = lr.level.autotune(dt)
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    ms = time_steps(torch, lambda: lr.level.imex_step(dt, None, nf), args.level_steps, 1)
    res["batched_eager"] = {"zone_updates_per_s": round(nzu / (ms * 1e-3), 1), "ms_per_step": round(ms, 3)}
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        ms = time_steps(torch, lambda: lr.level.imex_step(dt, None, nf, use_graph=True, stream=stream),
                        args.level_steps, 1)
    res["batched_graph"] = {"zone_updates_per_s": round(nzu / (ms * 1e-3), 1), "ms_per_step": round(ms, 3)}
    say("level IMEX batched graph (%s): %.2f ms/step" % (res["autotuned"], ms))
    torch.cuda.synchronize()
    mhd.profile_start()
    lr.level.imex_step(dt, None, nf)
    prof = mhd.profile_stop()
    res["kernels"] = kernel_table(prof, _Units(lr.ninterior, lr.npts, lr.nhalo1), 1, nfields=I.NU_M1)
    res["implicit_solves_not_converged"] = int(nf.item())
    res["finite"] = all(bool(torch.isfinite(b["U"]).all().item()) for b in lr.boxes)
    lr.level.close()
    del lr
    torch.cuda.empty_cache()
    return res


def glue_path(torch, mhd, I, args):
    """Mesh-refinement glue on star-sized data (32 fields): a fine 128^3 patch
    (dx 0.25, 3 ghosts) filled entirely by prolongation from its 2:1 parent
    (70^3 interior, dx 0.5), the restriction of the fine data back onto the 65^3
    coincident parent points, and the RK4 dense output (and its first
    derivative) on the fine patch.  Per-call times and HBM rates of the
    algorithmic bytes (every input value read once, every output written once)."""
    import numpy as np

    nf = I.NU
    ipf = I.Patch((128, 128, 128), (0.25,) * 3, (-16.0,) * 3, 3)
    ipc = I.Patch((70, 70, 70), (0.5,) * 3, (-17.5,) * 3, 3)
    Uc, _, _, _ = I.star_fields(ipc)
    pc, pf = mhd.patch_of(ipc), mhd.patch_of(ipf)
    # coarse padded index 0 at x = -19, fine padded index 0 at x = -16.75: the
    # coarse point i coincides with the fine point 2 i - 9
    off = (-9, -9, -9)
    Ucd = torch.as_tensor(Uc).cuda()
    Uf = torch.zeros((nf,) + ipf.shape, dtype=torch.float64, device="cuda")
    nfine = ipf.npts
    lo, hi = (0, 0, 0), tuple(n + 6 for n in ipf.n)
    ms = time_steps(torch, lambda: mhd.prolong(pc, Ucd, pf, Uf, nf, off, lo, hi), 10, 2)
    # reads: the coarse points under the fine patch; writes: every fine point
    ncoarse_read = ((134 + 1) // 2 + 5) ** 3
    b = 8.0 * nf * (nfine + ncoarse_read)
    res = {"workload": "128^3 fine patch (+3 ghosts) of the star from its 2:1 parent, 32 fields",
           "prolong": {"ms": round(ms, 4), "gbs": round(b / (ms * 1e-3) / 1e9, 1), "algorithmic_bytes": b}}
    clo = [max(0, (1 - o) // 2) for o in off]
    chi = [min(n + 6, (134 - 1 - o) // 2 + 1) for n, o in zip(ipc.n, off)]
    npts_r = int(np.prod([h - l for l, h in zip(clo, chi)]))
    Ub = Ucd.clone()
    ms = time_steps(torch, lambda: mhd.restrict(pf, Uf, pc, Ub, nf, off, clo, chi), 10, 2)
    b = 8.0 * nf * 2 * npts_r
    res["restrict"] = {"ms": round(ms, 4), "gbs": round(b / (ms * 1e-3) / 1e9, 1), "points": npts_r}
    L = [torch.rand_like(Uf) for _ in range(4)]
    out = torch.empty_like(Uf)
    for m in (0, 1):
        ms = time_steps(torch, lambda: mhd.dense_output(pf, nf, 0.5, 0.0625, m, Uf, L, out), 10, 2)
        b = 8.0 * nf * ipf.ninterior * (6 if m == 0 else 5)
        res["dense_output_d%d" % m] = {"ms": round(ms, 4), "gbs": round(b / (ms * 1e-3) / 1e9, 1)}
    say("glue: prolong %.3f ms (%.0f GB/s), restrict %.3f ms, dense output %.3f ms" % (
        res["prolong"]["ms"], res["prolong"]["gbs"], res["restrict"]["ms"], res["dense_output_d0"]["ms"]))
    del Ucd, Uf, Ub, L, out
    torch.cuda.empty_cache()
    return res


def diag_path(torch, mhd, I, run, ip):
    """Constraint monitors on the evolved star patch (the state the plain path
    left): per-call time of mhd_constraints, per-kernel event times, the HBM
    rate of the algorithmic bytes of the point kernel (23 evolved fields read
    once, 5 monitor fields written once, per interior point) and the monitor
    values themselves."""
    C5 = torch.zeros((5,) + ip.shape, dtype=torch.float64, device="cuda")
    sums = torch.zeros(7 * (ip.n[2] + 1), dtype=torch.float64, device="cuda")
    ms = time_steps(torch, lambda: mhd.constraints(run.patch, run.Un, C5, sums), 5, 1)
    mhd.profile_start()
    for _ in range(5):
        mhd.constraints(run.patch, run.Un, C5, sums)
    torch.cuda.synchronize()
    prof = mhd.profile_stop()
    kern = {k: round(t / n, 4) for k, (n, t) in prof.items()}
    b = 8.0 * (23 + 5) * ip.ninterior
    t = kern.get("k_constraints")
    s = sums[:7].cpu().tolist()
    res = {"workload": "constraint monitors of the evolved %d^3 star patch" % ip.n[0], "ms": round(ms, 4),
           "kernels_ms": kern, "k_constraints_gbs": round(b / (t * 1e-3) / 1e9, 1) if t else None,
           "algorithmic_bytes": b,
           "monitors": {"H_L2": s[0] ** 0.5, "M_L2": s[1] ** 0.5, "baryon_mass": s[2], "Theta_L2": s[3] ** 0.5,
                        "Z_L2": s[4] ** 0.5, "phi_L2": s[5] ** 0.5, "B_L2": s[6] ** 0.5}}
    say("constraints: %.3f ms per call (H_L2 %.3e, baryonic mass %.6f)" % (ms, res["monitors"]["H_L2"], s[2]))
    del C5, sums
    return res


def star_patch_paths(torch, mhd, I, args, mlp):
    """The 128^3 star patch (CCZ4 + GRMHD, plain con2prim and RK4 stage):
    per-kernel events, its own roofline entry and the learned variant."""
    from paper_2510_13965_amd.step import PatchRun

    ip, U, P, EM = I.tov_star_state(n=args.n)
    say("building the %d^3 star patch" % args.n)
    run = PatchRun(ip, U, I.EOS_IDEAL2, I.PARAMS, periodic=False, device="cuda")
    Pd = torch.as_tensor(P).to("cuda").contiguous()
    EMd = torch.as_tensor(EM).to("cuda").contiguous()
    mhd.prim2con(run.patch, run.eos, run.Un, Pd, EMd, 0)
    run.Us.copy_(run.Un)
    dt = 0.25 * ip.dx[0]
    if args.strip:
        mhd.set_tuning(args.strip)

    def step():
        run.step(dt)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    mhd.profile_start()
    ms_step = time_steps(torch, step, args.steps, 0)
    prof = mhd.profile_stop()
    nint = ip.ninterior
    res = {"workload": "TOV star K=100 Gamma=2 rho_c=1.28e-3, %d^3 interior, dx=%.4g, full CCZ4+GRMHD RHS + plain "
                       "con2prim + RK4 stage" % (args.n, ip.dx[0]),
           "interior_points": nint, "padded_points": ip.npts,
           "zone_updates_per_s": round(nint * 4 / (ms_step * 1e-3), 1), "ms_per_step": round(ms_step, 4),
           "kernels": kernel_table(prof, ip, args.steps),
           "roofline": roofline(prof, ip, FLOP_PER_UNIT_STAR, TRAFFIC_STAR),
           "finite": bool(torch.isfinite(run.Un).all().item()), "tuning": mhd.get_tuning()}
    say("star patch plain: %.3f ms/step" % ms_step)
    if mlp is not None:
        res["learned"] = learned_path(torch, mhd, I, run, step, args, nint, mlp)
    return run, ip, (U, P, EM), res


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2510_13965_amd import inputs as I
    from paper_2510_13965_amd import mhd

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    mhd.lib()
    w0 = time.perf_counter()
    mlp, train = train_star_mlp(torch, I)
    ms_value, head = headline_level_m1(torch, mhd, I, args, mlp)
    paths = {}
    if not args.headline_only:
        run, ip, (U, P, EM), paths["star128"] = star_patch_paths(torch, mhd, I, args, mlp)
        if not args.no_diag:
            paths["constraints"] = diag_path(torch, mhd, I, run, ip)
        del run
        torch.cuda.empty_cache()
        if not args.no_c2p_cells:
            paths["c2p_cells"] = c2p_cells_path(torch, mhd, I, args)
        if not args.no_m1:
            paths["m1"] = m1_path(torch, mhd, I, ip, U, P, EM, args)
            paths["imex"] = imex_path(torch, mhd, I, ip, U, P, EM, args)
        if not args.no_level:
            paths["level192"] = level_paths(torch, mhd, I, args, mlp)
        if not args.no_glue:
            paths["glue"] = glue_path(torch, mhd, I, args)
        if not args.no_level_imex:
            paths["level_imex"] = level_imex_path(torch, mhd, I, args)
    nzu = head["interior_points"] * 4
    value = nzu / (ms_value * 1e-3)
    out = {"metric": METRIC, "value": round(value, 1), "unit": "zone-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_value, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "batched AMR level of %d boxes (edges from {16,24,32,48,64}, three 2:1 levels "
                                  "dx=1,1/2,1/4) of the TOV star K=100 Gamma=2 rho_c=1.28e-3 with poloidal B, CCZ4 + "
                                  "GRMHD + 3 grey M1 species (44 fields), RK4 dt=%.4g; chosen form: learned "
                                  "con2prim guess + batched autotuned persistent launches. Radiation opacities "
                                  "kappa_a, kappa_s = 10^U(-3,0) * rho/1e-3 (proportional to density, up to 1 at "
                                  "the centre), not log-uniform [1e-8,1e-2]: density-independent opacities drive the "
                                  "1e-12 atmosphere to the velocity cap within a step. Timed in blocks of %d "
                                  "steps, each from the initial data (frozen ghosts: the level stays physical for "
                                  "~30 steps)" % (head["boxes"], head["dt"], HEADLINE_BLOCK),
                      "interior_points": head["interior_points"], "padded_points": head["padded_points"],
                      "rhs_evals_per_step": 4, "path": "learned+batched",
                      "plain_zone_updates_per_s": head["plain_per_box"]["zone_updates_per_s"],
                      "learned_batched_vs_plain": round(value / head["plain_per_box"]["zone_updates_per_s"], 3)},
           "headline": head, "train": train, "paths": paths, "roofline": head["roofline"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_level_m1(args)
    out["wall_s"] = round(time.perf_counter() - w0, 1)
    print(json.dumps(out), flush=True)


def train_star_mlp(torch, I):
    """The network of the learned con2prim guess, trained here (own kernels) on
    2^18 random states of the star workloads' distribution; training time is
    reported, not part of any step."""
    from paper_2510_13965_amd import learned

    t0 = time.perf_counter()
    X, T = learned.training_set(1 << 18, seed=I.SEED0 + 50, eos_cfg=I.EOS_IDEAL2, **learned.STAR_SAMPLING)
    prm, hist = learned.train(X, T, seed=7, epochs=24, batch=4096)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    say("network trained in %.1f s, loss %.3e -> %.3e" % (t_train, hist[0], hist[-1]))
    return prm, {"states": 1 << 18, "epochs": 24, "train_s": round(t_train, 2),
                 "loss_first_last": [hist[0], hist[-1]]}


def cpu_baseline_level_m1(args):
    """The FP64 oracle on the host cores: one evaluation (con2prim + right-hand
    side with radiation + RK4 stage) of each box of the seeded 16-box subset
    of the headline level, from the level's initial data; on all cores the
    process may use and on one core, median of 3 each."""
    import numpy as np

    from oracle import orc
    from paper_2510_13965_amd import inputs as I

    boxes = I.amr_level_boxes(seed=I.SEED0 + 5, nboxes=args.level_m1_boxes)
    sub = I.level_subset(len(boxes))
    Ab = I.star_field_amplitude()
    e = orc.make_eos(I.EOS_IDEAL2)
    par = orc.make_par(dict(I.PARAMS, evolve_m1=1))
    states = []
    for b in sub:
        ip, U, P, EM = I.amr_box_state(boxes[b], Ab)
        R, aux = I.m1_radiation(ip, P, I.SEED0 + 500 + b)
        g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
        orc.prim2con(g, e, U, P, EM, 0)
        states.append((ip, g, np.concatenate([U, R]), aux))
    nint = sum(ip.ninterior for ip, _, _, _ in states)
    dt = 0.25 * min(b["dx"][0] for b in boxes)

    def once(sample):
        t0 = time.perf_counter()
        for ip, g, U0, aux in sample:
            U = U0.copy()
            Pr = np.zeros((I.NP,) + ip.shape)
            k = np.zeros_like(U)
            acc = np.zeros_like(U)
            Us = U.copy()
            orc.con2prim(g, e, U, Pr, None, None)
            orc.rhs_full(g, par, e, U, Pr, aux, k)
            orc.rk4_stage_interior(g, I.NU_M1, 0, dt, U, k, acc, Us)
        return time.perf_counter() - t0

    cores = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp:
        cores = min(cores, int(omp))
    orc.set_threads(cores)
    t_all = sorted(once(states) for _ in range(3))[1]
    # one thread: the first box of the subset only (the whole subset would take minutes)
    one = states[:1]
    n_one = one[0][0].ninterior
    orc.set_threads(1)
    t_one = sorted(once(one) for _ in range(3))[1]
    orc.set_threads(cores)
    return {"value": round(nint / t_all, 1), "unit": "zone-updates/s", "cores": cores, "kind": "oracle",
            "sample": "one evaluation (con2prim + RHS with 3 grey M1 species + RK4 stage) of each of the %d boxes "
                      "of the seeded subset of the headline level (%d interior points) from its initial data, "
                      "median of 3: %.2f s on %d threads. On 1 thread, the subset's first box (%s, %d interior "
                      "points), median of 3: %.2f s"
                      % (len(states), nint, t_all, cores, "x".join(str(v) for v in one[0][0].n), n_one, t_one),
            "one_core": {"value": round(n_one / t_one, 1), "unit": "zone-updates/s", "cores": 1}}


# Algorithmic work per unit, counted by oracle/opcount.py (the oracle's own
# evaluation with an op-counting scalar type; add/sub, mul, div, sqrt and
# pow/exp/log count one flop each).  Units: interior points for the RHS
# kernels, padded points for con2prim and the GRMHD point fluxes, interior
# point-fields for the RK stage; the M1 point pass covers the interior and one
# ghost layer, and its row (an average over the padded points) is applied to
# those points.  The MHD and M1 updates count every interface
# once.  Star patch: the 128^3 star (M1 rows: three grey species on the same
# star).  Level with radiation: the 16-box subset of the 803-box level
# (inputs.level_subset), three grey species, summed over the boxes
# (python oracle/opcount.py --level-m1 803); its CCZ4 row includes the
# radiation's matter terms, while the closure they use is counted with the M1
# point step, where the kernels evaluate it.
FLOP_PER_UNIT_STAR = {
    "k_con2prim": 188.85,
    "k_mhd_point": 1608.0,
    "k_mhd_update": 5136.11,
    "ccz4 (4 kernels)": 10396.0,
    "k_rk4_stage": 4.75,
    "k_m1_point": 15301.03,
    "k_m1_update": 2855.5,
}
FLOP_PER_UNIT_LEVEL_M1 = {
    "k_con2prim": 233.58,
    "k_mhd_point": 1608.0,
    "k_mhd_update": 5048.19,
    "ccz4 (4 kernels)": 10651.0,
    "k_rk4_stage": 4.75,
    "k_m1_point": 11941.59,
    "k_m1_update": 2873.4,
}
# HBM bytes per launch of a kernel from rocprofv3 --pmc (FETCH_SIZE and
# WRITE_SIZE, each scaled by what the counter reads for a plain 1 GiB copy),
# valid only for the kernel sources they were taken on (sha256 of these files).
TRAFFIC_STAR = {"k_mhd_update": (2650625248.0, "2a8e9605e17bbe5a")}
TRAFFIC_LEVEL_M1 = {"k_m1_update": (119581269011.2, "c83ffef2a4ca171b"),
                    "k_m1_point": (48873636155.1, "c83ffef2a4ca171b"),
                    "k_mhd_update": (68506649479.9, "2a8e9605e17bbe5a")}
TRAFFIC_SOURCES = {
    "k_mhd_update": ["paper_2510_13965_amd/csrc/grmhd.hip", "paper_2510_13965_amd/csrc/dev_common.hpp"],
    "k_m1_point": ["paper_2510_13965_amd/csrc/m1.hip", "paper_2510_13965_amd/csrc/m1_dev.hpp",
                   "paper_2510_13965_amd/csrc/dev_common.hpp"],
    "k_m1_update": ["paper_2510_13965_amd/csrc/m1.hip", "paper_2510_13965_amd/csrc/m1_dev.hpp",
                    "paper_2510_13965_amd/csrc/dev_common.hpp"],
}


def sources_sha(files):
    import hashlib

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_table(prof, ip, steps, nfields=32, flops=None):
    """Per-kernel launches and event-timed durations, with the achieved FP64
    rate of the algorithmic flops where the count exists."""
    flops = FLOP_PER_UNIT_STAR if flops is None else flops
    units = {"k_con2prim": ip.npts, "k_mhd_point": ip.npts, "k_mhd_update": ip.ninterior,
             "k_rk4_stage": ip.ninterior * nfields, "k_m1_point": ip.nhalo1}
    tab = {}
    for k, (n, t) in prof.items():
        e = {"launches": n, "ms_per_launch": round(t / n, 4), "ms_per_step": round(t / steps, 4)}
        if k in units:
            e["fp64_tflops"] = round(flops[k] * units[k] / (t / n * 1e-3) / 1e12, 3)
        tab[k] = e
    cz = [k for k in prof if k.startswith("k_ccz4_")]
    if cz:
        t = sum(prof[k][1] for k in cz) / prof[cz[0]][0]
        tab["ccz4 (4 kernels)"] = {"ms_per_launch": round(t, 4),
                                   "fp64_tflops": round(flops["ccz4 (4 kernels)"] * ip.ninterior
                                                        / (t * 1e-3) / 1e12, 3)}
    return tab


def kernel_work(ip, flops, nfields):
    """Bound and algorithmic work of one launch of each kernel on this patch
    or level: FP64 flops (oracle op counts) for the arithmetic-bound kernels,
    minimum HBM bytes for the streaming ones (every input value read once,
    every output written once)."""
    nint, npad = ip.ninterior, ip.npts
    return {
        "k_mhd_update": ("alu", flops["k_mhd_update"] * nint),
        "k_mhd_point": ("alu", flops["k_mhd_point"] * npad),
        "k_con2prim": ("alu", flops["k_con2prim"] * npad),
        "k_m1_point": ("alu", flops["k_m1_point"] * ip.nhalo1),
        # every field read once, every output written once: U (19 metric and gauge fields, 12 radiation),
        # P (v, W), aux (9), the M1 workspace (closure 18, fluxes and speeds 45), the fluid's tau and
        # S_i read and written, 12 radiation right-hand sides written: 127 values per interior point
        "k_m1_update": ("hbm", nint * 8 * 127),
        # stages 0-2 read Un, k, acc and write acc, Unext; stage 3 reads Un, k, acc and writes Un
        "k_rk4_stage": ("hbm", nint * nfields * 8 * 4.75),
        # 22 CCZ4 fields read on the padded patch, 22 right-hand sides written
        "k_ccz4_stencil": ("hbm", 22 * 8 * (npad + nint)),
        # 11 fields read on the padded patch, 24 second-derivative fields written
        "k_ccz4_d2": ("hbm", 11 * 8 * npad + 24 * 8 * nint),
    }


def roofline(prof, ip, flops, traffic, nfields=32):
    """Roofline entry of the kernel with the largest share of the timed region
    (among those with an algorithmic work figure; the kernel with the largest
    share overall is named beside it).  Achieved = algorithmic work of one
    launch / its average event-timed duration."""
    work = kernel_work(ip, flops, nfields)
    top = max(prof, key=lambda k: prof[k][1])
    dom = max((k for k in prof if k in work), key=lambda k: prof[k][1])
    launches, tot = prof[dom]
    ms = tot / launches
    out = {"kernel": dom, "ms_per_launch": round(ms, 4)}
    if top != dom:
        out["largest_share"] = top
    bound, w = work[dom]
    if bound == "alu":
        ach = w / (ms * 1e-3) / 1e12
        out.update({"bound": "alu", "achieved": round(ach, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(ach / FP64_PEAK_TFLOPS, 4), "flop_per_launch": w})
    else:
        ach = w / (ms * 1e-3) / 1e9
        out.update({"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_launch": w})
    t = traffic.get(dom)
    out["traffic"] = t[0] if t and dom in TRAFFIC_SOURCES and t[1] == sources_sha(TRAFFIC_SOURCES[dom]) else None
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
