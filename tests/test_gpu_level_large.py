"""Batched level with the large boxes of the level workloads: six boxes of the
star on three 2:1 levels whose edges reach 48 and 64 (a 64^3 box among them),
so the level kernels run 3-4 LDS tiles per axis.

* The level's right-hand side (bracketed con2prim) equals per-box calls bit
  for bit, and on four boxes, the 64^3 one included, the FP64 oracle to 1e-10
  per field; the same with three grey M1 species (44 fields).
* With the learned con2prim guess (network trained on the star workloads'
  distribution), RK4 steps of the level, eager and replayed as a hipGraph,
  equal per-box steps with the learned guess bit for bit.
"""
import sys

import numpy as np
import pytest

from paper_2510_13965_amd import inputs as I

pytestmark = pytest.mark.gpu

PAR_M1 = dict(I.PARAMS, evolve_m1=1)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2510_13965_amd import mhd

    mhd.lib()
    return torch.device("cuda")


@pytest.fixture(scope="module")
def large_states(dev):
    """Six boxes (edges 16..64, one 64^3) with radiation; cons built on the device."""
    import torch
    from paper_2510_13965_amd import mhd

    boxes = I.amr_level_boxes(seed=I.SEED0 + 42, nboxes=6, edges=(16, 24, 32, 48, 64))
    Ab = I.star_field_amplitude()
    eos = mhd.make_eos(I.EOS_IDEAL2)
    out = []
    for b, box in enumerate(boxes):
        ip, U, P, EM = I.amr_box_state(box, Ab)
        R, aux = I.m1_radiation(ip, P, I.SEED0 + 900 + b)
        Ud = torch.empty((I.NU_M1,) + tuple(ip.shape), dtype=torch.float64, device="cuda")
        Ud[:I.NU].copy_(torch.as_tensor(U))
        Ud[I.NU:].copy_(torch.as_tensor(R))
        mhd.prim2con(mhd.patch_of(ip), eos, Ud, torch.as_tensor(P).cuda(), torch.as_tensor(EM).cuda(), 0)
        out.append((ip, Ud.cpu().numpy(), aux))
    ns = [ip.n for ip, _, _ in out]
    say("large level boxes", ns)
    assert (64, 64, 64) in ns and any(48 in n for n in ns)
    return out


def per_box(states, par, m1):
    import torch
    from paper_2510_13965_amd.step import PatchRun

    res = []
    for ip, U, aux in states:
        r = PatchRun(ip, U if m1 else U[:I.NU], I.EOS_IDEAL2, par, aux=aux if m1 else None)
        r.rhs_eval(r.Un)
        torch.cuda.synchronize()
        res.append(dict(k=r.k.cpu().numpy(), P=r.P.cpu().numpy(), flags=r.flags.cpu().numpy()))
    return res


def level_rhs(states, par, m1):
    import torch
    from paper_2510_13965_amd.step import LevelRun

    run = LevelRun([ip for ip, _, _ in states], [U if m1 else U[:I.NU] for _, U, _ in states], I.EOS_IDEAL2, par,
                   auxs=[aux for _, _, aux in states] if m1 else None)
    run.level.rhs(0, None)
    torch.cuda.synchronize()
    out = [dict(k=b["k"].cpu().numpy(), P=b["P"].cpu().numpy(), flags=b["flags"].cpu().numpy()) for b in run.boxes]
    run.level.close()
    return out


def oracle_box(orc, ip, U, aux, par, m1):
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    e = orc.make_eos(I.EOS_IDEAL2)
    Uo = (U if m1 else U[:I.NU]).copy()
    Po = np.zeros((I.NP,) + ip.shape)
    orc.con2prim(g, e, Uo, Po, None, None)
    ko = np.zeros_like(Uo)
    if m1:
        orc.rhs_full(g, orc.make_par(par), e, Uo, Po, aux, ko)
    else:
        orc.rhs(g, orc.make_par(par), e, Uo, Po, ko)
    return ko


@pytest.mark.parametrize("m1", [False, True], ids=["ccz4+grmhd", "with-m1"])
def test_large_level_rhs_bitwise_and_oracle(orc, large_states, m1):
    par = PAR_M1 if m1 else I.PARAMS
    nf = I.NU_M1 if m1 else I.NU
    say("case large level rhs vs per-box and oracle, m1=%s" % m1)
    ref = per_box(large_states, par, m1)
    got = level_rhs(large_states, par, m1)
    for b, (r, g) in enumerate(zip(ref, got)):
        for key in r:
            assert np.array_equal(r[key], g[key]), (b, key)
    # the oracle on four boxes: the 64^3 one and the next three largest
    order = sorted(range(len(large_states)), key=lambda b: -large_states[b][0].npts)[:4]
    for b in order:
        ip, U, aux = large_states[b]
        ko = oracle_box(orc, ip, U, aux, par, m1)
        sl = (slice(None),) + ip.interior()
        kg, ko = got[b]["k"][sl], ko[sl]
        worst = 0.0
        for f in range(nf):
            m = np.abs(ko[f]).max()
            if m > 0:
                e = np.abs(kg[f] - ko[f]).max() / m
                worst = max(worst, e)
                assert e <= 1e-10, (ip.n, f, e)
        say("  box", ip.n, "worst field error %.1e" % worst)


def test_large_level_learned_rk4_eager_and_graph(large_states):
    """Two RK4 steps of the level with the learned guess, eager and as a
    replayed hipGraph (with eager work and synchronisation between the
    replays), against per-box steps with the learned guess: bitwise."""
    import torch
    from paper_2510_13965_amd import learned
    from paper_2510_13965_amd.step import LevelRun, PatchRun

    say("case large level learned rk4 eager/graph, 2 steps")
    X, T = learned.training_set(1 << 14, seed=I.SEED0 + 45, eos_cfg=I.EOS_IDEAL2, **learned.STAR_SAMPLING)
    prm, hist = learned.train(X, T, seed=5, epochs=8, batch=1024)
    ips = [ip for ip, _, _ in large_states]
    Us = [U[:I.NU] for _, U, _ in large_states]
    dt = 0.25 * min(ip.dx[0] for ip in ips)
    boxes = [PatchRun(ip, U, I.EOS_IDEAL2, I.PARAMS) for ip, U in zip(ips, Us)]
    for r in boxes:
        r.use_learned(prm)
    eager = LevelRun(ips, Us, I.EOS_IDEAL2, I.PARAMS)
    graph = LevelRun(ips, Us, I.EOS_IDEAL2, I.PARAMS)
    eager.level.set_learned(prm)
    graph.level.set_learned(prm)
    stream = torch.cuda.Stream()
    fb = []
    for step in range(2):
        for r in boxes:
            r.step(dt)
        eager.level.rk4_step(dt)
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            graph.level.rk4_step(dt, use_graph=True, stream=stream)
        torch.cuda.synchronize()
        for b, r in enumerate(boxes):
            ref = r.Un.cpu().numpy()
            assert np.array_equal(ref, eager.boxes[b]["U"].cpu().numpy()), ("eager", step, b)
            assert np.array_equal(ref, graph.boxes[b]["U"].cpu().numpy()), ("graph", step, b)
            fb.append(((r.flags.cpu().numpy() & 32) != 0).mean())
    say("fallback share %.4f" % np.mean(fb))
    eager.level.close()
    graph.level.close()
