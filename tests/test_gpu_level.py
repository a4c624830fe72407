"""Batched levels (mhd_level_*): uneven boxes through one persistent kernel per
phase, eager or as a replayed hipGraph, under every tuning.

The per-point arithmetic is the single-patch kernels' own, so the bar is
bitwise equality with per-box calls of mhd_con2prim / mhd_rhs / mhd_rk_stage
(themselves parity-tested against the oracle); one box is also compared with
the oracle directly.
"""
import sys

import numpy as np
import pytest

from paper_2510_13965_amd import inputs as I

pytestmark = pytest.mark.gpu


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
def level_states(dev):
    """Eight uneven boxes on three levels of the star, cons built on the device."""
    import torch
    from paper_2510_13965_amd import mhd

    boxes = I.amr_level_boxes(seed=I.SEED0 + 30, nboxes=8, edges=(16, 24, 32))
    Ab = I.star_field_amplitude()
    eos = mhd.make_eos(I.EOS_IDEAL2)
    out = []
    for b in boxes:
        ip, U, P, EM = I.amr_box_state(b, Ab)
        Ud = torch.as_tensor(U).cuda()
        mhd.prim2con(mhd.patch_of(ip), eos, Ud, torch.as_tensor(P).cuda(), torch.as_tensor(EM).cuda(), 0)
        out.append((ip, Ud.cpu().numpy()))
    say("level boxes", [ip.n for ip, _ in out])
    return out


def per_box_rhs(states):
    import torch
    from paper_2510_13965_amd.step import PatchRun

    res = []
    vmax = 0.0
    for ip, U in states:
        r = PatchRun(ip, U, I.EOS_IDEAL2, I.PARAMS)
        r.rhs_eval(r.Un)
        torch.cuda.synchronize()
        vmax = max(vmax, float(r.vmax.item()))
        res.append(dict(k=r.k.cpu().numpy(), P=r.P.cpu().numpy(), flags=r.flags.cpu().numpy(), U=r.Un.cpu().numpy()))
    return res, vmax


def level_rhs(run, src=0):
    import torch

    ms = torch.zeros(1, dtype=torch.float64, device="cuda")
    run.level.rhs(src, ms)
    torch.cuda.synchronize()
    return [dict(k=b["k"].cpu().numpy(), P=b["P"].cpu().numpy(), flags=b["flags"].cpu().numpy(),
                 U=b["U"].cpu().numpy()) for b in run.boxes], float(ms.item())


def assert_same(ref, got, tag):
    for b, (r, g) in enumerate(zip(ref, got)):
        for key in r:
            assert np.array_equal(r[key], g[key]), (tag, b, key)


def test_level_rhs_bitwise_equals_per_box(level_states):
    from paper_2510_13965_amd.step import LevelRun

    say("case level rhs vs per-box, 8 boxes")
    ref, vref = per_box_rhs(level_states)
    run = LevelRun([ip for ip, _ in level_states], [U for _, U in level_states], I.EOS_IDEAL2, I.PARAMS)
    got, v = level_rhs(run)
    assert_same(ref, got, "default tuning")
    assert v == vref


@pytest.mark.parametrize("tun", [dict(strip=1, block_threads=64, grid_per_cu=0),
                                 dict(strip=16, block_threads=128, grid_per_cu=4),
                                 dict(strip=4, block_threads=256, grid_per_cu=1)])
def test_level_rhs_tuning_invariant(level_states, tun):
    from paper_2510_13965_amd.step import LevelRun

    say("case level rhs tuning", tun)
    ref, vref = per_box_rhs(level_states)
    run = LevelRun([ip for ip, _ in level_states], [U for _, U in level_states], I.EOS_IDEAL2, I.PARAMS)
    run.level.set_tuning(**tun)
    assert run.level.get_tuning() == tun
    got, v = level_rhs(run)
    assert_same(ref, got, str(tun))
    assert v == vref


def test_level_rk4_eager_and_graph_replays(level_states):
    """Two RK4 steps per-box, eager level and graph level; the graph is
    replayed with eager work between replays and checked after every replay."""
    import torch
    from paper_2510_13965_amd.step import LevelRun, PatchRun

    say("case level rk4 eager/graph, 8 boxes, 2 steps")
    dt = 0.25 * 0.25
    ips = [ip for ip, _ in level_states]
    Us = [U for _, U in level_states]
    boxes = [PatchRun(ip, U, I.EOS_IDEAL2, I.PARAMS) for ip, U in level_states]
    eager = LevelRun(ips, Us, I.EOS_IDEAL2, I.PARAMS)
    graph = LevelRun(ips, Us, I.EOS_IDEAL2, I.PARAMS)
    ms_e = torch.zeros(1, dtype=torch.float64, device="cuda")
    ms_g = torch.zeros(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    for step in range(3):
        for r in boxes:
            r.step(dt)
        eager.level.rk4_step(dt, ms_e)
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            graph.level.rk4_step(dt, ms_g, use_graph=True, stream=stream)
        stream.synchronize()
        torch.cuda.synchronize()
        for b, r in enumerate(boxes):
            ref = r.Un.cpu().numpy()
            assert np.array_equal(ref, eager.boxes[b]["U"].cpu().numpy()), ("eager", step, b)
            assert np.array_equal(ref, graph.boxes[b]["U"].cpu().numpy()), ("graph", step, b)
        assert float(ms_e.item()) == float(ms_g.item()) > 0.0
        say("step", step, "ok, max speed", float(ms_e.item()))


def test_level_autotune_keeps_results(level_states):
    import torch
    from paper_2510_13965_amd.step import LevelRun

    say("case level autotune")
    ref, vref = per_box_rhs(level_states)
    run = LevelRun([ip for ip, _ in level_states], [U for _, U in level_states], I.EOS_IDEAL2, I.PARAMS)
    U0 = [b["U"].clone() for b in run.boxes]
    t = run.level.autotune(0.0625)
    torch.cuda.synchronize()
    say("autotune chose", t)
    assert t["block_threads"] in (64, 128, 256) and t["strip"] in (1, 4, 16) and t["grid_per_cu"] in (0, 4, 16)
    for b, u in zip(run.boxes, U0):
        assert torch.equal(b["U"], u)   # the tuner only reads U
    got, v = level_rhs(run)
    assert_same(ref, got, "after autotune")


def test_level_autotune_cache(level_states, tmp_path):
    """A second level of the same box shapes takes the cached choice without
    timing anything, and its results are unchanged."""
    import time

    import torch
    from paper_2510_13965_amd.step import LevelRun

    say("case level autotune cache")
    cache = tmp_path / "tuning.json"
    ips, Us = [ip for ip, _ in level_states], [U for _, U in level_states]
    t1 = LevelRun(ips, Us, I.EOS_IDEAL2, I.PARAMS).level.autotune(0.0625, cache=cache)
    assert cache.exists()
    run = LevelRun(ips, Us, I.EOS_IDEAL2, I.PARAMS)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    t2 = run.level.autotune(0.0625, cache=cache)
    assert time.perf_counter() - w0 < 0.5
    assert t2 == t1 == run.level.get_tuning()
    ref, vref = per_box_rhs(level_states)
    got, v = level_rhs(run)
    assert_same(ref, got, "cached tuning")


def test_level_box_against_oracle(orc, level_states):
    """The level's RHS on its smallest box against the FP64 oracle (1e-10 per field)."""
    from paper_2510_13965_amd.step import LevelRun

    ip, U = min(level_states, key=lambda s: s[0].npts)
    say("case level box vs oracle", ip.n)
    run = LevelRun([ip], [U], I.EOS_IDEAL2, I.PARAMS)
    got, _ = level_rhs(run)
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    e = orc.make_eos(I.EOS_IDEAL2)
    Uo = U.copy()
    Po = np.zeros((I.NP,) + ip.shape)
    orc.con2prim(g, e, Uo, Po, None, None)
    ko = np.zeros_like(U)
    orc.rhs(g, orc.make_par(I.PARAMS), e, Uo, Po, ko)
    sl = (slice(None),) + ip.interior()
    kg, ko = got[0]["k"][sl], ko[sl]
    for f in range(I.NU):
        m = np.abs(ko[f]).max()
        if m > 0:
            assert np.abs(kg[f] - ko[f]).max() <= 1e-10 * m, f


def test_level_learned_equals_per_box_learned(level_states):
    """The level's con2prim with the learned guess (one fallback queue for all
    boxes) against per-box mhd_con2prim_learned + mhd_rhs: bitwise."""
    import torch
    from paper_2510_13965_amd import mhd
    from paper_2510_13965_amd.step import LevelRun, PatchRun

    say("case level learned vs per-box learned")
    r = np.random.default_rng(13)
    p = np.zeros(mhd.MLP_NBLOCK, dtype=np.float32)
    p[:mhd.MLP_NPARAM] = r.normal(0.0, 0.05, mhd.MLP_NPARAM)
    p[4866:4874] = 0.0
    p[4874:4882] = 0.2
    p[4864] = 3.0   # bias the guesses towards mu ~ 1/h0, where most points sit
    p[4865] = 3.0
    prm = torch.as_tensor(p).cuda()
    ref = []
    for ip, U in level_states:
        b = PatchRun(ip, U, I.EOS_IDEAL2, I.PARAMS)
        ws = torch.empty((mhd.con2prim_learned_workspace_size(b.patch) + 7) // 8, dtype=torch.float64, device="cuda")
        mhd.con2prim_learned(b.patch, b.eos, prm, b.Un, b.P, ws, b.flags, None, b.stats)
        mhd.rhs(b.patch, b.par, b.eos, b.Un, b.P, b.k, b.vmax, b.ws)
        torch.cuda.synchronize()
        ref.append(dict(k=b.k.cpu().numpy(), P=b.P.cpu().numpy(), flags=b.flags.cpu().numpy(), U=b.Un.cpu().numpy()))
    run = LevelRun([ip for ip, _ in level_states], [U for _, U in level_states], I.EOS_IDEAL2, I.PARAMS)
    run.level.set_learned(prm)
    got, _ = level_rhs(run)
    assert_same(ref, got, "learned")
    fb = np.mean([((g["flags"] & 32) != 0).mean() for g in got])
    say("fallback share with these weights %.3f" % fb)


# ---------------------------------------------------------------- levels with M1

PAR_M1 = dict(I.PARAMS, evolve_m1=1)


@pytest.fixture(scope="module")
def level_m1_states(dev):
    """Six uneven boxes of the star with three grey M1 species (radiation inputs
    following the matter, as on the single patch); cons built on the device."""
    import torch
    from paper_2510_13965_amd import mhd

    boxes = I.amr_level_boxes(seed=I.SEED0 + 31, nboxes=6, edges=(16, 24, 32))
    Ab = I.star_field_amplitude()
    eos = mhd.make_eos(I.EOS_IDEAL2)
    out = []
    for b, box in enumerate(boxes):
        ip, U, P, EM = I.amr_box_state(box, Ab)
        Ud = torch.as_tensor(U).cuda()
        mhd.prim2con(mhd.patch_of(ip), eos, Ud, torch.as_tensor(P).cuda(), torch.as_tensor(EM).cuda(), 0)
        U44, aux = I.m1_fields(ip, Ud.cpu().numpy(), P, I.SEED0 + 310 + b)
        out.append((ip, U44, aux))
    say("level M1 boxes", [ip.n for ip, _, _ in out])
    return out


def m1_level_run(states, **kw):
    from paper_2510_13965_amd.step import LevelRun

    return LevelRun([s[0] for s in states], [s[1] for s in states], I.EOS_IDEAL2, PAR_M1,
                    auxs=[s[2] for s in states], **kw)


def test_level_m1_rhs_bitwise_equals_per_box(level_m1_states):
    import torch
    from paper_2510_13965_amd.step import PatchRun

    say("case level M1 rhs vs per-box, 6 boxes")
    ref, vref = [], 0.0
    for ip, U, aux in level_m1_states:
        r = PatchRun(ip, U, I.EOS_IDEAL2, PAR_M1, aux=aux)
        r.rhs_eval(r.Un)
        torch.cuda.synchronize()
        vref = max(vref, float(r.vmax.item()))
        ref.append(dict(k=r.k.cpu().numpy(), P=r.P.cpu().numpy(), flags=r.flags.cpu().numpy(), U=r.Un.cpu().numpy()))
    for tun in (None, dict(strip=16, block_threads=128, grid_per_cu=4)):
        run = m1_level_run(level_m1_states)
        if tun:
            run.level.set_tuning(**tun)
        got, v = level_rhs(run)
        assert_same(ref, got, "M1 %s" % tun)
        assert v == vref


def test_level_m1_rk4_eager_and_graph_replays(level_m1_states):
    """Two RK4 steps (44 fields) per box, eager level and replayed graph level."""
    import torch
    from paper_2510_13965_amd.step import PatchRun

    say("case level M1 rk4 eager/graph, 6 boxes, 2 steps")
    dt = 0.25 * 0.25
    boxes = [PatchRun(ip, U, I.EOS_IDEAL2, PAR_M1, aux=aux) for ip, U, aux in level_m1_states]
    eager = m1_level_run(level_m1_states)
    graph = m1_level_run(level_m1_states)
    ms_e = torch.zeros(1, dtype=torch.float64, device="cuda")
    ms_g = torch.zeros(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    for step in range(2):
        for r in boxes:
            r.step(dt)
        eager.level.rk4_step(dt, ms_e)
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            graph.level.rk4_step(dt, ms_g, use_graph=True, stream=stream)
        stream.synchronize()
        torch.cuda.synchronize()
        for b, r in enumerate(boxes):
            ref = r.Un.cpu().numpy()
            assert np.isfinite(ref).all()
            assert np.array_equal(ref, eager.boxes[b]["U"].cpu().numpy()), ("eager", step, b)
            assert np.array_equal(ref, graph.boxes[b]["U"].cpu().numpy()), ("graph", step, b)
        assert float(ms_e.item()) == float(ms_g.item()) > 0.0
        say("step", step, "ok, max speed", float(ms_e.item()))


def test_level_m1_box_against_oracle(orc, level_m1_states):
    """The level's coupled RHS with radiation on its smallest box against the
    FP64 oracle (1e-10 per field, all 44 fields)."""
    ip, U, aux = min(level_m1_states, key=lambda s: s[0].npts)
    say("case level M1 box vs oracle", ip.n)
    run = m1_level_run([(ip, U, aux)])
    got, _ = level_rhs(run)
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    e = orc.make_eos(I.EOS_IDEAL2)
    Uo = U.copy()
    Po = np.zeros((I.NP,) + ip.shape)
    orc.con2prim(g, e, Uo, Po, None, None)
    ko = np.zeros_like(U)
    orc.rhs_full(g, orc.make_par(PAR_M1), e, Uo, Po, aux, ko)
    sl = (slice(None),) + ip.interior()
    kg, ko = got[0]["k"][sl], ko[sl]
    for f in range(I.NU_M1):
        m = np.abs(ko[f]).max()
        if m > 0:
            assert np.abs(kg[f] - ko[f]).max() <= 1e-10 * m, f
        else:
            assert np.abs(kg[f]).max() == 0.0, f


def test_level_m1_rejects_missing_aux(level_m1_states):
    from paper_2510_13965_amd import mhd

    say("case level M1 without aux")
    ip, U, aux = level_m1_states[0]
    with pytest.raises(mhd.MhdError, match="aux is required"):
        m1_level_run([(ip, U, None)])


def test_level_imex_bitwise_equals_per_box(level_m1_states):
    """IMEX(4,4,2) steps of the batched level (opacities and emissivities x100,
    kappa dt up to ~8: past the explicit stability limit), eager and as a
    replayed graph, against per-box ImexRun steps: bitwise."""
    import torch
    from paper_2510_13965_amd.step import ImexRun

    say("case level IMEX vs per-box IMEX, 6 boxes, 3 steps")
    dt = 0.25 * 0.25
    states = [(ip, U, aux * 1e2) for ip, U, aux in level_m1_states]
    boxes = [ImexRun(ip, U, aux, I.EOS_IDEAL2, I.PARAMS) for ip, U, aux in states]
    eager = m1_level_run(states, imex=True)
    graph = m1_level_run(states, imex=True)
    ms_e = torch.zeros(1, dtype=torch.float64, device="cuda")
    ms_g = torch.zeros(1, dtype=torch.float64, device="cuda")
    nf_e = torch.zeros(1, dtype=torch.int64, device="cuda")
    nf_g = torch.zeros(1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.Stream()
    for step in range(3):
        for r in boxes:
            r.step(dt)
        eager.level.imex_step(dt, ms_e, nf_e)
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            graph.level.imex_step(dt, ms_g, nf_g, use_graph=True, stream=stream)
        stream.synchronize()
        torch.cuda.synchronize()
        for b, r in enumerate(boxes):
            ref = r.Un.cpu().numpy()
            assert np.isfinite(ref).all()
            assert np.array_equal(ref, eager.boxes[b]["U"].cpu().numpy()), ("eager", step, b)
            assert np.array_equal(ref, graph.boxes[b]["U"].cpu().numpy()), ("graph", step, b)
        if step == 0:
            assert float(ms_e.item()) == max(float(r.vmax.item()) for r in boxes) > 0.0
        assert float(ms_e.item()) == float(ms_g.item())
        nf_ref = sum(int(r.nfail.item()) for r in boxes)
        assert int(nf_e.item()) == int(nf_g.item()) == nf_ref
        say("step", step, "ok, max speed", float(ms_e.item()), "unconverged solves", nf_ref)


def test_level_imex_needs_m1_and_stage_arrays(level_states, level_m1_states):
    from paper_2510_13965_amd import mhd
    from paper_2510_13965_amd.step import LevelRun

    say("case level IMEX argument checks")
    run = LevelRun([s[0] for s in level_states[:1]], [s[1] for s in level_states[:1]], I.EOS_IDEAL2, I.PARAMS)
    with pytest.raises(mhd.MhdError, match="must evolve M1"):
        run.level.set_imex([([None] * 4, [None] * 4)])
    m1 = m1_level_run(level_m1_states[:1])
    with pytest.raises(mhd.MhdError, match="no IMEX stage arrays"):
        m1.level.imex_step(0.0625)
