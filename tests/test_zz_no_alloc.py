"""The allocation-free con2prim entry point (mhd_con2prim_learned_noalloc)
against mhd_con2prim_learned on the same inputs: two calls in a row on one
device, the second on a smaller patch, every output bitwise equal (same
kernels; the shared queue is cleared at the start of each call)."""
import sys

import numpy as np
import pytest

from paper_2510_13965_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rand_params(seed, scale):
    r = np.random.default_rng(seed)
    p = np.zeros(4882, dtype=np.float32)
    p[:4866] = r.normal(0.0, scale, 4866)
    p[4866:4874] = r.normal(0.0, 1.0, 8)
    p[4874:4882] = r.uniform(0.5, 2.0, 8)
    return p


def cells(shape, seed):
    import torch
    from paper_2510_13965_amd import mhd

    n = int(np.prod(shape))
    ip, U, P, EM = I.c2p_cells(ncell=n, shape=shape, seed=seed)
    pt = mhd.patch_of(ip)
    Ud = torch.as_tensor(U).cuda()
    mhd.prim2con(pt, mhd.make_eos(I.EOS_PWP3), Ud, torch.as_tensor(P).cuda(), torch.as_tensor(EM).cuda(), 1)
    return ip, pt, Ud


def run(pt, ip, U0, prm, noalloc):
    import torch
    from paper_2510_13965_amd import mhd

    eos = mhd.make_eos(I.EOS_PWP3)
    U = U0.clone()
    P = torch.full((I.NP,) + ip.shape, -1.0, dtype=torch.float64, device="cuda")
    fl = torch.full(ip.shape, 255, dtype=torch.uint8, device="cuda")
    mu = torch.full((2,) + ip.shape, -1.0, dtype=torch.float64, device="cuda")
    st = torch.zeros(mhd.MHD_NSTAT, dtype=torch.int64, device="cuda")
    if noalloc:
        mhd.con2prim_learned_noalloc(pt, eos, prm, U, P, fl, mu, st)
    else:
        ws = torch.empty((mhd.con2prim_learned_workspace_size(pt) + 7) // 8, dtype=torch.float64, device="cuda")
        mhd.con2prim_learned(pt, eos, prm, U, P, ws, fl, mu, st)
    torch.cuda.synchronize()
    return [a.cpu().numpy() for a in (U, P, fl, mu, st)]


@pytest.mark.parametrize("scale", [0.05, 0.0])
def test_noalloc_equals_workspace_entry(scale):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    prm = torch.as_tensor(rand_params(21, scale)).cuda()
    # a large call first (many fallbacks fill the shared queue), then a smaller one
    for shape, seed in (((64, 64, 32), I.SEED0 + 61), ((24, 16, 8), I.SEED0 + 62)):
        say("case no-alloc con2prim, scale %g, shape %s" % (scale, shape))
        ip, pt, U0 = cells(shape, seed)
        a = run(pt, ip, U0, prm, noalloc=False)
        b = run(pt, ip, U0, prm, noalloc=True)
        for name, x, y in zip(("U", "P", "flags", "mu", "stats"), a, b):
            assert np.array_equal(x, y, equal_nan=True), name
        fb = a[4][2]
        say("  fallback points %d of %d" % (fb, np.prod(shape)))
        assert fb > 0


def test_noalloc_rejects_oversized_patch():
    import torch
    from paper_2510_13965_amd import mhd

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pt = mhd.make_patch((156, 156, 156), (0.1, 0.1, 0.1), ng=3)
    x = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(mhd.MhdError, match="at most"):
        mhd.con2prim_learned_noalloc(pt, mhd.make_eos(I.EOS_PWP3), x, x, x)
