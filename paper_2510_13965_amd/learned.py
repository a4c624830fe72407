"""Training driver of the learned con2prim starting guess.

Every arithmetic step runs in the library's HIP kernels (prim->cons, the plain
con2prim that provides the target roots, features, normalisation, forward and
backward passes, Adam); this module only allocates device buffers and loops
over mini-batches.  The initial weights are seeded random numbers drawn here
(He-uniform) and passed in.
"""
import numpy as np

from . import inputs as I
from . import mhd


def init_params(seed):
    """Parameter block (float32 numpy, MHD_MLP_NBLOCK) with He-uniform weights,
    zero biases, and identity feature normalisation."""
    r = np.random.Generator(np.random.Philox(seed))
    p = np.zeros(mhd.MLP_NBLOCK, dtype=np.float32)

    def he(shape, fan_in):
        b = np.sqrt(6.0 / fan_in)
        return r.uniform(-b, b, shape).astype(np.float32)

    p[0:512] = he(512, 8)
    p[576:4672] = he(4096, 64)
    p[4736:4864] = he(128, 64) * 0.1
    p[4874:4882] = 1.0
    return p


# sampling of the star workloads (ideal gas, static to mildly relativistic flow,
# weak fields, the star's density range and its atmosphere)
STAR_SAMPLING = dict(log_rho=(-12.0, -2.5), log_eps=(-11.0, 0.0), log_sigma=(-7.0, -1.0), log_wm1=(-14.0, -1.0),
                     static_frac=0.1)


def training_set(ncell, seed, eos_cfg=I.EOS_PWP3, device="cuda", **sampling):
    """(X, T) device tensors for `ncell` random con2prim states: raw features of
    the conserved state and the targets (log fractions of the plain solver's roots
    less their closed-form baselines).
    Rows of atmosphere states are NaN (skipped by the kernels).  `sampling`
    overrides the state distribution (inputs.c2p_cells)."""
    import torch

    ip, U, P, EM = I.c2p_cells(seed=seed, ncell=ncell, **sampling)
    pt = mhd.patch_of(ip)
    eos = mhd.make_eos(eos_cfg)
    Ud = torch.as_tensor(U).to(device)
    Pd = torch.as_tensor(P).to(device)
    EMd = torch.as_tensor(EM).to(device)
    mhd.prim2con(pt, eos, Ud, Pd, EMd, 1)
    Uc = Ud.clone()
    mu = torch.zeros((2,) + ip.shape, dtype=torch.float64, device=device)
    mhd.con2prim(pt, eos, Uc, torch.empty_like(Pd), None, mu, None)
    X = torch.empty((ip.npts, 8), dtype=torch.float32, device=device)
    T = torch.empty((ip.npts, 2), dtype=torch.float32, device=device)
    mhd.mlp_features(pt, eos, Ud, X, mu, T)
    return X, T


def train(X, T, seed=1, epochs=30, batch=4096, lr=3e-3, lr_final=2e-4, params=None):
    """Adam on mini-batches of consecutive rows (rows are i.i.d. draws); the
    learning rate decays geometrically from lr to lr_final.  Returns the
    parameter block (device float32) and the per-epoch mean loss."""
    import torch

    dev = X.device
    n = X.shape[0]
    p = torch.as_tensor(init_params(seed) if params is None else params).to(dev)
    mhd.mlp_normalize(p, X)
    grad = torch.zeros(mhd.MLP_NPARAM, dtype=torch.float32, device=dev)
    m = torch.zeros_like(grad)
    v = torch.zeros_like(grad)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    ws = torch.empty((mhd.mlp_grad_workspace_size(batch) + 3) // 4, dtype=torch.float32, device=dev)
    nb = max(1, n // batch)
    total = epochs * nb
    hist = []
    step = 0
    for ep in range(epochs):
        acc = torch.zeros(1, dtype=torch.float32, device=dev)
        for b in range(nb):
            step += 1
            rate = lr * (lr_final / lr) ** ((step - 1) / max(1, total - 1))
            Xb = X[b * batch:(b + 1) * batch]
            Tb = T[b * batch:(b + 1) * batch]
            mhd.mlp_grad(p, Xb, Tb, grad, ws, loss)
            mhd.mlp_adam(p, grad, m, v, step, rate)
            acc += loss
        hist.append(float(acc.item()) / nb)
    return p, hist
