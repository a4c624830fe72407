"""Seeded synthetic inputs for the MoL right-hand side.

This module builds *inputs only*: spacetime fields, primitive fluid fields and
magnetic fields on padded patches, and the parameter sets of the workloads.  It
contains none of the method's arithmetic (no cons/prim conversion, no RHS, no
EoS evaluation beyond the polytropic initial-data relation); both the HIP path
and the CPU oracle start from what it returns.

Array layout everywhere: numpy float64, shape (nfields, Nz, Ny, Nx) over the
padded patch (N = n + 2*ng per axis), x fastest.

Workloads (seeds 2510139650 + k):
  * perturbed flat patch: 32^3 interior, dx = 0.25, periodic; Minkowski plus
        Gaussian bumps of amplitude 1e-6 in the conformal metric and the lapse;
        ideal gas Gamma=2, rho=1e-3, eps=0.1, velocity bumps of 1e-3, uniform B^z
        with b^2/rho=0.01.  ``perturbed_flat_state(rich=True)`` also perturbs
        Khat, Theta, At_ij, Ghat^i and beta^i so that every term (both upwind
        branches included) is exercised.
  * TOV star patch: 128^3 interior, dx = 0.25 on [-16,16]^3; K=100, Gamma=2,
        rho_c=1.28e-3 in isotropic coordinates; poloidal B from
        A_phi ~ varpi^2 max(p - 0.04 p_max, 0)^2 scaled to max b^2/rho = 1e-3;
        atmosphere rho = 1e-12.
  * AMR level: 192 boxes, edges from {16,24,32,48,64}, three 2:1 levels,
        sampled from the star profile.
  * random con2prim cells: 2^24 cells of random (rho, eps_th, W, sigma_m,
        metric) states for the 3-piece piecewise polytrope + thermal EoS.
  * three grey M1 species on any of the patches (m1_fields).
"""
import math

import numpy as np

SEED0 = 2510139650

# field indices of the evolved vector U
GT = (0, 1, 2, 3, 4, 5)          # gt_xx, gt_xy, gt_xz, gt_yy, gt_yz, gt_zz
AT = (6, 7, 8, 9, 10, 11)
CHI, KHAT, THETA = 12, 13, 14
GHAT = (15, 16, 17)
ALPHA = 18
BETA = (19, 20, 21)
DBAR, DYBAR, TAUBAR = 22, 23, 24
SBAR = (25, 26, 27)
BBAR = (28, 29, 30)
PHIBAR = 31
NST, NMHD, NU = 22, 10, 32
# primitive slots
RHO, EPS, PRESS, VX, VY, VZ, WLOR, YE = range(8)
NP = 8
# EM slots (undensitized B^i and phi)
NEM = 4

EOS_IDEAL2 = dict(K0=0.0, Gamma=[2.0], rho_b=[], Gamma_th=2.0,
                  rho_atm=1e-12, rho_min=1.1e-12, rho_max=1.0, eps_max=1e3, W_max=50.0,
                  rho_low=1e-8, alpha_bh=0.2, h0=1.0, ye_min=0.0, ye_max=0.6, ye_atm=0.1)

# three-piece cold polytrope (the middle piece is the K=100, Gamma=2 polytrope)
EOS_PWP3 = dict(K0=0.01, Gamma=[4.0 / 3.0, 2.0, 2.75], rho_b=[1e-6, 1e-4], Gamma_th=1.8,
                rho_atm=1e-12, rho_min=1.1e-12, rho_max=1.0, eps_max=1e3, W_max=50.0,
                rho_low=1e-8, alpha_bh=0.2, h0=1.0, ye_min=0.0, ye_max=0.6, ye_atm=0.1)

PARAMS = dict(kappa_z=0.5, kappa_c=0.05, kappa_2=0.0, eta=1.4, beta0=[0.0, 0.0, 0.0],
              sigma_ko=0.1, c_b=1.0, kappa_b=1.0, alpha_mp5=4.0, f_beta=1.0, f_alpha_kind=0,
              evolve_st=1, evolve_mhd=1, couple_matter=1)


def rng(seed):
    return np.random.Generator(np.random.Philox(seed))


class Patch:
    """Geometry of one vertex-centred patch; coordinate of padded index i is
    x0 + (i - ng) * dx."""

    def __init__(self, n, dx, x0, ng=3):
        self.n = tuple(int(v) for v in n)
        self.dx = tuple(float(v) for v in dx)
        self.x0 = tuple(float(v) for v in x0)
        self.ng = int(ng)

    @property
    def shape(self):  # (Nz, Ny, Nx)
        return tuple(self.n[2 - a] + 2 * self.ng for a in range(3))

    @property
    def npts(self):
        s = self.shape
        return s[0] * s[1] * s[2]

    @property
    def ninterior(self):
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def nhalo1(self):
        """Points of the interior with one ghost layer."""
        return (self.n[0] + 2) * (self.n[1] + 2) * (self.n[2] + 2)

    def coords(self):
        """Z, Y, X coordinate arrays of shape (Nz, Ny, Nx)."""
        ax = [self.x0[a] + (np.arange(self.n[a] + 2 * self.ng) - self.ng) * self.dx[a]
              for a in range(3)]
        Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        return Z, Y, X

    def interior(self):
        g = self.ng
        return (slice(g, g + self.n[2]), slice(g, g + self.n[1]), slice(g, g + self.n[0]))


def empty_state(patch):
    U = np.zeros((NU,) + patch.shape)
    P = np.zeros((NP,) + patch.shape)
    EM = np.zeros((NEM,) + patch.shape)
    return U, P, EM


def flat_spacetime(U):
    for a in (0, 3, 5):
        U[GT[a]] = 1.0
    U[CHI] = 1.0
    U[ALPHA] = 1.0


# ----------------------------------------------------------------------- perturbed flat patch

def _bumps(r, patch, X, Y, Z, amp, count=4):
    """Sum of `count` Gaussians (minimum-image periodic distance, width L/10),
    amplitudes uniform in [-amp, amp], centres uniform in the periodic box."""
    L = [patch.n[a] * patch.dx[a] for a in range(3)]
    w = min(L) / 10.0
    out = np.zeros_like(X)
    for _ in range(count):
        c = [patch.x0[a] + r.uniform(0, L[a]) for a in range(3)]
        A = r.uniform(-amp, amp)
        d2 = 0.0
        for a, Q in enumerate((X, Y, Z)):
            d = Q - c[a]
            d = d - L[a] * np.round(d / L[a])
            d2 = d2 + d * d
        out += A * np.exp(-d2 / (2 * w * w))
    return out


def perturbed_flat_state(seed=SEED0 + 1, n=32, rich=False):
    patch = Patch((n, n, n), (0.25,) * 3, (0.0,) * 3)
    r = rng(seed)
    Z, Y, X = patch.coords()
    U, P, EM = empty_state(patch)
    flat_spacetime(U)
    for c in GT:
        U[c] += _bumps(r, patch, X, Y, Z, 1e-6)
    U[ALPHA] += _bumps(r, patch, X, Y, Z, 1e-6)
    if rich:
        for c in AT + (KHAT, THETA) + GHAT:
            U[c] += _bumps(r, patch, X, Y, Z, 1e-6)
        U[CHI] += _bumps(r, patch, X, Y, Z, 1e-6)
        for c in BETA:
            U[c] += _bumps(r, patch, X, Y, Z, 1e-3)
    P[RHO] = 1e-3
    P[EPS] = 0.1
    for c in (VX, VY, VZ):
        P[c] = _bumps(r, patch, X, Y, Z, 1e-3)
    P[YE] = 0.1
    EM[2] = math.sqrt(0.01 * 1e-3)
    if rich:
        EM[0] = _bumps(r, patch, X, Y, Z, 1e-4)
        EM[3] = _bumps(r, patch, X, Y, Z, 1e-5)
    return patch, U, P, EM


# ----------------------------------------------------------------------- TOV

class TOV:
    """Static spherical polytrope p = K rho^Gamma in isotropic coordinates.

    Integrates the Tolman-Oppenheimer-Volkoff equations in the areal radius r
    together with the isotropic radius rbar (d ln rbar/dr = 1/(r sqrt(1-2m/r)))
    and the lapse potential Phi, then matches to exterior Schwarzschild."""

    def __init__(self, K=100.0, Gamma=2.0, rho_c=1.28e-3, npts=20001):
        from scipy.integrate import solve_ivp

        self.K, self.G, self.rho_c = K, Gamma, rho_c

        def rho_of_p(p):
            return (max(p, 0.0) / K) ** (1.0 / Gamma)

        def e_of_p(p):
            rho = rho_of_p(p)
            return rho + K * rho ** Gamma / (Gamma - 1.0)

        def f(r, y):
            m, p, phi, lnrb = y
            e = e_of_p(p)
            den = r * (r - 2.0 * m)
            dp = -(e + p) * (m + 4 * math.pi * r ** 3 * p) / den
            return [4 * math.pi * r * r * e, dp, (m + 4 * math.pi * r ** 3 * p) / den,
                    1.0 / (r * math.sqrt(1.0 - 2.0 * m / r))]

        def surface(r, y):
            return y[1] - 1e-14 * K * rho_c ** Gamma

        surface.terminal = True
        surface.direction = -1
        r0 = 1e-6
        pc = K * rho_c ** Gamma
        y0 = [4.0 / 3.0 * math.pi * r0 ** 3 * e_of_p(pc), pc, 0.0, math.log(r0)]
        sol = solve_ivp(f, (r0, 100.0), y0, events=surface, rtol=1e-12, atol=1e-16,
                        dense_output=True, method="DOP853", max_step=0.01)
        R = float(sol.t_events[0][0])
        M = float(sol.y_events[0][0][0])
        r = np.linspace(r0, R, npts)
        y = sol.sol(r)
        rbs = 0.5 * (R - M + math.sqrt(R * R - 2 * M * R))   # isotropic surface radius
        lnrb = y[3] - y[3][-1] + math.log(rbs)
        phi = y[2] - y[2][-1] + 0.5 * math.log(1 - 2 * M / R)
        self.R, self.M, self.rbar_s = R, M, rbs
        self.r_tab = r
        self.rbar_tab = np.exp(lnrb)
        self.psi2_tab = r / self.rbar_tab
        self.alpha_tab = np.exp(phi)
        self.p_tab = np.maximum(y[1], 0.0)
        self.p_max = pc

    def profile(self, rbar):
        """psi^4, alpha, rho, p at isotropic radii rbar (array)."""
        rb = np.asarray(rbar, dtype=np.float64)
        inside = rb < self.rbar_s
        rbi = np.clip(rb, self.rbar_tab[0], self.rbar_s)
        psi2_in = np.interp(rbi, self.rbar_tab, self.psi2_tab)
        alpha_in = np.interp(rbi, self.rbar_tab, self.alpha_tab)
        p_in = np.interp(rbi, self.rbar_tab, self.p_tab)
        q = self.M / (2.0 * np.maximum(rb, 1e-300))
        psi_out = 1.0 + q
        alpha_out = (1.0 - q) / (1.0 + q)
        psi4 = np.where(inside, psi2_in ** 2, psi_out ** 4)
        alpha = np.where(inside, alpha_in, alpha_out)
        p = np.where(inside, p_in, 0.0)
        rho = (p / self.K) ** (1.0 / self.G)
        return psi4, alpha, rho, p


_TOV_CACHE = {}


def tov_default():
    if "c2" not in _TOV_CACHE:
        _TOV_CACHE["c2"] = TOV()
    return _TOV_CACHE["c2"]


def _curl4(A, dx, trim):
    """4th-order centred curl of the covariant potential A (3, Nz, Ny, Nx) on a
    grid with `trim` extra layers; returns (3, ...) trimmed by `trim`."""

    def d(f, axis, h):
        return (8.0 * (np.roll(f, -1, axis) - np.roll(f, 1, axis))
                - (np.roll(f, -2, axis) - np.roll(f, 2, axis))) / (12.0 * h)

    ax = {0: 2, 1: 1, 2: 0}   # x -> last array axis
    Ax, Ay, Az = A
    hx, hy, hz = dx
    cx = d(Az, ax[1], hy) - d(Ay, ax[2], hz)
    cy = d(Ax, ax[2], hz) - d(Az, ax[0], hx)
    cz = d(Ay, ax[0], hx) - d(Ax, ax[1], hy)
    s = (slice(trim, -trim),) * 3
    return np.stack([cx[s], cy[s], cz[s]])


def star_fields(patch, tov=None, b_axis=(0.0, 0.0, 1.0), Ab=None, bmag=1e-3, rho_atm=1e-12):
    """Spacetime, primitive and magnetic fields of the TOV star on `patch`.

    Returns U (spacetime part set), P (rho, eps, v=0, Ye), EM (B^i, phi=0) and the
    field amplitude Ab used (so that boxes of other patches can share it)."""
    tov = tov or tov_default()
    U, P, EM = empty_state(patch)
    Z, Y, X = patch.coords()
    rb = np.sqrt(X * X + Y * Y + Z * Z)
    psi4, alpha, rho, p = tov.profile(rb)
    for a in (0, 3, 5):
        U[GT[a]] = 1.0
    U[CHI] = 1.0 / psi4
    U[ALPHA] = alpha
    inside = rho > rho_atm
    rho = np.where(inside, rho, rho_atm)
    P[RHO] = rho
    P[EPS] = tov.K * rho ** (tov.G - 1.0) / (tov.G - 1.0)
    P[YE] = 0.1

    # poloidal field from A_k = Ab max(p - 0.04 p_max, 0)^2 (n x x)_k on a grid
    # with two extra layers, B^i = curl(A)^i / sqrt(gamma), sqrt(gamma) = psi^6
    big = Patch(patch.n, patch.dx, patch.x0, patch.ng + 2)
    Zb, Yb, Xb = big.coords()
    _, _, _, pb = tov.profile(np.sqrt(Xb * Xb + Yb * Yb + Zb * Zb))
    w = np.maximum(pb - 0.04 * tov.p_max, 0.0) ** 2
    n = np.asarray(b_axis, dtype=np.float64)
    n = n / np.linalg.norm(n)
    A = np.stack([w * (n[1] * Zb - n[2] * Yb), w * (n[2] * Xb - n[0] * Zb), w * (n[0] * Yb - n[1] * Xb)])
    curl = _curl4(A, patch.dx, 2)
    B = curl / psi4 ** 1.5
    if Ab is None:
        b2 = psi4 * (B[0] ** 2 + B[1] ** 2 + B[2] ** 2)
        ratio = np.where(inside, b2 / rho, 0.0)
        Ab = math.sqrt(bmag / ratio.max()) if ratio.max() > 0 else 0.0
    EM[0:3] = Ab * B
    return U, P, EM, Ab


def tov_star_state(seed=SEED0 + 2, n=128):
    r = rng(seed)
    L = 32.0
    dx = L / n
    patch = Patch((n, n, n), (dx,) * 3, (-L / 2 + dx / 2,) * 3)
    # seeded tilt of the magnetic axis, within 0.3 rad of z
    th = r.uniform(0.0, 0.3)
    ph = r.uniform(0.0, 2 * math.pi)
    axis = (math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th))
    U, P, EM, Ab = star_fields(patch, b_axis=axis)
    return patch, U, P, EM


# ----------------------------------------------------------------------- AMR level

def amr_level_boxes(seed=SEED0 + 3, nboxes=192, edges=(16, 24, 32, 48, 64)):
    """Box list of a batched AMR level: per box (n, dx, x0, level).

    Level l has dx = 1/2^l; the origin of a box is snapped to its own grid, and
    level-l boxes sit inside [-16,16]^3 scaled by 2^-l (2:1 nesting)."""
    r = rng(seed)
    boxes = []
    for _ in range(nboxes):
        lev = int(r.integers(0, 3))
        dx = 1.0 / 2 ** lev
        n = tuple(int(edges[r.integers(0, len(edges))]) for _ in range(3))
        half = 16.0 * 2.0 ** (-lev) * 2.0   # level extent: 32, 16, 8 (half-widths)
        x0 = []
        for a in range(3):
            ext = n[a] * dx
            lo, hi = -half, max(-half, half - ext)
            x0.append(dx * math.floor(r.uniform(lo, hi) / dx) + 0.5 * dx)
        boxes.append(dict(n=n, dx=(dx,) * 3, x0=tuple(x0), level=lev))
    return boxes


def level_subset(nboxes, k=16, seed=SEED0 + 6):
    """Seeded subset of k box indices (sorted) of a level of nboxes boxes: the
    boxes the oracle runs for the level workloads' CPU figures and sampled
    parity checks."""
    r = rng(seed)
    return sorted(int(i) for i in r.choice(nboxes, size=min(k, nboxes), replace=False))


def amr_box_state(box, Ab):
    patch = Patch(box["n"], box["dx"], box["x0"])
    U, P, EM, _ = star_fields(patch, Ab=Ab)
    return patch, U, P, EM


def star_field_amplitude():
    """Magnetic amplitude of the star (shared by the AMR-level boxes)."""
    if "Ab" not in _TOV_CACHE:
        _, _, _, Ab = star_fields(Patch((32, 32, 32), (1.0,) * 3, (-15.5,) * 3))
        _TOV_CACHE["Ab"] = Ab
    return _TOV_CACHE["Ab"]


# ----------------------------------------------------------------------- random con2prim cells

def c2p_cells(seed=SEED0 + 4, ncell=1 << 24, shape=None, log_rho=(-12.0, -3.0), log_eps=(-6.0, 0.0),
             log_sigma=(-4.0, 1.0), log_wm1=None, static_frac=0.0):
    """Random con2prim states laid out as a ghost-free patch.

    rho log-uniform [1e-12, 1e-3]; thermal specific energy log-uniform
    [1e-6, 1] (added to the cold part by the prim->cons map so every state is
    inside the EoS validity region); W uniform [1, 10]; magnetisation
    sigma = b^2/rho log-uniform [1e-4, 10]; random unit directions of v and B
    in the physical metric; gamma_ij = psi^4 (delta_ij + h_ij), psi^4 in [1,2],
    |h_ij| <= 0.1; alpha in [0.5, 1], |beta| <= 0.3 (unused by con2prim).
    The ranges (log10 bounds) can be changed; log_wm1 = (lo, hi) draws W - 1
    log-uniform instead, and a fraction static_frac of the states gets v = 0."""
    if shape is None:
        shape = (ncell, 1, 1)
    nx, ny, nz = shape
    assert nx * ny * nz == ncell
    patch = Patch((nx, ny, nz), (1.0,) * 3, (0.0,) * 3, ng=0)
    r = rng(seed)
    sh = patch.shape
    U, P, EM = empty_state(patch)
    psi4 = r.uniform(1.0, 2.0, sh)
    h = r.uniform(-0.1, 0.1, (6,) + sh)
    g = np.empty((3, 3) + sh)
    idx = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 1): 3, (1, 2): 4, (2, 2): 5}
    for (i, j), c in idx.items():
        g[i, j] = psi4 * ((1.0 if i == j else 0.0) + h[c])
        g[j, i] = g[i, j]
    det = (g[0, 0] * (g[1, 1] * g[2, 2] - g[1, 2] * g[2, 1]) - g[0, 1] * (g[1, 0] * g[2, 2] - g[1, 2] * g[2, 0])
           + g[0, 2] * (g[1, 0] * g[2, 1] - g[1, 1] * g[2, 0]))
    chi = det ** (-1.0 / 3.0)
    for (i, j), c in idx.items():
        U[GT[c]] = chi * g[i, j]
    U[CHI] = chi
    U[ALPHA] = r.uniform(0.5, 1.0, sh)
    bdir = r.normal(size=(3,) + sh)
    bdir /= np.linalg.norm(bdir, axis=0)
    bmag = r.uniform(0.0, 0.3, sh)
    for a in range(3):
        U[BETA[a]] = bmag * bdir[a]

    def unit_dir():
        d = r.normal(size=(3,) + sh)
        nrm = np.sqrt(np.einsum("i...,ij...,j...->...", d, g, d))
        return d / nrm

    rho = 10.0 ** r.uniform(log_rho[0], log_rho[1], sh)
    epsth = 10.0 ** r.uniform(log_eps[0], log_eps[1], sh)
    if log_wm1 is None:
        W = r.uniform(1.0, 10.0, sh)
    else:
        W = 1.0 + 10.0 ** r.uniform(log_wm1[0], log_wm1[1], sh)
    if static_frac > 0.0:
        W = np.where(r.uniform(0.0, 1.0, sh) < static_frac, 1.0, W)
    sig = 10.0 ** r.uniform(log_sigma[0], log_sigma[1], sh)
    vdir = unit_dir()
    vmag = np.sqrt(1.0 - 1.0 / (W * W))
    v = vmag * vdir
    bd = unit_dir()
    # b^2 = B^2/W^2 + (B.v)^2 = |B|^2 (1/W^2 + (bd.v)^2) = sigma rho
    bv = np.einsum("i...,ij...,j...->...", bd, g, v)
    Bm = np.sqrt(sig * rho / (1.0 / (W * W) + bv * bv))
    P[RHO] = rho
    P[EPS] = epsth
    P[VX], P[VY], P[VZ] = v
    P[YE] = 0.1
    EM[0:3] = Bm * bd
    return patch, U, P, EM


# ----------------------------------------------------------------------- M1 radiation

NU_M1 = 44       # evolved fields with three M1 species
NAUX = 9         # kappa_a, kappa_s, eta per species
NU_M1N = 47      # with the three neutrino number densities Nbar (fields 44..46)
NAUX_N = 15      # and per species the number opacity kappa0_a (9 + 2 s) and emissivity eta0 (10 + 2 s)


def _smooth01(r, patch, X, Y, Z, count=4):
    """Sum of `count` Gaussian bumps (width a quarter of the patch) scaled to [0, 1]."""
    L = [patch.n[a] * patch.dx[a] for a in range(3)]
    w = min(L) / 4.0
    f = np.zeros_like(X)
    for _ in range(count):
        c = [patch.x0[a] + r.uniform(0, L[a]) for a in range(3)]
        A = r.uniform(0.2, 1.0)
        f += A * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / (2 * w * w))
    lo, hi = f.min(), f.max()
    return (f - lo) / (hi - lo) if hi > lo else np.zeros_like(f)


def m1_fields(patch, U32, P, seed):
    """Three grey species on `patch`: returns U with 44 fields (U32 extended by
    Ebar, Fbar_i per species) and the 9 aux fields (kappa_a, kappa_s, eta).

    Ebar = 10^(-10 + 6 s(x)) with s a smooth field in [0, 1] (so Ebar spans
    [1e-10, 1e-4]); Fbar_i = f(x) Ebar d_i/|d| with d a smooth direction field
    and f = 0.95 (w s'(x) + 1 - w), s' smooth in [0, 1] and w = min(rho/1e-4, 1):
    random flux factors in dense matter, near free streaming where it thins out (|F|/E <= 0.95 wherever chi <= 1 and the conformal
    metric is flat, as on the star and the perturbed flat patches).
    Opacities scale with the density, as matter opacities do: kappa_a, kappa_s
    = khat rho / 1e-3 with khat log-uniform in [1e-3, 1] per point and species
    (so radiation streams freely through the atmosphere and kappa dt stays
    well inside the explicit RK4 stability interval at the star's densities);
    eta = kappa_a E_eq with E_eq = 1e-2 rho eps."""
    R, aux = m1_radiation(patch, P, seed)
    U = np.empty((NU_M1,) + patch.shape)
    U[:NU] = U32[:NU]
    U[NU:] = R
    return U, aux


def m1_radiation(patch, P, seed):
    """The radiation part of m1_fields alone: the 12 fields Ebar, Fbar_i of the
    three species (in U order from field 32) and the 9 aux fields; they depend
    on the primitives P and the seed only."""
    r = rng(seed)
    Z, Y, X = patch.coords()
    R = np.zeros((NU_M1 - NU,) + patch.shape)
    aux = np.zeros((NAUX,) + patch.shape)
    for s in range(3):
        Eb = 10.0 ** (-10.0 + 6.0 * _smooth01(r, patch, X, Y, Z))
        # free streaming (|F|/E -> 0.95) where the matter thins out
        wm = np.minimum(P[RHO] / 1e-4, 1.0)
        frac = 0.95 * (wm * _smooth01(r, patch, X, Y, Z) + (1.0 - wm))
        d = np.array([2.0 * _smooth01(r, patch, X, Y, Z) - 1.0 for _ in range(3)]) + 1e-3
        d /= np.sqrt((d * d).sum(0))
        R[4 * s] = Eb
        for a in range(3):
            R[4 * s + 1 + a] = frac * Eb * d[a]
        ka = 10.0 ** r.uniform(-3.0, 0.0, patch.shape) * (P[RHO] / 1e-3)
        ks = 10.0 ** r.uniform(-3.0, 0.0, patch.shape) * (P[RHO] / 1e-3)
        aux[3 * s] = ka
        aux[3 * s + 1] = ks
        aux[3 * s + 2] = ka * 1e-2 * P[RHO] * P[EPS]
    return R, aux


def m1n_fields(patch, U44, aux9, seed):
    """The three neutrino number densities on top of m1_fields' radiation:
    returns U with 47 fields (Nbar of species s at 44 + s) and 15 aux fields
    (kappa0_a at 9 + 2 s, eta0 at 10 + 2 s after the 9 energy ones).

    Nbar = Ebar / e_mean with a smooth mean neutrino energy e_mean =
    10^(-1.5 + s(x)) (s smooth in [0, 1]); kappa0_a = kappa_a 10^u with u
    uniform in [-0.5, 0.5] per point; eta0 = kappa0_a E_eq / e_mean with the
    energy moments' E_eq = eta / kappa_a (where kappa_a = 0, eta0 = 0)."""
    r = rng(seed)
    Z, Y, X = patch.coords()
    U = np.empty((NU_M1N,) + patch.shape)
    U[:NU_M1] = U44[:NU_M1]
    aux = np.zeros((NAUX_N,) + patch.shape)
    aux[:NAUX] = aux9[:NAUX]
    for sp in range(3):
        emean = 10.0 ** (-1.5 + _smooth01(r, patch, X, Y, Z))
        U[NU_M1 + sp] = U44[32 + 4 * sp] / emean
        ka, eta = aux9[3 * sp], aux9[3 * sp + 2]
        k0 = ka * 10.0 ** r.uniform(-0.5, 0.5, patch.shape)
        Eeq = np.divide(eta, ka, out=np.zeros_like(eta), where=ka > 0)
        aux[9 + 2 * sp] = k0
        aux[10 + 2 * sp] = k0 * Eeq / emean
    return U, aux
