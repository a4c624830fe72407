"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py may
import this module.  Arrays are numpy float64, C-contiguous, laid out as
(field, z, y, x) over the padded patch.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class Grid(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("ng", C.c_int), ("dx", C.c_double * 3)]


class Eos(C.Structure):
    _fields_ = [("npieces", C.c_int), ("K", C.c_double * 4), ("Gamma", C.c_double * 4),
                ("rho_b", C.c_double * 3), ("a", C.c_double * 4), ("Gamma_th", C.c_double),
                ("rho_atm", C.c_double), ("rho_min", C.c_double), ("rho_max", C.c_double),
                ("eps_max", C.c_double), ("W_max", C.c_double), ("rho_low", C.c_double),
                ("alpha_bh", C.c_double), ("h0", C.c_double), ("ye_min", C.c_double),
                ("ye_max", C.c_double), ("ye_atm", C.c_double)]


class Par(C.Structure):
    _fields_ = [("kappa_z", C.c_double), ("kappa_c", C.c_double), ("kappa_2", C.c_double),
                ("eta", C.c_double), ("beta0", C.c_double * 3), ("sigma_ko", C.c_double),
                ("c_b", C.c_double), ("kappa_b", C.c_double), ("alpha_mp5", C.c_double),
                ("f_beta", C.c_double), ("f_alpha_kind", C.c_int), ("evolve_st", C.c_int),
                ("evolve_mhd", C.c_int), ("couple_matter", C.c_int), ("evolve_m1", C.c_int),
                ("evolve_m1n", C.c_int), ("m_b", C.c_double), ("les_cm", C.c_double),
                ("couple_exchange", C.c_int)]


_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_u8p = C.POINTER(C.c_uint8)


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liborc.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        _LIB = _bind(C.CDLL(path))
    return _LIB


def use_library(path):
    """Bind this module to another build of the same sources (the op-counting
    build of opcount.py); returns the previous library."""
    global _LIB
    old = _LIB
    _LIB = _bind(C.CDLL(path))
    return old


def _bind(L):
    L.orc_eos_init_pwp.argtypes = [C.POINTER(Eos), C.c_int, C.c_double, _dp, _dp, C.c_double]
    L.orc_eps_cold.argtypes = [C.POINTER(Eos), C.c_double]
    L.orc_eps_cold.restype = C.c_double
    L.orc_press.argtypes = [C.POINTER(Eos), C.c_double, C.c_double]
    L.orc_press.restype = C.c_double
    L.orc_cs2.argtypes = [C.POINTER(Eos), C.c_double, C.c_double]
    L.orc_cs2.restype = C.c_double
    for name in ("orc_d1", "orc_d2", "orc_ko"):
        getattr(L, name).restype = C.c_double
    L.orc_d1.argtypes = [_dp, C.c_int64, C.c_int64, C.c_double]
    L.orc_d2.argtypes = [_dp, C.c_int64, C.c_int64, C.c_double]
    L.orc_d11.argtypes = [_dp, C.c_int64, C.c_int64, C.c_int64, C.c_double, C.c_double]
    L.orc_d11.restype = C.c_double
    L.orc_dup.argtypes = [_dp, C.c_int64, C.c_int64, C.c_double, C.c_double]
    L.orc_dup.restype = C.c_double
    L.orc_ko.argtypes = [_dp, C.c_int64, C.c_int64, C.c_double, C.c_double]
    L.orc_mp5.argtypes = [_dp, C.c_double]
    L.orc_mp5.restype = C.c_double
    L.orc_prim2con.argtypes = [C.POINTER(Grid), C.POINTER(Eos), _dp, _dp, _dp, C.c_int]
    L.orc_con2prim.argtypes = [C.POINTER(Grid), C.POINTER(Eos), _dp, _dp, _u8p, _dp]
    L.orc_con2prim.restype = C.c_int64
    L.orc_imex_step_scheme.argtypes = [C.POINTER(Grid), C.POINTER(Par), C.POINTER(Eos), _dp, _dp, C.c_double,
                                       C.c_int, C.c_int]
    L.orc_imex_step_scheme.restype = C.c_int64
    L.orc_imex_tableau.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.POINTER(C.c_int)]
    L.orc_imex_tableau.restype = None
    L.orc_les_rhs.argtypes = [C.POINTER(Grid), C.POINTER(Par), C.POINTER(Eos), _dp, _dp, _dp]
    L.orc_les_rhs.restype = None
    L.orc_les_point_fields.argtypes = [C.POINTER(Grid), C.POINTER(Eos), _dp, _dp, _dp]
    L.orc_les_point_fields.restype = None
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_set_threads.restype = None
    L.orc_m1_implicit_point.argtypes = [_dp, _dp, C.c_double, _dp, _dp] + [C.c_double] * 6 + [_dp, _dp]
    L.orc_m1_implicit_point.restype = None
    L.orc_c2p_prims_at.argtypes = [C.POINTER(Grid), C.POINTER(Eos), _dp, _dp, _dp, _u8p]
    L.orc_c2p_prims_at.restype = None
    L.orc_c2p_f_at.argtypes = [C.POINTER(Grid), C.POINTER(Eos), _dp, _dp, _dp, _dp]
    L.orc_c2p_f_at.restype = None
    L.orc_c2p_point.argtypes = [C.POINTER(Eos), _dp, _dp, _dp, _dp, C.c_double, _dp, _dp,
                                C.POINTER(C.c_int)]
    L.orc_c2p_point.restype = C.c_uint
    L.orc_rhs.argtypes = [C.POINTER(Grid), C.POINTER(Par), C.POINTER(Eos), _dp, _dp, _dp, _dp]
    L.orc_rk4_stage.argtypes = [C.c_int, C.c_double, C.c_int64, _dp, _dp, _dp, _dp]
    L.orc_rk4_stage_interior.argtypes = [C.POINTER(Grid), C.c_int, C.c_int, C.c_double,
                                         _dp, _dp, _dp, _dp]
    L.orc_fill_periodic.argtypes = [C.POINTER(Grid), _dp, C.c_int]
    if hasattr(L, "orc_ssprk3_combine"):
        L.orc_ssprk3_tableau.argtypes = [_dp, _dp]
        L.orc_ssprk3_combine.argtypes = [C.POINTER(Grid), C.c_int, C.c_int, C.c_double, _dp, _dp, _dp, _dp, _dp]
    if hasattr(L, "orc_prolong"):
        _i3 = C.POINTER(C.c_int)
        L.orc_lagrange_half.argtypes = [_dp]
        L.orc_prolong.argtypes = [C.POINTER(Grid), _dp, C.POINTER(Grid), _dp, C.c_int, _i3, _i3, _i3]
        L.orc_prolong.restype = C.c_int
        L.orc_restrict.argtypes = [C.POINTER(Grid), _dp, C.POINTER(Grid), _dp, C.c_int, _i3, _i3, _i3]
        L.orc_restrict.restype = C.c_int
        L.orc_dense_weights.argtypes = [C.c_double, C.c_int, _dp]
        L.orc_dense_output.argtypes = [C.POINTER(Grid), C.c_int, C.c_double, C.c_double, C.c_int, _dp, _dp, _dp,
                                       _dp, _dp, _dp]
    if hasattr(L, "orc_constraints"):
        L.orc_constraints.argtypes = [C.POINTER(Grid), _dp, _dp, _dp]
    if hasattr(L, "orc_m1_rhs"):
        L.orc_m1_eddington.argtypes = [C.c_double]
        L.orc_m1_eddington.restype = C.c_double
        L.orc_m1_closure.argtypes = [C.c_double, _dp, _dp, C.c_double, _dp, _dp, _dp, _dp, _dp, _dp,
                                     C.POINTER(C.c_int)]
        L.orc_m1_closure.restype = C.c_double
        L.orc_m1_rhs.argtypes = [C.POINTER(Grid), C.POINTER(Par), _dp, _dp, _dp, _dp, _dp]
        L.orc_rhs_full.argtypes = [C.POINTER(Grid), C.POINTER(Par), C.POINTER(Eos), _dp, _dp, _dp, _dp, _dp]
        L.orc_rhs_split.argtypes = [C.POINTER(Grid), C.POINTER(Par), C.POINTER(Eos), _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_m1_implicit.argtypes = [C.POINTER(Grid), _dp, _dp, _dp, C.c_double]
        L.orc_m1_implicit.restype = C.c_int64
        L.orc_m1_implicit_x.argtypes = [C.POINTER(Grid), _dp, _dp, _dp, C.c_double, C.c_int]
        L.orc_m1_implicit_x.restype = C.c_int64
        L.orc_imex_stiff_fields.argtypes = [C.POINTER(Par)]
        L.orc_imex_stiff_fields.restype = C.c_int
        L.orc_imex_step.argtypes = [C.POINTER(Grid), C.POINTER(Par), C.POINTER(Eos), _dp, _dp, C.c_double, C.c_int]
        L.orc_imex_step.restype = C.c_int64
    if hasattr(L, "orc_m1n_rhs"):
        L.orc_m1n_rhs.argtypes = [C.POINTER(Grid), C.POINTER(Par), _dp, _dp, _dp, _dp, _dp]
        L.orc_m1n_implicit.argtypes = [C.POINTER(Grid), _dp, _dp, _dp, C.c_double]
        L.orc_m1n_implicit_x.argtypes = [C.POINTER(Grid), _dp, _dp, _dp, C.c_double, C.c_int, C.c_double]
    if hasattr(L, "orc_mlp_forward"):
        L.orc_bf16.argtypes = [C.c_float]
        L.orc_bf16.restype = C.c_float
        L.orc_mlp_features.argtypes = [_dp, _dp, _dp, _dp, _dp]
        L.orc_mlp_baseline.argtypes = [C.c_double, _dp, _dp, _dp]
        L.orc_mlp_targets.argtypes = [C.c_double, _dp, _dp, _dp]
        L.orc_c2p_features.argtypes = [C.POINTER(Grid), C.POINTER(Eos), _dp, _dp, _fp, _fp]
        L.orc_mlp_forward.argtypes = [_dp, _fp, C.c_int64, C.c_int, _dp]
        L.orc_mlp_grad.argtypes = [_dp, _fp, _fp, C.c_int64, C.c_int, _dp]
        L.orc_mlp_grad.restype = C.c_double
        L.orc_mlp_adam.argtypes = [_dp, _dp, _dp, _dp, C.c_int, C.c_double, C.c_double, C.c_double,
                                   C.c_double]
    return L


def ptr(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    if a.dtype == np.uint8:
        return a.ctypes.data_as(_u8p)
    if a.dtype == np.float32:
        return a.ctypes.data_as(_fp)
    assert a.dtype == np.float64, a.dtype
    return a.ctypes.data_as(_dp)


# ---------------------------------------------------------------- structs

def make_grid(n, dx, ng=3):
    g = Grid()
    for i in range(3):
        g.n[i] = int(n[i])
        g.dx[i] = float(dx[i])
    g.ng = ng
    return g


def make_eos(cfg):
    """cfg: dict with K0, Gamma (list), rho_b (list), Gamma_th and thresholds."""
    e = Eos()
    G = (C.c_double * 4)(*(list(cfg["Gamma"]) + [0.0] * (4 - len(cfg["Gamma"]))))
    rb = (C.c_double * 3)(*(list(cfg.get("rho_b", [])) + [0.0] * (3 - len(cfg.get("rho_b", [])))))
    lib().orc_eos_init_pwp(C.byref(e), len(cfg["Gamma"]), cfg["K0"], G, rb, cfg["Gamma_th"])
    for k in ("rho_atm", "rho_min", "rho_max", "eps_max", "W_max", "rho_low", "alpha_bh", "h0",
              "ye_min", "ye_max", "ye_atm"):
        setattr(e, k, float(cfg[k]))
    return e


def make_par(cfg):
    p = Par()
    for k in ("kappa_z", "kappa_c", "kappa_2", "eta", "sigma_ko", "c_b", "kappa_b", "alpha_mp5",
              "f_beta"):
        setattr(p, k, float(cfg[k]))
    for i in range(3):
        p.beta0[i] = float(cfg["beta0"][i])
    p.f_alpha_kind = int(cfg["f_alpha_kind"])
    p.evolve_st = int(cfg["evolve_st"])
    p.evolve_mhd = int(cfg["evolve_mhd"])
    p.couple_matter = int(cfg["couple_matter"])
    p.evolve_m1 = int(cfg.get("evolve_m1", 0))
    p.evolve_m1n = int(cfg.get("evolve_m1n", 0))
    p.m_b = float(cfg.get("m_b", 1.0))
    p.les_cm = float(cfg.get("les_cm", 0.0))
    p.couple_exchange = int(cfg.get("couple_exchange", 0))
    return p


# ---------------------------------------------------------------- calls

def prim2con(g, e, U, P, EM, eps_mode=0):
    lib().orc_prim2con(C.byref(g), C.byref(e), ptr(U), ptr(P), ptr(EM), eps_mode)


def con2prim(g, e, U, P, flags=None, mu=None):
    return lib().orc_con2prim(C.byref(g), C.byref(e), ptr(U), ptr(P), ptr(flags), ptr(mu))


def rhs(g, par, e, U, P, out):
    ms = C.c_double(0.0)
    lib().orc_rhs(C.byref(g), C.byref(par), C.byref(e), ptr(U), ptr(P), ptr(out), C.byref(ms))
    return ms.value


def rk4_stage_interior(g, nfields, stage, dt, Un, k, acc, Unext):
    lib().orc_rk4_stage_interior(C.byref(g), nfields, stage, dt, ptr(Un), ptr(k), ptr(acc),
                                 ptr(Unext))


def rk4_stage(stage, dt, Un, k, acc, Unext):
    lib().orc_rk4_stage(stage, dt, Un.size, ptr(Un), ptr(k), ptr(acc), ptr(Unext))


def fill_periodic(g, U, nfields):
    lib().orc_fill_periodic(C.byref(g), ptr(U), nfields)


def ssprk3_tableau():
    A, b = np.zeros(9), np.zeros(3)
    lib().orc_ssprk3_tableau(ptr(A), ptr(b))
    return A.reshape(3, 3), b


def ssprk3_combine(g, nfields, stage, dt, Un, K, Unext):
    """Stage `stage` of SSP-RK(3,3) in Butcher form from the stage RHS list K."""
    ks = [ptr(x) if x is not None else None for x in (list(K) + [None, None, None])[:3]]
    lib().orc_ssprk3_combine(C.byref(g), int(nfields), int(stage), float(dt), ptr(Un), ks[0], ks[1], ks[2],
                             ptr(Unext))


def _int3(v):
    return (C.c_int * 3)(*[int(x) for x in v])


def lagrange_half():
    w = np.zeros(6)
    lib().orc_lagrange_half(ptr(w))
    return w


def prolong(gc, Uc, gf, Uf, nfields, off, lo, hi):
    """Fine padded box [lo, hi) of Uf from Uc (fine index = 2 coarse index + off); 0 or -1."""
    return lib().orc_prolong(C.byref(gc), ptr(Uc), C.byref(gf), ptr(Uf), int(nfields), _int3(off), _int3(lo),
                             _int3(hi))


def restrict(gf, Uf, gc, Uc, nfields, off, lo, hi):
    """Coarse padded box [lo, hi) of Uc copied from Uf; 0 or -1."""
    return lib().orc_restrict(C.byref(gf), ptr(Uf), C.byref(gc), ptr(Uc), int(nfields), _int3(off), _int3(lo),
                              _int3(hi))


def dense_weights(theta, m):
    b = np.zeros(4)
    lib().orc_dense_weights(float(theta), int(m), ptr(b))
    return b


def dense_output(g, nfields, theta, dt, m, Un, L, out):
    lib().orc_dense_output(C.byref(g), int(nfields), float(theta), float(dt), int(m), ptr(Un), ptr(L[0]), ptr(L[1]),
                           ptr(L[2]), ptr(L[3]), ptr(out))


def constraints(g, U):
    """Constraint monitors over the interior of the padded patch of grid g:
    returns (C, sums), C = (5, padded) with H, M_1..3, Z_i Z^i at interior
    points (zero elsewhere), sums = 7 (nz + 1) volume integrals (totals first,
    then one row per interior plane)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    out = np.zeros((5,) + U.shape[1:])
    sums = np.zeros(7 * (g.n[2] + 1))
    lib().orc_constraints(C.byref(g), ptr(U), ptr(out), ptr(sums))
    return out, sums


def c2p_prims_at(g, e, U, mu, P, flags=None):
    """Primitives and flags at the given mu (one value per padded point)."""
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    lib().orc_c2p_prims_at(C.byref(g), C.byref(e), ptr(U), ptr(mu), ptr(P), ptr(flags))


def c2p_f_at(g, e, U, mu):
    """f_a and f at the given mu (one value per padded point; NaN where the
    point is atmosphere)."""
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    fa = np.zeros_like(mu)
    f = np.zeros_like(mu)
    lib().orc_c2p_f_at(C.byref(g), C.byref(e), ptr(U), ptr(mu), ptr(fa), ptr(f))
    return fa, f


def c2p_point(e, cons, B, gdn, gup, alpha):
    cons = np.ascontiguousarray(cons, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    gdn = np.ascontiguousarray(gdn, dtype=np.float64)
    gup = np.ascontiguousarray(gup, dtype=np.float64)
    prim = np.zeros(8)
    mu = np.zeros(2)
    it = C.c_int(0)
    f = lib().orc_c2p_point(C.byref(e), ptr(cons), ptr(B), ptr(gdn), ptr(gup), float(alpha),
                            ptr(prim), ptr(mu), C.byref(it))
    return f, prim, mu, it.value


def mp5(f5, alpha=4.0):
    f5 = np.ascontiguousarray(f5, dtype=np.float64)
    return lib().orc_mp5(ptr(f5), alpha)


def eps_cold(e, rho):
    return lib().orc_eps_cold(C.byref(e), rho)


def press(e, rho, eps):
    return lib().orc_press(C.byref(e), rho, eps)


def cs2(e, rho, eps):
    return lib().orc_cs2(C.byref(e), rho, eps)


# ---------------------------------------------------------------- learned guess (MLP)

MLP_NPARAM = 4866
MLP_NBLOCK = 4882
MLP_OFF = dict(W1=0, b1=512, W2=576, b2=4672, W3=4736, b3=4864, mean=4866, istd=4874)


def bf16(x):
    """bfloat16 rounding (nearest-even) of binary32 values, elementwise."""
    a = np.asarray(x, dtype=np.float32)
    return np.array([lib().orc_bf16(float(v)) for v in a.ravel()], dtype=np.float32).reshape(a.shape)


def mlp_features(cons, B, gdn, gup):
    x = np.zeros(8)
    lib().orc_mlp_features(ptr(np.ascontiguousarray(cons, dtype=np.float64)),
                           ptr(np.ascontiguousarray(B, dtype=np.float64)),
                           ptr(np.ascontiguousarray(gdn, dtype=np.float64)),
                           ptr(np.ascontiguousarray(gup, dtype=np.float64)), ptr(x))
    return x


def mlp_baseline(h0, cons, gup):
    b = np.zeros(2)
    lib().orc_mlp_baseline(float(h0), ptr(np.ascontiguousarray(cons, dtype=np.float64)),
                           ptr(np.ascontiguousarray(gup, dtype=np.float64)), ptr(b))
    return b


def mlp_targets(h0, b, mu):
    t = np.zeros(2)
    lib().orc_mlp_targets(float(h0), ptr(np.ascontiguousarray(b, dtype=np.float64)),
                          ptr(np.ascontiguousarray(mu, dtype=np.float64)), ptr(t))
    return t


def c2p_features(g, e, U, mu=None):
    """Features X [N][8] and (if mu is given) targets T [N][2], binary32."""
    N = U[0].size
    X = np.zeros((N, 8), dtype=np.float32)
    T = np.zeros((N, 2), dtype=np.float32) if mu is not None else None
    lib().orc_c2p_features(C.byref(g), C.byref(e), ptr(U), ptr(mu), ptr(X), ptr(T))
    return X, T


def _prm(prm):
    return np.ascontiguousarray(prm, dtype=np.float64)


def mlp_forward(prm, X, emulate=1):
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.zeros((X.shape[0], 2))
    lib().orc_mlp_forward(ptr(_prm(prm)), ptr(X), X.shape[0], int(emulate), ptr(Y))
    return Y


def mlp_grad(prm, X, T, emulate=1):
    """(loss, gradient of the 4866 trainable parameters) over the batch."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    T = np.ascontiguousarray(T, dtype=np.float32)
    g = np.zeros(MLP_NPARAM)
    loss = lib().orc_mlp_grad(ptr(_prm(prm)), ptr(X), ptr(T), X.shape[0], int(emulate), ptr(g))
    return loss, g


def mlp_adam(prm, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays prm (>= 4866), m, v."""
    for a in (prm, m, v):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    lib().orc_mlp_adam(ptr(prm), ptr(np.ascontiguousarray(grad, dtype=np.float64)), ptr(m), ptr(v), int(step),
                       float(lr), float(beta1), float(beta2), float(eps))


# ---------------------------------------------------------------- M1 radiation

def m1_eddington(xi):
    return lib().orc_m1_eddington(float(xi))


def m1_closure(E, F, v, W, gdn, gup):
    """(xi, chi, P_ij (6, lower), J, H_i (lower), Brent iterations) of the Minerbo closure."""
    P = np.zeros(6)
    J = C.c_double()
    H = np.zeros(3)
    chi = C.c_double()
    it = C.c_int()
    f = lambda a: ptr(np.ascontiguousarray(a, dtype=np.float64))
    xi = lib().orc_m1_closure(float(E), f(F), f(v), float(W), f(gdn), f(gup), ptr(P), C.byref(J), ptr(H),
                              C.byref(chi), C.byref(it))
    return xi, chi.value, P, J.value, H, it.value


def rhs_full(g, par, e, U, P, aux, out):
    """L(U) with the M1 part when par.evolve_m1 (U: 44 fields, aux: 9 fields)."""
    ms = C.c_double(0.0)
    lib().orc_rhs_full(C.byref(g), C.byref(par), C.byref(e), ptr(U), ptr(P), ptr(aux), ptr(out), C.byref(ms))
    return ms.value


def rhs_split(g, par, e, U, P, aux, F, R):
    """Explicit part F (44 fields) and stiff radiation part R (12 fields) of L(U)."""
    ms = C.c_double(0.0)
    lib().orc_rhs_split(C.byref(g), C.byref(par), C.byref(e), ptr(U), ptr(P), ptr(aux), ptr(F), ptr(R),
                        C.byref(ms))
    return ms.value


def m1n_rhs(g, par, U, P, aux, out, stiff=None):
    """Number-density part of L(U) (47 fields, aux 15): out[44..46] written,
    the electron-fraction source added to out[23]."""
    lib().orc_m1n_rhs(C.byref(g), C.byref(par), ptr(U), ptr(P), ptr(aux), ptr(out), ptr(stiff))


def m1n_implicit(g, U, P, aux, adt):
    lib().orc_m1n_implicit(C.byref(g), ptr(U), ptr(P), ptr(aux), float(adt))


def les_rhs(g, par, e, U, P, out):
    """Adds the gradient SGS term of the induction equation to out[28..30]."""
    lib().orc_les_rhs(C.byref(g), C.byref(par), C.byref(e), ptr(U), ptr(P), ptr(out))


def les_point_fields(g, e, U, P):
    """(H_v^i, H_M^xy, H_M^xz, H_M^yz): 6 fields at the points two or more from
    the patch edge (zero elsewhere)."""
    out = np.zeros((6,) + U.shape[1:])
    lib().orc_les_point_fields(C.byref(g), C.byref(e), ptr(U), ptr(P), ptr(out))
    return out


def set_threads(n):
    """Threads of the oracle's parallel loops (for timing on n cores)."""
    lib().orc_set_threads(int(n))


def m1_implicit_point(gd6, v, W, V, Vs, chi, adt, alp, ka, ks, eta):
    """(G, dG/dV) of the implicit M1 equation at one point (App. C Jacobian)."""
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (gd6, v, V, Vs)]
    G = np.zeros(4)
    Jac = np.zeros(16)
    lib().orc_m1_implicit_point(ptr(a[0]), ptr(a[1]), float(W), ptr(a[2]), ptr(a[3]), float(chi), float(adt),
                                float(alp), float(ka), float(ks), float(eta), ptr(G), ptr(Jac))
    return G, Jac.reshape(4, 4)


def m1_implicit(g, U, P, aux, adt, couple=0):
    """Implicit collision solve of the three species in place on U; with
    couple, the fluid's taubar and Sbar_i lose what the radiation gained.
    Returns the count of solves that did not converge."""
    return int(lib().orc_m1_implicit_x(C.byref(g), ptr(U), ptr(P), ptr(aux), float(adt), int(couple)))


def m1n_implicit_x(g, U, P, aux, adt, couple=0, m_b=1.0):
    lib().orc_m1n_implicit_x(C.byref(g), ptr(U), ptr(P), ptr(aux), float(adt), int(couple), float(m_b))


def imex_stiff_fields(par):
    """Stiff fields of the split right-hand side for these parameters."""
    return int(lib().orc_imex_stiff_fields(C.byref(par)))


def imex_step(g, par, e, U, aux, dt, periodic=False, scheme=0):
    """One IMEX step in place on U (44 or 47 fields): scheme 0 IMEX(4,4,2),
    1 IMEX(3,3,2); returns the count of implicit solves that did not converge."""
    return int(lib().orc_imex_step_scheme(C.byref(g), C.byref(par), C.byref(e), ptr(U), ptr(aux), float(dt),
                                          int(bool(periodic)), int(scheme)))


def imex_tableau(scheme):
    """(AE, AI, BE, BI) of an IMEX scheme as numpy arrays (stages x stages)."""
    AE, AI, BE, BI = np.zeros(16), np.zeros(16), np.zeros(4), np.zeros(4)
    ns = C.c_int(0)
    lib().orc_imex_tableau(int(scheme), ptr(AE), ptr(AI), ptr(BE), ptr(BI), C.byref(ns))
    n = ns.value
    return AE.reshape(4, 4)[:n, :n], AI.reshape(4, 4)[:n, :n], BE[:n], BI[:n]
