"""Thin ctypes binding of libmhd.so (include/mhd.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Arrays are torch tensors on the HIP device (float64, laid out as
(field, z, y, x) over the padded patch, or any strided layout described by the
patch strides); the stream is torch's current stream unless one is given.
There is no CPU fallback: a missing library or device raises.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libmhd.so")

MHD_NST, MHD_NMHD, MHD_NU, MHD_NP, MHD_NEM = 22, 10, 32, 8, 4
MHD_NU_M1, MHD_NAUX = 44, 9
MHD_NU_M1N, MHD_NAUX_N = 47, 15
MHD_NSTAT = 8
EVOLVE_SPACETIME, EVOLVE_MHD, COUPLE_MATTER, EVOLVE_M1, EVOLVE_M1N, COUPLE_EXCHANGE = 1, 2, 4, 8, 16, 32
IMPLICIT_N, IMPLICIT_COUPLED = 1, 2
IMEX_442, IMEX_332 = 0, 1
FLAG = dict(ATMO=1, EPS_LO=2, EPS_HI=4, VEL_LIMIT=8, YE_RESET=16, FALLBACK=32, NOT_CONVERGED=64, FATAL=128)
STAT_FATAL, STAT_CORRECTED, STAT_FALLBACK, STAT_ITERATIONS = 0, 1, 2, 3


class Patch(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("ng", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
                ("sy", C.c_int64), ("sz", C.c_int64), ("sf", C.c_int64)]


class Eos(C.Structure):
    _fields_ = [("npieces", C.c_int32), ("reserved", C.c_int32), ("K", C.c_double * 4),
                ("Gamma", C.c_double * 4), ("rho_b", C.c_double * 3), ("a", C.c_double * 4),
                ("Gamma_th", C.c_double), ("rho_atm", C.c_double), ("rho_min", C.c_double),
                ("rho_max", C.c_double), ("eps_max", C.c_double), ("W_max", C.c_double),
                ("rho_low", C.c_double), ("alpha_bh", C.c_double), ("h0", C.c_double),
                ("ye_min", C.c_double), ("ye_max", C.c_double), ("ye_atm", C.c_double)]


class Params(C.Structure):
    _fields_ = [("kappa_z", C.c_double), ("kappa_c", C.c_double), ("kappa_2", C.c_double),
                ("eta", C.c_double), ("beta0", C.c_double * 3), ("sigma_ko", C.c_double),
                ("c_b", C.c_double), ("kappa_b", C.c_double), ("alpha_mp5", C.c_double),
                ("f_beta", C.c_double), ("f_alpha_kind", C.c_int32), ("flags", C.c_uint32), ("m_b", C.c_double),
                ("les_cm", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("strip", C.c_int32), ("block_threads", C.c_int32), ("grid_per_cu", C.c_int32),
                ("reserved", C.c_int32 * 5)]


class Box(C.Structure):
    _fields_ = [("patch", Patch), ("U", C.c_void_p), ("Us", C.c_void_p), ("P", C.c_void_p), ("k", C.c_void_p),
                ("acc", C.c_void_p), ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("flags", C.c_void_p), ("aux", C.c_void_p)]


class ImexBox(C.Structure):
    _fields_ = [("F", C.c_void_p * 4), ("R", C.c_void_p * 4)]


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 40), ("launches", C.c_int64), ("total_ms", C.c_double)]


_vp = C.c_void_p
_LIB = None

# name -> (restype, argtypes); the exported C symbols of include/mhd.h
SIGNATURES = {
    "mhd_last_error": (C.c_char_p, []),
    "mhd_abi_version": (C.c_int, []),
    "mhd_eos_init_pwp": (C.c_int, [C.POINTER(Eos)]),
    "mhd_prim2con": (C.c_int, [C.POINTER(Patch), C.POINTER(Eos), _vp, _vp, _vp, C.c_int, _vp]),
    "mhd_con2prim": (C.c_int, [C.POINTER(Patch), C.POINTER(Eos), _vp, _vp, _vp, _vp, _vp, _vp]),
    "mhd_rhs_workspace_size": (C.c_size_t, [C.POINTER(Patch)]),
    "mhd_rhs_workspace_size_m1": (C.c_size_t, [C.POINTER(Patch)]),
    "mhd_rhs_workspace_size_m1n": (C.c_size_t, [C.POINTER(Patch)]),
    "mhd_rhs": (C.c_int, [C.POINTER(Patch), C.POINTER(Params), C.POINTER(Eos), _vp, _vp, _vp, _vp, _vp, _vp,
                          C.c_size_t, _vp]),
    "mhd_rk_stage": (C.c_int, [C.POINTER(Patch), C.c_int, C.c_int, C.c_double, _vp, _vp, _vp, _vp, _vp]),
    "mhd_fill_ghosts_periodic": (C.c_int, [C.POINTER(Patch), _vp, C.c_int, _vp]),
    "mhd_set_tuning": (C.c_int, [C.POINTER(Tuning)]),
    "mhd_get_tuning": (C.c_int, [C.POINTER(Tuning)]),
    "mhd_con2prim_learned_workspace_size": (C.c_size_t, [C.POINTER(Patch)]),
    "mhd_con2prim_learned_noalloc": (C.c_int, [C.POINTER(Patch), C.POINTER(Eos), _vp, _vp, _vp, _vp, _vp, _vp,
                                               _vp]),
    "mhd_con2prim_learned": (C.c_int, [C.POINTER(Patch), C.POINTER(Eos), _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                       C.c_size_t, _vp]),
    "mhd_mlp_features": (C.c_int, [C.POINTER(Patch), C.POINTER(Eos), _vp, _vp, _vp, _vp, _vp]),
    "mhd_mlp_normalize": (C.c_int, [_vp, _vp, C.c_int64, _vp]),
    "mhd_mlp_forward": (C.c_int, [_vp, _vp, C.c_int64, _vp, _vp]),
    "mhd_mlp_grad_workspace_size": (C.c_size_t, [C.c_int64]),
    "mhd_mlp_grad": (C.c_int, [_vp, _vp, _vp, C.c_int64, _vp, _vp, _vp, C.c_size_t, _vp]),
    "mhd_mlp_adam": (C.c_int, [_vp, _vp, _vp, _vp, C.c_int, C.c_float, C.c_float, C.c_float, C.c_float, _vp]),
    "mhd_level_create": (C.c_int, [C.POINTER(Box), C.c_int, C.POINTER(Params), C.POINTER(Eos),
                                   C.POINTER(C.c_void_p)]),
    "mhd_level_destroy": (C.c_int, [_vp]),
    "mhd_level_set_tuning": (C.c_int, [_vp, C.POINTER(Tuning)]),
    "mhd_level_get_tuning": (C.c_int, [_vp, C.POINTER(Tuning)]),
    "mhd_level_rhs": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "mhd_level_rk4_step": (C.c_int, [_vp, C.c_double, _vp, C.c_int, _vp]),
    "mhd_level_autotune": (C.c_int, [_vp, C.c_double, _vp, C.POINTER(Tuning)]),
    "mhd_level_learned_workspace_size": (C.c_size_t, [_vp]),
    "mhd_level_set_learned": (C.c_int, [_vp, _vp, _vp, C.c_size_t]),
    "mhd_level_set_imex": (C.c_int, [_vp, C.POINTER(ImexBox), C.c_int]),
    "mhd_ssprk3_stage": (C.c_int, [C.POINTER(Patch), C.c_int, C.c_int, C.c_double, _vp, _vp, _vp, _vp, _vp]),
    "mhd_prolong": (C.c_int, [C.POINTER(Patch), _vp, C.POINTER(Patch), _vp, C.c_int, _vp, _vp, _vp, _vp]),
    "mhd_restrict": (C.c_int, [C.POINTER(Patch), _vp, C.POINTER(Patch), _vp, C.c_int, _vp, _vp, _vp, _vp]),
    "mhd_dense_output": (C.c_int, [C.POINTER(Patch), C.c_int, C.c_double, C.c_double, C.c_int, _vp,
                                   C.POINTER(C.c_void_p), _vp, _vp]),
    "mhd_level_imex_step": (C.c_int, [_vp, C.c_double, _vp, _vp, C.c_int, _vp]),
    "mhd_rhs_split": (C.c_int, [C.POINTER(Patch), C.POINTER(Params), C.POINTER(Eos), _vp, _vp, _vp, _vp, _vp, _vp,
                                _vp, C.c_size_t, _vp]),
    "mhd_imex_stiff_fields": (C.c_int, [C.c_int, C.c_int]),
    "mhd_imex_combine": (C.c_int, [C.POINTER(Patch), C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, _vp,
                                   C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), _vp, _vp]),
    "mhd_m1_implicit": (C.c_int, [C.POINTER(Patch), _vp, _vp, _vp, C.c_double, C.c_uint, C.c_double, _vp, _vp]),
    "mhd_constraints": (C.c_int, [C.POINTER(Patch), _vp, _vp, _vp, _vp]),
    "mhd_profile_start": (C.c_int, []),
    "mhd_profile_stop": (C.c_int, [C.POINTER(KernelTime), C.c_int, C.POINTER(C.c_int)]),
}


class MhdError(RuntimeError):
    pass


def lib():
    """Load libmhd.so (built in-tree by build.py); raises if it is missing."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIBPATH):
            raise MhdError("libmhd.so not built: run paper_2510_13965_amd/build.py (or __graft_entry__.build())")
        L = C.CDLL(LIBPATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _check(rc):
    if rc != 0:
        raise MhdError("libmhd error %d: %s" % (rc, lib().mhd_last_error().decode()))


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise MhdError("libmhd takes device tensors only (got a %s tensor)" % t.device)
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------ structs

def make_patch(n, dx, x0=(0.0, 0.0, 0.0), ng=3, strides=None):
    p = Patch()
    p.nx, p.ny, p.nz = (int(v) for v in n)
    p.ng = int(ng)
    p.dx, p.dy, p.dz = (float(v) for v in dx)
    p.x0, p.y0, p.z0 = (float(v) for v in x0)
    Nx, Ny, Nz = (int(n[a]) + 2 * ng for a in range(3))
    if strides is None:
        strides = (Nx, Nx * Ny, Nx * Ny * Nz)
    p.sy, p.sz, p.sf = (int(v) for v in strides)
    return p


def patch_of(ip, strides=None):
    """libmhd patch of an inputs.Patch."""
    return make_patch(ip.n, ip.dx, ip.x0, ip.ng, strides)


def make_eos(cfg):
    e = Eos()
    G = list(cfg["Gamma"])
    e.npieces = len(G)
    for i, g in enumerate(G):
        e.Gamma[i] = g
    for i, r in enumerate(cfg.get("rho_b", [])):
        e.rho_b[i] = r
    e.K[0] = cfg["K0"]
    e.Gamma_th = cfg["Gamma_th"]
    for k in ("rho_atm", "rho_min", "rho_max", "eps_max", "W_max", "rho_low", "alpha_bh", "h0",
              "ye_min", "ye_max", "ye_atm"):
        setattr(e, k, float(cfg[k]))
    _check(lib().mhd_eos_init_pwp(C.byref(e)))
    return e


def make_params(cfg):
    p = Params()
    for k in ("kappa_z", "kappa_c", "kappa_2", "eta", "sigma_ko", "c_b", "kappa_b", "alpha_mp5", "f_beta"):
        setattr(p, k, float(cfg[k]))
    for i in range(3):
        p.beta0[i] = float(cfg["beta0"][i])
    p.f_alpha_kind = int(cfg["f_alpha_kind"])
    fl = 0
    if cfg.get("evolve_st", 1):
        fl |= EVOLVE_SPACETIME
    if cfg.get("evolve_mhd", 1):
        fl |= EVOLVE_MHD
    if cfg.get("couple_matter", 1):
        fl |= COUPLE_MATTER
    if cfg.get("evolve_m1", 0):
        fl |= EVOLVE_M1
    if cfg.get("evolve_m1n", 0):
        fl |= EVOLVE_M1N
    if cfg.get("couple_exchange", 0):
        fl |= COUPLE_EXCHANGE
    p.flags = fl
    p.m_b = float(cfg.get("m_b", 1.0))
    p.les_cm = float(cfg.get("les_cm", 0.0))
    return p


# ------------------------------------------------------------------ calls

def prim2con(patch, eos, U, P, EM, eps_mode=0, stream=None):
    _check(lib().mhd_prim2con(C.byref(patch), C.byref(eos), _ptr(U), _ptr(P), _ptr(EM), eps_mode,
                              _stream(stream)))


def con2prim(patch, eos, U, P, flags=None, mu=None, stats=None, stream=None):
    _check(lib().mhd_con2prim(C.byref(patch), C.byref(eos), _ptr(U), _ptr(P), _ptr(flags), _ptr(mu),
                              _ptr(stats), _stream(stream)))


def rhs_workspace_size(patch):
    return int(lib().mhd_rhs_workspace_size(C.byref(patch)))


def rhs(patch, params, eos, U, P, out, max_speed=None, workspace=None, stream=None, aux=None):
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(lib().mhd_rhs(C.byref(patch), C.byref(params), C.byref(eos), _ptr(U), _ptr(P), _ptr(aux), _ptr(out),
                         _ptr(max_speed), _ptr(workspace), nbytes, _stream(stream)))


def rk_stage(patch, nfields, stage, dt, Un, k, acc, Unext, stream=None):
    _check(lib().mhd_rk_stage(C.byref(patch), nfields, stage, float(dt), _ptr(Un), _ptr(k), _ptr(acc),
                              _ptr(Unext), _stream(stream)))


def fill_ghosts_periodic(patch, U, nfields, stream=None):
    _check(lib().mhd_fill_ghosts_periodic(C.byref(patch), _ptr(U), nfields, _stream(stream)))


MLP_NPARAM, MLP_NBLOCK = 4866, 4882


def con2prim_learned_workspace_size(patch):
    return int(lib().mhd_con2prim_learned_workspace_size(C.byref(patch)))


def con2prim_learned(patch, eos, mlp, U, P, workspace, flags=None, mu=None, stats=None, stream=None):
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib().mhd_con2prim_learned(C.byref(patch), C.byref(eos), _ptr(mlp), _ptr(U), _ptr(P), _ptr(flags), _ptr(mu),
                                      _ptr(stats), _ptr(workspace), nbytes, _stream(stream)))


def con2prim_learned_noalloc(patch, eos, mlp, U, P, flags=None, mu=None, stats=None, stream=None):
    _check(lib().mhd_con2prim_learned_noalloc(C.byref(patch), C.byref(eos), _ptr(mlp), _ptr(U), _ptr(P), _ptr(flags),
                                              _ptr(mu), _ptr(stats), _stream(stream)))


def mlp_features(patch, eos, U, X, mu=None, T=None, stream=None):
    _check(lib().mhd_mlp_features(C.byref(patch), C.byref(eos), _ptr(U), _ptr(mu), _ptr(X), _ptr(T), _stream(stream)))


def mlp_normalize(mlp, X, n=None, stream=None):
    n = X.shape[0] if n is None else n
    _check(lib().mhd_mlp_normalize(_ptr(mlp), _ptr(X), int(n), _stream(stream)))


def mlp_forward(mlp, X, Y, n=None, stream=None):
    n = X.shape[0] if n is None else n
    _check(lib().mhd_mlp_forward(_ptr(mlp), _ptr(X), int(n), _ptr(Y), _stream(stream)))


def mlp_grad_workspace_size(n):
    return int(lib().mhd_mlp_grad_workspace_size(int(n)))


def mlp_grad(mlp, X, T, grad, workspace, loss=None, n=None, stream=None):
    n = X.shape[0] if n is None else n
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib().mhd_mlp_grad(_ptr(mlp), _ptr(X), _ptr(T), int(n), _ptr(grad), _ptr(loss), _ptr(workspace), nbytes,
                              _stream(stream)))


def mlp_adam(mlp, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().mhd_mlp_adam(_ptr(mlp), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr), float(beta1), float(beta2),
                              float(eps), _stream(stream)))


def _tuning(strip=4, block_threads=256, grid_per_cu=0):
    t = Tuning()
    t.strip, t.block_threads, t.grid_per_cu = int(strip), int(block_threads), int(grid_per_cu)
    return t


def _tuning_dict(t):
    return {"strip": t.strip, "block_threads": t.block_threads, "grid_per_cu": t.grid_per_cu}


def rhs_split(patch, params, eos, U, P, aux, out, stiff, max_speed=None, workspace=None, stream=None):
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(lib().mhd_rhs_split(C.byref(patch), C.byref(params), C.byref(eos), _ptr(U), _ptr(P), _ptr(aux), _ptr(out),
                               _ptr(stiff), _ptr(max_speed), _ptr(workspace), nbytes, _stream(stream)))


def imex_stiff_fields(nfields, coupled=False):
    n = int(lib().mhd_imex_stiff_fields(int(nfields), int(bool(coupled))))
    if n < 0:
        _check(n)
    return n


def imex_combine(patch, stage, dt, Un, F, R, Uout, stream=None, nfields=MHD_NU_M1, scheme=IMEX_442, coupled=False):
    """F, R: lists of up to 4 device tensors (stage explicit and stiff parts)."""
    fa = (C.c_void_p * 4)(*[(_ptr(F[j]) if j < len(F) and F[j] is not None else None) for j in range(4)])
    ra = (C.c_void_p * 4)(*[(_ptr(R[j]) if j < len(R) and R[j] is not None else None) for j in range(4)])
    _check(lib().mhd_imex_combine(C.byref(patch), int(scheme), int(nfields), int(bool(coupled)), int(stage),
                                  float(dt), _ptr(Un), fa, ra, _ptr(Uout), _stream(stream)))


def m1_implicit(patch, aux, U, P, adt, nfail=None, stream=None, evolve_n=False, coupled=False, m_b=1.0):
    flags = (IMPLICIT_N if evolve_n else 0) | (IMPLICIT_COUPLED if coupled else 0)
    _check(lib().mhd_m1_implicit(C.byref(patch), _ptr(aux), _ptr(U), _ptr(P), float(adt), flags, float(m_b),
                                 _ptr(nfail), _stream(stream)))


def set_tuning(strip):
    _check(lib().mhd_set_tuning(C.byref(_tuning(strip))))


def get_tuning():
    t = Tuning()
    _check(lib().mhd_get_tuning(C.byref(t)))
    return {"strip": t.strip}


class Level:
    """A batched level (mhd_level_*).  `boxes` is a list of dicts with the
    patch (mhd_patch_t) and device tensors U, Us, P, k, acc, ws and
    optionally flags and aux (required when params evolve M1); the tensors are
    kept alive with the level."""

    def __init__(self, boxes, params, eos):
        self._keep = boxes
        arr = (Box * len(boxes))()
        for b, d in enumerate(boxes):
            arr[b].patch = d["patch"]
            for name in ("U", "Us", "P", "k", "acc"):
                setattr(arr[b], name, _ptr(d[name]))
            arr[b].workspace = _ptr(d["ws"])
            arr[b].workspace_bytes = d["ws"].numel() * d["ws"].element_size()
            arr[b].flags = _ptr(d.get("flags"))
            arr[b].aux = _ptr(d.get("aux"))
        self._params, self._eos = params, eos
        h = C.c_void_p()
        _check(lib().mhd_level_create(arr, len(boxes), C.byref(params), C.byref(eos), C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().mhd_level_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, strip=4, block_threads=256, grid_per_cu=0):
        _check(lib().mhd_level_set_tuning(self.h, C.byref(_tuning(strip, block_threads, grid_per_cu))))

    def get_tuning(self):
        t = Tuning()
        _check(lib().mhd_level_get_tuning(self.h, C.byref(t)))
        return _tuning_dict(t)

    def rhs(self, src=0, max_speed=None, stats=None, stream=None):
        _check(lib().mhd_level_rhs(self.h, int(src), _ptr(max_speed), _ptr(stats), _stream(stream)))

    def rk4_step(self, dt, max_speed=None, use_graph=False, stream=None):
        _check(lib().mhd_level_rk4_step(self.h, float(dt), _ptr(max_speed), int(bool(use_graph)), _stream(stream)))

    def set_learned(self, mlp, device="cuda"):
        """Use the learned con2prim guess (mlp: device float32 parameter block), or
        the bracketed solver (mlp = None)."""
        import torch

        if mlp is None:
            _check(lib().mhd_level_set_learned(self.h, None, None, 0))
            self._lws = self._mlp = None
            return
        n = int(lib().mhd_level_learned_workspace_size(self.h))
        self._lws = torch.empty((n + 7) // 8, dtype=torch.float64, device=device)
        self._mlp = mlp
        _check(lib().mhd_level_set_learned(self.h, _ptr(mlp), _ptr(self._lws), self._lws.numel() * 8))

    def set_imex(self, stages):
        """IMEX stage arrays per box: stages[b] = (F, R), four device tensors each
        (F: 44 fields, R: 12 fields, the box's shape); None detaches them."""
        if stages is None:
            _check(lib().mhd_level_set_imex(self.h, None, 0))
            self._imex = None
            return
        arr = (ImexBox * len(stages))()
        for b, (F, R) in enumerate(stages):
            for st in range(4):
                arr[b].F[st] = _ptr(F[st])
                arr[b].R[st] = _ptr(R[st])
        self._imex = stages
        _check(lib().mhd_level_set_imex(self.h, arr, len(stages)))

    def imex_step(self, dt, max_speed=None, nfail=None, use_graph=False, stream=None):
        _check(lib().mhd_level_imex_step(self.h, float(dt), _ptr(max_speed), _ptr(nfail), int(bool(use_graph)),
                                         _stream(stream)))

    def autotune(self, dt, stream=None, cache=None):
        """Time the candidate launch shapes and keep the fastest (mhd_level_autotune).
        cache: path of an on-disk tuning cache (tuning.TuningCache); a level with
        the same device, library version, radiation switch and box shapes reuses
        the stored choice without timing anything."""
        key = None
        if cache is not None:
            import torch

            from .tuning import TuningCache, cache_key

            dims = [(b["patch"].nx, b["patch"].ny, b["patch"].nz) for b in self._keep]
            key = cache_key(dims, self._params.flags & EVOLVE_M1, torch.cuda.get_device_name(),
                            lib().mhd_abi_version())
            hit = TuningCache(cache).get(key)
            if hit is not None:
                self.set_tuning(**hit)
                return self.get_tuning()
        t = Tuning()
        _check(lib().mhd_level_autotune(self.h, float(dt), _stream(stream), C.byref(t)))
        chosen = _tuning_dict(t)
        if key is not None:
            TuningCache(cache).put(key, chosen)
        return chosen


def ssprk3_stage(patch, nfields, stage, dt, Un, k, acc, Unext, stream=None):
    _check(lib().mhd_ssprk3_stage(C.byref(patch), int(nfields), int(stage), float(dt), _ptr(Un), _ptr(k), _ptr(acc),
                                  _ptr(Unext), _stream(stream)))


def _i3(v):
    return (C.c_int32 * 3)(*[int(x) for x in v])


def prolong(coarse, Uc, fine, Uf, nfields, offset, lo, hi, stream=None):
    """Fine padded box [lo, hi) of Uf from Uc (mhd_prolong); offset: fine index of coarse index 0."""
    o, l, h = _i3(offset), _i3(lo), _i3(hi)
    _check(lib().mhd_prolong(C.byref(coarse), _ptr(Uc), C.byref(fine), _ptr(Uf), int(nfields), C.cast(o, _vp),
                             C.cast(l, _vp), C.cast(h, _vp), _stream(stream)))


def restrict(fine, Uf, coarse, Uc, nfields, offset, lo, hi, stream=None):
    """Coarse padded box [lo, hi) of Uc copied from the coincident fine points (mhd_restrict)."""
    o, l, h = _i3(offset), _i3(lo), _i3(hi)
    _check(lib().mhd_restrict(C.byref(fine), _ptr(Uf), C.byref(coarse), _ptr(Uc), int(nfields), C.cast(o, _vp),
                              C.cast(l, _vp), C.cast(h, _vp), _stream(stream)))


def dense_output(patch, nfields, theta, dt, deriv, Un, L, out, stream=None):
    """RK4 dense output (deriv 0) or its deriv-th time derivative from the four stage RHS arrays L."""
    arr = (C.c_void_p * 4)(*[_ptr(x) for x in L])
    _check(lib().mhd_dense_output(C.byref(patch), int(nfields), float(theta), float(dt), int(deriv), _ptr(Un), arr,
                                  _ptr(out), _stream(stream)))


def constraints(patch, U, C5, sums, stream=None):
    """Constraint monitors (mhd_constraints): H, M_i, Z_i Z^i into the 5-field
    array C5 at interior points, volume integrals into the device array sums of
    7 (nz + 1) doubles (totals first, then one row per interior plane)."""
    _check(lib().mhd_constraints(C.byref(patch), _ptr(U), _ptr(C5), _ptr(sums), _stream(stream)))


def profile_start():
    _check(lib().mhd_profile_start())


def profile_stop():
    """{kernel name: (launches, total ms)} since profile_start()."""
    out = (KernelTime * 32)()
    n = C.c_int(0)
    _check(lib().mhd_profile_stop(out, 32, C.byref(n)))
    return {out[i].name.decode(): (int(out[i].launches), float(out[i].total_ms)) for i in range(min(n.value, 32))}


def workspace_for(patch, device="cuda", m1=False, m1n=False):
    import torch

    if m1n:
        size = int(lib().mhd_rhs_workspace_size_m1n(C.byref(patch)))
    elif m1:
        size = int(lib().mhd_rhs_workspace_size_m1(C.byref(patch)))
    else:
        size = rhs_workspace_size(patch)
    n = (size + 7) // 8
    return torch.empty(n, dtype=torch.float64, device=device)
