"""The pins catch plausible slips: each case plants one wrong coefficient,
sign, index or operand in a copy of the oracle's C sources (built into a
temporary directory, never over oracle/liborc.so), binds the copy and checks
that at least one named pin fails on it.  The unmodified oracle passes the
same pins in their own test files.

The slips are the ones a reader of Sec. 2.1 (damping and gauge terms),
Sec. 3.3 (MP5 bounds) and Sec. 2.3 / App. C (number densities) could make:
kappa_z (2 - kappa_2) for (2 + kappa_2), a sign of eta, the 3/4 of the shift,
the 2/3 K of the Ghat damping, a dropped Theta term, the 4/3 curvature weight
of f^LC, the halves of f^MD, the alpha of f^UL, the arguments of d^M4 swapped,
the sign rule of the 4-argument minmod; a sign in Gamma, the normal part of
H^a dropped or flipped, the W on the shift, H^k without 1/J, the number
source with Gamma multiplied or N densitized, the electron-fraction source's
sign or baryon mass, and the lapse or emission of the implicit update; a
factor or sign of App. C's printed Jacobian of the implicit M1 equation;
the LES term's product part, second-derivative factor, index order, xi and
divergence assembly (App. A); the coupled exchange's fluid update (sign,
momentum index, the m_b of the lepton number) and its stiff slot's sign.
"""
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

from oracle import build as obuild

import test_oracle_coupled as CP
import test_oracle_gauge as G
import test_oracle_imex as IM
import test_oracle_les as LES
import test_oracle_m1n as NM
import test_oracle_stencils as S

NPINS = [NM.check_source_at_rest, NM.check_thick_limit, NM.check_thin_limit, NM.check_imex_relaxation]

ORACLE_DIR = os.path.dirname(obuild.__file__)

# (name, file, original text, planted slip, pins that must catch it)
MUTANTS = [
    ("theta damping kappa_2 sign", "ccz4.c", "par->kappa_z * (2.0 + par->kappa_2) * Th",
     "par->kappa_z * (2.0 - par->kappa_2) * Th", [G.check_z4_damping]),
    ("khat damping kappa_2 sign", "ccz4.c", "par->kappa_z * (1.0 - par->kappa_2) * Th",
     "par->kappa_z * (1.0 + par->kappa_2) * Th", [G.check_z4_damping]),
    ("khat damping dropped", "ccz4.c", "+ par->kappa_z * (1.0 - par->kappa_2) * Th);", ");",
     [G.check_z4_damping]),
    ("ghat damping 2/3 K dropped", "ccz4.c", "(par->kappa_z + 2.0 / 3.0 * Kfull)", "(par->kappa_z)",
     [G.check_z4_damping]),
    ("ghat damping Khat for K", "ccz4.c", "(par->kappa_z + 2.0 / 3.0 * Kfull)",
     "(par->kappa_z + 2.0 / 3.0 * Kh)", [G.check_z4_damping]),
    ("ghat damping sign", "ccz4.c", "t2 += -1.0 / chi * Z[i]", "t2 += 1.0 / chi * Z[i]",
     [G.check_z4_damping]),
    ("theta K-hat term", "ccz4.c", "2.0 / 3.0 * Th * (Kh - 2.0 * Th)", "2.0 / 3.0 * Th * (Kh + 2.0 * Th)",
     [G.check_z4_damping]),
    ("shift eta sign", "ccz4.c", "- par->eta * (beta[i] - par->beta0[i])",
     "+ par->eta * (beta[i] - par->beta0[i])", [G.check_lapse_shift]),
    ("shift beta0 sign", "ccz4.c", "(beta[i] - par->beta0[i])", "(beta[i] + par->beta0[i])",
     [G.check_lapse_shift]),
    ("shift 3/4", "ccz4.c", "0.75 * par->f_beta * Gh[i]", "0.5 * par->f_beta * Gh[i]", [G.check_lapse_shift]),
    ("1+log factor", "ccz4.c", "- 2.0 * alp * falpha * Kh", "- alp * falpha * Kh", [G.check_lapse_shift]),
    ("harmonic slicing f_alpha", "ccz4.c", "? 0.5 * alp : 1.0", "? alp : 1.0", [G.check_harmonic_lapse]),
    ("At Khat for K", "ccz4.c", "r += alp * (Kh * At[i][j] - 2.0 * AikAkj);",
     "r += alp * (Kfull * At[i][j] - 2.0 * AikAkj);", [G.check_z4_damping_with_At]),
    ("mp5 f^LC weight", "fd.c", "4.0 / 3.0 * dm4_minus", "1.0 * dm4_minus", [S.check_mp5_limited]),
    ("mp5 f^MD half", "fd.c", "- 0.5 * dm4_plus", "- 1.0 * dm4_plus", [S.check_mp5_limited]),
    ("mp5 f^MD sign", "fd.c", "- 0.5 * dm4_plus", "+ 0.5 * dm4_plus", [S.check_mp5_limited]),
    ("mp5 f^UL alpha", "fd.c", "double ful = f0 + alpha * dminus;", "double ful = f0 + 3.0 * dminus;",
     [S.check_mp5_limited]),
    ("mp5 d^M4 swapped", "fd.c", "double fmd = 0.5 * (f0 + fp1) - 0.5 * dm4_plus;",
     "double fmd = 0.5 * (f0 + fp1) - 0.5 * dm4_minus;", [S.check_mp5_limited]),
    ("mp5 d^M4 argument", "fd.c", "minmod4(4.0 * dm1 - d0, 4.0 * d0 - dm1, dm1, d0)",
     "minmod4(4.0 * dm1 - d0, 4.0 * d0 - dm1, dm1, dp1)", [S.check_mp5_limited]),
    ("mp5 f^LC D-", "fd.c", "f0 + 0.5 * dminus + 4.0 / 3.0", "f0 + 0.5 * dplus + 4.0 / 3.0",
     [S.check_mp5_limited]),
    ("N Gamma sign", "m1.c", "gam = s.W * (s.E - s.vF) / J;\n      GM[sp * N + p] = gam;",
     "gam = s.W * (s.E + s.vF) / J;\n      GM[sp * N + p] = gam;", NPINS),
    ("N four-vector H shift term sign", "m1.c", "Hu[d] = s.W * (J - s.E + s.vF) * U[(19 + d) * N + p] / alp;",
     "Hu[d] = -s.W * (J - s.E + s.vF) * U[(19 + d) * N + p] / alp;", NPINS),
    ("N H spatial projection only", "m1.c", "Hu[d] = s.W * (J - s.E + s.vF) * U[(19 + d) * N + p] / alp;",
     "Hu[d] = 0.0;", NPINS),
    ("N flux W on the shift", "m1.c", "(-s.W * bd + alp * s.W * s.v[d] + alp * Hu[d] / J)",
     "(-bd + alp * s.W * s.v[d] + alp * Hu[d] / J)", NPINS),
    ("N flux H over J", "m1.c", "(-s.W * bd + alp * s.W * s.v[d] + alp * Hu[d] / J)",
     "(-s.W * bd + alp * s.W * s.v[d] + alp * Hu[d])", NPINS),
    ("N source Gamma", "m1.c", "C[sp] = e0 - k0 * (u[q] / m.sqrtg) / GM[sp * N + q];",
     "C[sp] = e0 - k0 * (u[q] / m.sqrtg) * GM[sp * N + q];", NPINS),
    ("N source densitized N", "m1.c", "C[sp] = e0 - k0 * (u[q] / m.sqrtg) / GM[sp * N + q];",
     "C[sp] = e0 - k0 * u[q] / GM[sp * N + q];", NPINS),
    ("Ye source sign", "m1.c", "rhs[23 * N + q] -= alp * m.sqrtg * par->m_b * (C[0] - C[1])",
     "rhs[23 * N + q] -= alp * m.sqrtg * par->m_b * (C[1] - C[0])", NPINS),
    ("Ye source m_b dropped", "m1.c", "rhs[23 * N + q] -= alp * m.sqrtg * par->m_b * (C[0] - C[1])",
     "rhs[23 * N + q] -= alp * m.sqrtg * (C[0] - C[1])", NPINS),
    ("N implicit lapse", "m1.c", "(1.0 + adt * alp * k0 / gam)", "(1.0 + adt * k0 / gam)", NPINS),
    ("N implicit emission", "m1.c", "(Ns + adt * alp * e0)", "(Ns + adt * e0)", NPINS),
    ("App. C dJ/dE thick factor", "m1.c", "dthick * (3.0 - 2.0 * W2) * (W2 - 1.0)",
     "dthick * (3.0 - 2.0 * W2) * (W2 + 1.0)", [IM.check_implicit_jacobian]),
    ("App. C dH/dF last term sign", "m1.c", "dthin * W * tE0 * fh[i] * s->v[j];",
     "(-dthin) * W * tE0 * fh[i] * s->v[j];", [IM.check_implicit_jacobian]),
    ("App. C calJ_0j advection sign", "m1.c", "(ks * dJdF[j] + kas * s->v[j])", "(ks * dJdF[j] - kas * s->v[j])",
     [IM.check_implicit_jacobian]),
    ("coupled exchange: fluid energy gains", "m1.c", "if (couple) U[24 * N + q] -= U[(32 + 4 * sp) * N + q] - E0;",
     "if (couple) U[24 * N + q] += U[(32 + 4 * sp) * N + q] - E0;", [CP.check_implicit_conserves]),
    ("coupled exchange: momentum index", "m1.c", "if (couple) U[(25 + a) * N + q] -= U[(33 + 4 * sp + a) * N + q] - F0;",
     "if (couple) U[(25 + a) * N + q] -= U[(33 + 4 * sp + (2 - a)) * N + q] - F0;", [CP.check_implicit_conserves]),
    ("coupled exchange: lepton number m_b", "m1.c", "if (couple) U[23 * N + q] -= m_b * (dN[0] - dN[1]);",
     "if (couple) U[23 * N + q] -= (dN[0] - dN[1]);", [CP.check_number_update_conserves_lepton_number]),
    ("coupled exchange: stiff slot sign", "m1.c", "fs[0] = (sp == 0 ? 0.0 : fs[0]) - alp * m.sqrtg * Sn;",
     "fs[0] = (sp == 0 ? 0.0 : fs[0]) + alp * m.sqrtg * Sn;", [CP.check_split_slots]),
    ("LES product term sign", "les.c", "+ 2.0 * (bv - vb);", "- 2.0 * (bv - vb);", [LES.check_filter_expansion]),
    ("LES second derivative factor", "les.c", "rhs[c] += 2.0 * Cj[c].a2;", "rhs[c] += Cj[c].a2;",
     [LES.check_filter_expansion]),
    ("LES B index of H_v term", "les.c", "HM[c] = Pv[5 + ii] * Hv[kk] - Pv[5 + kk] * Hv[ii]",
     "HM[c] = Pv[5 + kk] * Hv[kk] - Pv[5 + ii] * Hv[ii]", [LES.check_filter_expansion]),
    ("LES xi 24", "les.c", "xi = cbrt(m.det) * D2 / 24.0;", "xi = cbrt(m.det) * D2 / 12.0;", [LES.check_assembly]),
    ("LES divergence sign", "les.c", "rhs[30 * N + p] += (gxz[p + st[0]] - gxz[p - st[0]]) / dx2 + ",
     "rhs[30 * N + p] += (gxz[p + st[0]] - gxz[p - st[0]]) / dx2 - ", [LES.check_assembly]),
]


def _build_mutant(tmp, fname, old, new):
    src = os.path.join(tmp, "src")
    shutil.copytree(ORACLE_DIR, src, ignore=shutil.ignore_patterns("*.so", "__pycache__", "*.py"))
    path = os.path.join(src, fname)
    text = open(path).read()
    assert text.count(old) == 1, (fname, old)
    open(path, "w").write(text.replace(old, new))
    out = os.path.join(tmp, "libmutant.so")
    srcs = [os.path.join(src, s) for s in obuild.SOURCES + obuild.EXTRA if os.path.exists(os.path.join(src, s))]
    subprocess.check_call(["gcc", "-std=gnu99", "-O1", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-w", "-o", out] + srcs + ["-lm"])
    return out


@pytest.fixture(scope="module")
def mutant_libs():
    tmp = tempfile.mkdtemp(prefix="orc_mut_")
    try:
        dirs = [os.path.join(tmp, "m%02d" % i) for i in range(len(MUTANTS))]
        for d in dirs:
            os.makedirs(d)
        with ThreadPoolExecutor(max_workers=4) as ex:
            libs = list(ex.map(lambda a: _build_mutant(a[0], *a[1][1:4]), zip(dirs, MUTANTS)))
        yield dict(zip([m[0] for m in MUTANTS], libs))
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


@pytest.mark.parametrize("mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_slip(orc, mutant_libs, mut):
    name, _, _, _, checks = mut
    old = orc.use_library(mutant_libs[name])
    try:
        caught = []
        for chk in checks:
            try:
                chk(orc)
            except AssertionError:
                caught.append(chk.__name__)
        assert caught, "no pin caught the planted slip: %s" % name
    finally:
        orc._LIB = old
