"""Mutation check of the oracle's pins.

Each entry below plants one plausible mistake in a copy of
oracle/casim_oracle.c (a dropped factor, a wrong exponent, Gamma argument,
density, latent heat, index or branch), compiles the copy into a temporary
directory and runs the oracle's pin tests against it.  Every mutation must
make at least one pin fail: a mistake that passes every pin would mean that
part of the oracle is not fixed by anything but itself.  The unmutated copy,
built the same way, must pass.  Everything runs on the CPU.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "casim_oracle.c")
PIN_TESTS = ["tests/test_oracle_pins.py", "tests/test_oracle_process_golden.py"]

# (name, text in casim_oracle.c, replacement)
MUTATIONS = [
    ("REVP 2pi -> pi", "r[REVP] = 2.0 * PI * Gl", "r[REVP] = PI * Gl"),
    ("DEPI 2pi -> pi", "r[DEPI] = 2.0 * PI * Gi", "r[DEPI] = PI * Gi"),
    ("DEPS lambda^-2 -> lambda^-3", "N0_S / (rho * ls * ls);", "N0_S / (rho * ls * ls * ls);"),
    ("GACW Gamma(3+b) -> Gamma(4+b)", "tgamma(3.0 + bg)", "tgamma(4.0 + bg)"),
    ("SACI efficiency dropped", "r[SACI] = exp(0.025 * (T - T_0)) * q[I] * coll", "r[SACI] = q[I] * coll"),
    ("SMLT L_f -> L_v", "N0_S / (rho * LF * ls * ls)", "N0_S / (rho * LV * ls * ls)"),
    ("D_v exponent 1", "pow(T / T_0, DV_EXP)", "(T / T_0)"),
    ("G_l T^2 -> T", "LV * LV / (K_A * R_V * T * T)", "LV * LV / (K_A * R_V * T)"),
    ("G_i T^2 -> T", "LS * LS / (K_A * R_V * T * T)", "LS * LS / (K_A * R_V * T)"),
    ("V_q without /6", "a * tgamma(4.0 + b) / (6.0 * lb)", "a * tgamma(4.0 + b) / lb"),
    ("V_n Gamma(1+b) -> Gamma(2+b)", "a * tgamma(1.0 + b) / lb", "a * tgamma(2.0 + b) / lb"),
    ("fall speeds rho0/rho without sqrt", "double rfac = sqrt(RHO_0 / rho);\n    double lb",
     "double rfac = RHO_0 / rho;\n    double lb"),
    ("collection rho0/rho without sqrt", "double rfac = sqrt(RHO_0 / rho);\n\n",
     "double rfac = RHO_0 / rho;\n\n"),
    ("ice slope with rho_w", "double rx = (cat == 0) ? RHO_W : RHO_I;", "double rx = RHO_W;"),
    ("graupel slope with rho_s", "double rx = (cat == 2) ? RHO_S : RHO_G;", "double rx = RHO_S;"),
    ("graupel fall speed with snow's a", "double a = FALL_A[cat], b", "double a = FALL_A[cat == 3 ? 2 : cat], b"),
    ("snow slope cube root", "pow(PI * rx * n0 / (rho * q), 0.25)", "cbrt(PI * rx * n0 / (rho * q))"),
    ("AUTO q_c exponent", "pow(q[C], 2.47)", "pow(q[C], 2.74)"),
    ("AUTO N_c without rho", "double Nc = n[C] * rho * 1e-6;", "double Nc = n[C] * 1e-6;"),
    ("ACCR exponent", "pow(q[C] * q[R], 1.15)", "pow(q[C] * q[R], 1.5)"),
    ("FRZR lambda^-7 -> lambda^-6", "pow(lr, -7.0)", "pow(lr, -6.0)"),
    ("FRZR without the -1", "(exp(BIGG_A * (T_0 - T)) - 1.0)", "exp(BIGG_A * (T_0 - T))"),
    ("IAUT without threshold", "(q[I] - Q_I0);", "q[I];"),
    ("SACW collects ice", "if (cP) r[SACW] = q[C] * coll;", "if (cP) r[SACW] = q[I] * coll;"),
    ("REVP while cloud present", "if (rP && q[C] == 0.0 && Sl < 1.0)", "if (rP && Sl < 1.0)"),
    ("adjustment dq with L_s", "double dq = CP * delta / LV;", "double dq = CP * delta / LS;"),
    ("Cooper coefficient", "5.0 * exp(0.304 * (T_0 - w->T))", "5.0 * exp(0.0304 * (T_0 - w->T))"),
    ("freezing heat with L_v", "        addT(w, d, LF * m / CP);\n    }\n    if (w->T > T_0",
     "        addT(w, d, LV * m / CP);\n    }\n    if (w->T > T_0"),
    ("rain number sink at cloud mean mass", "nsink[R] = sinkq[R] * mm_r;", "nsink[R] = sinkq[R] * mm_c;"),
    ("AUTO number times m_r0", "auto_ / M_R0", "auto_ * M_R0"),
    ("rain evaporation heat with L_s", "- revp * LV", "- revp * LS"),
    ("melting heat sign", "- (smlt + gmlt) * LF) / CP", "+ (smlt + gmlt) * LF) / CP"),
    ("substeps floor", "ceil(V_MAX[c] * dt / dzmin)", "floor(V_MAX[c] * dt / dzmin)"),
    ("sed number flux at V_q", "Fn[k] = rho[k] * n[k] * vn;", "Fn[k] = rho[k] * n[k] * vq;"),
    ("sed flux divergence with dz[0]", "(fin_q - Fq[k]) / (rho[k] * dz[k])", "(fin_q - Fq[k]) / (rho[k] * dz[0])"),
    ("ice saturation constant", "22.452 * Tc / (Tc + 272.55)", "22.452 * Tc / (Tc + 243.5)"),
]


def _build(src_text, outdir):
    os.makedirs(outdir, exist_ok=True)
    c = os.path.join(outdir, "casim_oracle.c")
    h = os.path.join(ROOT, "oracle", "casim_oracle.h")
    with open(c, "w") as f:
        f.write(src_text)
    so = os.path.join(outdir, "liboracle.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
                    "-shared", "-I", os.path.dirname(h), "-o", so, c, "-lm"], check=True,
                   capture_output=True)
    return so


def _run_pins(so):
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=so, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PIN_TESTS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    return r.returncode, r.stdout[-2000:]


def test_every_mutation_fails_a_pin(tmp_path):
    with open(SRC) as f:
        base = f.read()
    for name, old, new in MUTATIONS:
        assert base.count(old) == 1, "mutation target not unique or missing: %s" % name

    def job(i):
        if i < 0:
            return "unmutated", _run_pins(_build(base, str(tmp_path / "base")))
        name, old, new = MUTATIONS[i]
        return name, _run_pins(_build(base.replace(old, new), str(tmp_path / ("m%02d" % i))))

    workers = max(1, min(8, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(job, range(-1, len(MUTATIONS))))
    name, (rc, out) = results[0]
    assert rc == 0, "the unmutated oracle must pass its pins:\n" + out
    survivors = [name for name, (rc, out) in results[1:] if rc == 0]
    assert not survivors, "mutations that pass every pin: %s" % survivors
