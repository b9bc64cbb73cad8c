"""Writes process_points.json: expected process rates and fall speeds at
hand-picked states, computed WITHOUT the oracle.

    python tests/golden/gen_process_points.py

The oracle evaluates each rate as a closed-form moment of an exponential size
distribution.  This script reaches the same quantities by another route: it
takes the single-particle law of every process from its published source,
finds the distribution's slope by root-finding on the numerically integrated
mass, and integrates the single-particle law over the distribution by
adaptive quadrature.  A wrong power of the slope, a wrong Gamma argument, a
dropped factor of 2 or pi, a wrong latent heat or density, or a wrong
air-density correction in the oracle's closed forms therefore disagrees with
these values.  It imports nothing from ``oracle/`` and shares no code with
the GPU path.

Single-particle laws (D = diameter, m, per particle):
  * diffusional growth / evaporation of a sphere, unventilated (Mason 1971;
    Rogers & Yau 1989, ch. 7: dm/dt = 4 pi C (S - 1) G with capacitance
    C = D/2):  dm/dt = 2 pi D (S - 1) G(T, p), where
        G = 1 / (L^2 / (K_a R_v T^2) + R_v T / (D_v e_s)),
        D_v = 2.11e-5 (T / T0)^1.94 (1e5 / p)  (Pruppacher & Klett 1997,
        eq. 13-3, with the reference pressure 1000 hPa);
  * melting of a sphere, unventilated (Lin et al. 1983, eq. 32 without the
    ventilation and evaporation terms): dm/dt = 2 pi D K_a (T - T0) / L_f;
  * continuous collection of cloud or ice (Lin et al. 1983, eqs. 22, 24):
    dm/dt = (pi/4) D^2 V(D) E rho q_x;
  * Bigg (1953) immersion freezing, as used by Lin et al. (1983, eq. 26):
    a drop of volume v = (pi/6) D^3 freezes at the rate
    B' v (exp(A' (T0 - T)) - 1) per second;
  * terminal velocity V(D) = a D^b (rho0 / rho)^(1/2) (Liu & Orville 1969 for
    rain; Locatelli & Hobbs 1974 for snow and graupel; (700, 1) for ice).
Size distributions: N(D) = N0 exp(-lambda D) per m^3 of air.  Rain and
cloud ice carry a number n per kg (N0 = rho n lambda); snow and graupel have
fixed intercepts N0_s = 3e6, N0_g = 4e6 m^-4.  Particles are spheres of
density rho_w (rain), rho_i = 500 (ice), rho_s = 100, rho_g = 400 kg m^-3.
Rates per kg of air are (1/rho) * integral of dm/dt N(D) dD.  Mass-weighted
and number-weighted fall speeds are the m(D)- and 1-weighted means of V(D).

Ice autoconversion has no size integral: its value is the Lin et al. (1983,
eq. 21) expression 1e-3 exp(0.025 (T - T0)) (q_i - q_i0), evaluated here at
q_i0 = 1e-4.
"""
from __future__ import annotations

import json
import math
import os

from scipy import integrate, optimize

# ---- constants (the scheme's published values) ---------------------------
R_D, R_V = 287.04, 461.5
EPS = R_D / R_V
CP = 1005.0
LV, LS = 2.501e6, 2.834e6
LF = LS - LV
T0 = 273.15
K_A = 2.4e-2
DV0, DV_EXP = 2.11e-5, 1.94
RHO0 = 1.225
RHO_X = {"r": 1000.0, "i": 500.0, "s": 100.0, "g": 400.0}
N0_FIXED = {"s": 3e6, "g": 4e6}
FALL = {"r": (842.0, 0.8), "i": (700.0, 1.0), "s": (11.72, 0.41), "g": (19.3, 0.37)}
D_BOUNDS = {"r": (2e-5, 5e-3), "i": (1e-6, 1e-3), "s": (1e-5, 1e-2), "g": (1e-5, 1e-2)}
BIGG_A, BIGG_B = 0.66, 100.0
Q_I0 = 1e-4


def e_liquid(T):                     # Bolton (1980), Pa
    tc = T - T0
    return 611.2 * math.exp(17.67 * tc / (tc + 243.5))


def e_ice(T):                        # Buck (1981), over ice, Pa
    tc = T - T0
    return 611.15 * math.exp(22.452 * tc / (tc + 272.55))


def q_sat(e, p):
    return EPS * e / (p - (1.0 - EPS) * e)


def diffusivity(T, p):
    return DV0 * (T / T0) ** DV_EXP * (1e5 / p)


def growth_G(T, p, L, es):
    return 1.0 / (L * L / (K_A * R_V * T * T) + R_V * T / (diffusivity(T, p) * es))


def moment_integral(f, lam):
    """integral_0^inf f(D) exp(-lam D) dD by adaptive quadrature, cut at
    D = 80/lam (the tail beyond is below e^-70 of the integrand's scale)."""
    top = 80.0 / lam
    pts = [top * x for x in (0.005, 0.02, 0.05, 0.1, 0.2, 0.4)]
    val, err = integrate.quad(lambda D: f(D) * math.exp(-lam * D), 0.0, top, points=pts,
                              limit=400, epsabs=0.0, epsrel=1e-13)
    return val


class Dist:
    """Exponential distribution of category cat holding mass q (kg/kg) and,
    for rain and ice, number n (per kg), in air of density rho."""

    def __init__(self, cat, q, rho, n=None):
        self.cat, self.rho = cat, rho
        mass = lambda D: math.pi / 6.0 * RHO_X[cat] * D ** 3

        def n0_of(lam):
            return rho * n * lam if cat in ("r", "i") else N0_FIXED[cat]

        def resid(loglam):
            lam = math.exp(loglam)
            return math.log(moment_integral(mass, lam) * n0_of(lam) / rho) - math.log(q)
        loglam = optimize.brentq(resid, math.log(10.0), math.log(1e8), xtol=1e-15, rtol=1e-15, maxiter=500)
        self.lam = math.exp(loglam)
        self.n0 = n0_of(self.lam)
        lo, hi = D_BOUNDS[cat]
        # every state below is chosen with its mean diameter inside the clamps
        assert lo < 1.0 / self.lam < hi, (cat, 1.0 / self.lam)
        self.mass = mass

    def per_kg(self, dmdt):
        """(1/rho) integral dm/dt N(D) dD."""
        return self.n0 * moment_integral(dmdt, self.lam) / self.rho

    def speed(self, D):
        a, b = FALL[self.cat]
        return a * D ** b * math.sqrt(RHO0 / self.rho)

    def v_mass(self):
        return moment_integral(lambda D: self.mass(D) * self.speed(D), self.lam) / \
            moment_integral(self.mass, self.lam)

    def v_number(self):
        return moment_integral(self.speed, self.lam) / moment_integral(lambda D: 1.0, self.lam)


def rates_at(pt):
    """Expected values of the open-gate rates at state pt (dict)."""
    T, p, rho = pt["T"], pt["p"], pt["rho"]
    q, n = pt["q"], pt["n"]          # q: v c r i s g; n: -, c, r, i, s, g
    esl, esi = e_liquid(T), e_ice(T)
    Sl, Si = q[0] / q_sat(esl, p), q[0] / q_sat(esi, p)
    Gl, Gi = growth_G(T, p, LV, esl), growth_G(T, p, LS, esi)
    out = {}
    rain = Dist("r", q[2], rho, n[2]) if q[2] > 0 else None
    ice = Dist("i", q[3], rho, n[3]) if q[3] > 0 else None
    snow = Dist("s", q[4], rho) if q[4] > 0 else None
    grau = Dist("g", q[5], rho) if q[5] > 0 else None
    cold, hot = T < T0, T > T0
    # Khairoutdinov & Kogan (2000), eqs. 29 and 33: N_c in cm^-3
    if q[1] > 0 and n[1] > 0:
        out["AUTO"] = 1350.0 * q[1] ** 2.47 * (n[1] * rho * 1e-6) ** -1.79
    if q[1] > 0 and rain:
        out["ACCR"] = 67.0 * (q[1] * q[2]) ** 1.15
    if rain and q[1] == 0.0 and Sl < 1.0:
        out["REVP"] = rain.per_kg(lambda D: 2.0 * math.pi * D * (1.0 - Sl) * Gl)
    if ice and cold:
        out["DEPI"] = ice.per_kg(lambda D: 2.0 * math.pi * D * (Si - 1.0) * Gi)
    if snow and cold:
        out["DEPS"] = snow.per_kg(lambda D: 2.0 * math.pi * D * (Si - 1.0) * Gi)
    if ice and cold and q[3] > Q_I0:
        out["IAUT"] = 1e-3 * math.exp(0.025 * (T - T0)) * (q[3] - Q_I0)
    if snow and cold and ice:
        E = math.exp(0.025 * (T - T0))
        out["SACI"] = snow.per_kg(lambda D: math.pi / 4.0 * D * D * snow.speed(D) * E * rho * q[3])
    if snow and cold and q[1] > 0:
        out["SACW"] = snow.per_kg(lambda D: math.pi / 4.0 * D * D * snow.speed(D) * rho * q[1])
    if grau and cold and q[1] > 0:
        out["GACW"] = grau.per_kg(lambda D: math.pi / 4.0 * D * D * grau.speed(D) * rho * q[1])
    if rain and cold:
        frz = BIGG_B * (math.exp(BIGG_A * (T0 - T)) - 1.0)
        out["FRZR"] = rain.per_kg(lambda D: rain.mass(D) * frz * math.pi / 6.0 * D ** 3)
    if snow and hot:
        out["SMLT"] = snow.per_kg(lambda D: 2.0 * math.pi * D * K_A * (T - T0) / LF)
    if grau and hot:
        out["GMLT"] = grau.per_kg(lambda D: 2.0 * math.pi * D * K_A * (T - T0) / LF)
    return out


# Hand-picked states: two cold regimes (ice-supersaturated / subsaturated),
# a second cold point at other densities and masses, and a melting regime.
# Vapour is given as a fraction of liquid / ice saturation so the states are
# readable; the stored value is the resulting q_v.
def _states():
    pts = []

    def add(name, T, p, rho, qv, qc, nc, qr, nr, qi, ni, qs, ns, qg, ng):
        pts.append({"name": name, "T": T, "p": p, "rho": rho,
                    "q": [qv, qc, qr, qi, qs, qg], "n": [0.0, nc, nr, ni, ns, ng]})

    T, p = 255.0, 5.5e4
    qsl, qsi = q_sat(e_liquid(T), p), q_sat(e_ice(T), p)
    add("cold_supersat_ice", T, p, 0.75, 0.5 * (qsl + qsi), 2e-4, 1e8, 1e-4, 1e4, 2e-4, 1e5, 1.5e-4, 1e5,
        1e-4, 1e5)
    T, p = 263.0, 7e4
    qsl, qsi = q_sat(e_liquid(T), p), q_sat(e_ice(T), p)
    add("cold_second", T, p, 0.93, 0.95 * qsl, 5e-4, 2e8, 3e-4, 5e3, 1.2e-4, 3e5, 6e-5, 1e5, 4e-4, 1e5)
    T, p = 248.0, 4.5e4
    qsi = q_sat(e_ice(T), p)
    add("cold_subsat_ice", T, p, 0.63, 0.7 * qsi, 0.0, 0.0, 0.0, 0.0, 5e-5, 2e5, 8e-5, 1e5, 0.0, 0.0)
    T, p = 278.0, 8.5e4
    qsl = q_sat(e_liquid(T), p)
    add("melting", T, p, 1.05, 0.7 * qsl, 0.0, 0.0, 2e-4, 1e4, 0.0, 0.0, 1e-4, 1e5, 1.2e-4, 2e5)
    T, p = 291.0, 9.6e4
    qsl = q_sat(e_liquid(T), p)
    add("warm_evaporation", T, p, 1.14, 0.55 * qsl, 0.0, 0.0, 6e-5, 3e3, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    return pts


# Single-level sedimentation states with every speed below its cap.
def _fall_states():
    return [
        {"cat": "r", "q": 1e-4, "n": 1e4, "rho": 0.85},
        {"cat": "r", "q": 4e-4, "n": 2e3, "rho": 1.15},
        {"cat": "i", "q": 1e-4, "n": 1e5, "rho": 0.6},
        {"cat": "i", "q": 3e-5, "n": 4e5, "rho": 0.9},
        {"cat": "s", "q": 1e-4, "n": 1e5, "rho": 0.8},
        {"cat": "s", "q": 5e-4, "n": 1e5, "rho": 0.55},
        {"cat": "g", "q": 1e-4, "n": 1e5, "rho": 0.8},
        {"cat": "g", "q": 2e-3, "n": 1e5, "rho": 1.1},
    ]


def main():
    out = {
        "_source": __doc__.strip().split("\n\n")[0] + " See gen_process_points.py for the single-particle "
                   "laws and their sources (Mason 1971; Rogers & Yau 1989; Pruppacher & Klett 1997; "
                   "Lin et al. 1983; Bigg 1953; Liu & Orville 1969; Locatelli & Hobbs 1974).",
        "rel_tol": 1e-9,
        "rates": [],
        "fall": [],
    }
    for pt in _states():
        out["rates"].append({**pt, "expect": rates_at(pt)})
    for fs in _fall_states():
        d = Dist(fs["cat"], fs["q"], fs["rho"], fs["n"] if fs["cat"] in ("r", "i") else None)
        out["fall"].append({**fs, "v_mass": d.v_mass(), "v_number": d.v_number(), "inv_lambda": 1.0 / d.lam})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "process_points.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
