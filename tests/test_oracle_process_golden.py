"""Pins of the oracle's process rates and fall speeds against values reached
by another route: numerical integration of published single-particle laws
over exponential size distributions (tests/golden/gen_process_points.py,
which imports nothing of the oracle).  The oracle evaluates closed-form
moments, so agreement fixes every rate's magnitude -- its slope power, Gamma
argument, 2 pi factors, latent heat, diffusivity exponent and air-density
correction -- not only its sign and gate."""
import importlib.util
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RATES = ("AUTO", "ACCR", "REVP", "DEPI", "DEPS", "IAUT", "SACI", "SACW", "GACW", "FRZR", "SMLT", "GMLT")
CAT = {"r": 0, "i": 1, "s": 2, "g": 3}


def _golden():
    with open(os.path.join(GOLDEN, "process_points.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("idx", range(5))
def test_rates_match_integrated_single_particle_laws(oracle_lib, idx):
    g = _golden()
    pt = g["rates"][idx]
    got = oracle_lib.point_rates(pt["T"], pt["p"], pt["rho"], np.array(pt["q"]), np.array(pt["n"]))
    for j, name in enumerate(RATES):
        if name in pt["expect"]:
            want = pt["expect"][name]
            assert got[j] == pytest.approx(want, rel=g["rel_tol"]), (pt["name"], name, got[j], want)
        else:
            assert got[j] == 0.0, (pt["name"], name, got[j])


@pytest.mark.parametrize("idx", range(8))
def test_fall_speeds_from_single_level_surface_flux(oracle_lib, idx):
    """One level, one substep, every speed below its cap: the surface receives
    rho q V_q dt of mass and rho n V_n dt of number."""
    fs = _golden()["fall"][idx]
    c = CAT[fs["cat"]]
    st = np.zeros((14, 1, 1))
    st[0], st[1], st[2] = 280.0, 8e4, fs["rho"]
    st[6 + 2 * c] = fs["q"]
    st[7 + 2 * c] = fs["n"]
    dz, dt = np.array([1000.0]), 2.0
    assert oracle_lib.nsub(dz, dt) == [1, 1, 1, 1]
    tend, sfc = oracle_lib.step(st, dz, dt, stages=oracle_lib.ST_SED)
    vq = sfc[c, 0] / (fs["rho"] * fs["q"] * dt)
    vn = sfc[4 + c, 0] / (fs["rho"] * fs["n"] * dt)
    tol = _golden()["rel_tol"]
    assert vq == pytest.approx(fs["v_mass"], rel=tol), (fs, vq)
    assert vn == pytest.approx(fs["v_number"], rel=tol), (fs, vn)
    # the level loses what reaches the surface
    assert -tend[4 + 2 * c, 0, 0] * dt * fs["rho"] * dz[0] == pytest.approx(sfc[c, 0], rel=1e-13)


def test_golden_file_is_what_the_generator_writes(tmp_path):
    spec = importlib.util.spec_from_file_location("gen_process_points",
                                                  os.path.join(GOLDEN, "gen_process_points.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    g = _golden()
    for pt in g["rates"]:
        fresh = gen.rates_at(pt)
        assert set(fresh) == set(pt["expect"])
        for k, v in fresh.items():
            assert v == pytest.approx(pt["expect"][k], rel=1e-12)
    for fs in g["fall"]:
        d = gen.Dist(fs["cat"], fs["q"], fs["rho"], fs["n"] if fs["cat"] in ("r", "i") else None)
        assert d.v_mass() == pytest.approx(fs["v_mass"], rel=1e-12)
        assert d.v_number() == pytest.approx(fs["v_number"], rel=1e-12)
