"""The input generators use the constants the paper prints (golden fixture
tests/golden/paper_constants.json, each entry citing its section)."""
import json
import os

from paper_1810_03931_amd import inputs as I

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_keller_miksis_material_constants():
    g = GOLD["keller_miksis_material"]
    assert I.C_L == g["c_L_m_per_s"] and I.RHO_L == g["rho_L_kg_per_m3"]
    assert I.P_INF == g["P_inf_Pa"] and I.P_V == g["p_V_Pa"]
    assert I.SIGMA == g["sigma_N_per_m"] and I.MU_L == g["mu_L_Pa_s"] and I.GAMMA == g["gamma"]


def test_relief_valve_and_solver_settings():
    g = GOLD["relief_valve"]
    pb = I.relief_valve_sweep(64)
    assert tuple(pb.params[[0, 1, 2, 4], 0]) == (g["kappa"], g["delta"], g["beta"], g["r"])
    o, e = GOLD["ode_properties_example"], GOLD["event_properties_example"]
    for name in ("duffing_rkck45", "keller_miksis", "relief_valve"):
        opts = I.CONFIGS[name]().options if name != "keller_miksis" else \
            I.keller_miksis_sweep(256).options
        assert opts["rtol"] == o["rtol"] and opts["atol"] == o["atol"]
        assert opts["h_max"] == o["h_max"] and opts["h_min"] == o["h_min"]
        assert opts["grow"] == o["grow"] and opts["shrink"] == o["shrink"]
        for ev in opts.get("events", []):
            assert ev["tolerance"] == e["tolerance"] and ev["direction"] == e["direction_local_maximum"]
