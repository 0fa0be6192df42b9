"""Write tests/golden/riemann_exact.json from the exact shallow-water solutions
in oracle.exact (calls nothing but oracle/).  Run: python tests/golden/make_golden.py"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact  # noqa: E402


def main():
    dam = exact.riemann(2.0, 0.0, 1.0, 0.0, 1.0)
    inc = exact.riemann(1.5, 0.5, 1.0, 0.0, 1.0)
    hw, sref = exact.wall_reflection(inc.hs, inc.us, 1.0)
    out = {
        "note": "exact shallow-water Riemann solutions, g = 1, written by make_golden.py",
        "dam_break": {"hl": 2.0, "hr": 1.0, "h_star": dam.hs, "u_star": dam.us,
                      "shock_speed": dam.sr, "rarefaction_head": dam.ul - 2.0 ** 0.5,
                      "rarefaction_tail": dam.wave_speeds()["left_tail"]},
        "wall_reflection": {"h_in": 1.5, "u_in": 0.5, "h0": 1.0, "h_mid": inc.hs, "u_mid": inc.us,
                            "incident_shock_speed": inc.sr, "left_shock_speed": inc.sl,
                            "h_wall": hw, "reflected_shock_speed": sref},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "riemann_exact.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=2)
    print(path)


if __name__ == "__main__":
    main()
