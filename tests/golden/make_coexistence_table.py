"""Writes coexistence.txt from the oracle's multiprecision solvers only
(critical point and spinodals of Eq. 15, Maxwell rule of Eq. 11, mechanical
stability condition of Eq. 9).  Run: python tests/golden/make_coexistence_table.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import coexist  # noqa: E402

TR = (0.5, 0.6, 0.7, 0.8, 0.9)
EPS = (0.0, 1.0, 1.86, 2.0)


def main():
    Tc, rc, pc = coexist.critical_point()
    lines = ["# Carnahan-Starling coexistence, a = 0.5, b = 4 (eta = rho), R = 1, G = -1",
             "# critical point: T_c %.16e rho_c %.16e p_c %.16e" % (Tc, rc, pc),
             "# columns: T/Tc T rho_s_gas rho_s_liq maxwell_rho_g maxwell_rho_l maxwell_p0"
             + "".join(" eq9_eps%s_rho_g eq9_eps%s_rho_l" % (e, e) for e in EPS),
             "# nan: Eq. 9 has no solution with p0 >= 0"]
    for tr in TR:
        T = coexist.temperature(tr)
        sg, sl = coexist.spinodals(T)
        g, l, p0 = coexist.maxwell(T)
        row = [tr, T, sg, sl, g, l, p0]
        for e in EPS:
            sol = coexist.mechanical_stability(T, e)
            row += [sol[0], sol[1]] if sol else [float("nan"), float("nan")]
        lines.append(" ".join("%.12e" % v for v in row))
        print(lines[-1], flush=True)
    with open(os.path.join(HERE, "coexistence.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
