"""Writes colella_exact_j4m.json: the exact solution (gamma = 2) of Colella's explosion tube
(Sec. 5.1.4 states, pressure ratio 1e5) at t = 0.02 on the 4000-cell tube of the
benchmark (dx = 2.5e-4, jump at x = 0.5), sampled at the cell centres of every fourth cell
(j = 4m, m = 0..999), with the positions of its waves and the mask of the cells at least
MARGIN from every wave and from both ends of the tube (the shock reaches x = 1 at
t = 0.0197 and the rarefaction head leaves through x = 0 at t = 0.011, so both ends have
seen a wave pass through the outflow sides by t = 0.02).  Uses only oracle.riemann (the
textbook exact Riemann solver).  Run from the repository root:
    python tests/golden/make_colella_exact.py
"""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import riemann  # noqa: E402

LEFT, RIGHT = (1.0, 0.0, 0.0, 1000.0), (1.0, 0.0, 0.0, 0.01)
NX, DX, T_END, X0, GAMMA = 4000, 2.5e-4, 0.02, 0.5, 2.0
MARGIN = 0.02


def main():
    j = np.arange(0, NX, 4)
    x = (j + 0.5) * DX
    rho, u, T = riemann.tube_solution(LEFT, RIGHT, x, X0, T_END, GAMMA)
    pl, pr = LEFT[0] * LEFT[3], RIGHT[0] * RIGHT[3]
    ps, us = riemann.star_state((LEFT[0], 0.0, pl), (RIGHT[0], 0.0, pr), GAMMA)
    al = math.sqrt(GAMMA * pl / LEFT[0])
    ar = math.sqrt(GAMMA * pr / RIGHT[0])
    head = X0 - al * T_END
    tail = X0 + (us - al * (ps / pl) ** ((GAMMA - 1) / (2 * GAMMA))) * T_END
    contact = X0 + us * T_END
    shock_speed = ar * math.sqrt((GAMMA + 1) / (2 * GAMMA) * ps / pr + (GAMMA - 1) / (2 * GAMMA))
    shock = X0 + shock_speed * T_END
    smooth = np.ones(len(x), dtype=bool)
    for w in (tail, contact, shock):
        smooth &= np.abs(x - w) > MARGIN
    smooth &= (x > MARGIN) & (x < 1.0 - MARGIN)
    out = {"about": "exact gamma = 2 solution of the Colella tube at t = 0.02, cells j = 4m of 4000 (dx = 2.5e-4), "
                    "written by tests/golden/make_colella_exact.py from oracle.riemann",
           "j": j.tolist(), "rho": rho.tolist(), "u": u.tolist(), "T": T.tolist(),
           "waves": {"rarefaction_head": head, "rarefaction_tail": tail, "contact": contact, "shock": shock},
           "star": {"p": ps, "u": us}, "margin": MARGIN, "smooth": smooth.astype(int).tolist()}
    with open(os.path.join(HERE, "colella_exact_j4m.json"), "w") as fh:
        json.dump(out, fh, indent=0)


if __name__ == "__main__":
    main()
