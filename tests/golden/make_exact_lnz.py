"""Write exact_lnz.json: ln Z of the periodic L x L Ising model (Kaufman's
closed form, oracle/exact.py) along the linear schedules of the named
workloads and at the end points used by the schedule comparisons.

Run from the repository root:  python tests/golden/make_exact_lnz.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import mpmath  # noqa: E402

from oracle import exact  # noqa: E402


def schedule(beta_final, n):
    return [(beta_final * i) / n for i in range(n + 1)]


def main():
    mpmath.mp.prec = 160
    out = {"_about": "ln Z (natural log) of the periodic L x L Ising model, J = 1, from "
                     "Kaufman's formula; written by tests/golden/make_exact_lnz.py",
           "schedules": {}, "points": {}}
    for L, bf, n in ((8, 0.44, 101), (64, 0.4407, 200), (128, 1.0, 400), (32, 0.4407, 200)):
        betas = schedule(bf, n)
        out["schedules"]["L%d_%g_%d" % (L, bf, n)] = {
            "L": L, "beta_final": bf, "n_steps": n,
            "ln_z": [float(exact.ln_z_kaufman(L, b)) for b in betas]}
    for L in (16, 32, 64, 128):
        for bf in (0.4407, 0.44, 1.0):
            out["points"]["L%d_%g" % (L, bf)] = float(exact.ln_z_kaufman(L, bf))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_lnz.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
