"""Write tests/golden/bruteforce_o3v4.json from the Fock-space brute force only.

The paper prints no numerical Green's-function values for any system, so this
fixture is generated here: G_qp(omega) of the retarded IP term (paper, Theory section,
compact GFCC expression with the X_p linear system) for one tiny synthetic
system, computed by ``oracle.fockspace`` (no working equations).  Run from the
repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.fockspace import IPBruteForce  # noqa: E402
from synth import make_system  # noqa: E402

SPEC = dict(n_occ=3, n_vir=4, n_chol=5, seed=424242, sigma_L=0.3, sigma_t1=0.08)
OMEGAS = [-1.1, -0.6, -0.35, -0.1]
ETA = 0.02


def main():
    s = make_system(SPEC["n_occ"], SPEC["n_vir"], SPEC["n_chol"], SPEC["seed"],
                    sigma_L=SPEC["sigma_L"], sigma_t1=SPEC["sigma_t1"])
    bf = IPBruteForce(s)
    rows = []
    for w in OMEGAS:
        for p in range(s.n_occ):
            for q in range(s.n_occ):
                g = bf.greens_so(w, ETA, p, q)
                rows.append({"omega": w, "p": p, "q": q, "re": g.real, "im": g.imag})
    out = {"source": "oracle.fockspace brute force; paper, Theory section (compact GFCC form, IP term)",
           "system": SPEC, "eta": ETA, "G_qp": rows}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bruteforce_o3v4.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
