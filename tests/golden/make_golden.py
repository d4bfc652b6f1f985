"""Write tests/golden/exact_values.json from the exact references in oracle.exact.

The paper prints no numerical worked example, so the stored values are exact
spin-model results (enumeration, transfer matrix, closed forms) at the
workloads the tests use.  Run from the repository root:

    python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact as E  # noqa: E402


def main():
    vals = []

    def add(kind, args, value, cite):
        vals.append(dict(kind=kind, args=args, value=value, cite=cite))

    for h in (0.0, 0.1):
        r = E.brute_force(E.torus_adjacency((4, 4)), 0.4, h=h)
        add("brute_force", dict(L=[4, 4], beta=0.4, h=h), {k: r[k] for k in ("be", "m", "m2", "am")},
            "Sec. 2 partition sum, 2^16 states")
    for beta in (0.4, E.BETA_C_2D):
        r = E.row_transfer_2d(8, 8, beta)
        add("row_transfer_2d", dict(L=[8, 8], beta=beta), r, "8x8 torus, row transfer matrix")
    r = E.ring_1d(12, 0.5, h=0.1)
    add("ring_1d", dict(N=12, beta=0.5, h=0.1), r, "periodic chain closed form")
    for N in (8, 12, 16):
        r = E.infinite_range(N, 1.0)
        add("infinite_range", dict(N=N, betaJ=1.0), {"be": r["be"]}, "App. A energy formula")
    for beta in (0.4, E.BETA_C_2D, 0.5):
        add("onsager", dict(beta=beta), {"be": E.onsager_energy(beta)}, "Onsager 2D energy")
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_values.json")
    with open(out, "w") as f:
        json.dump(dict(source="oracle.exact", values=vals), f, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
