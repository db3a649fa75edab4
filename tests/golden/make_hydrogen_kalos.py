"""Writes hydrogen_kalos.json: the oracle's iteration of Sec. 6.2 (mu, E and rho's leaf count per step)
for the cases the GPU parity test runs.  Calls only the oracle.

    python tests/golden/make_hydrogen_kalos.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import hydrogen as H  # noqa: E402

CASES = [dict(k=5, eps=1e-3, L=10.0, jmax=7, mu0=0.8, iters=3),
         dict(k=6, eps=1e-4, L=12.0, jmax=8, mu0=1.2, iters=2)]


def main():
    out = []
    for c in CASES:
        leaves = []
        hist = H.kalos(c["k"], c["eps"], c["L"], c["jmax"], mu0=c["mu0"], iters=c["iters"], leaves=leaves)
        out.append(dict(c, mu=[m for m, _ in hist], E=[e for _, e in hist], rho_leaves=leaves))
        print(out[-1], flush=True)
    with open(os.path.join(HERE, "hydrogen_kalos.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
