"""Write the stored expected values used by the GPU parity tests.

Calls only the oracle (and the seeded input recipes); run from the repo root:
    python tests/golden/make_golden.py
Writes tests/golden/config2_jk_blocks.json: J and K shell blocks of the
40-atom s,s,p,d workload (Schwarz tau = 1e-10), each computed by the oracle's
plain block sums J_ab = sum (ab|cd) D_cd and K_ab = sum (ac|bd) D_cd.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2412_13203_amd import inputs  # noqa: E402

# sampled shell blocks (A, B): every pair class, diagonal and off-diagonal,
# first / middle / last atoms (4 shells per atom: s, s, p, d)
BLOCKS = [(0, 0), (5, 1), (2, 2), (3, 3), (3, 78), (83, 3), (159, 159), (158, 40), (123, 67), (97, 98)]


def main():
    cfg = inputs.make_config(2)
    b, D = cfg["basis"], cfg["D"]
    Q = oracle.schwarz(b)
    Js, Ks = oracle.jk_blocks(b, D, cfg["tau"], BLOCKS, Q)
    out = {
        "what": "J and K shell blocks, 40-atom s,s,p,d lattice workload, seed 2, tau 1e-10, oracle block sums",
        "tau": cfg["tau"],
        "blocks": [list(x) for x in BLOCKS],
        "J": [[float(v) for v in j.ravel()] for j in Js],
        "K": [[float(v) for v in k.ravel()] for k in Ks],
    }
    with open(os.path.join(HERE, "config2_jk_blocks.json"), "w") as fh:
        json.dump(out, fh)
    print("wrote", len(BLOCKS), "blocks")


if __name__ == "__main__":
    main()
