"""Write the stored expected values used by the GPU parity tests.

Calls only the oracle (and the seeded input recipes); run from the repo root:
    python tests/golden/make_golden.py
Writes
  tests/golden/config2_jk_blocks.json: J and K shell blocks of the 40-atom
    s,s,p,d workload (Schwarz tau = 1e-10), each computed by the oracle's
    plain block sums J_ab = sum (ab|cd) D_cd and K_ab = sum (ac|bd) D_cd;
  tests/golden/grad_small.json: E2 and its nuclear gradient at fixed D
    (oracle, every quartet, no screening) for the 4-atom s,s,p workload, a
    4-atom cut of the 60-atom s,s,p,d workload, and 3 atoms of s,p,d shells
    with 1-4 primitives and two coincident centres;
  tests/golden/scf_small.json: the converged energy of the oracle's RHF loop
    on the 4-atom cut of the 40-atom s,s,p,d workload.
    python tests/golden/make_golden.py [jk] [grad] [scf]
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


def grad_cases():
    """The small gradient workloads (seeded recipes; shared with the tests)."""
    import numpy as np
    cases = {}
    c1 = inputs.make_config(1)
    cases["config1"] = (c1["basis"], c1["D"])
    c5 = inputs.make_config(5, natom=4)
    cases["config5_4atoms"] = (c5["basis"], c5["D"])
    rng = np.random.default_rng(31)
    b = inputs.random_shells(rng, 3, [0, 1, 2], box=2.5, nprim_range=(1, 4), exp_range=(0.2, 8.0))
    b["xyz"][2] = b["xyz"][0]  # atoms 0 and 2 coincide
    C = rng.standard_normal((b["nbf"], 4)) * 0.5
    D = C @ C.T
    cases["mixed_k_coincident"] = (b, 0.5 * (D + D.T))
    return cases


def main_grad():
    out = {"what": "E2 and dE2/dR at fixed D, oracle over every quartet (no screening)", "cases": {}}
    for name, (b, D) in grad_cases().items():
        J, K, _ = oracle.build_jk(b, D, 0.0)
        g = oracle.grad_e2(b, D)
        out["cases"][name] = {"e2": oracle.e2(J, K, D), "grad": [[float(v) for v in r] for r in g]}
        print(name, "natom", b["xyz"].shape[0], "nbf", b["nbf"], flush=True)
    with open(os.path.join(HERE, "grad_small.json"), "w") as fh:
        json.dump(out, fh, indent=1)


def main_scf():
    from oracle import scf
    out = {"what": "converged RHF energy of the oracle's loop (tau as the recipe, e_tol 1e-12, err_tol 1e-9)",
           "cases": {}}
    cfg = inputs.make_config(2, natom=4)
    Z, nocc = inputs.scf_system(cfg)
    r = scf.rhf(cfg["basis"], Z, nocc, tau=cfg["tau"], e_tol=1e-12, err_tol=1e-9)
    assert r["converged"]
    out["cases"]["config2_4atoms"] = {"energy": r["energy"], "iterations": r["iterations"], "nocc": nocc,
                                      "Z": [float(z) for z in Z]}
    print("config2_4atoms", r["energy"], r["iterations"], flush=True)
    with open(os.path.join(HERE, "scf_small.json"), "w") as fh:
        json.dump(out, fh, indent=1)


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
    what = sys.argv[1:] or ["jk", "grad", "scf"]
    if "jk" in what:
        main()
    if "grad" in what:
        main_grad()
    if "scf" in what:
        main_scf()
