"""Seeded synthetic molecules: geometry, contracted Cartesian shells, density.

This module is the only code shared by the HIP path and the oracle.  It draws
random numbers and lays them out; it computes no integral.

A basis is a dict of numpy arrays (all host memory):

  xyz            (natom, 3) float64, bohr
  shell_atom     (nshell,)  int32
  shell_l        (nshell,)  int32, 0..3
  shell_nprim    (nshell,)  int32, 1..6
  shell_prim_off (nshell,)  int32, offset into exps / coefs
  exps, coefs    (nprim,)   float64; coefs are final (they multiply the
                 unnormalized primitive Gaussians x^i y^j z^k exp(-a r^2))
  nbf            int, number of Cartesian basis functions

Shells follow the contracted form of Eq. 1 (Section 2.2): a fixed linear
combination of primitive Gaussians that share one angular momentum.  Inside a
shell the Cartesian components are ordered lexicographically (xx, xy, xz, yy,
yz, zz for d).  Normalization: each primitive is scaled to unit norm of its
x^l component, then the whole contraction is rescaled so the contracted x^l
component has unit self-overlap; every component of the shell shares that one
factor.

Workloads (the recipes below; sizes follow the five configurations named in
the design notes):
  1: 4 atoms uniform in a 4-bohr box (min separation 1.2), shells s,s,p,
     K=3, exponents log-uniform in [0.1, 50]; C is N x 4, N(0,1)*0.3.
  2: 40 atoms, jittered cubic lattice (2.5 bohr, +-0.3), shells s,s,p,d,
     K=3, exponents in [0.08, 80]; C is N x 80, N(0,1)/sqrt(N).
  3: as 2 with 120 atoms, C is N x 240.
  4: 64 molecules, atoms ~ U{8..96}, shells s,s,p,d,f, K ~ U{1..6}; per
     molecule C is N x 2*atoms.
  5: as 2 with 60 atoms, C is N x 120.
D = (C C^T + (C C^T)^T) / 2, so it is bit-symmetric.
"""
from __future__ import annotations

import math

import numpy as np

L_NAMES = "spdf"


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def cart_components(l: int):
    """Lexicographic Cartesian exponent triples (i, j, k), i+j+k = l."""
    out = []
    for i in range(l, -1, -1):
        for j in range(l - i, -1, -1):
            out.append((i, j, l - i - j))
    return out


def _dfact(n: int) -> int:
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def normalize_shell(l: int, exps: np.ndarray, coefs: np.ndarray) -> np.ndarray:
    """Fold primitive and contraction normalization into the coefficients."""
    exps = np.asarray(exps, dtype=np.float64)
    c = np.asarray(coefs, dtype=np.float64).copy()
    df = float(_dfact(2 * l - 1))
    prim_norm = (2.0 * exps / math.pi) ** 0.75 * (4.0 * exps) ** (l / 2.0) / math.sqrt(df)
    c = c * prim_norm
    # self-overlap of the contracted x^l component
    s = 0.0
    for i in range(len(exps)):
        for j in range(len(exps)):
            p = exps[i] + exps[j]
            s += c[i] * c[j] * (math.pi / p) ** 1.5 * df / (2.0 * p) ** l
    return c / math.sqrt(s)


def _lattice(rng, natom: int, spacing: float = 2.5, jitter: float = 0.3) -> np.ndarray:
    n = int(math.ceil(natom ** (1.0 / 3.0) - 1e-12))
    sites = []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                sites.append((i, j, k))
    sites = np.array(sites[:natom], dtype=np.float64)
    return spacing * sites + rng.uniform(-jitter, jitter, size=(natom, 3))


def _random_box(rng, natom: int, box: float, min_sep: float) -> np.ndarray:
    pos = []
    while len(pos) < natom:
        x = rng.uniform(0.0, box, size=3)
        if all(np.linalg.norm(x - y) >= min_sep for y in pos):
            pos.append(x)
    return np.array(pos, dtype=np.float64)


def make_basis(rng, xyz: np.ndarray, shell_ls, exp_lo: float, exp_hi: float,
               nprim=3, nprim_range=None) -> dict:
    """Draw shells atom by atom, in the listed order; per shell: [K], exps, coefs."""
    shell_atom, shell_l, shell_nprim, shell_off = [], [], [], []
    exps, coefs = [], []
    off = 0
    for a in range(xyz.shape[0]):
        for l in shell_ls:
            if nprim_range is not None:
                k = int(rng.integers(nprim_range[0], nprim_range[1] + 1))
            else:
                k = nprim
            e = np.exp(rng.uniform(math.log(exp_lo), math.log(exp_hi), size=k))
            c = rng.uniform(0.1, 1.0, size=k)
            c = normalize_shell(l, e, c)
            shell_atom.append(a)
            shell_l.append(l)
            shell_nprim.append(k)
            shell_off.append(off)
            exps.extend(e.tolist())
            coefs.extend(c.tolist())
            off += k
    basis = {
        "xyz": np.ascontiguousarray(xyz, dtype=np.float64),
        "shell_atom": np.array(shell_atom, dtype=np.int32),
        "shell_l": np.array(shell_l, dtype=np.int32),
        "shell_nprim": np.array(shell_nprim, dtype=np.int32),
        "shell_prim_off": np.array(shell_off, dtype=np.int32),
        "exps": np.array(exps, dtype=np.float64),
        "coefs": np.array(coefs, dtype=np.float64),
    }
    basis["nbf"] = int(sum(ncart(l) for l in shell_l))
    return basis


def ao_offsets(basis: dict) -> np.ndarray:
    off = np.zeros(len(basis["shell_l"]) + 1, dtype=np.int64)
    off[1:] = np.cumsum([ncart(int(l)) for l in basis["shell_l"]])
    return off


def density(rng, nbf: int, ncol: int, scale: float) -> np.ndarray:
    C = rng.standard_normal(size=(nbf, ncol)) * scale
    P = C @ C.T
    return np.ascontiguousarray(0.5 * (P + P.T))


# Per-configuration recipes: (seed, natom, geometry, shells, exponent range,
# density columns per atom or fixed, density scale rule, Schwarz tau, fp32 tau)
CONFIGS = {
    1: dict(seed=1, natom=4, geom="box", shells=(0, 0, 1), erange=(0.1, 50.0),
            ncol=4, scale="0.3", tau=0.0, fp32_tau=0.0),
    2: dict(seed=2, natom=40, geom="lattice", shells=(0, 0, 1, 2), erange=(0.08, 80.0),
            ncol=80, scale="isqrtN", tau=1e-10, fp32_tau=0.0),
    3: dict(seed=3, natom=120, geom="lattice", shells=(0, 0, 1, 2), erange=(0.08, 80.0),
            ncol=240, scale="isqrtN", tau=1e-10, fp32_tau=1e-4),
    5: dict(seed=5, natom=60, geom="lattice", shells=(0, 0, 1, 2), erange=(0.08, 80.0),
            ncol=120, scale="isqrtN", tau=0.0, fp32_tau=0.0),
}


def make_config(i: int, seed: int | None = None, natom: int | None = None) -> dict:
    """Workload `i` (1, 2, 3 or 5) as {'basis', 'D', 'tau', 'fp32_tau', 'name'}.

    `natom` overrides the atom count (smaller parity cases of the same recipe);
    the density then keeps the same columns-per-atom ratio.
    """
    cfg = CONFIGS[i]
    seed = cfg["seed"] if seed is None else seed
    rng = np.random.default_rng(seed)
    na = cfg["natom"] if natom is None else natom
    if cfg["geom"] == "box":
        xyz = _random_box(rng, na, 4.0, 1.2)
    else:
        xyz = _lattice(rng, na)
    basis = make_basis(rng, xyz, cfg["shells"], *cfg["erange"])
    n = basis["nbf"]
    ncol = cfg["ncol"] if natom is None or i == 1 else max(1, round(cfg["ncol"] * na / cfg["natom"]))
    scale = 0.3 if cfg["scale"] == "0.3" else 1.0 / math.sqrt(n)
    D = density(rng, n, ncol, scale)
    return {"basis": basis, "D": D, "tau": cfg["tau"], "fp32_tau": cfg["fp32_tau"],
            "name": f"config{i}", "seed": seed, "natom": na, "ncol": ncol}


def scf_system(cfg: dict) -> tuple:
    """Nuclear charges and occupied orbitals of a workload's SCF problem.

    The workloads define no elements; the reading used here: as many doubly
    occupied orbitals as the recipe's density has columns, and that many
    electron pairs shared evenly among the atoms, Z_A = 2 nocc / natom (2 for
    the 4-atom recipe, 4 for the lattice recipes)."""
    nocc = int(cfg["ncol"])
    na = int(cfg["natom"])
    Z = np.full(na, 2.0 * nocc / na)
    return Z, nocc


def make_batch(nmol: int = 64, seed: int = 4, atom_range=(8, 96), shells=(0, 0, 1, 2, 3)) -> list:
    """Workload 4: molecule m draws from default_rng([seed, m])."""
    mols = []
    for m in range(nmol):
        rng = np.random.default_rng([seed, m])
        na = int(rng.integers(atom_range[0], atom_range[1] + 1))
        xyz = _lattice(rng, na)
        basis = make_basis(rng, xyz, tuple(shells), 0.08, 80.0, nprim_range=(1, 6))
        n = basis["nbf"]
        D = density(rng, n, 2 * na, 1.0 / math.sqrt(n))
        mols.append({"basis": basis, "D": D, "tau": 1e-10, "natom": na})
    return mols


def random_shells(rng, natom: int, shell_ls, box: float = 3.0, nprim_range=(1, 3),
                  exp_range=(0.2, 5.0)) -> dict:
    """Small random basis for property tests: atoms uniform in a box."""
    xyz = rng.uniform(0.0, box, size=(natom, 3))
    return make_basis(rng, xyz, shell_ls, *exp_range, nprim_range=nprim_range)


def basis_subset(basis: dict, shells) -> dict:
    """A basis made of the listed shells (in that order), same atoms."""
    shells = list(shells)
    exps, coefs, off = [], [], []
    o = 0
    for s in shells:
        p0 = int(basis["shell_prim_off"][s])
        k = int(basis["shell_nprim"][s])
        exps.extend(basis["exps"][p0:p0 + k])
        coefs.extend(basis["coefs"][p0:p0 + k])
        off.append(o)
        o += k
    out = {
        "xyz": basis["xyz"].copy(),
        "shell_atom": basis["shell_atom"][shells].astype(np.int32),
        "shell_l": basis["shell_l"][shells].astype(np.int32),
        "shell_nprim": basis["shell_nprim"][shells].astype(np.int32),
        "shell_prim_off": np.array(off, dtype=np.int32),
        "exps": np.array(exps, dtype=np.float64),
        "coefs": np.array(coefs, dtype=np.float64),
    }
    out["nbf"] = int(sum(ncart(int(l)) for l in out["shell_l"]))
    return out
