"""Plain FP64 CPU oracle for ERIs, J/K and the E2 nuclear gradient.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path never imports this
package, and this package imports nothing from the product.

The C source (oracle.c) is built with gcc -O2 -fopenmp (no fast-math) into
oracle/_build/liboracle.so by `build()`.  Each wrapper below names the
passage of the paper that defines what it computes; the C file's header
gives the algorithm (McMurchie-Davidson Hermite expansion, Boys function by
series / erf in long double).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile oracle.c into _build/liboracle.so (always recompiles)."""
    os.makedirs(os.path.join(_HERE, "_build"), exist_ok=True)
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           os.path.join(_HERE, "oracle.c"), "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


class _Basis(ctypes.Structure):
    _fields_ = [
        ("natom", ctypes.c_int),
        ("xyz", ctypes.POINTER(ctypes.c_double)),
        ("nshell", ctypes.c_int),
        ("shell_atom", ctypes.POINTER(ctypes.c_int)),
        ("shell_l", ctypes.POINTER(ctypes.c_int)),
        ("shell_nprim", ctypes.POINTER(ctypes.c_int)),
        ("shell_prim_off", ctypes.POINTER(ctypes.c_int)),
        ("exps", ctypes.POINTER(ctypes.c_double)),
        ("coefs", ctypes.POINTER(ctypes.c_double)),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = ctypes.CDLL(_SO)
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


class _BasisHandle:
    """Keeps the contiguous arrays alive while the C struct points at them."""

    def __init__(self, basis: dict):
        self.xyz = np.ascontiguousarray(basis["xyz"], dtype=np.float64)
        self.atom = np.ascontiguousarray(basis["shell_atom"], dtype=np.int32)
        self.l = np.ascontiguousarray(basis["shell_l"], dtype=np.int32)
        self.nprim = np.ascontiguousarray(basis["shell_nprim"], dtype=np.int32)
        self.off = np.ascontiguousarray(basis["shell_prim_off"], dtype=np.int32)
        self.exps = np.ascontiguousarray(basis["exps"], dtype=np.float64)
        self.coefs = np.ascontiguousarray(basis["coefs"], dtype=np.float64)
        self.s = _Basis(self.xyz.shape[0], _dptr(self.xyz), len(self.l), _iptr(self.atom), _iptr(self.l),
                        _iptr(self.nprim), _iptr(self.off), _dptr(self.exps), _dptr(self.coefs))
        self.nshell = len(self.l)
        self.ncart = (self.l + 1) * (self.l + 2) // 2
        self.ao_off = np.concatenate([[0], np.cumsum(self.ncart)]).astype(np.int64)
        self.nbf = int(self.ao_off[-1])

    @property
    def ref(self):
        return ctypes.byref(self.s)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def nthreads() -> int:
    return int(_load().orc_nthreads())


def boys(mmax: int, T: float) -> np.ndarray:
    """F_m(T), m = 0..mmax: the auxiliary function behind the analytic [00|00] (Section 2.2)."""
    out = np.zeros(mmax + 1)
    _check(_load().orc_boys(ctypes.c_int(mmax), ctypes.c_double(T), _dptr(out)), "boys")
    return out


def eri_block(basis: dict, A: int, B: int, C: int, D: int) -> np.ndarray:
    """Contracted (AB|CD) block, Eq. 2; shape (na, nb, nc, nd)."""
    h = _BasisHandle(basis)
    A, B, C, D = int(A), int(B), int(C), int(D)
    n = [int(h.ncart[s]) for s in (A, B, C, D)]
    out = np.zeros(n)
    _check(_load().orc_eri_block(h.ref, A, B, C, D, _dptr(out)), "eri_block")
    return out


def eri_tensor(basis: dict) -> np.ndarray:
    """Full (N, N, N, N) ERI tensor (only for tiny bases)."""
    h = _BasisHandle(basis)
    N = h.nbf
    out = np.zeros((N, N, N, N))
    _check(_load().orc_eri_tensor(h.ref, _dptr(out)), "eri_tensor")
    return out


def schwarz(basis: dict) -> np.ndarray:
    """Q[A, B] = sqrt(max (ab|ab)) over the components of shells A, B."""
    h = _BasisHandle(basis)
    Q = np.zeros((h.nshell, h.nshell))
    _check(_load().orc_schwarz(h.ref, _dptr(Q)), "schwarz")
    return Q


def pair_index(A: int, B: int) -> int:
    A, B = max(A, B), min(A, B)
    return A * (A + 1) // 2 + B


def jk_rows(basis: dict, D: np.ndarray, tau: float, rows, Q=None):
    """Accumulate Jt, Kt over unique quartets whose bra pair is in `rows`.

    Returns (Jt, Kt, nquartets); J = Jt + Jt^T and K = Kt + Kt^T when rows
    covers every pair.  The Fock-matrix pieces of Section 2.1.
    """
    h = _BasisHandle(basis)
    if Q is None:
        Q = schwarz(basis)
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    D = np.ascontiguousarray(D, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    N = h.nbf
    Jt = np.zeros((N, N))
    Kt = np.zeros((N, N))
    nq = ctypes.c_longlong(0)
    _check(_load().orc_jk_rows(h.ref, _dptr(D), ctypes.c_double(tau), _dptr(Q), ctypes.c_int(len(rows)),
                               _iptr(rows), _dptr(Jt), _dptr(Kt), ctypes.byref(nq)), "jk_rows")
    return Jt, Kt, int(nq.value)


def build_jk(basis: dict, D: np.ndarray, tau: float = 0.0, Q=None):
    """Whole J and K over all unique quartets (8-fold scatter)."""
    ns = len(basis["shell_l"])
    rows = np.arange(ns * (ns + 1) // 2, dtype=np.int32)
    Jt, Kt, nq = jk_rows(basis, D, tau, rows, Q)
    return Jt + Jt.T, Kt + Kt.T, nq


def jk_blocks(basis: dict, D: np.ndarray, tau: float, blocks, Q=None):
    """J and K shell blocks by the plain sums J_ab = sum (ab|cd) D_cd,
    K_ab = sum (ac|bd) D_cd over all shells C, D.  blocks: list of (A, B).
    Returns two lists of (na, nb) arrays."""
    h = _BasisHandle(basis)
    if Q is None:
        Q = schwarz(basis)
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    D = np.ascontiguousarray(D, dtype=np.float64)
    blk = np.ascontiguousarray(np.asarray(blocks, dtype=np.int32).reshape(-1, 2))
    sizes = [int(h.ncart[a] * h.ncart[b]) for a, b in blk]
    tot = int(sum(sizes))
    Jb = np.zeros(tot)
    Kb = np.zeros(tot)
    _check(_load().orc_jk_blocks(h.ref, _dptr(D), ctypes.c_double(tau), _dptr(Q), ctypes.c_int(len(blk)),
                                 _iptr(blk), _dptr(Jb), _dptr(Kb)), "jk_blocks")
    Js, Ks, o = [], [], 0
    for (a, b), s in zip(blk, sizes):
        shp = (int(h.ncart[a]), int(h.ncart[b]))
        Js.append(Jb[o:o + s].reshape(shp))
        Ks.append(Kb[o:o + s].reshape(shp))
        o += s
    return Js, Ks


def overlap_block(basis: dict, A: int, B: int) -> np.ndarray:
    h = _BasisHandle(basis)
    A, B = int(A), int(B)
    out = np.zeros((int(h.ncart[A]), int(h.ncart[B])))
    _check(_load().orc_overlap_block(h.ref, A, B, _dptr(out)), "overlap_block")
    return out


def one_electron(basis: dict, Z) -> tuple:
    """Whole one-electron matrices (S, T, V), each N x N: overlap, kinetic
    energy -1/2 nabla^2 and attraction to point nuclei of charge Z[atom] at
    the atom centres.  With J and K they make the Fock matrix of the SCF loop
    (Section 2.1)."""
    h = _BasisHandle(basis)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    if Z.shape != (h.xyz.shape[0],):
        raise ValueError("one charge per atom")
    N = h.nbf
    S, T, V = np.zeros((N, N)), np.zeros((N, N)), np.zeros((N, N))
    _check(_load().orc_one_electron(h.ref, _dptr(Z), _dptr(S), _dptr(T), _dptr(V)), "one_electron")
    return S, T, V


def nuclear_repulsion(xyz, Z) -> float:
    """sum_{A<B} Z_A Z_B / |R_A - R_B|."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    return float(_load().orc_nuclear_repulsion(ctypes.c_int(xyz.shape[0]), _dptr(xyz), _dptr(Z)))


def e2(J: np.ndarray, K: np.ndarray, D: np.ndarray) -> float:
    """E2 = 1/2 Tr(DJ) - 1/4 Tr(DK)."""
    return float(0.5 * np.sum(D * J) - 0.25 * np.sum(D * K))


def grad_e2(basis: dict, D: np.ndarray) -> np.ndarray:
    """dE2/dR for every atom at fixed D, shape (natom, 3) (tiny bases only)."""
    h = _BasisHandle(basis)
    D = np.ascontiguousarray(D, dtype=np.float64)
    g = np.zeros((h.xyz.shape[0], 3))
    _check(_load().orc_grad_e2(h.ref, _dptr(D), _dptr(g)), "grad_e2")
    return g


def _setup_signatures():
    lib = _load()
    lib.orc_boys.restype = ctypes.c_int
    lib.orc_nthreads.restype = ctypes.c_int
    lib.orc_nuclear_repulsion.restype = ctypes.c_double


_setup_signatures()
