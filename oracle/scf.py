"""Plain restricted Hartree-Fock loop on the CPU oracle's integrals.

TEST INFRASTRUCTURE ONLY (see the package docstring): the reference that the
GPU self-consistent-field driver is checked against.

The paper places the Fock build inside the SCF iteration (Section 2.1): each
iteration forms the Fock matrix F = H + J - K/2 from the current density,
diagonalizes it and rebuilds the density from the occupied orbitals.  Closed
shell, D the total density (2 C_occ C_occ^T), so that the electronic energy is
    E_elec = 1/2 Tr(D (H + F)) = Tr(DH) + 1/2 Tr(DJ) - 1/4 Tr(DK)
and the total energy adds the repulsion of the point nuclei.  Every step is
numpy on the oracle's S, T, V, J and K:
  * canonical orthogonalization: S = U s U^T, X = U_k s_k^{-1/2} over the
    eigenvalues s_k > lindep (a near-dependent basis drops those directions);
  * core-Hamiltonian start: the first density comes from H alone;
  * Pulay's DIIS on the orthogonalized commutator e = X^T (F D S - S D F) X,
    extrapolating the Fock matrix from the last `ndiis` ones;
  * convergence: |E_n - E_{n-1}| < e_tol and max |e| < err_tol.
"""
from __future__ import annotations

import numpy as np

from . import build_jk, nuclear_repulsion, one_electron


def orthogonalizer(S: np.ndarray, lindep: float = 1e-8) -> np.ndarray:
    s, U = np.linalg.eigh(S)
    keep = s > lindep
    return U[:, keep] / np.sqrt(s[keep])


def density_from_fock(F: np.ndarray, X: np.ndarray, nocc: int) -> tuple:
    """Aufbau: the nocc lowest orbitals of X^T F X, D = 2 C_occ C_occ^T."""
    e, Cp = np.linalg.eigh(X.T @ F @ X)
    C = X @ Cp
    Co = C[:, :nocc]
    D = 2.0 * Co @ Co.T
    return 0.5 * (D + D.T), e


def rhf(basis: dict, Z, nocc: int, tau: float = 0.0, max_iter: int = 100, e_tol: float = 1e-12,
        err_tol: float = 1e-9, ndiis: int = 8, lindep: float = 1e-8) -> dict:
    Z = np.asarray(Z, dtype=np.float64)
    S, T, V = one_electron(basis, Z)
    H = T + V
    enuc = nuclear_repulsion(basis["xyz"], Z)
    X = orthogonalizer(S, lindep)
    if nocc > X.shape[1]:
        raise ValueError("more occupied orbitals than independent basis functions")
    D, _ = density_from_fock(H, X, nocc)
    focks, errs, energies = [], [], []
    e_old = None
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        J, K, _ = build_jk(basis, D, tau)
        F = H + J - 0.5 * K
        e_tot = 0.5 * float(np.sum(D * (H + F))) + enuc
        energies.append(e_tot)
        err = X.T @ (F @ D @ S - S @ D @ F) @ X
        emax = float(np.max(np.abs(err)))
        if e_old is not None and abs(e_tot - e_old) < e_tol and emax < err_tol:
            converged = True
            break
        e_old = e_tot
        focks.append(F)
        errs.append(err)
        if len(focks) > ndiis:
            focks.pop(0)
            errs.pop(0)
        Fx = diis_extrapolate(focks, errs)
        D, _ = density_from_fock(Fx, X, nocc)
    return {"energy": energies[-1], "energies": energies, "D": D, "converged": converged, "iterations": it,
            "enuc": enuc, "H": H, "S": S}


def diis_extrapolate(focks, errs) -> np.ndarray:
    """Pulay: minimize |sum c_i e_i| subject to sum c_i = 1."""
    n = len(focks)
    if n == 1:
        return focks[0]
    B = np.zeros((n + 1, n + 1))
    for i in range(n):
        for j in range(n):
            B[i, j] = float(np.sum(errs[i] * errs[j]))
    B[n, :n] = B[:n, n] = -1.0
    rhs = np.zeros(n + 1)
    rhs[n] = -1.0
    c = np.linalg.lstsq(B, rhs, rcond=None)[0][:n]
    return sum(ci * Fi for ci, Fi in zip(c, focks))
