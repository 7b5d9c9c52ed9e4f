"""Restricted closed-shell self-consistent-field driver around the library.

The paper places the Fock build inside the SCF iteration (Section 2.1): every
iteration forms F = H + J - K/2 from the current density, diagonalizes it and
builds the next density from the occupied orbitals; the ERIs take nearly all
of its time.  Here every integral comes from the gfx950 library through its
C ABI (one-electron S, T, V and the nuclear repulsion once per geometry;
J and K every iteration, `mjk_build_jk`), and the dense linear algebra around
them runs in torch on the same device:

  * canonical orthogonalization X = U s^{-1/2} over the eigenvalues of S
    above `lindep` (a near-dependent basis loses those directions);
  * the first density from the core Hamiltonian H = T + V;
  * Pulay's DIIS on the orthogonalized commutator X^T (F D S - S D F) X over
    the last `ndiis` Fock matrices;
  * D = 2 C_occ C_occ^T (total density), energy 1/2 Tr(D (H + F)) + E_nuc;
  * convergence when the energy changes by less than `e_tol` and the largest
    commutator element is below `err_tol`.

`incremental=True` builds J and K of the density change instead,
J(D_n) = J(D_{n-1}) + J(D_n - D_{n-1}) (J and K are linear in D), with the
screening of each difference build weighted by the difference itself: a
quartet is skipped when its Schwarz bound times the largest element of the
difference density in the shell rows it touches is below `inc_tau` (default
the plan's Schwarz threshold; `mjk_plan_set_density_screen`).  Every
`rebuild_every` iterations (and in the first) the full J and K are rebuilt,
which bounds the drift; iterations whose density changes by more than
`inc_start` anywhere build in full (the screen would keep nearly every
quartet); once the largest commutator element is within 10x of `err_tol`
the run finishes with full builds, and an iteration that meets the
convergence test on an incremental build is repeated with a full build of
the same density before the loop stops.
"""
from __future__ import annotations

import time

import numpy as np

from . import mjk


def _eigh(M):
    import torch
    e, U = torch.linalg.eigh(M)
    return e, U


class RHF:
    """SCF problem of one molecule: basis, nuclear charges and occupied orbitals."""

    def __init__(self, basis: dict, Z, nocc: int, tau: float = 1e-10, fp32_tau: float = 0.0, device: int = 0,
                 lindep: float = 1e-8):
        import torch
        self.torch = torch
        self.dev = torch.device(f"cuda:{device}")
        self.nocc = int(nocc)
        t0 = time.perf_counter()
        self.plan = mjk.Plan(basis, tau=tau, fp32_tau=fp32_tau, device=device)
        S, T, V, enuc = self.plan.one_electron(Z)
        self.S, self.H = S, T + V
        self.enuc = float(enuc)
        s, U = _eigh(S)
        keep = s > lindep
        self.X = (U[:, keep] / torch.sqrt(s[keep])).contiguous()
        if self.nocc > self.X.shape[1]:
            raise ValueError("more occupied orbitals than independent basis functions")
        torch.cuda.synchronize(self.dev)
        self.setup_s = time.perf_counter() - t0

    def density(self, F):
        """Aufbau density D = 2 C_occ C_occ^T of the nocc lowest orbitals of F."""
        e, Cp = _eigh(self.X.T @ F @ self.X)
        Co = self.X @ Cp[:, :self.nocc]
        D = 2.0 * Co @ Co.T
        return 0.5 * (D + D.T), e

    def run(self, max_iter: int = 100, e_tol: float = 1e-10, err_tol: float = 1e-8, ndiis: int = 8, D0=None,
            incremental: bool = False, rebuild_every: int = 8, inc_tau: float | None = None,
            inc_start: float = 1e-2, log=None) -> dict:
        torch = self.torch
        stream = torch.cuda.current_stream(self.dev)
        D = self.density(self.H)[0] if D0 is None else torch.as_tensor(D0, dtype=torch.float64, device=self.dev)
        n = D.shape[0]
        J = torch.zeros((n, n), dtype=torch.float64, device=self.dev)
        K = torch.zeros_like(J)
        dJ, dK = torch.empty_like(J), torch.empty_like(J)
        D_prev = None
        focks, errs = [], []
        energies, t_iter, t_jk, kept, was_full = [], [], [], [], []
        e_old, converged, it, confirm, inc_off = None, False, 0, False, False
        inc_tau = self.plan.tau if inc_tau is None else inc_tau
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        for it in range(1, max_iter + 1):
            ev[0].record(stream)
            full = not incremental or inc_off or D_prev is None or confirm or (it - 1) % rebuild_every == 0
            if not full:
                dD = D - D_prev
                # while the density still moves by more than inc_start the
                # screen would keep nearly every quartet: build in full
                full = float(dD.abs().max()) > inc_start
            if full:
                self.plan.set_density_screen(None)
                self.plan.build_jk(D, J, K)
            else:
                self.plan.set_density_screen(dD, inc_tau)
                self.plan.build_jk(dD, dJ, dK)
                J += dJ
                K += dK
            kept.append(self.plan.kept_quartets())
            was_full.append(full)
            ev[1].record(stream)
            D_prev = D
            F = self.H + J - 0.5 * K
            e_tot = 0.5 * float(torch.sum(D * (self.H + F))) + self.enuc
            err = self.X.T @ (F @ D @ self.S - self.S @ D @ F) @ self.X
            emax = float(err.abs().max())
            energies.append(e_tot)
            done = e_old is not None and abs(e_tot - e_old) < e_tol and emax < err_tol
            # an incremental build that looks converged is confirmed by a full
            # build of the same density; if that full build does not confirm
            # it, the screening noise is at the convergence threshold and the
            # remaining iterations build J and K in full
            if confirm and not done:
                inc_off = True
            # near convergence the screening noise is of the size of the
            # remaining error: finish with full builds
            if emax < 10.0 * err_tol:
                inc_off = True
            confirm = done and not full
            if not done:
                focks.append(F)
                errs.append(err)
                if len(focks) > ndiis:
                    focks.pop(0)
                    errs.pop(0)
                D = self.density(_diis(focks, errs))[0]
            ev[2].record(stream)
            ev[2].synchronize()
            t_iter.append(ev[0].elapsed_time(ev[2]))
            t_jk.append(ev[0].elapsed_time(ev[1]))
            if log is not None:
                log(f"iteration {it}: E = {e_tot:.10f}, max |FDS - SDF| = {emax:.2e}, "
                    f"{'full' if full else 'incremental'} J/K {t_jk[-1]:.1f} ms of {t_iter[-1]:.1f} ms")
            e_old = e_tot
            if done and full:
                converged = True
                break
        self.plan.set_density_screen(None)
        return {"energy": energies[-1], "energies": energies, "iterations": it, "converged": converged,
                "D": D_prev, "ms_per_iter": t_iter, "ms_jk": t_jk, "kept_quartets": kept, "full_build": was_full,
                "enuc": self.enuc}


def _diis(focks, errs):
    """Pulay extrapolation: minimize |sum c_i e_i| subject to sum c_i = 1."""
    n = len(focks)
    if n == 1:
        return focks[0]
    import torch
    E = torch.stack([e.reshape(-1) for e in errs])
    B = np.zeros((n + 1, n + 1))
    B[:n, :n] = (E @ E.T).cpu().numpy()
    B[n, :n] = B[:n, n] = -1.0
    rhs = np.zeros(n + 1)
    rhs[n] = -1.0
    c = np.linalg.lstsq(B, rhs, rcond=None)[0][:n]
    out = torch.zeros_like(focks[0])
    for ci, Fi in zip(c, focks):
        out += float(ci) * Fi
    return out
