"""CPU tests of the SCF driver's linear algebra (the steps around the
library's integrals, Section 2.1's iteration): the aufbau density and Pulay's
DIIS extrapolation, on CPU tensors (the driver runs them on the GPU)."""
import numpy as np
import pytest
import torch

from paper_2412_13203_amd import scf


def _driver(S, nocc):
    """An RHF object with only the orthogonalizer and occupation set."""
    r = object.__new__(scf.RHF)
    r.torch = torch
    r.nocc = nocc
    s, U = torch.linalg.eigh(S)
    r.X = (U / torch.sqrt(s)).contiguous()
    return r


def _spd(rng, n):
    A = rng.standard_normal((n, n))
    return A @ A.T / n + np.eye(n)


def test_density_is_idempotent_and_counts_electrons():
    rng = np.random.default_rng(11)
    n, nocc = 9, 3
    S = torch.tensor(_spd(rng, n))
    F = torch.tensor(rng.standard_normal((n, n)))
    F = 0.5 * (F + F.T)
    r = _driver(S, nocc)
    D, e = r.density(F)
    assert torch.allclose(D, D.T, atol=1e-14)
    assert torch.allclose(D @ S @ D, 2 * D, atol=1e-12)
    assert abs(float(torch.trace(D @ S)) - 2 * nocc) < 1e-12
    # the occupied space is spanned by the nocc lowest solutions of F C = S C e
    ev = np.sort(np.linalg.eigvals(np.linalg.solve(S.numpy(), F.numpy())).real)
    assert np.allclose(np.sort(e.numpy())[:nocc], ev[:nocc], atol=1e-10)


def test_diis_minimizes_the_error_norm_with_unit_weight_sum():
    rng = np.random.default_rng(12)
    n, m = 5, 4
    focks = [torch.tensor(rng.standard_normal((n, n))) for _ in range(m)]
    errs = [torch.tensor(rng.standard_normal((n, n))) for _ in range(m)]
    F = scf._diis(focks, errs)
    # the weights: least squares of sum c_i e_i subject to sum c_i = 1, solved
    # here through the null space of the constraint
    E = np.stack([e.numpy().ravel() for e in errs], axis=1)
    N = np.vstack([np.eye(m - 1), -np.ones((1, m - 1))])
    c0 = np.zeros(m)
    c0[-1] = 1.0
    y = np.linalg.lstsq(E @ N, -E @ c0, rcond=None)[0]
    c = c0 + N @ y
    ref = sum(ci * Fi.numpy() for ci, Fi in zip(c, focks))
    assert np.allclose(F.numpy(), ref, atol=1e-10)
    assert scf._diis(focks[:1], errs[:1]) is focks[0]


def test_diis_reproduces_a_vanishing_error_combination():
    """If sum c_i e_i = 0 for weights summing to one, DIIS returns sum c_i F_i."""
    rng = np.random.default_rng(13)
    n = 4
    e1 = torch.tensor(rng.standard_normal((n, n)))
    errs = [e1, -e1]
    focks = [torch.tensor(rng.standard_normal((n, n))) for _ in range(2)]
    F = scf._diis(focks, errs)
    assert torch.allclose(F, 0.5 * (focks[0] + focks[1]), atol=1e-12)


@pytest.mark.parametrize("n,nocc", [(6, 1), (6, 6)])
def test_density_edge_occupations(n, nocc):
    rng = np.random.default_rng(14)
    S = torch.tensor(_spd(rng, n))
    F = torch.tensor(np.diag(np.arange(n, dtype=float)))
    D, _ = _driver(S, nocc).density(F)
    assert abs(float(torch.trace(D @ S)) - 2 * nocc) < 1e-12
    if nocc == n:  # every orbital doubly occupied: D = 2 S^-1
        assert torch.allclose(D, 2 * torch.linalg.inv(S), atol=1e-10)
