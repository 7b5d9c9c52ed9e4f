"""Pins for the oracle's J, K and E2 (two-electron Fock pieces, Section 2.1).

  * the plain einsum of the full ERI tensor against the oracle's eight-fold
    scatter (build_jk) and its per-block plain sums (jk_blocks);
  * a rank-1 density D = c c^T gives Tr(DJ) = Tr(DK);
  * a probe density D = E_ij + E_ji gives J = 2 (..|ij), tying J to eri_block;
  * Tr(DJ) >= 0 and Tr(DK) >= 0 for a positive semidefinite D;
  * screened minus unscreened J/K stays within the summed Schwarz bounds.
"""
import numpy as np
import pytest

import oracle
from paper_2412_13203_amd import inputs


@pytest.fixture(scope="module")
def cfg1():
    cfg = inputs.make_config(1)
    T = oracle.eri_tensor(cfg["basis"])
    return cfg, T


def test_scatter_matches_einsum(cfg1):
    cfg, T = cfg1
    D = cfg["D"]
    J, K, nq = oracle.build_jk(cfg["basis"], D, 0.0)
    Jref = np.einsum("mnls,ls->mn", T, D)
    Kref = np.einsum("mlns,ls->mn", T, D)
    assert np.max(np.abs(J - Jref)) < 1e-13
    assert np.max(np.abs(K - Kref)) < 1e-13
    ns = len(cfg["basis"]["shell_l"])
    npair = ns * (ns + 1) // 2
    assert nq == npair * (npair + 1) // 2


def test_blocks_match_einsum(cfg1):
    cfg, T = cfg1
    D = cfg["D"]
    b = cfg["basis"]
    off = inputs.ao_offsets(b)
    Jref = np.einsum("mnls,ls->mn", T, D)
    Kref = np.einsum("mlns,ls->mn", T, D)
    blocks = [(0, 0), (2, 5), (5, 2), (11, 3), (8, 8)]
    Js, Ks = oracle.jk_blocks(b, D, 0.0, blocks)
    for (A, B), Jb, Kb in zip(blocks, Js, Ks):
        sa, sb = slice(off[A], off[A + 1]), slice(off[B], off[B + 1])
        assert np.max(np.abs(Jb - Jref[sa, sb])) < 1e-13
        assert np.max(np.abs(Kb - Kref[sa, sb])) < 1e-13


def test_rank1_density(cfg1):
    cfg, _ = cfg1
    b = cfg["basis"]
    c = np.random.default_rng(4).standard_normal(b["nbf"])
    D = np.outer(c, c)
    J, K, _ = oracle.build_jk(b, D, 0.0)
    assert abs(np.sum(D * J) - np.sum(D * K)) < 1e-12 * abs(np.sum(D * J))


def test_probe_density(cfg1):
    cfg, T = cfg1
    b = cfg["basis"]
    N = b["nbf"]
    i, j = 3, 11
    D = np.zeros((N, N))
    D[i, j] = D[j, i] = 1.0
    J, K, _ = oracle.build_jk(b, D, 0.0)
    assert np.max(np.abs(J - 2 * T[:, :, i, j])) < 1e-13
    # and K = (.i|.j) + (.j|.i)
    assert np.max(np.abs(K - (T[:, i, :, j] + T[:, j, :, i]))) < 1e-13


def test_traces_nonnegative():
    cfg = inputs.make_config(2, natom=3)
    b, D = cfg["basis"], cfg["D"]
    J, K, _ = oracle.build_jk(b, D, 0.0)
    assert np.sum(D * J) > 0
    assert np.sum(D * K) > 0
    e2 = oracle.e2(J, K, D)
    # for a PSD D, 1/2 Tr DJ - 1/4 Tr DK >= 1/4 Tr DJ > 0 (Tr DK <= Tr DJ)
    assert np.sum(D * K) <= np.sum(D * J) * (1 + 1e-12)
    assert e2 > 0


def test_screening_error_bounded():
    cfg = inputs.make_config(2, natom=4)
    b, D = cfg["basis"], cfg["D"]
    Q = oracle.schwarz(b)
    J0, K0, n0 = oracle.build_jk(b, D, 0.0, Q)
    tau = 1e-6
    J1, K1, n1 = oracle.build_jk(b, D, tau, Q)
    assert n1 < n0
    # every skipped quartet has |(ab|cd)| <= Q_AB Q_CD < tau; each feeds at most
    # 8 * 6 * 10^2 element updates weighted by |D| <= max|D|
    ns = len(b["shell_l"])
    pairs = [(A, B) for A in range(ns) for B in range(A + 1)]
    qp = np.array([Q[A, B] for A, B in pairs])
    prod = np.outer(qp, qp)
    skipped = np.tril(prod < tau)
    bound = np.sum(prod[skipped]) * 8 * 36 * np.max(np.abs(D))
    assert np.max(np.abs(J1 - J0)) <= bound
    assert np.max(np.abs(K1 - K0)) <= bound
    assert np.max(np.abs(J1 - J0)) > 0


def test_rows_partition():
    cfg = inputs.make_config(1)
    b, D = cfg["basis"], cfg["D"]
    ns = len(b["shell_l"])
    npair = ns * (ns + 1) // 2
    rows = np.arange(npair)
    Jt, Kt, n = oracle.jk_rows(b, D, 0.0, rows)
    Ja, Ka, na = oracle.jk_rows(b, D, 0.0, rows[::2])
    Jb, Kb, nb = oracle.jk_rows(b, D, 0.0, rows[1::2])
    assert na + nb == n
    assert np.max(np.abs(Ja + Jb - Jt)) < 1e-13
    assert np.max(np.abs(Ka + Kb - Kt)) < 1e-13
