"""Pins for the oracle's nuclear gradient of E2 = 1/2 Tr(DJ) - 1/4 Tr(DK).

The density is held fixed; basis functions move with their atoms.  Checked
against central finite differences of the oracle's own E2 (h = 1e-4 bohr,
truncation ~ h^2 E''' ~ 1e-8, so 1e-6 is a safe bar), the translational sum
rule sum_A g_A = 0 and, for an s-only basis, the rotational rule
sum_A R_A x g_A = 0.
"""
import numpy as np

import oracle
from paper_2412_13203_amd import inputs


def _e2(basis, D):
    J, K, _ = oracle.build_jk(basis, D, 0.0)
    return oracle.e2(J, K, D)


def _small(seed, ls, natom=3):
    rng = np.random.default_rng(seed)
    b = inputs.random_shells(rng, natom, ls, box=2.5, nprim_range=(1, 2), exp_range=(0.3, 3.0))
    C = rng.standard_normal((b["nbf"], 3)) * 0.4
    D = C @ C.T
    return b, 0.5 * (D + D.T)


def test_gradient_vs_finite_differences():
    b, D = _small(21, [0, 1, 2])
    g = oracle.grad_e2(b, D)
    h = 1e-4
    for atom in range(b["xyz"].shape[0]):
        for x in range(3):
            bp = dict(b)
            bm = dict(b)
            bp["xyz"] = b["xyz"].copy()
            bm["xyz"] = b["xyz"].copy()
            bp["xyz"][atom, x] += h
            bm["xyz"][atom, x] -= h
            fd = (_e2(bp, D) - _e2(bm, D)) / (2 * h)
            assert abs(fd - g[atom, x]) < 1e-6, (atom, x, fd, g[atom, x])


def test_translational_sum_rule():
    b, D = _small(22, [1, 2], natom=3)
    g = oracle.grad_e2(b, D)
    assert np.max(np.abs(g.sum(axis=0))) < 1e-10 * max(1.0, np.max(np.abs(g)))


def test_rotational_sum_rule_s_only():
    b, D = _small(23, [0, 0], natom=4)
    g = oracle.grad_e2(b, D)
    torque = np.sum(np.cross(b["xyz"], g), axis=0)
    assert np.max(np.abs(torque)) < 1e-10 * max(1.0, np.max(np.abs(g)))
