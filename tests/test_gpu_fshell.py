"""GPU parity with f shells (l = 3, ten Cartesian components; Eq. 1-2's
classes up to (ff|ff)), through the C ABI, against the FP64 CPU oracle.

  * eri_class for every ordered class (la lb | lc ld) with l <= 3, 1-3
    primitives per shell, one random quartet per class: 1e-10 absolute;
  * Schwarz factors of a basis with f shells (the split diagonal classes run
    through the pass/staging kernels): Q^2 within 1e-10, Q within 1e-11
    relative;
  * full J and K of a 3-atom cut of the batched recipe (s, s, p, d, f per
    atom, 1-6 primitives per shell): 1e-10 absolute, exact quartet count;
  * mixed precision leaves every quartet of a class with an f shell in FP64.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2412_13203_amd import inputs, mjk

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def need_f():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    if mjk.lib().mjk_lmax() < 3:
        pytest.skip("library built without f shells")
    mjk.context(0)


def _np(t):
    return t.detach().cpu().numpy()


def _spdf_basis(seed, nprim=(1, 3)):
    rng = np.random.default_rng(seed)
    return inputs.random_shells(rng, 3, [0, 1, 2, 3], box=2.5, nprim_range=nprim, exp_range=(0.15, 8.0))


def test_eri_class_every_ordered_class_to_f():
    b = _spdf_basis(301)
    ls = b["shell_l"]
    by_l = {l: [s for s in range(len(ls)) if ls[s] == l] for l in range(4)}
    rng = np.random.default_rng(6)
    quartets = [[int(rng.choice(by_l[l])) for l in combo] for combo in itertools.product(range(4), repeat=4)]
    plan = mjk.Plan(b)
    blocks = plan.eri_class(quartets)
    worst = 0.0
    for q, g in zip(quartets, blocks):
        ref = oracle.eri_block(b, *q)
        d = float(np.max(np.abs(_np(g) - ref)))
        worst = max(worst, d)
        assert d <= TOL, (q, [int(ls[s]) for s in q], d)
    print(f"eri_class to (ff|ff): {len(quartets)} quartets, worst abs diff {worst:.2e}", flush=True)


def test_schwarz_with_f_shells():
    b = _spdf_basis(302)
    plan = mjk.Plan(b, tau=1e-10)
    Qg = plan.schwarz()
    Qo = oracle.schwarz(b)
    d2 = float(np.max(np.abs(Qg ** 2 - Qo ** 2)))
    assert d2 <= TOL, d2
    big = Qo > 1e-6
    rel = float(np.max(np.abs(Qg - Qo)[big] / Qo[big]))
    assert rel < 1e-11, rel


def _batch_cut(natom=3):
    m = inputs.make_batch(nmol=1, atom_range=(8, 8))[0]
    b = m["basis"]
    shells = [s for s in range(len(b["shell_l"])) if b["shell_atom"][s] < natom]
    sb = inputs.basis_subset(b, shells)
    rng = np.random.default_rng(9)
    n = sb["nbf"]
    C = rng.standard_normal((n, 2 * natom)) / np.sqrt(n)
    D = C @ C.T
    return sb, 0.5 * (D + D.T)


def test_f_shells_full_jk_vs_oracle():
    b, D = _batch_cut(3)
    print(f"3-atom cut, nbf {b['nbf']}, primitives per shell {list(b['shell_nprim'])}", flush=True)
    plan = mjk.Plan(b, tau=0.0)
    J, K = plan.build_jk(D)
    Jo, Ko, nq = oracle.build_jk(b, D, 0.0)
    dj = float(np.max(np.abs(_np(J) - Jo)))
    dk = float(np.max(np.abs(_np(K) - Ko)))
    print(f"  max |dJ| {dj:.2e}, max |dK| {dk:.2e}", flush=True)
    assert dj <= TOL and dk <= TOL
    assert plan.stats["nquartet_kept"] == nq


def test_f_classes_stay_fp64_under_mixed_precision():
    b, D = _batch_cut(2)
    p64 = mjk.Plan(b, tau=0.0)
    p32 = mjk.Plan(b, tau=0.0, fp32_tau=1e30)  # every other quartet in FP32
    J64, K64 = p64.build_jk(D)
    J32, K32 = p32.build_jk(D)
    assert p32.stats["nquartet_fp32"] > 0
    # quartets with an f shell are FP64 in both plans: eri_class agrees bitwise
    ls = b["shell_l"]
    f = [s for s in range(len(ls)) if ls[s] == 3]
    s0 = [s for s in range(len(ls)) if ls[s] == 0]
    q = [[f[0], s0[0], f[-1], s0[-1]], [f[0], f[-1], f[0], f[-1]]]
    for x, y in zip(p64.eri_class(q), p32.eri_class(q)):
        assert np.array_equal(_np(x), _np(y))
    # and the FP32 part is close, not exact
    assert float(np.max(np.abs(_np(J32) - _np(J64)))) < 1e-4
