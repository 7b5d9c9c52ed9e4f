"""GPU mixed precision: quartets with Q_AB Q_CD < fp32_tau run their
recurrence, contraction and HRR in FP32; geometry, Boys and the J/K
digestion stay FP64.  Bar: |E2(mixed) - E2(oracle FP64)| <= 1e-6 Eh."""
import numpy as np
import pytest

import oracle
from paper_2412_13203_amd import inputs, mjk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available()
    mjk.context(0)


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def cut120():
    """10 atoms of the 120-atom s,s,p,d recipe (seed 3), full oracle J/K."""
    cfg = inputs.make_config(3, natom=10)
    b, D = cfg["basis"], cfg["D"]
    Jo, Ko, nq = oracle.build_jk(b, D, cfg["tau"])
    return cfg, Jo, Ko, nq


def test_mixed_e2_within_bar(cut120):
    cfg, Jo, Ko, nq = cut120
    b, D = cfg["basis"], cfg["D"]
    plan = mjk.Plan(b, tau=cfg["tau"], fp32_tau=cfg["fp32_tau"])
    assert plan.stats["nquartet_fp32"] > 0
    assert plan.stats["nquartet_kept"] == nq
    J, K = plan.build_jk(D)
    e_mixed = oracle.e2(_np(J), _np(K), D)
    e_ref = oracle.e2(Jo, Ko, D)
    print(f"E2 oracle {e_ref:.12f}  mixed {e_mixed:.12f}  diff {e_mixed - e_ref:.3e}; "
          f"{plan.stats['nquartet_fp32']} of {nq} quartets in FP32")
    assert abs(e_mixed - e_ref) <= 1e-6
    # element-wise sanity only (the contract is E2): each FP32 quartet has
    # |(ab|cd)| <= Q_AB Q_CD < 1e-4 and ~1e-7 relative FP32 error; a J/K element
    # sums thousands of them, so errors up to ~1e-6 are expected, 1e-5 is the bound
    dj = float(np.max(np.abs(_np(J) - Jo)))
    dk = float(np.max(np.abs(_np(K) - Ko)))
    print(f"max |dJ| {dj:.3e}  max |dK| {dk:.3e}")
    assert dj <= 1e-5 and dk <= 1e-5


def test_fp32_tau_zero_is_fp64(cut120):
    cfg, Jo, Ko, _ = cut120
    plan = mjk.Plan(cfg["basis"], tau=cfg["tau"], fp32_tau=0.0)
    assert plan.stats["nquartet_fp32"] == 0
    J, K = plan.build_jk(cfg["D"])
    assert float(np.max(np.abs(_np(J) - Jo))) <= 1e-10
    assert float(np.max(np.abs(_np(K) - Ko))) <= 1e-10


def test_everything_fp32_is_close_not_exact():
    cfg = inputs.make_config(1)
    b, D = cfg["basis"], cfg["D"]
    plan = mjk.Plan(b, tau=0.0, fp32_tau=1e30)
    assert plan.stats["nquartet_fp32"] == plan.stats["nquartet_kept"]
    J, K = plan.build_jk(D)
    Jo, Ko, _ = oracle.build_jk(b, D, 0.0)
    dJ = float(np.max(np.abs(_np(J) - Jo)))
    # FP32 recurrence: relative ~1e-6 of the largest integrals, never 1e-10 exact
    assert 1e-12 < dJ <= 1e-4 * np.max(np.abs(Jo))
    assert abs(oracle.e2(_np(J), _np(K), D) - oracle.e2(Jo, Ko, D)) <= 1e-4 * abs(oracle.e2(Jo, Ko, D))
