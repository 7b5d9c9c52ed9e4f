"""mjk_build_jk_static (the entry point that allocates nothing: work counters
and staging in the library's static device scratch) against mjk_build_jk on
the same inputs, through the C ABI: the 40-atom s,s,p,d workload, then a
smaller 8-atom cut of it (the scratch keeps the first call's contents), each
to 1e-10 per J and K element (the FP64 parity bar)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_static_scratch_build_matches_build_jk():
    import torch

    from paper_2412_13203_amd import inputs, mjk
    for natom in (40, 8):
        cfg = inputs.make_config(2, natom=natom)
        b, D = cfg["basis"], cfg["D"]
        print(f"no-alloc entry point: {natom}-atom cut, nbf {b['nbf']}", flush=True)
        Dd = torch.as_tensor(D, dtype=torch.float64, device="cuda:0").contiguous()
        ref = mjk.Plan(b, tau=cfg["tau"])
        J0, K0 = ref.build_jk(Dd)
        plan = mjk.Plan(b, tau=cfg["tau"], flags=mjk.FLAG_NO_STAGING)
        assert plan.stats["workspace_bytes"] < ref.stats["workspace_bytes"]
        J = torch.full_like(Dd, float("nan"))
        K = torch.full_like(Dd, float("nan"))
        plan.build_jk_static(Dd, J, K)
        torch.cuda.synchronize()
        dj = float((J - J0).abs().max())
        dk = float((K - K0).abs().max())
        print(f"  max|dJ| {dj:.2e} max|dK| {dk:.2e}", flush=True)
        assert dj <= 1e-10 and dk <= 1e-10, (natom, dj, dk)
        # the existing entry point refuses a plan without staging
        with pytest.raises(mjk.MjkError) as ei:
            plan.build_jk(Dd)
        assert ei.value.code == -6
        # a regular plan may use the static entry point too
        J2 = torch.empty_like(Dd)
        K2 = torch.empty_like(Dd)
        ref.build_jk_static(Dd, J2, K2)
        torch.cuda.synchronize()
        assert float((J2 - J0).abs().max()) <= 1e-10 and float((K2 - K0).abs().max()) <= 1e-10
