"""GPU tests of the boundary's smaller entry points, through the C ABI:
the device Boys function against the oracle's (Section 2.2's analytic
[00|00] is a prefactor times F_m(T)), the E2 backward (upstream gradient
times dE2/dD = J - K/2 and times dE2/dR), and the per-context error message."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _mods():
    import torch

    from paper_2412_13203_amd import inputs, mjk
    return torch, mjk, inputs


def test_boys_matches_oracle():
    """Every order the class kernels use (0..13) on arguments spanning the
    table (grid points, midpoints, both sides of the switch to the
    asymptotic branch at T = 40) and far beyond; bar 2e-14 relative (the
    oracle's series is long double; the device's Taylor step is ~1e-17)."""
    torch, mjk, _ = _mods()
    rng = np.random.default_rng(3)
    T = np.concatenate([[0.0, 1e-12, 1.0 / 32, 1.0 / 16, 0.5, 1.0, 7.96875, 39.96875, 39.999999, 40.0,
                         40.000001, 45.5, 100.0, 1e3, 1e6],
                        rng.uniform(0, 40, 200), np.exp(rng.uniform(np.log(40), np.log(1e5), 40))])
    for mmax in (0, 1, 4, 8, 12, 13):
        F = mjk.boys(T, mmax).cpu().numpy()
        ref = np.array([oracle.boys(mmax, float(t)) for t in T])
        rel = np.abs(F - ref) / np.abs(ref)
        print(f"boys mmax {mmax}: max rel err {rel.max():.2e}", flush=True)
        assert rel.max() <= 2e-14, (mmax, T[np.argmax(rel.max(axis=1))], rel.max())


def test_boys_rejects_bad_order_and_marks_bad_arguments():
    torch, mjk, _ = _mods()
    with pytest.raises(mjk.MjkError) as ei:
        mjk.boys([1.0], 14)
    assert ei.value.code == -2
    assert "mmax" in mjk.context_last_error()
    F = mjk.boys([-1.0, float("nan"), 2.0], 3).cpu().numpy()
    assert np.isnan(F[0]).all() and np.isnan(F[1]).all() and np.isfinite(F[2]).all()


def test_e2_backward_matches_pieces():
    torch, mjk, inputs = _mods()
    cfg = inputs.make_config(5, natom=4)
    b, D = cfg["basis"], cfg["D"]
    plan = mjk.Plan(b, grad=True)
    Dd = torch.as_tensor(D, dtype=torch.float64, device="cuda:0").contiguous()
    J, K = plan.build_jk(Dd)
    g = plan.grad_e2(Dd)
    gout = torch.tensor(-2.5, dtype=torch.float64, device="cuda:0")
    gD, gR = plan.e2_backward(Dd, J, K, gout)
    torch.cuda.synchronize()
    assert float((gD - (-2.5) * (J - 0.5 * K)).abs().max()) <= 1e-13 * float(J.abs().max())
    assert float((gR - (-2.5) * g).abs().max()) <= 1e-13 * float(g.abs().max())
    gD1, gR1 = plan.e2_backward(Dd, J, K, None, want_R=False)
    assert gR1 is None and float((gD1 - (J - 0.5 * K)).abs().max()) == 0.0
    # a plan without the gradient flag gives gD but refuses gR
    p2 = mjk.Plan(b)
    J2, K2 = p2.build_jk(Dd)
    gD2, _ = p2.e2_backward(Dd, J2, K2, None, want_R=False)
    with pytest.raises(mjk.MjkError) as ei:
        p2.e2_backward(Dd, J2, K2, None, want_D=False)
    assert ei.value.code == -6
    assert "MJK_FLAG_GRAD" in mjk.context_last_error()


def test_autograd_with_cpu_density():
    """D on the host with requires_grad: its gradient comes back on the host
    in D's dtype (the library works on a device copy)."""
    torch, mjk, inputs = _mods()
    cfg = inputs.make_config(5, natom=3)
    b, D = cfg["basis"], cfg["D"]
    coords = torch.tensor(b["xyz"], dtype=torch.float64, requires_grad=True)
    Dc = torch.tensor(D, dtype=torch.float64, requires_grad=True)
    e = mjk.E2.apply(coords, Dc, b)
    assert e.device == Dc.device
    (0.5 * e).backward()
    assert Dc.grad is not None and Dc.grad.device == Dc.device and Dc.grad.dtype == Dc.dtype
    plan = mjk.Plan(b, grad=True)
    Dd = Dc.detach().to("cuda:0").contiguous()
    J, K = plan.build_jk(Dd)
    g = plan.grad_e2(Dd)
    torch.cuda.synchronize()
    np.testing.assert_allclose(Dc.grad.numpy(), 0.5 * (J - 0.5 * K).cpu().numpy(), rtol=0,
                               atol=1e-13 * float(J.abs().max()))
    np.testing.assert_allclose(coords.grad.numpy(), 0.5 * g.cpu().numpy(), rtol=0,
                               atol=1e-13 * float(g.abs().max()))


def test_context_error_message():
    torch, mjk, inputs = _mods()
    cfg = inputs.make_config(1)
    plan = mjk.Plan(cfg["basis"])
    with pytest.raises(mjk.MjkError) as ei:
        plan.set_tiles([3] * mjk.num_classes())
    assert ei.value.code == -1
    msg = mjk.context_last_error()
    assert "quartets per lane" in msg and msg in str(ei.value)
