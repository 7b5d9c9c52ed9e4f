"""GPU tests of the SCF driver around the library (Section 2.1: the Fock
matrix, one-electron Hamiltonian plus J - K/2, is rebuilt from the density
at every iteration), through the C ABI:

  * mjk_one_electron (S, T, V, nuclear repulsion; Obara-Saika on the GPU)
    against the oracle's McMurchie-Davidson matrices, every element;
  * the converged RHF energy of the GPU driver (library integrals, torch
    linear algebra) against the oracle's RHF loop: config 1 computed here,
    the 4-atom cut of the 40-atom s,s,p,d recipe from the stored value
    (tests/golden/scf_small.json, written by make_golden.py from the oracle);
  * density-weighted screening (mjk_plan_set_density_screen): it never keeps
    more quartets than the Schwarz screen, keeps them all for a density change
    of 1 in every row, drops quartets for a small one with a J/K error inside the
    skipped bound, and None restores the plain lists exactly;
  * the work lists do not depend on the number of host threads that build
    them;
  * the incremental SCF (difference densities with that screening) converges
    to the energy of the full builds.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import scf as oscf

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _mods():
    import torch

    from paper_2412_13203_amd import inputs, mjk, scf
    return torch, mjk, inputs, scf


def _cases(inputs):
    c1 = inputs.make_config(1)
    c2 = inputs.make_config(2, natom=8)
    rng = np.random.default_rng(77)
    lmax = min(3, _lmax())
    b = inputs.random_shells(rng, 3, list(range(lmax + 1)), box=2.5, nprim_range=(1, 6), exp_range=(0.1, 30.0))
    b["xyz"][2] = b["xyz"][0]  # coincident centres: PC = 0 for some nuclei
    return {"config1": (c1["basis"], inputs.scf_system(c1)[0]),
            "config2_8atoms": (c2["basis"], inputs.scf_system(c2)[0]),
            "lmax_shells_coincident": (b, np.array([1.0, 3.5, 0.0]))}


def _lmax():
    from paper_2412_13203_amd import mjk
    return mjk.lib().mjk_lmax()


@pytest.mark.parametrize("name", ["config1", "config2_8atoms", "lmax_shells_coincident"])
def test_one_electron_vs_oracle(name):
    torch, mjk, inputs, _ = _mods()
    b, Z = _cases(inputs)[name]
    print(f"one-electron case {name}: nbf {b['nbf']}", flush=True)
    plan = mjk.Plan(b, tau=0.0)
    S, T, V, enuc = plan.one_electron(Z)
    torch.cuda.synchronize()
    So, To, Vo = oracle.one_electron(b, Z)
    for M, R, what in ((S, So, "S"), (T, To, "T"), (V, Vo, "V")):
        d = np.abs(M.cpu().numpy() - R)
        bar = 1e-10 + 1e-13 * np.abs(R)
        print(f"  {what}: max |d| {d.max():.2e} (max |ref| {np.abs(R).max():.2e})", flush=True)
        assert (d <= bar).all(), (what, d.max())
    assert np.array_equal(S.cpu().numpy(), S.cpu().numpy().T)
    en = oracle.nuclear_repulsion(b["xyz"], Z)
    assert abs(float(enuc) - en) <= 1e-12 * max(1.0, abs(en))


def test_one_electron_optional_outputs_and_errors():
    torch, mjk, inputs, _ = _mods()
    b, Z = _cases(inputs)["config1"]
    plan = mjk.Plan(b)
    S, T, V, _ = plan.one_electron(Z)
    with pytest.raises(mjk.MjkError):
        plan.one_electron(Z[:-1])
    with pytest.raises(mjk.MjkError):
        plan.one_electron(np.full(len(Z), np.nan))


def _gpu_rhf(b, Z, nocc, tau, **kw):
    torch, mjk, inputs, scf = _mods()
    r = scf.RHF(b, Z, nocc, tau=tau).run(**kw)
    print(f"  GPU RHF: E = {r['energy']:.12f}, {r['iterations']} iterations, converged {r['converged']}",
          flush=True)
    return r


def test_rhf_config1_matches_oracle():
    torch, mjk, inputs, scf = _mods()
    cfg = inputs.make_config(1)
    Z, nocc = inputs.scf_system(cfg)
    ro = oscf.rhf(cfg["basis"], Z, nocc, tau=0.0)
    r = _gpu_rhf(cfg["basis"], Z, nocc, 0.0, e_tol=1e-12, err_tol=1e-9)
    assert ro["converged"] and r["converged"]
    print(f"  oracle RHF: E = {ro['energy']:.12f}", flush=True)
    assert abs(r["energy"] - ro["energy"]) <= 1e-10
    D = r["D"].cpu().numpy()
    assert np.max(np.abs(D - ro["D"])) <= 1e-6  # the density converges to first order only


def test_rhf_config2_cut_matches_stored_oracle():
    torch, mjk, inputs, scf = _mods()
    with open(os.path.join(HERE, "golden", "scf_small.json")) as fh:
        ref = json.load(fh)["cases"]["config2_4atoms"]
    cfg = inputs.make_config(2, natom=4)
    Z, nocc = inputs.scf_system(cfg)
    r = _gpu_rhf(cfg["basis"], Z, nocc, cfg["tau"], e_tol=1e-12, err_tol=1e-9)
    assert r["converged"]
    assert abs(r["energy"] - ref["energy"]) <= 1e-10, (r["energy"], ref["energy"])


def test_density_screen_bounds_and_restores():
    torch, mjk, inputs, _ = _mods()
    cfg = inputs.make_config(2, natom=8)
    b = cfg["basis"]
    tau = 1e-10
    plan = mjk.Plan(b, tau=tau)
    n0 = plan.kept_quartets()
    D = torch.as_tensor(cfg["D"], device="cuda:0")
    J0, K0 = plan.build_jk(D)
    # a density change with |dD| >= 1 in every shell row keeps every
    # quartet the Schwarz screen keeps
    big = torch.ones_like(D)
    plan.set_density_screen(big)
    assert plan.kept_quartets() == n0
    # a small one drops quartets; the dropped contributions are bounded
    rng = np.random.default_rng(5)
    E = rng.standard_normal(D.shape) * 1e-6
    dD = torch.as_tensor(0.5 * (E + E.T), device="cuda:0")
    plan.set_density_screen(dD)
    n1 = plan.kept_quartets()
    print(f"  density screen: kept {n1} of {n0}", flush=True)
    assert n1 < n0
    Js, Ks = plan.build_jk(dD)
    plan.set_density_screen(None)
    assert plan.kept_quartets() == n0
    Jf, Kf = plan.build_jk(dD)
    torch.cuda.synchronize()
    # each skipped quartet changes an element of J or K by at most
    # 8 tau-sized terms (8-fold symmetry); the bound is loose by design
    bound = 8.0 * tau * (n0 - n1)
    dj = float((Js - Jf).abs().max())
    dk = float((Ks - Kf).abs().max())
    print(f"  screened vs full: max |dJ| {dj:.2e}, max |dK| {dk:.2e}, bound {bound:.2e}", flush=True)
    assert dj <= bound and dk <= bound
    # and the plain lists give the plain result again
    J2, K2 = plan.build_jk(D)
    torch.cuda.synchronize()
    assert float((J2 - J0).abs().max()) <= 1e-12 and float((K2 - K0).abs().max()) <= 1e-12


def test_work_lists_do_not_depend_on_host_threads(monkeypatch):
    """The planner builds the work lists of the bin pairs on host threads;
    one thread and the default count give the same lists (kept counts,
    primitive quartets, FP32 split) and the same J and K, for the Schwarz
    lists and for a density-weighted screen."""
    torch, mjk, inputs, _ = _mods()
    cfg = inputs.make_config(2, natom=8)
    b = cfg["basis"]
    D = torch.as_tensor(cfg["D"], device="cuda:0")
    rng = np.random.default_rng(8)
    E = rng.standard_normal(D.shape) * 1e-6
    dD = torch.as_tensor(0.5 * (E + E.T), device="cuda:0")
    keys = ("nquartet_kept", "nquartet_fp32", "nprim_quartet_kept", "ncart_eri_kept")
    res = []
    for threads in ("1", None):
        if threads is None:
            monkeypatch.delenv("OMP_NUM_THREADS", raising=False)
        else:
            monkeypatch.setenv("OMP_NUM_THREADS", threads)
        plan = mjk.Plan(b, tau=1e-10, fp32_tau=1e-7)
        st = tuple(plan.stats[k] for k in keys)
        J, K = plan.build_jk(D)
        plan.set_density_screen(dD)
        st_d = tuple(plan.stats[k] for k in keys)
        Jd, Kd = plan.build_jk(dD)
        torch.cuda.synchronize()
        res.append((st, st_d, J, K, Jd, Kd))
    (a, ad, *ma), (c, cd, *mc) = res
    print(f"  one thread vs default: {a} / {ad}", flush=True)
    assert a == c and ad == cd
    assert a[1] > 0 and ad[0] < a[0]
    for x, y in zip(ma, mc):
        assert float((x - y).abs().max()) <= 1e-12


def test_incremental_rhf_matches_full():
    torch, mjk, inputs, scf = _mods()
    cfg = inputs.make_config(2, natom=8)
    Z, nocc = inputs.scf_system(cfg)
    full = _gpu_rhf(cfg["basis"], Z, nocc, cfg["tau"], e_tol=1e-9, err_tol=1e-7)
    inc = _gpu_rhf(cfg["basis"], Z, nocc, cfg["tau"], e_tol=1e-9, err_tol=1e-7, incremental=True)
    assert full["converged"] and inc["converged"]
    print(f"  kept quartets per iteration (incremental): {inc['kept_quartets']}", flush=True)
    assert min(inc["kept_quartets"][1:]) < inc["kept_quartets"][0]
    assert inc["full_build"][-1]  # the converged energy comes from a full build
    # the energy is stationary: density errors of the order of the screening
    # move it to second order only
    assert abs(full["energy"] - inc["energy"]) <= 1e-8
