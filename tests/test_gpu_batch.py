"""GPU parity of the batched path: many molecules of uneven size in one
launch per class, with per-class tiles (quartets per lane) from Algorithm 2.

Each molecule's J and K must equal those of a separate single-molecule plan
(same kernels, different work split: 1e-12 absolute, summation order only)
and, for the smallest molecules, the FP64 oracle (1e-10 absolute)."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _mods():
    import torch

    from paper_2412_13203_amd import inputs, mjk
    return torch, mjk, inputs


def _batch_inputs(inputs, mjk, nmol=6, atom_range=(3, 9)):
    shells = (0, 0, 1, 2, 3) if mjk.lib().mjk_lmax() >= 3 else (0, 0, 1, 2)
    return inputs.make_batch(nmol=nmol, seed=4, atom_range=atom_range, shells=shells)


def _single(torch, mjk, mol):
    plan = mjk.Plan(mol["basis"], tau=mol["tau"])
    D = torch.as_tensor(mol["D"], dtype=torch.float64, device="cuda:0").contiguous()
    J, K = plan.build_jk(D)
    torch.cuda.synchronize()
    return J.cpu().numpy(), K.cpu().numpy(), plan.stats["nquartet_kept"]


def _max_abs(a, b):
    return float(np.max(np.abs(a - b)))


def test_batch_matches_single_plans_and_tiles():
    torch, mjk, inputs = _mods()
    mols = _batch_inputs(inputs, mjk)
    print("batch natoms", [m["natom"] for m in mols], flush=True)
    bt = mjk.Batch([m["basis"] for m in mols], tau=1e-10)
    D = bt.pack([m["D"] for m in mols])
    J, K = bt.build_jk(D)
    torch.cuda.synchronize()
    Js, Ks = bt.unpack(J), bt.unpack(K)
    for m, mol in enumerate(mols):
        Jr, Kr, nq = _single(torch, mjk, mol)
        assert bt.nq_per_mol[m] == nq
        assert _max_abs(Js[m].cpu().numpy(), Jr) <= 1e-12, m
        assert _max_abs(Ks[m].cpu().numpy(), Kr) <= 1e-12, m
    # other quartets-per-lane tables change only the summation order
    nc = mjk.num_classes()
    for qpl in ([2] * nc, [16] * nc, [1 << (q % 5) for q in range(nc)]):
        bt.set_tiles(qpl)
        J2, K2 = bt.build_jk(D)
        torch.cuda.synchronize()
        assert _max_abs(J2.cpu().numpy(), J.cpu().numpy()) <= 1e-12
        assert _max_abs(K2.cpu().numpy(), K.cpu().numpy()) <= 1e-12


def test_batch_smallest_vs_oracle():
    torch, mjk, inputs = _mods()
    import oracle
    mols = _batch_inputs(inputs, mjk, nmol=12, atom_range=(2, 6))
    order = sorted(range(len(mols)), key=lambda m: mols[m]["basis"]["nbf"])[:2]
    sel = [mols[m] for m in order]
    bt = mjk.Batch([m["basis"] for m in sel], tau=1e-10)
    J, K = bt.build_jk(bt.pack([m["D"] for m in sel]))
    torch.cuda.synchronize()
    for m, mol in enumerate(sel):
        Jo, Ko, nq = oracle.build_jk(mol["basis"], mol["D"], mol["tau"])
        print(f"molecule nbf {mol['basis']['nbf']}: oracle quartets {nq}", flush=True)
        assert bt.nq_per_mol[m] == nq
        assert _max_abs(bt.unpack(J)[m].cpu().numpy(), Jo) <= 1e-10
        assert _max_abs(bt.unpack(K)[m].cpu().numpy(), Ko) <= 1e-10


def test_autotune_and_stamps():
    torch, mjk, inputs = _mods()
    mols = _batch_inputs(inputs, mjk, nmol=8, atom_range=(4, 12))
    bt = mjk.Batch([m["basis"] for m in mols], tau=1e-10)
    D = bt.pack([m["D"] for m in mols])
    J0, K0 = bt.build_jk(D)
    torch.cuda.synchronize()
    J0, K0 = J0.cpu().numpy(), K0.cpu().numpy()
    nkb = mjk.lib().mjk_num_kbuckets()
    qpl = bt.autotune(D, reps=1, per_bucket=False)
    assert len(qpl) == mjk.num_classes() and all(v in (1, 2, 4, 8, 16) for v in qpl)
    # per (class, bra K-bucket), through a cache file: the second call finds
    # the table there and sets it without tuning
    import tempfile
    cache = os.path.join(tempfile.mkdtemp(), "tiles.json")
    qb = bt.autotune(D, reps=1, per_bucket=True, cache=cache, key="test")
    assert len(qb) == mjk.num_classes() * nkb and all(v in (1, 2, 4, 8, 16) for v in qb)
    bt.set_tiles([1] * len(qb))
    assert bt.autotune(D, reps=1, per_bucket=True, cache=cache, key="test") == qb
    with open(cache) as fh:
        assert len(json.load(fh)) == 1
    bt.set_stamps(True)
    J, K = bt.build_jk(D)
    torch.cuda.synchronize()
    assert _max_abs(J.cpu().numpy(), J0) <= 1e-12
    assert _max_abs(K.cpu().numpy(), K0) <= 1e-12
    times = bt.mol_times()
    for (t0, t1), nq in zip(times, bt.nq_per_mol):
        if nq > 0:
            assert 0.0 <= t0 <= t1
    assert max(t1 for _, t1 in times) > 0.0


def test_batch_rejects_bad_tiles():
    torch, mjk, inputs = _mods()
    mols = _batch_inputs(inputs, mjk, nmol=2, atom_range=(2, 3))
    bt = mjk.Batch([m["basis"] for m in mols])
    with pytest.raises(mjk.MjkError):
        bt.set_tiles([3] * mjk.num_classes())
    with pytest.raises(mjk.MjkError):
        bt.set_tiles([1] * (mjk.num_classes() - 1))
    with pytest.raises(mjk.MjkError):
        bt.set_tiles([1] * (mjk.num_classes() * mjk.lib().mjk_num_kbuckets() + 1))
    bt.set_tiles([2] * (mjk.num_classes() * mjk.lib().mjk_num_kbuckets()))
