"""The seeded input recipes: determinism, geometry rules and sizes."""
import hashlib

import numpy as np

from paper_2412_13203_amd import inputs


def _digest(cfg):
    h = hashlib.sha256()
    b = cfg["basis"]
    for k in ("xyz", "shell_atom", "shell_l", "shell_nprim", "shell_prim_off", "exps", "coefs"):
        h.update(np.ascontiguousarray(b[k]).tobytes())
    h.update(np.ascontiguousarray(cfg["D"]).tobytes())
    return h.hexdigest()


def test_deterministic():
    assert _digest(inputs.make_config(1)) == _digest(inputs.make_config(1))
    assert _digest(inputs.make_config(2)) == _digest(inputs.make_config(2))
    assert _digest(inputs.make_config(2)) != _digest(inputs.make_config(2, seed=99))


def test_config_sizes():
    c1 = inputs.make_config(1)
    assert c1["basis"]["nbf"] == 20 and len(c1["basis"]["shell_l"]) == 12
    c2 = inputs.make_config(2)
    assert c2["basis"]["nbf"] == 440 and len(c2["basis"]["shell_l"]) == 160
    c5 = inputs.make_config(5)
    assert c5["basis"]["nbf"] == 660
    assert c2["D"].shape == (440, 440)
    assert np.array_equal(c2["D"], c2["D"].T)


def test_geometry_rules():
    c1 = inputs.make_config(1)
    xyz = c1["basis"]["xyz"]
    assert np.all((xyz >= 0) & (xyz <= 4))
    d = np.linalg.norm(xyz[:, None] - xyz[None], axis=-1)
    assert np.min(d[np.triu_indices(4, 1)]) >= 1.2
    c2 = inputs.make_config(2)
    xyz = c2["basis"]["xyz"]
    sites = np.round((xyz) / 2.5)
    assert np.max(np.abs(xyz - 2.5 * sites)) <= 0.3
    assert len({tuple(s) for s in sites}) == 40


def test_exponent_ranges():
    b = inputs.make_config(2)["basis"]
    assert b["exps"].min() >= 0.08 and b["exps"].max() <= 80
    assert np.all(b["shell_nprim"] == 3)


def test_batch_recipe():
    mols = inputs.make_batch(nmol=3)
    for m in mols:
        b = m["basis"]
        assert 8 <= m["natom"] <= 96
        assert set(np.unique(b["shell_l"])) == {0, 1, 2, 3}
        assert b["shell_nprim"].min() >= 1 and b["shell_nprim"].max() <= 6
