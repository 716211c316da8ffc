"""The stored extended-precision references (tests/golden/extended_*.npz,
written by tests/golden/make_extended_refs.py from the oracle alone) still
match the oracle: a few of their atoms are recomputed by the extended build
and must agree bit for bit, and each file covers the atoms and
configurations its recipe names."""
import os

import numpy as np
import pytest

from golden import make_extended_refs as M


@pytest.mark.parametrize("name", sorted(M.references()))
def test_reference_matches_oracle(orc, name):
    if not os.path.exists(M.path_of(name)):
        pytest.fail(f"{M.path_of(name)} missing: run python tests/golden/make_extended_refs.py {name}")
    K, atoms, cfg_ids, cfgs = M.load(name)
    wl, parts = M.references()[name]
    assert K.shape == (len(parts), parts[0][2].size, wl["k_last"] - wl["k_first"] + 1)
    for j, (c, cfg_id, a) in enumerate(parts):
        assert int(cfgs[j]) == c and int(cfg_ids[j]) == cfg_id
        assert np.array_equal(atoms[j], a)
    # recompute the first and last atom of the first and last configuration
    for j in sorted({0, len(parts) - 1}):
        c, cfg_id, a = parts[j]
        L = M.oracle_laser(wl["lasers"][c], wl.get("field_order", 5))
        pick = a[[0, -1]]
        r = orc.chain(L, wl["seed"], cfg_id, pick, wl["r_factor"] * L.w0, orc.rayleigh(L),
                      wl["k_first"], wl["k_last"], extended=True)
        got = r["K"].reshape(2, -1)
        want = K[j][[0, -1]]
        assert np.array_equal(got, want, equal_nan=True), (name, j)
    assert np.isfinite(K).sum() > 0
