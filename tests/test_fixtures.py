"""The oracle-made liquid fixture (tests/golden/make_liquid_state.py) is a
valid dense-liquid state of the 1000-molecule system."""
import os

import numpy as np

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                       "liquid_1000_T0.75_sweep500.npz")


def test_liquid_fixture_is_a_valid_dense_liquid(oracle_mod):
    f = np.load(FIXTURE)
    com, quat, types, sweep = f["com"], f["quat"], f["types"], int(f["sweep"])
    assert com.shape == (1000, 3) and quat.shape == (1000, 4) and types.shape == (1000, 3)
    assert sweep == 500
    L = oracle_mod.box_length(1000)
    assert np.all((com >= 0) & (com < L))
    assert np.allclose((quat * quat).sum(1), 1.0, atol=1e-12)
    assert np.all(np.sort(types, axis=1) == [0, 1, 2])
    o = oracle_mod.System(oracle_mod.Params(n_molecules=1000, temperature=0.75, colours_per_axis=2,
                                            cells_per_side=4), lattice=False)
    o.set_state(com, quat, types, sweep)
    e = o.energy()
    # the stored energy is the oracle's, and the state is far below the
    # lattice start (E/M ~ 1.6e5): a dense liquid
    assert e == float(f["energy"])
    assert abs(f["e_acc"] - e) <= 1e-9 * abs(e)
    assert 1.0 < e / 1000 < 50.0
