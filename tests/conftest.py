import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

H2_MECH = os.path.join(ROOT, "synth", "data", "h2_synth_9sp_24r.mech")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def h2_path():
    return H2_MECH


@pytest.fixture(scope="session")
def h2_mech():
    import synth
    return synth.read_mech(H2_MECH)


@pytest.fixture(scope="session")
def h2_oracle():
    import oracle
    return oracle.Mech(H2_MECH)


@pytest.fixture(scope="session")
def npchem(h2_mech):
    from npchem import NpChem
    return NpChem(h2_mech)


@pytest.fixture(scope="session")
def cfg1(h2_mech):
    from synth import fields
    return fields.ignition_cells(h2_mech)


def random_states(mech, n, seed=7, T_range=(300.0, 2800.0), radicals=True):
    """Random (T, Y) states with all species present (for identity tests)."""
    rng = np.random.default_rng(seed)
    K = mech.n_species
    out = []
    for _ in range(n):
        T = rng.uniform(*T_range)
        Y = rng.uniform(0.0, 1.0, K) if radicals else np.zeros(K)
        Y = Y ** 3 + 1e-6
        Y /= Y.sum()
        out.append((T, Y))
    return out
