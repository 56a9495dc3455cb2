import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle
    oracle.build(force=False)
    return oracle


def boundary_coins(oracle_mod, rng_seed, count, e=0):
    """Worlds w whose coin for edge slot e is a multiple of 256 (between 512
    and 2^32 - 512): for those, p = coin / 2^32 is a float32 exactly, so its
    threshold floor(p * 2^32) equals the coin itself.  Returns [(w, coin)]."""
    out = []
    w = 0
    while len(out) < count:
        c = oracle_mod.coin(rng_seed, w, e)
        if c % 256 == 0 and 512 <= c < 2 ** 32 - 512:
            out.append((w, c))
        w += 1
    return out


def dyadic_p(c):
    """float32 probability equal to c / 2^32 (c a multiple of 256)."""
    import numpy as np
    p = np.float32(c / 2.0 ** 32)
    assert int(np.float64(p) * 2.0 ** 32) == c
    return float(p)
