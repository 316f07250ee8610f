"""What the trained warm-start network gains over the method without it, on media
it has not seen (held-out seeds of its training distribution): the initial
slowness map it predicts from a 1540 m/s beamform is closer to the true map than
the homogeneous 1540 m/s guess and than the plain method's best global speed
(the adaptive-grid sweep)."""
import numpy as np
import pytest

import gpu_setup as G

pytestmark = pytest.mark.gpu

HELD_OUT = range(9000, 9008)


@pytest.fixture(scope="module")
def net():
    G.ensure_built()
    from paper_2608_06853_amd import warmstart
    return warmstart.load_network("true")


def test_network_initial_map_beats_homogeneous_and_sweep(net):
    from paper_2608_06853_amd import warmstart
    r = warmstart.evaluate_init({"true": net}, HELD_OUT)
    print("held-out initial-map RMSE (m/s):", r, flush=True)
    assert r["net_true"] < 0.75 * r["homogeneous_1540"]
    assert r["net_true"] < 0.75 * r["sweep"]
