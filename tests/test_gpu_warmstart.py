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


def test_learned_start_runs_end_to_end():
    """The learned warm start (network map, else a sweep narrowed around the
    network's speed, else the full sweep) runs through to the plain method's
    target on a held-out medium."""
    import afsynth
    from paper_2608_06853_amd import warmstart
    net = warmstart.load_network("plain")
    r = warmstart.s_to_target(afsynth.configs.C4, net, seed=9001)
    print({k: r[k] for k in ("learned_start", "learned_iters", "learned_reached", "learned_seconds",
                             "learned_init_seconds", "plain_seconds", "plain_sweep_seconds")},
          flush=True)
    assert r["learned_start"] in ("map", "local_sweep", "sweep")
    assert r["learned_iters"] >= 1 and np.isfinite(r["learned_seconds"])
