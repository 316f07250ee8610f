"""What the trained warm-start networks give on media they have not seen (held-out
seeds of their training distribution, 4096 training media).

* The deployed network (trained on the plain method's converged solutions): its
  initial map is closer to the true map than the homogeneous 1540 m/s guess, and
  its mean speed starts a local search of the sweep's lattice that needs far fewer
  loss evaluations than the 41-speed sweep.  (Its map itself is not taken as the
  start on these media: its CMPE is above that of the best uniform speed nearby,
  and the plain objective judges the start by that; the seconds-to-target figures
  are in the benchmark's s_to_target report.)
* The network trained on the true maps: what the features carry about the medium
  (its initial map is much closer to the truth than either guess)."""
import numpy as np
import pytest

import gpu_setup as G

pytestmark = pytest.mark.gpu

HELD_OUT = range(9000, 9008)


@pytest.fixture(scope="module")
def nets():
    G.ensure_built()
    from paper_2608_06853_amd import warmstart
    return {k: warmstart.load_network(k) for k in ("plain", "true")}


@pytest.fixture(scope="module")
def rmse(nets):
    from paper_2608_06853_amd import warmstart
    r = warmstart.evaluate_init(nets, HELD_OUT)
    print("held-out initial-map RMSE (m/s):", r, flush=True)
    return r


def test_deployed_network_beats_homogeneous(rmse):
    assert rmse["net_plain"] < rmse["homogeneous_1540"]
    assert rmse["net_plain"] < rmse["sweep"]


def test_true_label_network_carries_the_medium(rmse):
    assert rmse["net_true"] < 0.75 * rmse["homogeneous_1540"]
    assert rmse["net_true"] < 0.75 * rmse["sweep"]


def test_learned_start_runs_end_to_end(nets):
    """The deployed warm start (the network's map if its CMPE is not above that of
    the best uniform speed of a local lattice search around its mean speed, else
    that speed, else the full sweep) reaches the plain method's target on a
    held-out medium with a fraction of the sweep's evaluations."""
    import afsynth
    from paper_2608_06853_amd import warmstart
    r = warmstart.s_to_target(afsynth.configs.C4, nets["plain"], seed=9001)
    print({k: r[k] for k in ("learned_start", "learned_speeds_evaluated", "learned_iters",
                             "learned_reached", "learned_seconds", "plain_seconds",
                             "plain_best_speed")}, flush=True)
    assert r["learned_start"] in ("map", "local_sweep")
    assert r["learned_reached"] and np.isfinite(r["learned_seconds"])
    assert r["learned_speeds_evaluated"] <= 15
