"""Pins of the oracle's receive-channel images and lag-one coherence: closed forms
of the coherence on constructed channels, and the channel images against the
block-pair images of the configured blocking (their sums are the same image)."""
import numpy as np

import afsynth
import problems
from oracle import coherence, model


def test_loc_identical_channels_is_one():
    rng = np.random.default_rng(0)
    v = rng.standard_normal((4, 9)) + 1j * rng.standard_normal((4, 9))
    X = np.broadcast_to(v.reshape(1, -1), (12, 36)) * np.arange(1, 13)[:, None]
    assert np.allclose(coherence.lag_one_coherence(X, 9), 1.0, atol=1e-14)


def test_loc_phase_ramp_is_cosine():
    # X_r = exp(j theta r) v: Re(X_r conj X_{r+1}) / |.|^2 = cos(theta)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(18) + 1j * rng.standard_normal(18)
    for th in (0.3, 1.2, 2.5):
        X = np.exp(1j * th * np.arange(10))[:, None] * v[None, :]
        assert np.allclose(coherence.lag_one_coherence(X, 9), np.cos(th), atol=1e-13)


def test_loc_skips_channels_without_energy():
    rng = np.random.default_rng(2)
    v = rng.standard_normal(9) + 1j * rng.standard_normal(9)
    X = np.tile(v, (6, 1))
    X[0] = 0.0                      # outside the aperture: pair (0, 1) is skipped
    X[3] = -v                       # pairs (2, 3) and (3, 4) give -1
    loc = coherence.lag_one_coherence(X, 9)
    assert abs(loc[0] - (1.0 - 1.0 - 1.0 + 1.0) / 4.0) < 1e-14
    assert coherence.lag_one_coherence(np.zeros((5, 9)), 9)[0] == 0.0


def test_loc_incoherent_channels_near_zero():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((64, 9 * 500)) + 1j * rng.standard_normal((64, 9 * 500))
    loc = coherence.lag_one_coherence(X, 9)
    assert abs(loc.mean()) < 0.01 and np.abs(loc).max() < 0.35


def test_channel_images_sum_to_the_block_image():
    cfg = afsynth.configs.MICRO.with_(
        img=afsynth.ImgCfg(n_depth=3, n_angle=4, depth_min=8.0, depth_max=20.0))
    med = afsynth.medium_for(cfg)
    iq = problems.simulate_iq(cfg, med, n_seg=32)
    prob = problems.problem(cfg, iq)
    s = problems.true_slowness(cfg, med, prob)
    X = coherence.channel_images(prob, s)
    f = model.forward(prob, s, problems.loss_params(cfg), keep=True)
    img = f["bblk"].sum(axis=(0, 1))
    assert np.abs(X.sum(axis=0) - img).max() < 1e-12 * np.abs(img).max()
    # a channel outside a point's apodisation is empty there
    assert np.all(X[~prob.apod()] == 0)
