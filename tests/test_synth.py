"""The seeded input generator: compiled chord sums equal the numpy formulas,
phantoms are reproducible and stay in range, and the noise model holds."""
import numpy as np
import pytest

import synth
from synth import phantom as P


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "tiny_helical", "fan2d_128"])
def test_compiled_chords_match_numpy(name):
    cfg = synth.get_config(name)
    ph = synth.make_phantom(cfg)
    a = P.analytic_sinogram(cfg, ph, use_c=True)
    b = P.analytic_sinogram(cfg, ph, use_c=False)
    assert np.abs(a - b).max() <= 1e-11 * np.abs(b).max()


def test_phantom_reproducible_and_in_range():
    cfg = synth.get_config("fan2d_128")
    a, b = synth.make_phantom(cfg), synth.make_phantom(cfg)
    for k in ("cx", "cy", "ax", "ay", "phi", "amp"):
        assert np.array_equal(a[k], b[k])
    x = synth.pixelize(cfg, a, ss=2)
    inside = x[x > 0]
    assert inside.min() >= 0.015 * 0.2 and x.max() <= 0.025 + 1e-12


def test_noise_model():
    cfg = synth.get_config("fan2d_128")
    d = synth.make_problem_data(cfg, workers=1)
    assert np.all(d["w"] >= 0) and np.all(d["w"] == np.round(d["w"]))
    pos = d["w"] > 0
    np.testing.assert_allclose(d["y"][pos], np.log(cfg["I0"] / d["w"][pos]))
    assert np.all(d["y"][~pos] == 0)
    # the mean count follows I0 exp(-ybar) within Poisson scatter
    lam = cfg["I0"] * np.exp(-d["ybar"])
    z = (d["w"] - lam) / np.sqrt(lam)
    assert abs(z.mean()) < 0.05 and abs(z.std() - 1.0) < 0.05
