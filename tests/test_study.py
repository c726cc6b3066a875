"""Host-side scoring of the beta sweep (no GPU)."""
import numpy as np

from paper_1601_08201_amd import study


def test_scores_of_exact_and_scaled_images():
    rng = np.random.default_rng(0)
    S, Q = 12, 7
    x = rng.random(S * Q)
    x.reshape(S, Q)[3] = 0.0
    assert study.spatial_error(x, x, S, Q) == 0.0
    assert study.spectral_error(x, x, S, Q) < 1e-15
    # the spectral score ignores each spectrum's scale, the spatial one does not
    y = (x.reshape(S, Q) * rng.uniform(0.5, 2.0, (S, 1))).ravel()
    assert study.spectral_error(y, x, S, Q) < 1e-15
    assert study.spatial_error(y, x, S, Q) > 0.05
    # a uniformly scaled image has spatial error |scale - 1|
    assert abs(study.spatial_error(1.25 * x, x, S, Q) - 0.25) < 1e-12


def test_spectral_error_of_orthogonal_and_empty_spectra():
    S, Q = 2, 4
    t = np.array([1, 0, 0, 0, 0, 0, 0, 0], float)
    f = np.array([0, 1, 0, 0, 5, 5, 5, 5], float)
    # bin 0: orthogonal spectra (error 1); bin 1 is empty in the phantom (ignored)
    assert study.spectral_error(f, t, S, Q) == 1.0
    assert study.spectral_error(np.zeros(8), t, S, Q) == 1.0
    assert study.spatial_error(np.zeros(8), np.zeros(8), S, Q) == 0.0


def test_select_picks_smallest_spatial_error_per_grouping():
    res = [dict(grouping=g, beta=b, spatial_error=e, spectral_error=0.0)
           for g, b, e in [(0, 0.1, 0.3), (0, 0.2, 0.1), (0, 0.4, 0.2), (1, 0.1, 0.05), (1, 0.2, 0.5)]]
    best = study.select(res)
    assert best[0]["beta"] == 0.2 and best[1]["beta"] == 0.1
