"""Pins of the FP64 oracle's factored forward model (the PSF, attenuation and
background of Section 4.1's simulation): the Gaussian taps, the 2-D blur H and
the attenuation factors, against closed forms, library convolutions and
symmetry; and the recipe of the physics inputs (scatter and random fractions)."""
import math

import numpy as np
import pytest

import oracle
from paper_2409_13344_amd import synth

TO_SIGMA = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))


@pytest.mark.parametrize("fwhm", [2.0, 4.0, 5.62])
def test_taps_width_and_mass(fwhm):
    """Sum 1, symmetric; with a wide support the tap at t = FWHM/2 is half the central
    one (the definition of FWHM) and the second moment is sigma^2."""
    w = oracle.psf_taps(fwhm)
    R = (len(w) - 1) // 2
    assert R == oracle.psf_radius(fwhm) == math.ceil(3.0 * fwhm * TO_SIGMA)
    assert abs(w.sum() - 1.0) < 1e-15 and np.allclose(w, w[::-1], rtol=0, atol=1e-18)
    wide = oracle.psf_taps(fwhm, R=60)
    if float(fwhm / 2).is_integer():
        h = int(fwhm / 2)
        assert abs(wide[60 + h] / wide[60] - 0.5) < 1e-14
    t = np.arange(-60, 61)
    sig = fwhm * TO_SIGMA
    # sampling a Gaussian changes its second moment by O(4 pi^2 sigma^4 exp(-2 pi^2 sigma^2))
    # (Poisson summation); that bound, with a margin of 10, or 1e-9
    tol = max(1e-9, 10 * 4 * math.pi ** 2 * sig ** 4 * math.exp(-2 * math.pi ** 2 * sig ** 2))
    assert abs((t * t * wide).sum() - sig ** 2) < tol


def test_blur_is_separable_convolution_and_self_adjoint():
    """H x equals a row-then-column numpy convolution with the taps (zero outside the
    image); <H x, y> = <x, H y>; constants are kept away from the border; a centred
    delta spreads with variance 2 sigma^2."""
    n, fwhm = 24, 4.0
    w = oracle.psf_taps(fwhm)
    R = (len(w) - 1) // 2
    rng = np.random.default_rng(3)
    x = rng.standard_normal(n * n)
    y = rng.standard_normal(n * n)
    Hx = oracle.psf_apply(n, fwhm, x)
    img = x.reshape(n, n)
    rows = np.array([np.convolve(r, w, mode="same") for r in img])
    ref = np.array([np.convolve(c, w, mode="same") for c in rows.T]).T
    assert np.allclose(Hx, ref.ravel(), rtol=0, atol=1e-13)
    assert abs(Hx @ y - x @ oracle.psf_apply(n, fwhm, y)) < 1e-11 * np.abs(Hx).sum()
    one = oracle.psf_apply(n, fwhm, np.ones(n * n)).reshape(n, n)
    assert np.allclose(one[R:n - R, R:n - R], 1.0, rtol=0, atol=1e-14)
    assert one[0, 0] < 0.5
    e = np.zeros(n * n)
    e[(n // 2) * n + n // 2] = 1.0
    h = oracle.psf_apply(n, fwhm, e).reshape(n, n)
    r = np.arange(n) - n // 2
    var = (h * (r[:, None] ** 2 + r[None, :] ** 2)).sum()
    assert abs(h.sum() - 1.0) < 1e-14
    assert abs(var - 2 * (w * np.arange(-R, R + 1) ** 2).sum()) < 1e-12


def test_attenuation_closed_form_chords():
    """Uniform mu over the whole square: n_i = exp(-mu * chord length of ray i through
    the square), the chord in closed form."""
    geom = synth.Geometry(16, 22, 24)
    G = synth.siddon_matrix(geom)
    mu0 = 0.07
    att = oracle.attenuation(G, np.full(geom.d, mu0))
    for a in range(geom.n_angles):
        phi = a * math.pi / geom.n_angles
        for b in range(geom.n_bins):
            s = (b - (geom.n_bins - 1) / 2.0) * geom.ds
            L = synth.chord_length_square(phi, s, geom.n / 2.0)
            assert abs(att[a * geom.n_bins + b] - math.exp(-mu0 * L)) < 1e-12
    # and the physics inputs use exactly these factors for their water disc
    pp = synth.make_physics_problem(geom, [1], tc=1e5, G=G)
    assert np.allclose(pp.att, oracle.attenuation(G, pp.mu), rtol=1e-13, atol=0)


def test_factored_matrix_is_the_product():
    """factored_matrix(G, n, fwhm, att) applied to x equals att * G (H x)."""
    geom = synth.Geometry(12, 18, 16)
    G = synth.siddon_matrix(geom)
    att = np.random.default_rng(1).uniform(0.2, 1.0, geom.m)
    A = oracle.factored_matrix(G, geom.n, 3.0, att)
    x = np.random.default_rng(2).uniform(0.0, 2.0, geom.d)
    ref = att * oracle.forward(G, oracle.psf_apply(geom.n, 3.0, x))
    assert np.allclose(oracle.forward(A, x), ref, rtol=1e-12, atol=1e-12)
    r = np.random.default_rng(3).standard_normal(geom.m)
    assert np.allclose(oracle.back(A, r), oracle.psf_apply(geom.n, 3.0, oracle.back(G, att * r)),
                       rtol=1e-12, atol=1e-12)


def test_physics_recipe_fractions():
    """The expected counts follow Section 4.1's definitions: SF = Sc/(Tc+Sc) and
    RF = Rc/(Tc+Sc+Rc), TC = Tc+Sc+Rc; the background is Sc + Rc."""
    geom = synth.Geometry(32, 48, 40)
    pp = synth.make_physics_problem(geom, [7], tc=4e5, fov_mm=32 * 2.34)
    # expected (noise-free) trues from the unblurred truth through the same physics
    from scipy.ndimage import gaussian_filter
    img = pp.f_true[0].reshape(32, 32)
    blurred = gaussian_filter(img, pp.fwhm_px * TO_SIGMA, mode="constant", truncate=3.0).ravel()
    T = pp.att * oracle.forward(pp.G, blurred)
    gam = pp.gamma[0].astype(np.float64)
    R = gam.min() * np.ones_like(gam)      # randoms are the uniform floor of the background
    S = gam - R
    tc = T.sum() + gam.sum()
    assert abs(tc - 4e5) < 1e-4 * 4e5
    assert abs(S.sum() / (T.sum() + S.sum()) - 0.25) < 1e-3
    assert abs(R.sum() / tc - 0.25) < 1e-3
    assert abs(pp.g[0].sum() / tc - 1.0) < 0.01
    assert 2.5 < pp.fwhm_px < 3.0
