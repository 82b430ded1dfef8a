"""Pins of the synthetic input generator (system matrix, phantoms, data).

The system matrix is input data for both the GPU library and the oracle, so it
is pinned against geometry that does not depend on the Siddon builder.
"""
import math

import numpy as np
import pytest

from paper_2409_13344_amd import synth


def _dense(A):
    M = np.zeros((A.n_rows, A.n_cols))
    for i in range(A.n_rows):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            M[i, A.col[k]] += A.val[k]
    return M


@pytest.mark.parametrize("geom", [synth.Geometry(8, 12, 16), synth.Geometry(7, 11, 10),
                                  synth.Geometry(64, 96, 90)])
def test_row_sums_are_chord_lengths(geom):
    """Sum of a row = length of the ray inside the square (independent edge intersection)."""
    A = synth.siddon_matrix(geom)
    sums = np.add.reduceat(np.append(A.val, 0.0), A.row_ptr[:-1])
    sums[np.diff(A.row_ptr) == 0] = 0.0
    half = geom.n / 2.0
    for a in range(geom.n_angles):
        phi = a * math.pi / geom.n_angles
        for b in range(geom.n_bins):
            s = (b - (geom.n_bins - 1) / 2.0) * geom.ds
            ref = synth.chord_length_square(phi, s, half)
            assert abs(sums[a * geom.n_bins + b] - ref) <= 1e-9 * max(1.0, ref)


def test_matrix_structure():
    geom = synth.Geometry(64, 96, 90)
    A = synth.siddon_matrix(geom)
    assert A.row_ptr[0] == 0 and np.all(np.diff(A.row_ptr) >= 0)
    assert A.col.min() >= 0 and A.col.max() < geom.d
    assert np.all(A.val > 0)
    for i in range(0, A.n_rows, 97):
        cols = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert len(np.unique(cols)) == len(cols)
        assert len(cols) <= 2 * geom.n - 1
    # every pixel lies on the path of at least one ray per angle on average: column sums ~ NPA
    colsum = np.zeros(geom.d)
    np.add.at(colsum, A.col, A.val)
    assert abs(colsum.mean() - geom.n_angles) < 0.05 * geom.n_angles


@pytest.mark.parametrize("geom", [synth.Geometry(8, 12, 16), synth.Geometry(16, 22, 24)])
def test_quarter_turn_symmetry(geom):
    """Ray (phi + pi/2, s) is ray (phi, s) turned by 90 degrees: (x, y) -> (-y, x),
    i.e. pixel (r, c) -> (c, N-1-r)."""
    A = _dense(synth.siddon_matrix(geom))
    n, R, NA = geom.n, geom.n_bins, geom.n_angles
    r, c = np.divmod(np.arange(n * n), n)
    rot = c * n + (n - 1 - r)
    for a in range(NA // 2):
        for b in range(R):
            row = A[a * R + b]
            row2 = A[(a + NA // 2) * R + b]
            np.testing.assert_allclose(row2[rot], row, atol=1e-9)


def test_problem_scaling_and_reproducibility():
    geom = synth.Geometry(16, 22, 24)
    p1 = synth.make_problem(geom, [5, 6], tc=5e4, rf=0.1)
    p2 = synth.make_problem(geom, [5, 6], tc=5e4, rf=0.1)
    np.testing.assert_array_equal(p1.g, p2.g)
    assert np.all(p1.g == np.round(p1.g))
    colsum = np.zeros(geom.d)
    np.add.at(colsum, p1.A.col, p1.A.val)
    for k in range(2):
        # sum(A f_true) = (1 - rf) TC and sum(gamma) = rf TC
        assert abs(colsum @ p1.f_true[k] - 0.9 * 5e4) < 1e-6 * 5e4
        assert abs(p1.gamma[k].astype(np.float64).sum() - 0.1 * 5e4) < 1e-4 * 5e4
        # phantom support inside the field-of-view disk
        xs = np.arange(16) - 7.5
        X, Y = np.meshgrid(xs, xs)
        assert np.all(p1.f_true[k].reshape(16, 16)[X ** 2 + Y ** 2 > 64.0] == 0.0)
    assert not np.array_equal(p1.g[0], p1.g[1])


def test_ranges_per_seed():
    geom = synth.Geometry(16, 22, 24)
    p = synth.make_problem(geom, list(range(10)), tc_range=(1e5, 1e7), rf_range=(0.05, 0.2))
    assert np.all((p.tc >= 1e5) & (p.tc <= 1e7)) and np.all((p.rf >= 0.05) & (p.rf <= 0.2))
    assert len(np.unique(p.tc)) == 10


def test_disc_phantom_inside_fov_and_scaled():
    geom = synth.Geometry(32, 48, 30)
    pr = synth.make_problem(geom, [7, 8], tc=1e5, rf=0.1, phantom="disc")
    for k in range(2):
        f = pr.f_true[k].reshape(32, 32)
        vals = np.unique(f[f > 0])
        assert len(vals) == 1                      # uniform activity
        r, c = np.nonzero(f > 0)
        ctr = 15.5
        assert np.max(np.hypot(r - ctr, c - ctr)) <= 16.0   # inside the FOV disc
        assert 0.2 < (f > 0).mean() < 0.7
    with pytest.raises(ValueError):
        synth.make_problem(geom, [7], phantom="square")
