"""Pins of the banded-C oracle (Sec. III-C eq:ftcg, eq:cr, eq:dif3) against
facts fixed by the mathematics: the r = 1 reduction to the diagonal weights
of eq:difopt, the unconstrained optimum C = T^dagger of eq:dif3 (numpy's
pinv of the whole matrix), the normal equations of every column's least
squares problem, monotonicity of the residual in the band, and the
orientation of the apply c = C fhat. Planted mistakes at the end show that
each plausible slip fails one of them.
"""
import numpy as np
import pytest

import oracle as O
import oracle.band_ref as OB
from paper_1706_08575_amd import synth as S


def _raster_1d(m, seed):
    rng = np.random.default_rng(seed)
    return (np.arange(m) - m / 2 + rng.uniform(-0.25, 0.25, m)).reshape(m, 1)


def _raster_2d(seed):
    # a small polar SAS raster (raster order: pulse by pulse)
    return S.make_sas(seed, n=32, pulses=12, per_pulse=24)[0]


def _dense_T(k, R):
    d = k[:, None, :] - k[None, :, :]
    return np.prod(np.sinc(d), axis=2) * (np.max(np.abs(d), axis=2) <= R)


def test_r1_is_the_diagonal_optimum():
    for k in (_raster_1d(200, 1), _raster_2d(2)):
        B = O.band_columns(k, 1, 8.0)
        a = O.frame_weights(k, 8.0)
        assert B.shape == (len(k), 1)
        assert np.max(np.abs(B[:, 0] - a) / a) < 1e-12


def test_full_band_is_the_pseudo_inverse():
    # band covering every sample, no truncation: each column solves the
    # unrestricted problem, so C = T^dagger (eq:dif3); pinv is numpy's SVD
    # pseudo-inverse of the whole matrix, a different routine from the
    # per-column lstsq
    for k in (_raster_1d(40, 3), S.make_sas(4, n=16, pulses=5, per_pulse=8)[0]):
        m = len(k)
        B = O.band_columns(k, m, float("inf"))
        C = O.band_dense(B, m)
        P = np.linalg.pinv(_dense_T(k, np.inf))
        assert np.max(np.abs(C - P)) < 1e-9 * np.max(np.abs(P))


def test_columns_satisfy_normal_equations():
    # each column c of C on J(n) makes the residual T c - e_n orthogonal to
    # the columns T[:, J(n)] (optimality of the least-squares problem), and
    # is zero off J(n)
    for k, r in ((_raster_1d(120, 5), 4), (_raster_2d(6), 3)):
        m = len(k)
        T = _dense_T(k, 8.0)
        C = O.band_dense(O.band_columns(k, r, 8.0), r)
        for n in (0, 1, m // 2, m - 2, m - 1):
            J = np.arange(max(0, n - r + 1), min(m, n + r))
            res = T @ C[:, n] - np.eye(m)[:, n]
            assert np.max(np.abs(T[:, J].T @ res)) < 1e-10
            off = np.setdiff1d(np.arange(m), J)
            assert np.all(C[off, n] == 0)


def test_residual_decreases_with_band():
    # a wider band is a larger feasible set: ||T C_r - I||_F cannot grow
    k = _raster_2d(7)
    T = _dense_T(k, 8.0)
    prev = np.inf
    for r in (1, 2, 3, 5, 8):
        C = O.band_dense(O.band_columns(k, r, 8.0), r)
        res = np.linalg.norm(T @ C - np.eye(len(k)))
        assert res <= prev * (1 + 1e-12)
        prev = res
    # and strictly better than the diagonal weights for a jittered raster
    C1 = O.band_dense(O.band_columns(k, 1, 8.0), 1)
    assert prev < 0.9 * np.linalg.norm(T @ C1 - np.eye(len(k)))


def test_apply_orientation():
    # c = C fhat: a unit sample at n yields column n of C (support J(n));
    # the row of C would be a different vector for a non-symmetric C
    k = _raster_1d(60, 9)
    r = 3
    B = O.band_columns(k, r, 8.0)
    C = O.band_dense(B, r)
    assert np.max(np.abs(C - C.T)) > 1e-6          # the band solution is not symmetric
    for n in (0, 7, 59):
        e = np.zeros(60, dtype=np.complex128)
        e[n] = 1.0
        c = O.band_apply(B, e, r)
        assert np.max(np.abs(c - C[:, n])) < 1e-15
    f = S.random_values(10, 60)
    assert np.max(np.abs(O.band_apply(B, f, r) - C @ f)) < 1e-13


# ---------------------------------------------------------------------------
# planted mistakes
# ---------------------------------------------------------------------------

_good_cols = OB.band_columns
_good_apply = OB.band_apply
_good_gram = OB._gram


def _cols_shifted(k, r, R=8.0, cols=None):
    B = _good_cols(k, r, R, cols)
    return np.roll(B, 1, axis=1)                    # band off by one


def _apply_transposed(B, fhat, r):
    C = OB.band_dense(B, r)
    return C.T @ np.asarray(fhat, dtype=np.complex128)


def _gram_untruncated(ki, kj, R):
    return _good_gram(ki, kj, np.inf)


PLANTS = {
    "band_off_by_one": ("band_columns", _cols_shifted),
    "apply_transposed": ("band_apply", _apply_transposed),
    "gram_not_truncated": ("_gram", _gram_untruncated),
}
PINS = [test_r1_is_the_diagonal_optimum, test_full_band_is_the_pseudo_inverse,
        test_columns_satisfy_normal_equations, test_residual_decreases_with_band, test_apply_orientation]


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_band_planted_mistake_is_caught(plant, monkeypatch):
    name, fn = PLANTS[plant]
    monkeypatch.setattr(OB, name, fn)
    monkeypatch.setattr(O, name, fn, raising=False)
    failed = []
    for pin in PINS:
        try:
            pin()
        except (AssertionError, ValueError, IndexError):
            failed.append(pin.__name__)
    assert failed, plant
