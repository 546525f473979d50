"""Pins of the oracle's forward model A = R_t^{-1} H R_z (Section 2, eq. (3)).

Each check ties the oracle to something other than itself: hand-derived
fixtures, the direct-summation form of the convolution, the adjoint identity,
and the physical arrival time fixed by the continuous model eq. (2).
"""
import math

import numpy as np
import pytest

from oracle import cnlos_oracle as O
from tests.conftest import load_golden_matrix


def test_resample_matrix_matches_hand_derivation():
    rows, _ = load_golden_matrix("resample_m4.txt")
    np.testing.assert_allclose(O.resample_matrix(4), np.array(rows), atol=1e-15)


@pytest.mark.parametrize("m", [4, 16, 128, 1024])
def test_resample_columns_sum_to_one_and_rows_are_contiguous(m):
    S = O.resample_matrix(m)
    np.testing.assert_allclose(S.sum(axis=0), np.ones(m), atol=1e-12)
    for q in range(m):
        nz = np.nonzero(S[q])[0]
        assert nz.size >= 1
        assert nz[-1] - nz[0] + 1 == nz.size
        assert nz.size <= math.ceil(math.sqrt(m)) + 1
    # every squared-distance bin is reached and total mass is m (sum of columns)
    assert abs(S.sum() - m) < 1e-9


def test_literal_falloff_weights_match_hand_values():
    rows, _ = load_golden_matrix("falloff_literal_m4.txt")
    np.testing.assert_allclose(O.falloff_weights(4, O.FALLOFF_LITERAL), np.array(rows[0]),
                               rtol=1e-15)
    np.testing.assert_array_equal(O.falloff_weights(4, O.FALLOFF_COMPENSATED), np.ones(4))


def test_kernel_offsets_unit_slope_fixture():
    rows, extra = load_golden_matrix("kernel_offsets_unit_slope.txt")
    n, m, bin_ps = 2, 4, 1000.0
    R = O.range_metres(m, bin_ps)
    wall = n * R / math.sqrt(m)
    dq, Z = O.kernel_offsets(n, n, m, wall, wall, bin_ps)
    np.testing.assert_array_equal(dq, np.array(rows, dtype=np.int64))
    assert Z == int(extra[0][0])


def test_kernel_unit_sum_and_evenness():
    op = O.make_operator(6, 4, 32, 1.0, 0.8, 32.0)
    # h has unit sum: Hhat at zero frequency is 1
    assert abs(op.Hhat[0, 0, 0] - 1.0) < 1e-12
    # h is even in dx and dy, so Hhat is even in kx and ky
    H = op.Hhat
    np.testing.assert_allclose(H, H[(-np.arange(12)) % 12][:, :, :], atol=1e-12)
    np.testing.assert_allclose(H, H[:, (-np.arange(8)) % 8, :], atol=1e-12)


@pytest.mark.parametrize("falloff", [O.FALLOFF_COMPENSATED, O.FALLOFF_LITERAL])
@pytest.mark.parametrize("shape,wall", [((4, 4, 16), (1.0, 1.0)), ((4, 2, 8), (0.6, 0.3)),
                                        ((3, 5, 16), (1.2, 2.0))])
def test_direct_summation_equals_fft_form(falloff, shape, wall):
    nx, ny, m = shape
    rng = np.random.default_rng(3)
    mask = (rng.random((nx, ny)) < 0.6).astype(np.uint8)
    op = O.make_operator(nx, ny, m, wall[0], wall[1], 32.0, falloff=falloff, mask=mask)
    u = rng.random(shape)
    for masked in (False, True):
        a = O.apply_A_direct(u, op, masked)
        b = O.apply_A(u, op, masked)
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)


@pytest.mark.parametrize("falloff", [O.FALLOFF_COMPENSATED, O.FALLOFF_LITERAL])
def test_adjoint_identity(falloff):
    nx, ny, m = 8, 8, 32
    rng = np.random.default_rng(7)
    mask = (rng.random((nx, ny)) < 0.5).astype(np.uint8)
    op = O.make_operator(nx, ny, m, 1.0, 1.0, 32.0, falloff=falloff, mask=mask)
    x = rng.standard_normal((nx, ny, m))
    y = rng.standard_normal((nx, ny, m))
    for masked in (False, True):
        lhs = float((O.apply_A(x, op, masked) * y).sum())
        rhs = float((x * O.apply_AT(y, op, masked)).sum())
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_adjoint_equals_explicit_transpose_tiny():
    nx, ny, m = 3, 3, 8
    op = O.make_operator(nx, ny, m, 0.5, 0.5, 64.0, falloff=O.FALLOFF_LITERAL,
                         mask=np.array([[1, 0, 1], [1, 1, 0], [0, 1, 1]]))
    V = nx * ny * m
    Amat = np.zeros((V, V))
    for c in range(V):
        e = np.zeros(V)
        e[c] = 1.0
        Amat[:, c] = O.apply_A_direct(e.reshape(nx, ny, m), op, masked=True).ravel()
    y = np.random.default_rng(0).standard_normal(V)
    np.testing.assert_allclose(O.apply_AT(y.reshape(nx, ny, m), op, masked=True).ravel(),
                               Amat.T @ y, atol=1e-10)


def test_point_scatterer_arrives_at_round_trip_time():
    """A single voxel at depth z0 shows up, at scan point (i, j), in the bin of
    the one-way distance sqrt(lateral^2 + z0^2) (eq. (2): delta(2d - tc))."""
    n, m, wall, bin_ps = 8, 64, 0.4, 32.0
    op = O.make_operator(n, n, m, wall, wall, bin_ps)
    R = O.range_metres(m, bin_ps)
    dx_m = wall / n
    bin_m = R / m
    i0, j0, k0 = 3, 5, 30
    u = np.zeros((n, n, m))
    u[i0, j0, k0] = 1.0
    tau = O.apply_A(u, op)
    z0 = (k0 + 0.5) * bin_m
    checked = 0
    for i in range(n):
        for j in range(n):
            d = math.sqrt(((i - i0) * dx_m) ** 2 + ((j - j0) * dx_m) ** 2 + z0 ** 2)
            expect = int(math.floor(d / bin_m))
            if expect >= m - 1:
                continue
            got = int(np.argmax(tau[i, j]))
            assert abs(got - expect) <= 1, (i, j, got, expect)
            checked += 1
    assert checked > n * n // 2


def test_operator_is_nonnegative_and_translation_invariant_laterally():
    n, m = 8, 32
    op = O.make_operator(n, n, m, 1.0, 1.0, 32.0)
    u = np.zeros((n, n, m))
    u[2, 2, 10] = 1.0
    a = O.apply_A(u, op)
    assert a.min() >= -1e-12
    u2 = np.zeros((n, n, m))
    u2[3, 4, 10] = 1.0
    b = O.apply_A(u2, op)
    # shifting the scatterer shifts the response (away from the borders)
    np.testing.assert_allclose(a[2, 2], b[3, 4], atol=1e-12)
    np.testing.assert_allclose(a[1, 3], b[2, 5], atol=1e-12)


def test_normalize_measurement():
    rng = np.random.default_rng(1)
    tau = rng.random((4, 4, 16))
    mask = np.zeros((4, 4), dtype=np.uint8)
    mask[1, 2] = mask[3, 0] = 1
    y, s = O.normalize_measurement(tau, mask, O.FALLOFF_COMPENSATED)
    assert abs(y.max() - 1.0) < 1e-15
    assert np.all(y[mask == 0] == 0)
    r3 = ((np.arange(16) + 0.5) / 16) ** 3
    np.testing.assert_allclose(y[1, 2] * s, tau[1, 2] * r3, rtol=1e-14)
    with pytest.raises(ValueError):
        O.normalize_measurement(tau, np.zeros((4, 4)), O.FALLOFF_COMPENSATED)
    bad = tau.copy()
    bad[1, 2, 3] = np.nan
    with pytest.raises(ValueError):
        O.normalize_measurement(bad, mask, O.FALLOFF_COMPENSATED)


def test_power_iteration_bounds_operator_norm():
    nx, ny, m = 4, 4, 8
    op = O.make_operator(nx, ny, m, 0.5, 0.5, 64.0,
                         mask=np.eye(4, dtype=np.uint8) + np.eye(4, k=1, dtype=np.uint8))
    V = nx * ny * m
    Amat = np.zeros((V, V))
    for c in range(V):
        e = np.zeros(V)
        e[c] = 1.0
        Amat[:, c] = O.apply_A(e.reshape(nx, ny, m), op, masked=True).ravel()
    smax2 = np.linalg.norm(Amat, 2) ** 2
    est = O.power_norm2(lambda x: O.apply_A(x, op, True), lambda y: O.apply_AT(y, op, True),
                        (nx, ny, m), 15)
    assert est <= smax2 * (1 + 1e-12)
    assert est >= 0.5 * smax2
    est200 = O.power_norm2(lambda x: O.apply_A(x, op, True), lambda y: O.apply_AT(y, op, True),
                           (nx, ny, m), 400)
    assert abs(est200 - smax2) <= 1e-3 * smax2


def test_sampled_column_helpers_match_full_operator():
    """The direct-summation column helpers used at sizes the FFT oracle cannot
    hold agree with the full operator on a small grid."""
    from tests.gpu_helpers import sampled_columns_A, sampled_columns_AT
    n, m, wall, bin_ps = 8, 32, 0.7, 32.0
    rng = np.random.default_rng(21)
    u = rng.random((n, n, m))
    y = rng.standard_normal((n, n, m))
    cols = [(0, 0), (7, 7), (3, 5), (6, 1)]
    for falloff in (O.FALLOFF_COMPENSATED, O.FALLOFF_LITERAL):
        op = O.make_operator(n, n, m, wall, wall, bin_ps, falloff)
        full = O.apply_A(u, op)
        fullT = O.apply_AT(y, op)
        a = sampled_columns_A(u, n, m, wall, wall, bin_ps, falloff, cols)
        b = sampled_columns_AT(y, n, m, wall, wall, bin_ps, falloff, cols)
        for c in cols:
            np.testing.assert_allclose(a[c], full[c], rtol=1e-11, atol=1e-12 * np.abs(full).max())
            np.testing.assert_allclose(b[c], fullT[c], rtol=1e-11, atol=1e-12 * np.abs(fullT).max())
