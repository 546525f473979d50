"""Pins of the oracle's non-confocal operator (Section 2's general model with
unit normals, the volumetric albedo weight 1/(d_i^2 d_d^2)), and of the
midpoint approximation used for the non-confocal experiment of Section 5.

The operator is a direct sum (no FFT form exists: it is not shift-invariant);
these tests tie it to the adjoint identity, to closed forms of single
scatterers, to Helmholtz reciprocity, to the confocal operator in the limit
where illumination and detection coincide, and to the geometric bounds that
make the midpoint approximation second order in the source-detector
separation."""
import math

import numpy as np
import pytest

from oracle import cnlos_oracle as O


def _geo(illum=(0.1, -0.2), n=4, m=32):
    return O.NonConfocalGeometry(n, m, 0.8, 64.0, illum)


@pytest.mark.parametrize("literal", [True, False])
def test_adjoint_identity(literal):
    g = _geo()
    rng = np.random.default_rng(1)
    u = rng.random((g.n, g.n, g.m))
    t = rng.standard_normal((g.n, g.n, g.m))
    a = float((O.apply_nonconfocal(u, g, literal) * t).sum())
    b = float((u * O.apply_nonconfocal_T(t, g, literal)).sum())
    assert abs(a - b) <= 1e-12 * abs(a)


def test_transpose_is_the_explicit_matrix_transpose():
    g = _geo(n=3, m=16)
    V = g.n * g.n * g.m
    M = np.zeros((V, V))
    for c in range(V):
        e = np.zeros(V)
        e[c] = 1.0
        M[:, c] = O.apply_nonconfocal(e.reshape(g.n, g.n, g.m), g).ravel()
    for r in range(0, V, 7):
        e = np.zeros(V)
        e[r] = 1.0
        np.testing.assert_allclose(O.apply_nonconfocal_T(e.reshape(g.n, g.n, g.m), g).ravel(),
                                   M[r], rtol=1e-13, atol=0.0)


def test_scatterer_under_a_coincident_source_and_detector():
    """Illumination at detector (i0, j0) and a voxel right below it at depth
    z_k: d_i = d_d = z_k, the path 2 z_k lands in bin floor(2 z_k / (c dt)) with
    weight 1 / z_k^4; every other bin of that column is empty."""
    n, m = 4, 32
    x = (np.arange(n) + 0.5) * 0.8 / n - 0.4
    i0, j0, k = 1, 2, 9
    g = O.NonConfocalGeometry(n, m, 0.8, 64.0, (x[i0], x[j0]))
    u = np.zeros((n, n, m))
    u[i0, j0, k] = 2.0
    tau = O.apply_nonconfocal(u, g)
    z = (k + 0.5) * O.range_metres(m, 64.0) / m
    b = int(math.floor(2 * z / (299792458.0 * 64e-12)))
    assert b == k                                  # depth bins and time bins share R / m
    col = tau[i0, j0]
    assert abs(col[b] - 2.0 / z ** 4) <= 1e-12 * col[b]
    assert np.count_nonzero(col) == 1


def test_reciprocity_of_source_and_detector():
    """Swapping the illuminated and the detecting wall point leaves the
    transient unchanged (the path length and the weight are symmetric)."""
    n, m = 4, 32
    x = (np.arange(n) + 0.5) * 0.8 / n - 0.4
    rng = np.random.default_rng(2)
    u = rng.random((n, n, m))
    a, b = (0, 3), (2, 1)
    ta = O.apply_nonconfocal(u, O.NonConfocalGeometry(n, m, 0.8, 64.0, (x[a[0]], x[a[1]])))
    tb = O.apply_nonconfocal(u, O.NonConfocalGeometry(n, m, 0.8, 64.0, (x[b[0]], x[b[1]])))
    np.testing.assert_allclose(ta[b], tb[a], rtol=1e-13)


def test_confocal_limit_matches_the_confocal_operator_arrival():
    """With the illumination on a detector point, that detector's column is a
    confocal measurement: a point scatterer arrives there in the bin where the
    confocal light-cone operator (eq. (3), literal falloff) puts its peak, to
    within one bin (the two discretize the cone differently)."""
    n, m = 8, 64
    W, dt = 0.4, 32.0          # every path below stays inside the 64-bin window
    x = (np.arange(n) + 0.5) * W / n - W / 2
    op = O.make_operator(n, n, m, W, W, dt, O.FALLOFF_LITERAL)
    for (i0, j0), (p, q, k) in (((2, 3), (5, 4, 30)), ((6, 1), (4, 3, 45)), ((4, 4), (4, 4, 20))):
        g = O.NonConfocalGeometry(n, m, W, dt, (x[i0], x[j0]))
        u = np.zeros((n, n, m))
        u[p, q, k] = 1.0
        nc = O.apply_nonconfocal(u, g)[i0, j0]
        conf = O.apply_A(u, op)[i0, j0]
        assert abs(int(np.argmax(nc)) - int(np.argmax(conf))) <= 1, ((i0, j0), (p, q, k))


def test_midpoint_approximation_bounds_the_arrival_bin():
    """For illumination x_i and detector x_d with midpoint x_m and half
    separation h, 2 d(x_m, x) <= d_i + d_d <= 2 sqrt(d(x_m, x)^2 + h^2): the
    midpoint approximation is exact at h = 0 and second order in h.  Every
    detector's arrival bin of a point scatterer lies in the bins of that
    interval."""
    n, m = 6, 64
    W, dt = 0.8, 32.0
    g = O.NonConfocalGeometry(n, m, W, dt, (0.13, -0.07))
    x = g.lateral()
    z = g.depth()
    cdt = g.bin_length()
    p, q, k = 3, 1, 40
    u = np.zeros((n, n, m))
    u[p, q, k] = 1.0
    tau = O.apply_nonconfocal(u, g)
    X = np.array([x[p], x[q], z[k]])
    for i in range(n):
        for j in range(n):
            xm = np.array([(g.illum[0] + x[i]) / 2, (g.illum[1] + x[j]) / 2, 0.0])
            h2 = ((x[i] - g.illum[0]) ** 2 + (x[j] - g.illum[1]) ** 2) / 4.0
            dm = float(np.linalg.norm(X - xm))
            lo = math.floor(2 * dm / cdt)
            hi = math.floor(2 * math.sqrt(dm * dm + h2) / cdt)
            nz = np.nonzero(tau[i, j])[0]
            if hi < m:                              # the whole interval is in the window
                assert nz.size == 1, (i, j)
            assert nz.size <= 1 and all(lo <= b <= hi for b in nz), (i, j, nz, lo, hi)


def test_midpoint_geometry_is_a_half_scale_grid():
    g = O.NonConfocalGeometry(8, 64, 0.8, 32.0, (0.2, -0.1))
    wall, centre = O.nonconfocal_midpoint_geometry(g)
    assert wall == 0.4 and centre == (0.1, -0.05)
    # the midpoints of the illumination point and the detector grid are the
    # n x n grid of that extent and centre
    xm = (g.illum[0] + g.lateral()) / 2
    np.testing.assert_allclose(xm, (np.arange(8) + 0.5) * wall / 8 - wall / 2 + centre[0],
                               atol=1e-15)
