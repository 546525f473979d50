"""GPU parity of the non-confocal operator (Section 2's general model with one
illumination point, by direct summation) and its transpose, through the C ABI,
against the FP64 oracle; and Section 5's midpoint route (non-confocal
transients reconstructed by the confocal solver) against the oracle doing the
same.

Both sides decide each path's time bin in FP64 with the same operations, so
the supports (which bins receive anything) must agree exactly.  The values
are FP64 sums stored as FP32: 1e-6 relative L2 and elementwise, well above
FP32 rounding (6e-8) and far below the error of one misplaced path."""
import math

import numpy as np
import pytest

from oracle import cnlos_oracle as O
from paper_2301_00406_amd import cnlos as C
from paper_2301_00406_amd import scenes
from tests.gpu_helpers import f32, max_rel, need_gpu, rel_l2, say, to_dev, to_host

pytestmark = pytest.mark.gpu
TOL = 1e-6

GEOMS = [
    # (n, m, wall, bin_ps, illumination): tiny, ragged bin counts (not multiples
    # of the 64-lane chunk), illumination off the grid and outside the wall
    (4, 32, 0.8, 64.0, (0.1, -0.2)),
    (6, 40, 0.6, 48.0, (0.0, 0.0)),
    (8, 100, 1.0, 32.0, (0.37, 0.05)),
    (11, 64, 0.5, 32.0, (-0.4, 0.3)),
    (12, 130, 0.9, 24.0, (0.6, -0.7)),
]


def _geoms(n, m, wall, dt, illum, literal):
    return (C.nc_geometry(n, m, wall, dt, illum, literal),
            O.NonConfocalGeometry(n, m, wall, dt, illum))


@pytest.mark.parametrize("literal", [True, False])
@pytest.mark.parametrize("geom", GEOMS)
def test_forward_and_transpose_match_the_oracle(geom, literal):
    torch = need_gpu()
    n, m, wall, dt, illum = geom
    say(f"nonconfocal parity n={n} m={m} literal={literal}")
    g, og = _geoms(n, m, wall, dt, illum, literal)
    u = f32(scenes.random_volume((n, n, m), 11 + n))
    t = f32(scenes.random_signed((n, n, m), 13 + m))
    tau = to_host(C.nc_apply(g, to_dev(torch, u)))
    ut = to_host(C.nc_apply_T(g, to_dev(torch, t)))
    torch.cuda.synchronize()
    ref_tau = O.apply_nonconfocal(u, og, literal)
    ref_ut = O.apply_nonconfocal_T(t, og, literal)
    # the same bins are reached (u > 0 everywhere: a bin is nonzero iff a path lands there)
    assert np.array_equal(tau != 0.0, ref_tau != 0.0)
    assert rel_l2(tau, ref_tau) <= TOL and max_rel(tau, ref_tau) <= TOL
    assert rel_l2(ut, ref_ut) <= TOL and max_rel(ut, ref_ut) <= TOL


def test_adjoint_identity_and_determinism_at_32x32x256():
    torch = need_gpu()
    n, m = 32, 256
    say("nonconfocal adjoint identity 32x32x256")
    g = C.nc_geometry(n, m, 1.0, 32.0, (0.2, 0.1), True)
    u = to_dev(torch, scenes.random_volume((n, n, m), 5))
    t = to_dev(torch, scenes.random_signed((n, n, m), 6))
    Au = C.nc_apply(g, u)
    Au2 = C.nc_apply(g, u)
    Atr = C.nc_apply_T(g, t)
    Atr2 = C.nc_apply_T(g, t)
    torch.cuda.synchronize()
    assert torch.equal(Au, Au2) and torch.equal(Atr, Atr2)
    # t is signed, so the inner products cancel: the FP32 rounding of the
    # stored outputs is measured against the sums of the terms' magnitudes
    pa, pb = to_host(Au) * to_host(t), to_host(u) * to_host(Atr)
    a, b = float(pa.sum()), float(pb.sum())
    scale = max(float(np.abs(pa).sum()), float(np.abs(pb).sum()))
    assert abs(a - b) <= 1e-6 * scale


def test_point_scatterers_at_64x64x512():
    """At the size the oracle cannot sum, single scatterers have a closed form:
    every detector's transient holds one value 1/(d_i^2 d_d^2) in the bin of
    d_i + d_d (when inside the window), nothing elsewhere."""
    torch = need_gpu()
    n, m, wall, dt = 64, 512, 0.7, 16.0
    illum = (0.05, -0.1)
    say("nonconfocal point scatterers 64x64x512")
    g = C.nc_geometry(n, m, wall, dt, illum, True)
    x = (np.arange(n) + 0.5) * wall / n - wall / 2.0
    R = m * 299792458.0 * (dt * 1e-12) / 2.0
    cdt = 299792458.0 * dt * 1e-12
    for (p, q, k) in ((3, 60, 100), (32, 31, 7), (50, 10, 400)):
        u = np.zeros((n, n, m), np.float32)
        u[p, q, k] = 1.0
        tau = to_host(C.nc_apply(g, to_dev(torch, u)))
        # the operations of the definition, in its order (products, no powers)
        z = (k + 0.5) * R / m
        ex, ey = x[p] - illum[0], x[q] - illum[1]
        di = math.sqrt((ex * ex + ey * ey) + z * z)
        fx, fy = x[p] - x[:, None], x[q] - x[None, :]
        dd = np.sqrt((fx * fx + fy * fy) + z * z)
        b = np.floor((di + dd) / cdt).astype(np.int64)
        w = 1.0 / (di * di * dd * dd)
        exp = np.zeros((n, n, m))
        I, J = np.nonzero(b < m)
        exp[I, J, b[I, J]] = w[I, J]
        assert np.array_equal(tau != 0.0, exp != 0.0), (p, q, k)
        assert max_rel(tau, exp) <= TOL, (p, q, k)


def test_midpoint_route_matches_the_oracle():
    """Section 5's non-confocal experiment: transients of one illumination
    point, read at the midpoints as confocal data (wall extent W/2) and
    reconstructed by Algorithm 1.  Each side builds its own measurement from
    the same scene with its own non-confocal operator."""
    torch = need_gpu()
    n, m, W, dt = 8, 64, 0.8, 64.0
    illum = (0.1, -0.05)
    say("nonconfocal midpoint route 8x8x64, Algorithm 1, 20 iterations")
    rng = np.random.Generator(np.random.PCG64(77))
    u_true = np.zeros((n, n, m))
    scenes.add_planar_rect(u_true, rng, size_lo=2, size_hi=4)
    g, og = _geoms(n, m, W, dt, illum, True)
    wall, _ = C.nc_midpoint(g)
    mask = np.ones((n, n), np.uint8)
    raw_ref = O.apply_nonconfocal(u_true, og, True)
    raw_ref = raw_ref / raw_ref.max()
    raw_dev = C.nc_apply(g, to_dev(torch, u_true))
    raw_dev = raw_dev / raw_dev.max()
    op = O.make_operator(n, n, m, wall, wall, dt, mask=mask)
    tau0, _ = O.normalize_measurement(f32(raw_ref), mask, O.FALLOFF_COMPENSATED)
    L0 = 2.0 * O.power_norm2(lambda v: O.apply_A(v, op, True), lambda y: O.apply_AT(y, op, True),
                             tau0.shape)
    prm = O.Params(a=5e-5, b=5e-5, mu=0.1)
    iters = 20
    ref = O.run_alg1(tau0, op, prm, iters, L0=L0)
    cfg = C.default_config(nx=n, ny=n, nt=m, wall_w_m=wall, wall_h_m=wall, bin_ps=dt,
                           model=C.MODEL_OBJECT, max_iters=iters, L0=L0, a_u=5e-5, b_u=5e-5, mu=0.1)
    P = C.Problem(cfg, mask)
    P.set_measurement(raw_dev.contiguous())
    P.run()
    got = to_host(P.volume())
    P.close()
    assert rel_l2(got, ref.u) <= 1e-3
