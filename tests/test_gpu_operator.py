"""GPU parity of the light-cone-transform operator A = R_t^{-1} H R_z (eq. (3))
and its adjoint, through the C ABI, against the FP64 oracle.

Tolerance: 1e-5 relative L2 per operator application.  FP32 FFT round-off
grows like eps32 * log2(P) ~ 1e-6 for the largest padded grid, so 1e-5 leaves a
margin of ten while still catching any indexing or scaling mistake (those
give O(1) errors)."""
import numpy as np
import pytest

from oracle import cnlos_oracle as O
from paper_2301_00406_amd import cnlos as C
from paper_2301_00406_amd import scenes
from tests.gpu_helpers import (f32, need_gpu, rel_l2, sampled_columns_A, sampled_columns_AT,
                               say, to_dev, to_host)

pytestmark = pytest.mark.gpu
TOL_OP = 1e-5

SHAPES = [
    # (n, m, wall, bin_ps): tiny, the 16x16x128 workload, odd aspect ratios
    (8, 16, 0.5, 64.0),
    (16, 128, 1.0, 32.0),
    (32, 64, 0.6, 32.0),
    (8, 256, 0.3, 16.0),
    (16, 2048, 1.0, 8.0),
    (128, 32, 2.0, 64.0),     # the n = 128 plane kernel (split by ky parity), full volume
]


def _mask(n, seed, frac=0.5):
    rng = np.random.Generator(np.random.PCG64(seed))
    return scenes.density_mask(n, frac, rng)


def _op_problem(n, m, wall, bin_ps, falloff, mask):
    cfg = C.default_config(nx=n, ny=n, nt=m, wall_w_m=wall, wall_h_m=wall, bin_ps=bin_ps,
                           falloff=falloff, model=C.MODEL_OPERATOR)
    return C.Problem(cfg, mask)


@pytest.mark.parametrize("falloff", [C.FALLOFF_COMPENSATED, C.FALLOFF_LITERAL])
@pytest.mark.parametrize("shape", SHAPES)
def test_apply_A_and_AT_match_oracle(shape, falloff):
    torch = need_gpu()
    n, m, wall, bin_ps = shape
    say(f"operator parity n={n} m={m} falloff={falloff}")
    mask = _mask(n, 7 + n + m)
    P = _op_problem(n, m, wall, bin_ps, falloff, mask)
    op = O.make_operator(n, n, m, wall, wall, bin_ps, falloff, mask)
    u = f32(scenes.random_volume((n, n, m), seed=n * 1000 + m))
    y = f32(scenes.random_signed((n, n, m), seed=n * 1000 + m + 1))
    ud, yd = to_dev(torch, u), to_dev(torch, y)
    for masked in (False, True):
        got = to_host(P.apply_A(ud, masked))
        assert rel_l2(got, O.apply_A(u, op, masked)) <= TOL_OP
        got = to_host(P.apply_AT(yd, masked))
        assert rel_l2(got, O.apply_AT(y, op, masked)) <= TOL_OP
    P.close()


def test_adjoint_identity_on_gpu():
    torch = need_gpu()
    n, m = 32, 256
    mask = _mask(n, 3)
    P = _op_problem(n, m, 0.8, 16.0, C.FALLOFF_COMPENSATED, mask)
    x = to_dev(torch, scenes.random_signed((n, n, m), 11))
    y = to_dev(torch, scenes.random_signed((n, n, m), 12))
    for masked in (False, True):
        ax = P.apply_A(x, masked).double()
        aty = P.apply_AT(y, masked).double()
        lhs = float((ax * y.double()).sum())
        rhs = float((x.double() * aty).sum())
        assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), 1e-30)


def test_point_scatterer_on_gpu_matches_oracle_and_physics():
    torch = need_gpu()
    n, m, wall, bin_ps = 16, 128, 1.0, 32.0
    mask = np.ones((n, n), np.uint8)
    P = _op_problem(n, m, wall, bin_ps, C.FALLOFF_COMPENSATED, mask)
    u = np.zeros((n, n, m))
    u[5, 9, 70] = 1.0
    got = to_host(P.apply_A(to_dev(torch, u)))
    op = O.make_operator(n, n, m, wall, wall, bin_ps)
    assert rel_l2(got, O.apply_A(u, op)) <= TOL_OP
    # arrival bin of the one-way distance sqrt(lateral^2 + z0^2)
    R = O.range_metres(m, bin_ps)
    z0 = 70.5 * R / m
    d = np.sqrt(((7 - 5) * wall / n) ** 2 + ((12 - 9) * wall / n) ** 2 + z0 ** 2)
    assert abs(int(np.argmax(got[7, 12])) - int(d / (R / m))) <= 1


def test_medium_workload_operator_full_size():
    """64x64x512 (padded FFT 128x128x1024): full-volume parity on the scene
    (compensated falloff) and on a dense volume (both falloffs).  The literal
    weight rhat^-3 reaches (2m)^3 ~ 1e9 in the first bins, so on a sparse scene
    with empty near-wall bins it amplifies FP32 round-off of the convolution
    far above the signal there; literal parity is checked on dense input."""
    torch = need_gpu()
    sc = scenes.scene_medium()
    say("operator parity 64x64x512")
    cases = [(C.FALLOFF_COMPENSATED, f32(sc.u_true)),
             (C.FALLOFF_COMPENSATED, f32(scenes.random_volume(sc.shape, 77))),
             (C.FALLOFF_LITERAL, f32(scenes.random_volume(sc.shape, 78)))]
    for falloff, u in cases:
        P = _op_problem(sc.n, sc.m, sc.wall_w, sc.bin_ps, falloff, sc.mask)
        op = O.make_operator(sc.n, sc.n, sc.m, sc.wall_w, sc.wall_h, sc.bin_ps, falloff, sc.mask)
        got = to_host(P.apply_A(to_dev(torch, u), masked=True))
        ref = O.apply_A(u, op, masked=True)
        assert rel_l2(got, ref) <= TOL_OP, falloff
        y = f32(ref / np.abs(ref).max())
        got2 = to_host(P.apply_AT(to_dev(torch, y), masked=True))
        assert rel_l2(got2, O.apply_AT(y, op, masked=True)) <= TOL_OP, falloff
        P.close()


def test_large_workload_operator_sampled_columns():
    """128x128x1024 (padded FFT 256x256x2048): sampled scan columns computed one
    by one by direct summation."""
    torch = need_gpu()
    n, m, wall, bin_ps = 128, 1024, 2.0, 16.0
    say("operator parity 128x128x1024 (sampled)")
    rng = np.random.Generator(np.random.PCG64(5))
    mask = np.ones((n, n), np.uint8)
    P = _op_problem(n, m, wall, bin_ps, C.FALLOFF_COMPENSATED, mask)
    u = f32(rng.random((n, n, m)))
    cols = [(0, 0), (127, 127), (64, 3), (17, 100), (90, 45), (127, 0)]
    got = to_host(P.apply_A(to_dev(torch, u)))
    ref = sampled_columns_A(u, n, m, wall, wall, bin_ps, O.FALLOFF_COMPENSATED, cols)
    for c in cols:
        assert rel_l2(got[c], ref[c]) <= TOL_OP, c
    y = f32(rng.standard_normal((n, n, m)))
    got = to_host(P.apply_AT(to_dev(torch, y)))
    ref = sampled_columns_AT(y, n, m, wall, wall, bin_ps, O.FALLOFF_COMPENSATED, cols)
    for c in cols:
        assert rel_l2(got[c], ref[c]) <= TOL_OP, c
