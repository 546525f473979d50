"""Launch plans (the autotuner): cnlos_tune measures the plane kernels'
candidate LDS row pads on a problem and keeps the fastest for its shape.  The
pads only move values within LDS, so every plan must give bitwise the same
reconstruction; the expected values are the library's own runs under the
default plan (no oracle is needed for that claim)."""
import itertools

import numpy as np
import pytest

from paper_2301_00406_amd import cnlos as C
from paper_2301_00406_amd import scenes
from tests.gpu_helpers import need_gpu, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _scene(n, m, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = scenes.density_mask(n, 0.4, rng)
    raw = np.abs(scenes.random_signed((n, n, m), seed)) * 5.0
    return mask, raw


def test_tune_measures_every_candidate_and_later_problems_use_the_plan():
    torch = need_gpu()
    n, m = 32, 128
    say(f"tune {n}x{n}x{m}")
    mask, raw = _scene(n, m, 3)
    cfg = C.default_config(nx=n, ny=n, nt=m, model=C.MODEL_DUAL, max_iters=4, init_iters=2)
    P = C.Problem(cfg, mask)
    assert P.plan() == {"conv_row_pad": 2, "solve_row_pad": 8, "tuned": False,
                        "conv_plane_us": [0.0] * 3, "solve_plane_us": [0.0] * 3}
    P.set_measurement(to_dev(torch, raw))
    pl = P.tune()
    assert pl["tuned"]
    assert all(t > 0 for t in pl["conv_plane_us"] + pl["solve_plane_us"])
    # the fastest candidate, unless it beats the default by 3 % or less
    for key, pads, default, us in (("conv_row_pad", [1, 2, 4], 2, pl["conv_plane_us"]),
                                   ("solve_row_pad", [2, 4, 8], 8, pl["solve_plane_us"])):
        best = pads[int(np.argmin(us))]
        exp = best if min(us) < 0.97 * us[pads.index(default)] else default
        assert pl[key] == exp, (key, pl)
    # the tuned problem still runs from the start with its measurement
    P.run()
    assert P.info()["iter"] == 6
    Q = C.Problem(cfg, mask)
    got = Q.plan()
    assert (got["conv_row_pad"], got["solve_row_pad"]) == (pl["conv_row_pad"], pl["solve_row_pad"])
    R = C.Problem(C.default_config(nx=n, ny=n, nt=2 * m, model=C.MODEL_OBJECT), mask)
    assert (R.plan()["conv_row_pad"], R.plan()["solve_row_pad"]) == (2, 8)
    with pytest.raises(C.CnlosError):
        Q.set_plan(3, 8)
    O = C.Problem(C.default_config(nx=n, ny=n, nt=m, model=C.MODEL_OPERATOR), mask)
    with pytest.raises(C.CnlosError) as e:
        O.tune()
    assert e.value.status == C.ESTATE
    for h in (P, Q, R, O):
        h.close()


@pytest.mark.parametrize("n,m", [(16, 64), (64, 32), (128, 16)])
def test_every_plan_gives_bitwise_the_same_reconstruction(n, m):
    torch = need_gpu()
    say(f"plans bitwise {n}x{n}x{m}")
    mask, raw = _scene(n, m, n + m)
    cfg = C.default_config(nx=n, ny=n, nt=m, model=C.MODEL_DUAL, max_iters=5, init_iters=3)
    P = C.Problem(cfg, mask)
    P.set_measurement(to_dev(torch, raw))
    P.run()
    ref = to_host(P.volume())
    ref_sig = to_host(P.signal())
    ref_log = P.log()
    for cp, sp in itertools.product((1, 2, 4), (2, 4, 8)):
        P.set_plan(cp, sp)
        P.reset()
        P.run()
        np.testing.assert_array_equal(to_host(P.volume()), ref, err_msg=str((cp, sp)))
        np.testing.assert_array_equal(to_host(P.signal()), ref_sig, err_msg=str((cp, sp)))
        np.testing.assert_array_equal(P.log(), ref_log, err_msg=str((cp, sp)))
    P.close()
