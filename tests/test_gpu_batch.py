"""Batches through the C ABI: several scenes advanced by one launch per kernel
(launch grid z = scene).  A batch changes where each reconstruction runs, not
what it computes, and every reduction is in a fixed order, so each member's
result must equal the same scene run alone bit for bit; the alone runs are
tied to the FP64 oracle by the single-scene parity tests, and one member is
also checked against the oracle directly here."""
import numpy as np
import pytest

from oracle import cnlos_oracle as O
from paper_2301_00406_amd import cnlos as C
from paper_2301_00406_amd import scenes
from tests.gpu_helpers import f32, need_gpu, rel_l2, say, synth_measurement, to_dev, to_host

pytestmark = pytest.mark.gpu

OBJ = dict(a_u=5e-5, b_u=5e-5, mu=0.1)
DUAL = dict(a_u=5e-4, b_u=5e-5, a_tau=3e-3, b_tau=5e-4, warm_a=1.5e-4, warm_b=4e-5, mu=0.1,
            lam=200.0)


def _scene(n, m, seed, wall=1.0, bin_ps=32.0, density=0.5):
    sc = scenes.scene_custom(n, m, seed, wall=wall, bin_ps=bin_ps, density=density)
    return sc, synth_measurement(sc, seed + 7)


def _cfg(sc, model, params, **kw):
    return C.default_config(nx=sc.n, ny=sc.n, nt=sc.m, wall_w_m=sc.wall_w, wall_h_m=sc.wall_h,
                            bin_ps=sc.bin_ps, model=model, **params, **kw)


def _alone(torch, sc, raw, cfg):
    P = C.Problem(cfg, sc.mask)
    P.set_measurement(to_dev(torch, raw))
    rep = P.run()
    out = (P.volume().cpu().numpy(), P.log(), rep)
    if cfg.model == C.MODEL_DUAL:
        out = out + (P.signal().cpu().numpy(),)
    P.close()
    return out


def _check_members(torch, B, items, cfgs):
    for i, (sc, raw) in enumerate(items):
        alone = _alone(torch, sc, raw, cfgs[i])
        m = B.members[i]
        u = m.volume().cpu().numpy()
        assert np.array_equal(u, alone[0]), f"member {i}: volume differs from the alone run"
        assert np.array_equal(m.log(), alone[1]), f"member {i}: energy log differs"
        if cfgs[i].model == C.MODEL_DUAL:
            assert np.array_equal(m.signal().cpu().numpy(), alone[3]), f"member {i}: tau differs"


def test_object_batch_equals_alone_runs_bitwise():
    torch = need_gpu()
    say("batch: 3 object-model scenes 16x16x128, uneven iteration budgets")
    items = [_scene(16, 128, 500 + i, density=0.3 + 0.2 * i) for i in range(3)]
    cfgs = [_cfg(sc, C.MODEL_OBJECT, OBJ, max_iters=it) for (sc, _), it in zip(items, (20, 31, 26))]
    B = C.Batch(cfgs, [sc.mask for sc, _ in items])
    for m, (_, raw) in zip(B.members, items):
        m.set_measurement(to_dev(torch, raw))
    st, reps = B.run()
    assert st == C.OK
    assert [r["iters_done"] for r in reps] == [20, 31, 26]
    _check_members(torch, B, items, cfgs)
    # one member against the oracle directly
    sc, raw = items[1]
    op = O.make_operator(sc.n, sc.n, sc.m, sc.wall_w, sc.wall_h, sc.bin_ps, mask=sc.mask)
    tau0, _ = O.normalize_measurement(f32(raw), sc.mask, O.FALLOFF_COMPENSATED)
    L0 = B.members[1].info()["L0_obj"]
    ref = O.run_alg1(tau0, op, O.Params(a=5e-5, b=5e-5, mu=0.1), 31, L0=L0)
    assert rel_l2(to_host(B.members[1].volume()), ref.u) <= 1e-3
    B.close()


def test_dual_batch_with_rejections_equals_alone_runs_bitwise():
    """Small L0 forces backtracking rejections at different iterations per
    scene, so members sit at different iteration counts (and stages) inside
    the same launches; per-scene warm-start lengths differ too."""
    torch = need_gpu()
    say("batch: 3 dual-model scenes 32x32x256 with forced rejections")
    items = [_scene(32, 256, 600 + i, wall=0.8, bin_ps=24.0 + 4 * i, density=0.25 + 0.1 * i)
             for i in range(3)]
    cfgs = [_cfg(sc, C.MODEL_DUAL, DUAL, init_iters=ii, max_iters=mi, L0=l0, L0_dual=ld)
            for (sc, _), ii, mi, l0, ld in zip(items, (4, 6, 5), (8, 6, 9), (1e-3, 0.0, 2e-3),
                                               (0.0, 1e-2, 0.0))]
    B = C.Batch(cfgs, [sc.mask for sc, _ in items])
    for m, (_, raw) in zip(B.members, items):
        m.set_measurement(to_dev(torch, raw))
    st, reps = B.run()
    assert st == C.OK, C.last_error()
    assert [r["iters_done"] for r in reps] == [12, 12, 14]
    assert sum(r["bt_rejects"] for r in reps) > 0
    _check_members(torch, B, items, cfgs)
    B.close()


def test_run_many_overlapping_batches_of_different_shapes():
    torch = need_gpu()
    say("run_many: a 16x16x128 object batch and a 32x32x256 dual batch on two streams")
    s1 = torch.cuda.Stream()
    s2 = torch.cuda.Stream()
    it1 = [_scene(16, 128, 700 + i) for i in range(2)]
    it2 = [_scene(32, 256, 800 + i, wall=0.8, bin_ps=24.0) for i in range(2)]
    c1 = [_cfg(sc, C.MODEL_OBJECT, OBJ, max_iters=15) for sc, _ in it1]
    c2 = [_cfg(sc, C.MODEL_DUAL, DUAL, init_iters=3, max_iters=5) for sc, _ in it2]
    B1 = C.Batch(c1, [sc.mask for sc, _ in it1], stream=s1)
    B2 = C.Batch(c2, [sc.mask for sc, _ in it2], stream=s2)
    for B, items, s in ((B1, it1, s1), (B2, it2, s2)):
        with torch.cuda.stream(s):
            for m, (_, raw) in zip(B.members, items):
                m.set_measurement(to_dev(torch, raw))
        s.synchronize()
    st, reps = C.run_many([B1, B2])
    assert st == C.OK
    assert [r["iters_done"] for r in reps[0]] == [15, 15]
    assert [r["iters_done"] for r in reps[1]] == [8, 8]
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        _check_members(torch, B1, it1, c1)
    with torch.cuda.stream(s2):
        _check_members(torch, B2, it2, c2)
    B1.close()
    B2.close()


def test_batch_member_failure_does_not_stop_the_others():
    torch = need_gpu()
    say("batch: one member exhausts backtracking, the other finishes")
    items = [_scene(16, 128, 900 + i) for i in range(2)]
    cfgs = [_cfg(items[0][0], C.MODEL_OBJECT, OBJ, max_iters=10, L0=1e-9, bt_max_trials=0),
            _cfg(items[1][0], C.MODEL_OBJECT, OBJ, max_iters=10)]
    B = C.Batch(cfgs, [sc.mask for sc, _ in items])
    for m, (_, raw) in zip(B.members, items):
        m.set_measurement(to_dev(torch, raw))
    st, reps = B.run()
    assert st == C.EBACKTRACK
    assert reps[0]["status"] == C.EBACKTRACK and reps[1]["status"] == C.OK
    assert reps[1]["iters_done"] == 10
    alone = _alone(torch, *items[1], cfgs[1])
    assert np.array_equal(B.members[1].volume().cpu().numpy(), alone[0])
    B.close()
