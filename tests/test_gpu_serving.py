"""Serving with continuous batching through the C ABI: requests of mixed
shapes arrive while others run, are admitted into slot groups as slots and
arena memory free up, and each result must equal the same request run alone
bit for bit (one launch serves every slot of a group; reductions are in a
fixed order per scene)."""
import numpy as np
import pytest

from paper_2301_00406_amd import cnlos as C
from paper_2301_00406_amd import scenes
from tests.gpu_helpers import need_gpu, say, synth_measurement, to_dev

pytestmark = pytest.mark.gpu

OBJ = dict(a_u=5e-5, b_u=5e-5, mu=0.1)
DUAL = dict(a_u=5e-4, b_u=5e-5, a_tau=3e-3, b_tau=5e-4, warm_a=1.5e-4, warm_b=4e-5, mu=0.1,
            lam=200.0)


def _requests(torch):
    """Uneven requests: three shapes, both models, per-request masks, noise
    levels and iteration budgets."""
    out = []
    shapes = [(16, 128, "object"), (32, 256, "dual"), (16, 256, "object"), (32, 256, "dual"),
              (16, 128, "object"), (16, 256, "object"), (32, 256, "dual"), (16, 128, "object")]
    for i, (n, m, model) in enumerate(shapes):
        sc = scenes.scene_custom(n, m, 3000 + i, wall=1.0, bin_ps=32.0 * 128 / m,
                                 density=0.2 + 0.05 * i, peak=5.0 + 5 * i)
        raw = synth_measurement(sc, 3100 + i)
        if model == "dual":
            cfg = C.default_config(nx=n, ny=n, nt=m, wall_w_m=1.0, wall_h_m=1.0, bin_ps=sc.bin_ps,
                                   model=C.MODEL_DUAL, init_iters=3 + i % 3, max_iters=6 + i,
                                   **DUAL)
        else:
            cfg = C.default_config(nx=n, ny=n, nt=m, wall_w_m=1.0, wall_h_m=1.0, bin_ps=sc.bin_ps,
                                   model=C.MODEL_OBJECT, max_iters=12 + 2 * i, **OBJ)
        out.append((cfg, sc.mask, to_dev(torch, raw)))
    return out


def _hq_bytes(cfg):
    """One lane-ordered H^: every kt plane's full 2n x 2n spectrum, complex64,
    in a 256-byte aligned block."""
    b = (cfg.nt + 1) * 4 * cfg.nx * cfg.nx * 8
    return (b + 255) // 256 * 256


def _group_bytes(cfg, slots):
    """Arena bytes of a slot group: one H^ for the group's geometry, and slots
    whose workspaces hold everything else."""
    return slots * (C.workspace_bytes(cfg) - _hq_bytes(cfg)) + _hq_bytes(cfg)


def _alone(torch, cfg, mask, raw):
    P = C.Problem(cfg, mask)
    P.set_measurement(raw)
    P.run()
    u = P.volume().cpu().numpy()
    P.close()
    return u


def _serve(torch, reqs, arena_bytes, slots, rounds, arrivals):
    """arrivals[i]: the step before which request i is submitted."""
    S = C.Server(arena_bytes, slots=slots, rounds=rounds)
    outs = [torch.zeros(tuple(r[2].shape), dtype=torch.float32, device="cuda") for r in reqs]
    done = {}
    step = 0
    max_groups = 0
    while len(done) < len(reqs):
        for i, a in enumerate(arrivals):
            if a == step:
                cfg, mask, raw = reqs[i]
                S.submit(cfg, mask, raw, outs[i], i)
        S.step()
        max_groups = max(max_groups, S.usage()[1])
        for c in S.poll():
            done[c["id"]] = c
        step += 1
        assert step < 2000, "serving loop did not drain"
    S.close()
    return outs, done, max_groups


def test_served_results_equal_alone_runs_bitwise():
    torch = need_gpu()
    say("serving: 8 requests, 3 shapes, staggered arrivals, 2 slots per group")
    reqs = _requests(torch)
    arrivals = [0, 0, 1, 2, 2, 4, 6, 7]
    outs, done, groups = _serve(torch, reqs, 4 << 30, slots=2, rounds=3, arrivals=arrivals)
    assert groups >= 2
    for i, (cfg, mask, raw) in enumerate(reqs):
        c = done[i]
        assert c["status"] == C.OK, (i, c)
        planned = cfg.max_iters + (cfg.init_iters if cfg.model == C.MODEL_DUAL else 0)
        assert c["iters"] == planned
        ref = _alone(torch, cfg, mask, raw)
        assert np.array_equal(outs[i].cpu().numpy(), ref), f"request {i} differs from its alone run"


def test_admission_waits_for_arena_memory():
    """An arena that holds one slot group of the largest shape and nothing
    beside it: requests of other shapes wait in the queue until that group
    drains, then run."""
    torch = need_gpu()
    say("serving: arena for one large group at a time")
    r = _requests(torch)
    reqs = [r[1], r[0], r[2]]            # 32x256 dual first, then 16x128 and 16x256 object
    # room for the slot group of the large shape and nothing beside it
    arena = _group_bytes(reqs[0][0], 2) + (1 << 20)
    assert all(_group_bytes(q[0], 2) > (1 << 20) for q in reqs[1:])
    outs, done, groups = _serve(torch, reqs, arena, slots=2, rounds=4, arrivals=[0, 0, 0])
    for i, (cfg, mask, raw) in enumerate(reqs):
        assert done[i]["status"] == C.OK
        assert np.array_equal(outs[i].cpu().numpy(), _alone(torch, cfg, mask, raw))
    # the small requests were admitted only once the large group had drained
    for i in (1, 2):
        assert done[i]["queued_steps"] >= done[0]["served_steps"]


def test_group_creation_failure_gives_exactly_one_completion_per_request():
    """A slot group that cannot be created (failure injected by the library's
    test hook after its arena range and stream exist): the request that needed
    it completes once with the error, its arena range comes back, and every
    other request, queued before or after it, completes once and equals its
    alone run."""
    torch = need_gpu()
    say("serving: injected slot-group creation failure")
    r = _requests(torch)
    reqs = [r[0], r[1], r[2], r[4]]      # 16x128 object, 32x256 dual, 16x256 object, 16x128 object
    S = C.Server(4 << 30, slots=2, rounds=3)
    outs = [torch.zeros(tuple(q[2].shape), dtype=torch.float32, device="cuda") for q in reqs]
    S.fail_next_groups(1)
    for i, (cfg, mask, raw) in enumerate(reqs):
        S.submit(cfg, mask, raw, outs[i], i)
    done = {}
    for step in range(400):
        S.step()
        used, groups = S.usage()
        # the failed group's range was given back: what is in use is exactly
        # the groups that exist
        assert used <= 2 * sum(C.workspace_bytes(q[0]) for q in reqs[1:3]) + \
            2 * C.workspace_bytes(reqs[0][0])
        for c in S.poll():
            assert c["id"] not in done, f"second completion for request {c['id']}"
            done[c["id"]] = c
        if len(done) == len(reqs):
            break
    S.close()
    assert sorted(done) == [0, 1, 2, 3]
    assert done[0]["status"] == C.EHIP and done[0]["iters"] == 0
    for i in (1, 2, 3):
        assert done[i]["status"] == C.OK, (i, done[i])
        cfg, mask, raw = reqs[i]
        assert np.array_equal(outs[i].cpu().numpy(), _alone(torch, cfg, mask, raw)), i


def test_served_requests_match_the_oracle():
    """One object-model and one dual-model request, served beside others, agree
    with the FP64 oracle to the per-volume tolerance (1e-3 relative L2).  The
    step constants are the oracle's power estimates, passed in the requests."""
    import dataclasses
    from oracle import cnlos_oracle as O
    from tests.gpu_helpers import f32, rel_l2
    torch = need_gpu()
    say("serving: served results against the oracle")
    reqs = _requests(torch)
    checks = {}
    for i in (0, 1):
        n, m = reqs[i][0].nx, reqs[i][0].nt
        sc = scenes.scene_custom(n, m, 3000 + i, wall=1.0, bin_ps=32.0 * 128 / m,
                                 density=0.2 + 0.05 * i, peak=5.0 + 5 * i)
        raw = f32(synth_measurement(sc, 3100 + i))
        op = O.make_operator(n, n, m, 1.0, 1.0, sc.bin_ps, O.FALLOFF_COMPENSATED, sc.mask)
        tau0, _ = O.normalize_measurement(raw, sc.mask, O.FALLOFF_COMPENSATED)
        L0o = 2 * O.power_norm2(lambda x: O.apply_A(x, op, True),
                                lambda y: O.apply_AT(y, op, True), tau0.shape)
        cfg = reqs[i][0]
        cfg.L0 = L0o
        if cfg.model == C.MODEL_DUAL:
            L0d = 2 * O.power_norm2(lambda x: O.apply_A(x, op, False),
                                    lambda y: O.apply_AT(y, op, False), tau0.shape)
            cfg.L0_dual = L0d
            p = O.Params(a=DUAL["warm_a"], b=DUAL["warm_b"], mu=DUAL["mu"], a_u=DUAL["a_u"],
                         b_u=DUAL["b_u"], a_tau=DUAL["a_tau"], b_tau=DUAL["b_tau"],
                         lam=DUAL["lam"])
            _, s2 = O.run_alg2(tau0, op, p, cfg.max_iters, cfg.init_iters, L0_obj=L0o,
                               L0_dual=L0d)
            checks[i] = s2.u
        else:
            p = O.Params(a=OBJ["a_u"], b=OBJ["b_u"], mu=OBJ["mu"])
            checks[i] = O.run_alg1(tau0, op, p, cfg.max_iters, L0=L0o).u
    outs, done, _ = _serve(torch, reqs, 4 << 30, slots=2, rounds=3,
                           arrivals=[0, 0, 1, 2, 2, 4, 6, 7])
    for i, ref in checks.items():
        assert done[i]["status"] == C.OK
        err = rel_l2(outs[i].double().cpu().numpy(), ref)
        say(f"  request {i}: rel L2 vs oracle {err:.2e}")
        assert err <= 1e-3


def test_a_slot_group_holds_one_kernel_spectrum():
    """H^ depends only on the geometry (eq. (3)): a slot group keeps one copy
    for all its slots, so its arena footprint is one H^ plus the slots'
    workspaces without theirs, and requests of another wall extent get a group
    of their own."""
    torch = need_gpu()
    say("serving: one H^ per slot group")
    reqs = _requests(torch)
    cfg, mask, raw = reqs[1]                       # 32x256 dual
    S = C.Server(4 << 30, slots=4, rounds=2)
    out = [torch.zeros(tuple(raw.shape), dtype=torch.float32, device="cuda") for _ in range(3)]
    S.submit(cfg, mask, raw, out[0], 0)
    S.submit(cfg, mask, raw, out[1], 1)
    S.step()
    used, groups = S.usage()
    assert groups == 1 and used == _group_bytes(cfg, 4)
    other = C.default_config(**{f: getattr(cfg, f) for f, _ in C.Config._fields_})
    other.wall_w_m = other.wall_h_m = 0.9
    S.submit(other, mask, raw, out[2], 2)
    S.step()
    used, groups = S.usage()
    assert groups == 2 and used == 2 * _group_bytes(cfg, 4)
    done = {}
    for _ in range(400):
        for c in S.poll():
            done[c["id"]] = c
        if len(done) == 3:
            break
        S.step()
    S.close()
    assert all(done[i]["status"] == C.OK for i in range(3))
    ref = _alone(torch, cfg, mask, raw)
    assert np.array_equal(out[0].cpu().numpy(), ref) and np.array_equal(out[1].cpu().numpy(), ref)
    assert np.array_equal(out[2].cpu().numpy(), _alone(torch, other, mask, raw))
