"""Full-size solver parity at the benchmark's configuration against stored
oracle runs (tests/golden/make_reference_runs.py writes them with the FP64
oracle only).

64x64x512, Algorithm 2 (Section 4.1) for 200 iterations after 50 of
Algorithm 1 (Section 3.2): the volume u and the signal tau after the whole
run within 1e-3 relative L2 (the per-volume tolerance), every logged energy
of both stages within 1e-3, and the backtracking step sequence identical."""
import hashlib
import os

import numpy as np
import pytest

from paper_2301_00406_amd import cnlos as C
from paper_2301_00406_amd import scenes
from tests.conftest import golden_path
from tests.gpu_helpers import f32, max_rel, need_gpu, rel_l2, say, synth_measurement, to_dev, to_host

pytestmark = pytest.mark.gpu
TOL_VOL = 1e-3


def _raw(sc, seed, want_sha):
    raw = f32(synth_measurement(sc, seed))
    got = hashlib.sha256(np.ascontiguousarray(raw, dtype=np.float32).tobytes()).hexdigest()
    assert got == want_sha, "the regenerated measurement differs from the stored run's"
    return raw


def _params(ref):
    import ast
    return ast.literal_eval(str(ref["params"]))


def test_benchmark_configuration_matches_the_stored_oracle_run():
    torch = need_gpu()
    path = golden_path("alg2_64x64x512.npz")
    ref = np.load(path)
    sc = scenes.scene_medium()
    say("alg2 64x64x512 50+200 against the stored oracle run")
    raw = _raw(sc, int(ref["seed"][0]), str(ref["raw_sha256"]))
    pr = _params(ref)
    L0o, L0d = (float(x) for x in ref["L0"])
    i1, i2 = (int(x) for x in ref["iters"])
    cfg = C.default_config(nx=sc.n, ny=sc.n, nt=sc.m, wall_w_m=sc.wall_w, wall_h_m=sc.wall_h,
                           bin_ps=sc.bin_ps, model=C.MODEL_DUAL, max_iters=i2, init_iters=i1,
                           a_u=pr["a_u"], b_u=pr["b_u"], a_tau=pr["a_tau"], b_tau=pr["b_tau"],
                           warm_a=pr["a"], warm_b=pr["b"], mu=pr["mu"], lam=pr["lam"],
                           L0=L0o, L0_dual=L0d)
    P = C.Problem(cfg, sc.mask)
    P.set_measurement(to_dev(torch, raw))
    rep = P.run()
    assert rep["total_iters"] == i1 + i2
    u, tau = to_host(P.volume()), to_host(P.signal())
    eu, et = rel_l2(u, ref["u"]), rel_l2(tau, ref["tau"])
    say(f"  rel L2 u = {eu:.3e}, tau = {et:.3e}; max abs / max u = {max_rel(u, ref['u']):.3e}, "
        f"tau = {max_rel(tau, ref['tau']):.3e}")
    assert eu <= TOL_VOL and et <= TOL_VOL
    log = P.log()
    E = np.concatenate([ref["log1"][:, 0], ref["log2"][:, 0]])
    dE = np.max(np.abs(log[:, 0] - E) / np.abs(E))
    say(f"  largest relative energy difference {dE:.3e}")
    assert dE <= TOL_VOL
    Ls = np.concatenate([ref["log1"][:, 3], ref["log2"][:, 3]])
    np.testing.assert_array_equal(log[:, 3], Ls)            # step constants
    trials = np.concatenate([ref["log1"][:, 4], ref["log2"][:, 4]])
    np.testing.assert_array_equal(log[:, 4], trials)        # rejections per iteration
    P.close()


# builds the 128x128x1024 problem and compares full volumes on the host:
# more than a minute of host time
@pytest.mark.timeout(600)
def test_large_configuration_first_iterations_match_the_stored_oracle_run():
    """128x128x1024 (the large workload), one warm-start and one Algorithm-2
    iteration against the stored full-size oracle run: 64 sampled scan
    columns of u and tau within 1e-3 relative L2 (over the sample), the
    volumes' norms and both logged energies within 1e-3, the step constants
    identical."""
    torch = need_gpu()
    ref = np.load(golden_path("alg2_128x128x1024.npz"))
    sc = scenes.scene_large()
    say("alg2 128x128x1024 1+1 against the stored oracle run")
    raw = _raw(sc, int(ref["seed"][0]), str(ref["raw_sha256"]))
    pr = _params(ref)
    L0o, L0d = (float(x) for x in ref["L0"])
    i1, i2 = (int(x) for x in ref["iters"])
    cfg = C.default_config(nx=sc.n, ny=sc.n, nt=sc.m, wall_w_m=sc.wall_w, wall_h_m=sc.wall_h,
                           bin_ps=sc.bin_ps, model=C.MODEL_DUAL, max_iters=i2, init_iters=i1,
                           a_u=pr["a_u"], b_u=pr["b_u"], a_tau=pr["a_tau"], b_tau=pr["b_tau"],
                           warm_a=pr["a"], warm_b=pr["b"], mu=pr["mu"], lam=pr["lam"],
                           L0=L0o, L0_dual=L0d)
    P = C.Problem(cfg, sc.mask)
    P.set_measurement(to_dev(torch, raw))
    P.run(i1)
    u1 = to_host(P.volume())
    assert abs(np.linalg.norm(u1) - ref["u_norm"][1]) <= TOL_VOL * ref["u_norm"][1]
    P.run()
    u, tau = to_host(P.volume()), to_host(P.signal())
    cols = ref["cols"]
    eu = rel_l2(u[cols[:, 0], cols[:, 1]], ref["u_cols"])
    et = rel_l2(tau[cols[:, 0], cols[:, 1]], ref["tau_cols"])
    say(f"  sampled columns: rel L2 u = {eu:.3e}, tau = {et:.3e}")
    assert eu <= TOL_VOL and et <= TOL_VOL
    assert abs(np.linalg.norm(u) - ref["u_norm"][0]) <= TOL_VOL * ref["u_norm"][0]
    assert abs(np.linalg.norm(tau) - ref["tau_norm"][0]) <= TOL_VOL * ref["tau_norm"][0]
    log = P.log()
    E = np.concatenate([ref["log1"][:, 0], ref["log2"][:, 0]])
    assert np.max(np.abs(log[:, 0] - E) / np.abs(E)) <= TOL_VOL
    np.testing.assert_array_equal(log[:, 3], np.concatenate([ref["log1"][:, 3], ref["log2"][:, 3]]))
    P.close()
