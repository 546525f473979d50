"""Pins of the oracle's ADMM pieces (Sections 3-4): difference operators, the
FFT-diagonal solve (eq. (11)), shrinkage (eq. (7)), curvature and phi, the FISTA
recurrence, backtracking, and whole-run invariants and special cases."""
import dataclasses
import math

import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.optimize as sopt
import scipy.sparse.linalg as spla

from oracle import cnlos_oracle as O


# --------------------------------------------------------------------------
# difference operators and the diagonal solve
# --------------------------------------------------------------------------

def test_grad_adjoint_identity():
    rng = np.random.default_rng(0)
    u = rng.standard_normal((5, 6, 7))
    p = rng.standard_normal((3, 5, 6, 7))
    assert abs(float((O.grad(u) * p).sum()) - float((u * O.grad_adj(p)).sum())) < 1e-11


def test_grad_adj_grad_is_minus_periodic_laplacian():
    u = np.random.default_rng(1).standard_normal((6, 5, 8))
    lap = ndi.laplace(u, mode="wrap")
    np.testing.assert_allclose(O.grad_adj(O.grad(u)), -lap, atol=1e-12)


def test_grad_matches_hand_stencil():
    u = np.arange(24, dtype=float).reshape(2, 3, 4) ** 2
    g = O.grad(u)
    assert g[0, 0, 1, 2] == u[1, 1, 2] - u[0, 1, 2]
    assert g[0, 1, 1, 2] == u[0, 1, 2] - u[1, 1, 2]        # periodic wrap in x
    assert g[1, 1, 2, 3] == u[1, 0, 3] - u[1, 2, 3]        # wrap in y
    assert g[2, 0, 0, 3] == u[0, 0, 0] - u[0, 0, 3]        # wrap in t


def test_solve_diag_residual_by_stencil():
    rng = np.random.default_rng(2)
    rhs = rng.standard_normal((8, 4, 16))
    for c, mu in ((3.0, 0.1), (1.0 + 2.0, 800.0), (0.7, 5.0)):
        x = O.solve_diag(rhs, c, mu)
        res = c * x + mu * O.grad_adj(O.grad(x)) - rhs
        assert np.abs(res).max() < 1e-12 * max(1.0, mu)


def test_laplacian_symbol_on_a_cosine_mode():
    shape = (8, 16, 32)
    w = (3, 5, 7)
    idx = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    mode = np.cos(sum(2 * np.pi * w[a] * idx[a] / shape[a] for a in range(3)))
    lam = sum(4 * math.sin(math.pi * w[a] / shape[a]) ** 2 for a in range(3))
    np.testing.assert_allclose(O.grad_adj(O.grad(mode)), lam * mode, atol=1e-12)
    np.testing.assert_allclose(O.solve_diag(mode, 2.0, 0.5), mode / (2.0 + 0.5 * lam), atol=1e-12)


# --------------------------------------------------------------------------
# shrinkage
# --------------------------------------------------------------------------

def test_shrink_is_the_prox_of_the_weighted_norm():
    rng = np.random.default_rng(3)
    for _ in range(20):
        a = rng.standard_normal(3) * 2
        b = abs(rng.standard_normal()) * 1.5
        got = O.shrink(a.reshape(3, 1), b).ravel()
        obj = lambda v: b * np.linalg.norm(v) + 0.5 * np.sum((v - a) ** 2)
        best = sopt.minimize(obj, a, method="Nelder-Mead",
                             options=dict(xatol=1e-12, fatol=1e-14, maxiter=20000)).x
        assert obj(got) <= obj(best) + 1e-10
        # optimality: either zero with |a| <= b, or a scaled copy of a
        if np.linalg.norm(a) <= b:
            assert np.all(got == 0)
        else:
            np.testing.assert_allclose(got, a * (1 - b / np.linalg.norm(a)), rtol=1e-14)


def test_shrink_special_cases():
    a = np.array([[0.0, 1.0, -2.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    np.testing.assert_array_equal(O.shrink(a, 0.0), a)              # b = 0: identity
    assert np.all(O.shrink(a, 5.0) == 0)                            # |a| <= b: zero
    # zero vector: 0 (no 0/0)
    assert np.all(np.isfinite(O.shrink(np.zeros((3, 4)), 0.3)))
    # scalar case is soft thresholding
    x = np.linspace(-3, 3, 61)
    v = np.zeros((3, 61))
    v[0] = x
    np.testing.assert_allclose(O.shrink(v, 0.7)[0], np.sign(x) * np.maximum(np.abs(x) - 0.7, 0),
                               atol=1e-15)


# --------------------------------------------------------------------------
# curvature and phi
# --------------------------------------------------------------------------

def test_curvature_of_zero_and_bounds():
    assert np.all(O.curvature(np.zeros((4, 4, 4)), 1e-3) == 0)
    u = np.random.default_rng(4).standard_normal((6, 6, 6)) * 100
    assert np.abs(O.curvature(u, 1e-3)).max() <= 6.0


def test_curvature_of_a_plane_is_zero_in_the_interior():
    idx = np.meshgrid(*[np.arange(16)] * 3, indexing="ij")
    u = 0.3 * idx[0] - 0.7 * idx[1] + 0.2 * idx[2]
    k = O.curvature(u, 1e-3)
    assert np.abs(k[2:-2, 2:-2, 2:-2]).max() < 1e-12


@pytest.mark.parametrize("r", [8, 12])
def test_curvature_of_sphere_level_sets(r):
    """u = |x - c| has level sets that are spheres; mean curvature div(n) = 2/r."""
    n = 2 * r + 16
    c = n / 2 + 0.31
    idx = np.meshgrid(*[np.arange(n, dtype=float)] * 3, indexing="ij")
    rad = np.sqrt(sum((idx[a] - c) ** 2 for a in range(3)))
    k = O.curvature(rad, 1e-3)
    # the backward divergence of forward-difference normals is centred half a
    # voxel off the grid point; compare at the matching radius
    rs = np.sqrt(sum((idx[a] - c - 0.5) ** 2 for a in range(3)))
    shell = np.abs(rs - r) < 0.5
    rel = (k[shell] - 2.0 / rs[shell]) / (2.0 / rs[shell])
    assert abs(rel.mean()) < 0.01
    assert np.abs(rel).max() < 0.8 * 8 / r


def test_curvature_of_cylinder_level_sets():
    n, r = 40, 10
    c = n / 2 + 0.27
    idx = np.meshgrid(*[np.arange(n, dtype=float)] * 3, indexing="ij")
    rad = np.sqrt((idx[0] - c) ** 2 + (idx[1] - c) ** 2)
    k = O.curvature(rad, 1e-3)
    rs = np.sqrt((idx[0] - c - 0.5) ** 2 + (idx[1] - c - 0.5) ** 2)
    shell = np.abs(rs - r) < 0.5
    rel = (k[shell] - 1.0 / rs[shell]) / (1.0 / rs[shell])
    assert abs(rel.mean()) < 0.01
    assert np.abs(rel).max() < 0.1


def test_phi_variants_and_tv_special_case():
    k = np.array([-2.0, 0.0, 0.5, 3.0])
    np.testing.assert_allclose(O.phi_of(k, 0.1, 0.2, O.PHI_TSC), 0.1 + 0.2 * k ** 2)
    np.testing.assert_allclose(O.phi_of(k, 0.1, 0.2, O.PHI_TAC), 0.1 + 0.2 * np.abs(k))
    np.testing.assert_allclose(O.phi_of(k, 0.1, 0.2, O.PHI_TRV), np.sqrt(0.1 + 0.2 * k ** 2))
    for kind in (O.PHI_TSC, O.PHI_TAC):
        np.testing.assert_array_equal(O.phi_of(k, 0.3, 0.0, kind), 0.3)   # b = 0: TV


# --------------------------------------------------------------------------
# FISTA and backtracking
# --------------------------------------------------------------------------

def test_fista_recurrence_identity():
    t = 1.0
    for k in range(1, 200):
        tn = O.fista_next(t)
        assert abs(tn * tn - tn - t * t) <= 1e-12 * tn * tn
        assert tn >= (k + 1) / 2.0
        t = tn


def test_backtracking_condition_is_the_quadratic_identity():
    """For f = 1/2 |B u - y|^2 the Beck-Teboulle test equals |B d|^2 <= L |d|^2."""
    n, m = 4, 16
    rng = np.random.default_rng(5)
    mask = (rng.random((n, n)) < 0.5).astype(np.uint8)
    op = O.make_operator(n, n, m, 0.8, 0.8, 32.0, mask=mask)
    y = O.apply_A(rng.random((n, n, m)), op, True)
    ub = rng.standard_normal((n, n, m))
    d = rng.standard_normal((n, n, m)) * 1e-2
    f = lambda x: 0.5 * float(((O.apply_A(x, op, True) - y) ** 2).sum())
    g = O.apply_AT(O.apply_A(ub, op, True) - y, op, True)
    lhs = f(ub + d) - f(ub) - float((d * g).sum())
    Bd = O.apply_A(d, op, True)
    assert abs(lhs - 0.5 * float((Bd * Bd).sum())) <= 1e-9 * abs(lhs)


def test_backtracking_rejects_small_L_and_keeps_L_monotone():
    sc_n, m = 4, 16
    rng = np.random.default_rng(6)
    op = O.make_operator(sc_n, sc_n, m, 0.8, 0.8, 32.0)
    tau0 = O.apply_A(rng.random((sc_n, sc_n, m)), op, True)
    est = O.power_norm2(lambda x: O.apply_A(x, op, True), lambda y: O.apply_AT(y, op, True),
                        tau0.shape)
    p = O.Params(a=1e-4, b=1e-4, mu=0.1)
    st = O.run_alg1(tau0, op, p, 12, L0=est / 16)
    Ls = [e[3] for e in st.log]
    assert sum(e[4] for e in st.log) >= 1                   # at least one rejection
    assert all(b >= a for a, b in zip(Ls, Ls[1:]))          # L never decreases
    with pytest.raises(O.BacktrackingExhausted):
        O.run_alg1(tau0, op, O.Params(a=1e-4, b=1e-4, mu=0.1, bt_max_trials=1), 3,
                   L0=est / 1e6)


# --------------------------------------------------------------------------
# whole-run special cases and invariants
# --------------------------------------------------------------------------

def chambolle_rof(f: np.ndarray, lam: float, iters: int = 20000, step: float = 1.0 / 12.5):
    """Independent ROF solver (Chambolle's dual projection): minimizes
    1/2 |u - f|^2 + lam * sum |grad u| with the same periodic gradient."""
    p = np.zeros((3,) + f.shape)
    for _ in range(iters):
        g = O.grad(O.div_back(p) - f / lam)
        p = (p + step * g) / (1.0 + step * np.sqrt((g * g).sum(axis=0)))
    return f - lam * O.div_back(p)


@pytest.mark.slow
def test_alg1_with_identity_operator_solves_rof():
    """A = I, full mask, b = 0: Algorithm 1 is TV denoising (phi = a)."""
    rng = np.random.default_rng(8)
    f = np.zeros((6, 6, 6))
    f[1:4, 2:5, 2:4] = 1.0
    f += 0.2 * rng.standard_normal(f.shape)
    a = 0.15
    ref = chambolle_rof(f, a)
    p = O.Params(a=a, b=0.0, mu=1.0, bt=False)
    st = O.run_alg1(f, None, p, 3000, fwd=lambda x: x, adj=lambda y: y, L0=2.0)
    assert np.linalg.norm(st.u - ref) <= 1e-4 * np.linalg.norm(ref)


def test_alg1_without_regularization_reaches_least_squares():
    """a = b = 0: the iteration is accelerated preconditioned gradient descent on
    f = 1/2 |A_D u - tau0|^2; its value must reach the least-squares optimum."""
    n, m = 4, 8
    rng = np.random.default_rng(9)
    mask = (rng.random((n, n)) < 0.7).astype(np.uint8)
    op = O.make_operator(n, n, m, 0.6, 0.6, 64.0, mask=mask)
    tau0 = O.apply_A(rng.random((n, n, m)), op, True) + 0.01 * rng.standard_normal((n, n, m)) * mask[:, :, None]
    V = n * n * m
    Amat = np.zeros((V, V))
    for c in range(V):
        e = np.zeros(V)
        e[c] = 1.0
        Amat[:, c] = O.apply_A(e.reshape(n, n, m), op, True).ravel()
    xs = spla.lsqr(Amat, tau0.ravel(), atol=1e-14, btol=1e-14, iter_lim=100000)[0]
    fstar = 0.5 * float(((Amat @ xs - tau0.ravel()) ** 2).sum())
    f0 = 0.5 * float((tau0 ** 2).sum())
    st = O.run_alg1(tau0, op, O.Params(a=0.0, b=0.0, mu=1e-3, eta=1e-3), 400)
    r = O.apply_A(st.u, op, True) - tau0
    fT = 0.5 * float((r * r).sum())
    assert fT >= fstar - 1e-12
    assert (fT - fstar) <= 2e-3 * (f0 - fstar)


def _small_problem(seed=11, n=8, m=32):
    from paper_2301_00406_amd import scenes
    sc = scenes.scene_custom(n, m, seed, wall=0.8, bin_ps=32.0, density=0.5, n_planes=2,
                             n_shells=0, peak=30.0)
    opL = O.make_operator(n, n, m, sc.wall_w, sc.wall_h, sc.bin_ps, O.FALLOFF_LITERAL)
    clean = O.apply_A(sc.u_true, opL)
    raw = scenes.poisson_counts(clean, sc.peak, sc.background, np.random.default_rng(seed))
    tau0, _ = O.normalize_measurement(raw, sc.mask, O.FALLOFF_COMPENSATED)
    op = O.make_operator(n, n, m, sc.wall_w, sc.wall_h, sc.bin_ps, mask=sc.mask)
    return sc, op, tau0


def _windowed_decrease(vals, win=5):
    means = [np.mean(vals[i:i + win]) for i in range(0, len(vals) - win + 1, win)]
    return all(b <= a * (1 + 1e-9) for a, b in zip(means, means[1:]))


def test_alg1_energy_decreases():
    sc, op, tau0 = _small_problem()
    # the Bowling parameters printed with the full-sampling comparison figure
    st = O.run_alg1(tau0, op, O.Params(a=5e-5, b=5e-5, mu=0.1), 40)
    E = [e[0] for e in st.log]
    assert E[-1] < E[0]
    assert _windowed_decrease(E, 10)
    primal = [e[1] for e in st.log]
    assert np.mean(primal[-10:]) < np.mean(primal[:10])


def test_alg2_energy_decreases_and_substeps():
    sc, op, tau0 = _small_problem(seed=12)
    p = O.Params(a=5e-4, b=5e-4, mu=0.1, a_u=5e-4, b_u=5e-5, a_tau=3e-3, b_tau=5e-4,
                 lam=200.0)
    s1, s2 = O.run_alg2(tau0, op, p, 30, init_iters=10)
    E = [e[0] for e in s2.log]
    assert E[-1] < E[0]
    assert _windowed_decrease(E, 10)


def test_f_step_is_the_pointwise_minimizer():
    rng = np.random.default_rng(13)
    lam, mu3 = 200.0, 2.0
    tau0, taubar, Lam3 = rng.standard_normal((3, 50))
    kept = rng.random(50) < 0.5
    f = np.where(kept, (lam * tau0 + mu3 * taubar - Lam3) / (lam + mu3), taubar - Lam3 / mu3)
    obj = lambda x: (0.5 * lam * kept * (x - tau0) ** 2 + Lam3 * (x - taubar)
                     + 0.5 * mu3 * (x - taubar) ** 2)
    for dlt in (1e-3, -1e-3):
        assert np.all(obj(f + dlt) >= obj(f))


def test_tau_step_solves_its_quadratic():
    rng = np.random.default_rng(14)
    shape = (4, 4, 16)
    Au, f, Lam3 = rng.standard_normal((3,) + shape)
    w, Lam2 = rng.standard_normal((2, 3) + shape)
    mu2, mu3 = 800.0, 2.0
    rhs = Au + mu3 * f + Lam3 + mu2 * O.grad_adj(w + Lam2 / mu2)
    tau = O.solve_diag(rhs, 1.0 + mu3, mu2)

    def L(t):
        g = w - O.grad(t)
        return (0.5 * ((Au - t) ** 2).sum() + (Lam2 * g).sum() + 0.5 * mu2 * (g * g).sum()
                + (Lam3 * (f - t)).sum() + 0.5 * mu3 * ((f - t) ** 2).sum())
    base = L(tau)
    for _ in range(5):
        assert L(tau + 1e-4 * rng.standard_normal(shape)) >= base


def test_v_step_decreases_its_subobjective():
    rng = np.random.default_rng(15)
    shape = (4, 4, 8)
    ub = rng.standard_normal(shape)
    Lam = rng.standard_normal((3,) + shape)
    phi = 0.1 + rng.random(shape)
    mu = 0.5
    v = O.shrink(O.grad(ub) - Lam / mu, phi / mu)

    def obj(vv):
        return float((phi * np.sqrt((vv * vv).sum(axis=0))).sum() + (Lam * (vv - O.grad(ub))).sum()
                     + 0.5 * mu * ((vv - O.grad(ub)) ** 2).sum())
    base = obj(v)
    for _ in range(10):
        assert obj(v + 1e-3 * rng.standard_normal(v.shape)) >= base - 1e-12


# --------------------------------------------------------------------------
# momentum restart (an option; Algorithms 1-2 print the plain extrapolation)
# --------------------------------------------------------------------------

def test_momentum_restart_rule():
    """t resets to 1 only on an energy rise beyond the tolerance; never on the
    first accepted iterate (no previous energy)."""
    class S:
        pass
    st = S()
    st.t, st.E_prev = 7.5, float("nan")
    O.momentum_restart(st, 1e9)
    assert st.t == 7.5
    st.E_prev = 100.0
    O.momentum_restart(st, 100.0 * (1.0 + 0.5 * O.RESTART_TOL))
    assert st.t == 7.5
    O.momentum_restart(st, 99.0)
    assert st.t == 7.5
    O.momentum_restart(st, 100.0 * (1.0 + 2.0 * O.RESTART_TOL))
    assert st.t == 1.0


def test_restart_zeroes_the_next_extrapolation():
    """With the restart switched on, after a restarted step the extrapolated
    point equals the new iterate; with it off (the printed step) t keeps growing."""
    from tests.test_oracle_alg2_pins import _dual_problem
    op, tau0, p, L0o, L0d = _dual_problem()
    t_printed = O.run_alg1(tau0, op, p, 8, L0=L0o).t
    assert t_printed > 4.0
    p = dataclasses.replace(p, fista_restart=True)
    fwdD = lambda x: O.apply_A(x, op, True)
    adjD = lambda y: O.apply_AT(y, op, True)
    st = O.alg1_init(tau0.shape, p, L0o)
    for _ in range(6):
        O.alg1_step(st, tau0, fwdD, adjD, p)
    st.E_prev = 0.5 * st.log[-1][0]         # the next accepted energy reads as a rise
    O.alg1_step(st, tau0, fwdD, adjD, p)
    assert st.t == 1.0
    O.alg1_step(st, tau0, fwdD, adjD, p)
    np.testing.assert_array_equal(st.ubar, st.u)
