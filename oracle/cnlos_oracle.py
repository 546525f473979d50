"""FP64 CPU oracle for curvature-regularized confocal NLOS reconstruction.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously-correct
reference against which the HIP library is checked.  Only the test-suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
path never does.  It shares no code with the HIP library: everything below is
written from the paper (Ding et al., "Curvature regularization for
non-line-of-sight imaging from under-sampled data", arXiv 2301.00406), in
float64, with NumPy/SciPy FFTs as the only library steps.

Where the paper is silent the oracle takes the following readings (listed with
their reasons in the design notes):

* grid: unit voxel spacing on all three axes for the difference operators;
  scan point i at x_i = (i + 1/2) W / n - W / 2; bin k covers [k, k+1) R / m
  with R = m c dt / 2.
* R_z (Section 2, eq. (3)): the change of variables zeta = z^2 integrated over
  each squared-distance bin, giving S[q, k] = m * |[sqrt(q/m), sqrt((q+1)/m))
  intersect [k/m, (k+1)/m)|; every column of S sums to one.
* H (eq. (3)): the kernel of the continuous model eq. (2) after the change of
  variables, h[dx, dy, dq] = 1/Z iff dq = floor(m s_h (dx^2 + dy^2) + 1/2) < m,
  s_h = (W / (n R))^2 (anisotropic: dx and dy use their own wall extents),
  applied as a linear (zero-padded) convolution cropped to the volume.
* R_t^{-1} (eq. (3)): diag(w) S^T.  LITERAL falloff: w_k = rhat_k^{-3} with
  rhat_k = (k + 1/2)/m.  COMPENSATED falloff (the solver default): w_k = 1 and
  the measurement is pre-multiplied by rhat_k^3 and normalized to unit maximum.
* difference operators: periodic forward differences for nabla, nabla^* its
  exact adjoint (minus the backward-difference divergence); periodicity is
  what makes the FFT solve of eq. (11) exact.
* shrinkage eq. (7): isotropic over the 3-vector, 0 where |a| = 0.
* curvature (Section 3): div^-(nabla^+ u / sqrt(|nabla^+ u|^2 + eta^2)).
* backtracking (named in the abstract, not defined): Beck-Teboulle on the
  linearized data term, factor bt_factor, L never decreases.
* Alg. 2 sub-problems (Section 4.1 gives only the Lagrangian): closed forms
  derived from it, solved in the order v, w, f, u, tau, multipliers.  The
  extrapolated signal taubar is the data of the linearized u-step; the
  signal-domain splitting steps (w, f) start from the last accepted tau.
  Taking w and f at taubar as well makes the printed iteration unstable: the
  w-step then leaves Lambda2 = mu2 grad(taubar - tau+), the extrapolation's
  step scaled by mu2 (800 in Section 5.1), and the energy of eq. (13) grows
  without bound on synthetic scenes (the oracle keeps that reading behind
  ``Params.tau_split_at_bar`` to show it).
* FISTA (Algorithms 1-2): the printed extrapolation by default; a
  function-value restart (O'Donoghue and Candes) is available as an option
  (``Params.fista_restart``).
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Callable, Optional

import numpy as np
import scipy.fft as sfft

C_LIGHT = 299792458.0
WORKERS = int(os.environ.get("CNLOS_ORACLE_WORKERS", "0")) or (os.cpu_count() or 1)

FALLOFF_COMPENSATED = 0
FALLOFF_LITERAL = 1
PHI_TSC, PHI_TAC, PHI_TRV = 0, 1, 2


def _fftn(x):
    return sfft.fftn(x, workers=WORKERS)


def _ifftn(x):
    return sfft.ifftn(x, workers=WORKERS)


# ============================================================================
# Forward model: A = R_t^{-1} H R_z  (Section 2, eq. (3); continuous eq. (2))
# ============================================================================

def range_metres(m: int, bin_ps: float) -> float:
    """One-way distance covered by m bins: R = m c dt / 2 (light goes out and back)."""
    return m * C_LIGHT * (bin_ps * 1e-12) / 2.0


def resample_matrix(m: int) -> np.ndarray:
    """R_z as an m x m matrix S: depth bin k -> squared-distance bin q.

    The continuous change of variables zeta = z^2 maps u(z) to u(sqrt(zeta)) /
    (2 sqrt(zeta)); integrating it over bin q of zeta gives the integral of u
    over z in [sqrt(q/m), sqrt((q+1)/m)).  With u constant on each depth bin
    [k/m, (k+1)/m) this is the overlap length times m.
    """
    S = np.zeros((m, m))
    for q in range(m):
        lo, hi = math.sqrt(q / m), math.sqrt((q + 1) / m)
        for k in range(m):
            a, b = max(lo, k / m), min(hi, (k + 1) / m)
            if b > a:
                S[q, k] = m * (b - a)
    return S


def kernel_offsets(nx: int, ny: int, m: int, wall_w: float, wall_h: float, bin_ps: float):
    """Support of the shift-invariant kernel h of eq. (3).

    After the change of variables v = (tc/2)^2 the confocal model eq. (2) is a
    convolution in (x, y, v) with the cone h = delta(x^2 + y^2 - v).  In bin
    units, lateral offset (dx, dy) lands in v-bin dq = round(m ((dx Wx/nx)^2 +
    (dy Wy/ny)^2) / R^2).  Returns dq[dx + nx - 1, dy + ny - 1] (-1 outside the
    volume) and Z, the number of supported offsets (h has unit sum).
    """
    R = range_metres(m, bin_ps)
    sx = (wall_w / (nx * R)) * (wall_w / (nx * R))
    sy = (wall_h / (ny * R)) * (wall_h / (ny * R))
    dq = -np.ones((2 * nx - 1, 2 * ny - 1), dtype=np.int64)
    for dx in range(-(nx - 1), nx):
        for dy in range(-(ny - 1), ny):
            x = float(m) * (sx * float(dx * dx) + sy * float(dy * dy))
            q = int(math.floor(x + 0.5))
            if q < m:
                dq[dx + nx - 1, dy + ny - 1] = q
    Z = int((dq >= 0).sum())
    return dq, Z


def falloff_weights(m: int, falloff: int) -> np.ndarray:
    """The radiometric part of R_t^{-1}: w_k = rhat_k^{-3} (LITERAL) or 1."""
    if falloff == FALLOFF_LITERAL:
        r = (np.arange(m) + 0.5) / m
        return r ** -3
    return np.ones(m)


@dataclasses.dataclass
class LCTOperator:
    nx: int
    ny: int
    m: int
    S: np.ndarray          # (m, m)
    dq: np.ndarray         # (2nx-1, 2ny-1)
    Z: int
    w: np.ndarray          # (m,)
    Hhat: np.ndarray       # (2nx, 2ny, 2m) complex128, FFT of the padded kernel
    mask: np.ndarray       # (nx, ny) float64 0/1


def make_operator(nx, ny, m, wall_w, wall_h, bin_ps, falloff=FALLOFF_COMPENSATED,
                  mask=None) -> LCTOperator:
    S = resample_matrix(m)
    dq, Z = kernel_offsets(nx, ny, m, wall_w, wall_h, bin_ps)
    hpad = np.zeros((2 * nx, 2 * ny, 2 * m))
    for a in range(2 * nx - 1):
        for b in range(2 * ny - 1):
            q = dq[a, b]
            if q >= 0:
                dx, dy = a - (nx - 1), b - (ny - 1)
                hpad[dx % (2 * nx), dy % (2 * ny), q] = 1.0 / Z
    Hhat = _fftn(hpad)
    mk = np.ones((nx, ny)) if mask is None else np.asarray(mask, dtype=np.float64)
    return LCTOperator(nx, ny, m, S, dq, Z, falloff_weights(m, falloff), Hhat, mk)


def resample(u: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Apply S along the last (depth/time) axis: out[..., q] = sum_k S[q,k] u[..., k]."""
    return u @ S.T


def resample_T(g: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Apply S^T along the last axis: out[..., k] = sum_q S[q,k] g[..., q]."""
    return g @ S


def apply_A_direct(u: np.ndarray, op: LCTOperator, masked: bool = False) -> np.ndarray:
    """A u by direct summation of the linear convolution (tiny grids only)."""
    nx, ny, m = op.nx, op.ny, op.m
    ut = resample(u, op.S)
    g = np.zeros_like(ut)
    for i in range(nx):
        for j in range(ny):
            for i2 in range(nx):
                for j2 in range(ny):
                    q0 = op.dq[i - i2 + nx - 1, j - j2 + ny - 1]
                    if q0 < 0:
                        continue
                    g[i, j, q0:] += ut[i2, j2, :m - q0] / op.Z
    tau = resample_T(g, op.S) * op.w
    if masked:
        tau = tau * op.mask[:, :, None]
    return tau


def _conv_padded(x: np.ndarray, op: LCTOperator, adjoint: bool) -> np.ndarray:
    nx, ny, m = op.nx, op.ny, op.m
    pad = np.zeros((2 * nx, 2 * ny, 2 * m))
    pad[:nx, :ny, :m] = x
    H = np.conj(op.Hhat) if adjoint else op.Hhat
    return _ifftn(_fftn(pad) * H)[:nx, :ny, :m].real


def apply_A(u: np.ndarray, op: LCTOperator, masked: bool = False) -> np.ndarray:
    """A u = diag(w) S^T H S u (per scan column), via the zero-padded FFT
    convolution; masked=True applies the sampling operator D (A_D = D A)."""
    tau = resample_T(_conv_padded(resample(u, op.S), op, adjoint=False), op.S) * op.w
    if masked:
        tau = tau * op.mask[:, :, None]
    return tau


def apply_AT(tau: np.ndarray, op: LCTOperator, masked: bool = False) -> np.ndarray:
    """A^T tau = S^T H^T S diag(w) tau; H^T is correlation (conjugate spectrum)."""
    y = tau * op.mask[:, :, None] if masked else tau
    y = y * op.w
    return resample_T(_conv_padded(resample(y, op.S), op, adjoint=True), op.S)


# ============================================================================
# Difference operators and the FFT-diagonal solve (Section 3.1, eq. (11))
# ============================================================================

def grad(u: np.ndarray) -> np.ndarray:
    """Periodic forward differences, stacked (3, ...)."""
    return np.stack([np.roll(u, -1, axis=a) - u for a in range(3)])


def grad_adj(p: np.ndarray) -> np.ndarray:
    """nabla^*: the adjoint of grad, minus the backward-difference divergence."""
    return -sum(p[a] - np.roll(p[a], 1, axis=a) for a in range(3))


def div_back(p: np.ndarray) -> np.ndarray:
    return -grad_adj(p)


def laplacian_symbol(shape) -> np.ndarray:
    """Eigenvalues of nabla^* nabla on the periodic grid: sum_d 4 sin^2(pi w_d / n_d)."""
    sig = np.zeros(shape)
    for a, n in enumerate(shape):
        s = 4.0 * np.sin(np.pi * np.arange(n) / n) ** 2
        idx = [None, None, None]
        idx[a] = slice(None)
        sig = sig + s[tuple(idx)]
    return sig


def solve_diag(rhs: np.ndarray, c: float, mu: float) -> np.ndarray:
    """(c I + mu nabla^* nabla)^{-1} rhs by FFT (eq. (11))."""
    return _ifftn(_fftn(rhs) / (c + mu * laplacian_symbol(rhs.shape))).real


# ============================================================================
# Shrinkage, curvature, phi (Section 3, eqs. (6)-(7))
# ============================================================================

def shrink(a: np.ndarray, b) -> np.ndarray:
    """shrinkage(a, b) = max(|a| - b, 0) a / |a| with |.| the Euclidean norm
    over the leading component axis; 0 where |a| = 0."""
    nrm = np.sqrt((a * a).sum(axis=0))
    scale = np.where(nrm > 0, np.maximum(nrm - b, 0.0) / np.where(nrm > 0, nrm, 1.0), 0.0)
    return a * scale


def curvature(u: np.ndarray, eta: float) -> np.ndarray:
    """kappa = div(grad u / |grad u|), regularized by eta where grad u vanishes."""
    g = grad(u)
    nrm = np.sqrt((g * g).sum(axis=0) + eta * eta)
    return div_back(g / nrm)


def phi_of(kappa: np.ndarray, a: float, b: float, kind: int = PHI_TSC) -> np.ndarray:
    if kind == PHI_TSC:
        return a + b * kappa * kappa
    if kind == PHI_TAC:
        return a + b * np.abs(kappa)
    if kind == PHI_TRV:
        return np.sqrt(a + b * kappa * kappa)
    raise ValueError(kind)


def tv_weighted(u: np.ndarray, phi: np.ndarray) -> float:
    g = grad(u)
    return float((phi * np.sqrt((g * g).sum(axis=0))).sum())


# Optional momentum restart (not part of Algorithms 1-2, which print the plain
# extrapolation; enabled by Params.fista_restart): restart the extrapolation
# sequence (t = 1, so the next extrapolation weight is 0) whenever the energy
# of an accepted iterate exceeds the previous one by more than RESTART_TOL
# (function-value restart, O'Donoghue and Candes 2015).  The tolerance keeps
# the decision away from round-off ties.
RESTART_TOL = 1e-3


def momentum_restart(st, E: float) -> None:
    """Reset the FISTA sequence of state ``st`` after an energy rise."""
    if np.isfinite(st.E_prev) and E > st.E_prev * (1.0 + RESTART_TOL):
        st.t = 1.0


def fista_next(t: float) -> float:
    """t^{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2 (Algorithm 1)."""
    return (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0


# ============================================================================
# Measurement normalization, step constant
# ============================================================================

def normalize_measurement(tau_raw: np.ndarray, mask: np.ndarray, falloff: int):
    """Compensated: mask * rhat^3 * tau / max(...).  Literal: mask * tau / max(...)."""
    m = tau_raw.shape[-1]
    y = tau_raw * np.asarray(mask, dtype=np.float64)[:, :, None]
    if falloff == FALLOFF_COMPENSATED:
        y = y * (((np.arange(m) + 0.5) / m) ** 3)
    s = float(y.max())
    if not np.isfinite(s) or s <= 0:
        raise ValueError("measurement has no positive finite value on the kept scan points")
    return y / s, s


def power_norm2(fwd: Callable, adj: Callable, shape, iters: int = 15) -> float:
    """Estimate ||B||^2 = largest eigenvalue of B^T B by power iteration from the
    all-ones vector.  Returns the last ||B^T B x|| with ||x|| = 1."""
    x = np.ones(shape)
    x /= np.linalg.norm(x)
    est = 0.0
    for _ in range(iters):
        y = adj(fwd(x))
        est = float(np.linalg.norm(y))
        if est == 0.0:
            return 0.0
        x = y / est
    return est


# ============================================================================
# Algorithm 1: object-domain curvature ADMM (Section 3.2)
# ============================================================================

@dataclasses.dataclass
class Params:
    a: float = 5e-5
    b: float = 5e-5
    mu: float = 0.1
    phi_kind: int = PHI_TSC
    eta: float = 1e-3
    L0: float = 0.0              # <= 0: 2 * power estimate
    bt: bool = True
    bt_factor: float = 2.0
    bt_max_trials: int = 20
    eps: float = 0.0             # 0 = fixed iteration count
    power_iters: int = 15
    fista_restart: bool = False  # True: function-value restart; False: the printed step
    tau_split_at_bar: bool = False  # Alg. 2: w, f from taubar (the unstable reading)
    # Algorithm 2 (a, b, mu above drive Algorithm 1 and the warm start)
    a_u: float = 5e-4
    b_u: float = 5e-5
    a_tau: float = 3e-3
    b_tau: float = 5e-4
    mu1: float = 1.0
    mu2: float = 800.0
    mu3: float = 2.0
    lam: float = 200.0


class BacktrackingExhausted(RuntimeError):
    pass


@dataclasses.dataclass
class Alg1State:
    u: np.ndarray
    ubar: np.ndarray
    v: np.ndarray
    Lam: np.ndarray
    phi: np.ndarray
    t: float
    L: float
    k: int = 0
    E_prev: float = float("nan")
    log: list = dataclasses.field(default_factory=list)


def alg1_init(shape, p: Params, L: float) -> Alg1State:
    z = np.zeros(shape)
    return Alg1State(u=z.copy(), ubar=z.copy(), v=np.zeros((3,) + shape),
                     Lam=np.zeros((3,) + shape), phi=np.full(shape, p.a), t=1.0, L=L)


def backtrack(fq: Callable, gradf: np.ndarray, f_at_ubar: float, ubar: np.ndarray,
              solve_at: Callable, L: float, p: Params):
    """Beck-Teboulle: accept u+ = solve_at(L) when
    f(u+) <= f(ubar) + <u+ - ubar, grad f(ubar)> + (L/2) ||u+ - ubar||^2,
    otherwise L <- bt_factor L.  Returns (u+, f(u+), L, rejections)."""
    trials = 0
    while True:
        up = solve_at(L)
        fp = fq(up)
        d = up - ubar
        if (not p.bt) or fp <= f_at_ubar + float((d * gradf).sum()) + 0.5 * L * float((d * d).sum()):
            return up, fp, L, trials
        trials += 1
        if trials > p.bt_max_trials:
            raise BacktrackingExhausted(f"no acceptable step after {trials} trials")
        L *= p.bt_factor


def alg1_step(st: Alg1State, tau0: np.ndarray, fwd: Callable, adj: Callable, p: Params) -> None:
    """One iteration of Algorithm 1, at the extrapolated point ubar.

    fwd/adj are A_D and A_D^T (mask included); tau0 is the normalized data,
    zero off the kept scan points.
    """
    mu = p.mu
    # v-subproblem, eq. (7)
    st.v = shrink(grad(st.ubar) - st.Lam / mu, st.phi / mu)
    # linearized u-subproblem, eqs. (9)-(11)
    r = fwd(st.ubar) - tau0
    gf = adj(r)
    f_bar = 0.5 * float((r * r).sum())
    c = -gf + mu * grad_adj(st.v + st.Lam / mu)

    def solve_at(L):
        return solve_diag(L * st.ubar + c, L, mu)

    def fq(x):
        rr = fwd(x) - tau0
        return 0.5 * float((rr * rr).sum())

    u_new, f_new, st.L, trials = backtrack(fq, gf, f_bar, st.ubar, solve_at, st.L, p)
    # multiplier, eq. (12)
    st.Lam = st.Lam + mu * (st.v - grad(u_new))
    # FISTA extrapolation
    t_new = fista_next(st.t)
    ubar = u_new + ((st.t - 1.0) / t_new) * (u_new - st.u)
    u_old = st.u
    st.u, st.ubar, st.t = u_new, ubar, t_new
    # curvature weight refresh
    st.phi = phi_of(curvature(st.u, p.eta), p.a, p.b, p.phi_kind)
    # energy eq. (4), residuals
    E = f_new + tv_weighted(st.u, st.phi)
    gp = st.v - grad(st.u)
    primal = math.sqrt(float((gp * gp).sum()))
    gd = grad(st.u - u_old)
    dual = mu * math.sqrt(float((gd * gd).sum()))
    rel = abs(st.E_prev - E) / abs(E) if np.isfinite(st.E_prev) and E != 0 else float("inf")
    st.log.append((E, primal, dual, st.L, trials, rel))
    if p.fista_restart:
        momentum_restart(st, E)
    st.E_prev = E
    st.k += 1


def run_alg1(tau0, op: LCTOperator, p: Params, iters: int, fwd=None, adj=None,
             L0: Optional[float] = None, state: Optional[Alg1State] = None) -> Alg1State:
    """Algorithm 1 on the masked operator A_D (or on fwd/adj if given)."""
    if fwd is None:
        fwd = lambda x: apply_A(x, op, masked=True)
        adj = lambda y: apply_AT(y, op, masked=True)
    shape = tau0.shape if state is None else state.u.shape
    if state is None:
        if L0 is None:
            L0 = p.L0 if p.L0 > 0 else 2.0 * power_norm2(fwd, adj, shape, p.power_iters)
        state = alg1_init(shape, p, L0)
    for _ in range(iters):
        alg1_step(state, tau0, fwd, adj, p)
        if p.eps > 0 and state.log[-1][5] <= p.eps:
            break
    return state


# ============================================================================
# Algorithm 2: dual-domain (signal + object) curvature ADMM (Section 4.1)
# ============================================================================

@dataclasses.dataclass
class Alg2State:
    u: np.ndarray
    ubar: np.ndarray
    tau: np.ndarray
    taubar: np.ndarray
    v: np.ndarray
    w: np.ndarray
    f: np.ndarray
    Lam1: np.ndarray
    Lam2: np.ndarray
    Lam3: np.ndarray
    phi_u: np.ndarray
    phi_tau: np.ndarray
    t: float
    L: float
    k: int = 0
    E_prev: float = float("nan")
    log: list = dataclasses.field(default_factory=list)


def alg2_init(u0: np.ndarray, p: Params, L: float) -> Alg2State:
    shape = u0.shape
    z = np.zeros(shape)
    return Alg2State(u=u0.copy(), ubar=u0.copy(), tau=z.copy(), taubar=z.copy(),
                     v=np.zeros((3,) + shape), w=np.zeros((3,) + shape), f=z.copy(),
                     Lam1=np.zeros((3,) + shape), Lam2=np.zeros((3,) + shape), Lam3=z.copy(),
                     phi_u=phi_of(curvature(u0, p.eta), p.a_u, p.b_u, p.phi_kind),
                     phi_tau=phi_of(curvature(z, p.eta), p.a_tau, p.b_tau, p.phi_kind),
                     t=1.0, L=L)


def alg2_step(st: Alg2State, tau0: np.ndarray, mask: np.ndarray, fwd: Callable,
              adj: Callable, p: Params) -> None:
    """One iteration of Algorithm 2 at (ubar, taubar).  fwd/adj are the
    unmasked A and A^T; mask selects the measured scan points."""
    mu1, mu2, mu3, lam = p.mu1, p.mu2, p.mu3, p.lam
    D = np.asarray(mask, dtype=np.float64)[:, :, None] * np.ones_like(tau0)
    # v and w: weighted shrinkage on both gradients; the signal-domain
    # splitting steps (w, f) start from the last accepted tau
    ts = st.taubar if p.tau_split_at_bar else st.tau
    st.v = shrink(grad(st.ubar) - st.Lam1 / mu1, st.phi_u / mu1)
    st.w = shrink(grad(ts) - st.Lam2 / mu2, st.phi_tau / mu2)
    # f: pointwise minimizer of lam/2 |f - tau0|^2_D + <Lam3, f - tau> + mu3/2 |f - tau|^2
    st.f = np.where(D > 0, (lam * tau0 + mu3 * ts - st.Lam3) / (lam + mu3), ts - st.Lam3 / mu3)
    # u: linearized data term 1/2 |A u - taubar|^2 at ubar, FFT solve
    r = fwd(st.ubar) - st.taubar
    gf = adj(r)
    f_bar = 0.5 * float((r * r).sum())
    c = -gf + mu1 * grad_adj(st.v + st.Lam1 / mu1)

    def solve_at(L):
        return solve_diag(L * st.ubar + c, L, mu1)

    def fq(x):
        rr = fwd(x) - st.taubar
        return 0.5 * float((rr * rr).sum())

    u_new, _, st.L, trials = backtrack(fq, gf, f_bar, st.ubar, solve_at, st.L, p)
    Au = fwd(u_new)
    # tau: exact quadratic minimization, ((1+mu3) I + mu2 nabla^* nabla) tau = rhs
    rhs = Au + mu3 * st.f + st.Lam3 + mu2 * grad_adj(st.w + st.Lam2 / mu2)
    tau_new = solve_diag(rhs, 1.0 + mu3, mu2)
    # multipliers
    st.Lam1 = st.Lam1 + mu1 * (st.v - grad(u_new))
    st.Lam2 = st.Lam2 + mu2 * (st.w - grad(tau_new))
    st.Lam3 = st.Lam3 + mu3 * (st.f - tau_new)
    # FISTA on u and tau
    t_new = fista_next(st.t)
    beta = (st.t - 1.0) / t_new
    u_old, tau_old = st.u, st.tau
    st.ubar = u_new + beta * (u_new - st.u)
    st.taubar = tau_new + beta * (tau_new - st.tau)
    st.u, st.tau, st.t = u_new, tau_new, t_new
    # curvature weights
    st.phi_u = phi_of(curvature(st.u, p.eta), p.a_u, p.b_u, p.phi_kind)
    st.phi_tau = phi_of(curvature(st.tau, p.eta), p.a_tau, p.b_tau, p.phi_kind)
    # energy eq. (13)
    d1 = Au - st.tau
    d2 = D * (st.tau - tau0)
    E = (0.5 * float((d1 * d1).sum()) + 0.5 * lam * float((d2 * d2).sum())
         + tv_weighted(st.u, st.phi_u) + tv_weighted(st.tau, st.phi_tau))
    gp = st.v - grad(st.u)
    primal = math.sqrt(float((gp * gp).sum()))
    gd = grad(st.u - u_old)
    dual = mu1 * math.sqrt(float((gd * gd).sum()))
    rel = abs(st.E_prev - E) / abs(E) if np.isfinite(st.E_prev) and E != 0 else float("inf")
    st.log.append((E, primal, dual, st.L, trials, rel))
    if p.fista_restart:
        momentum_restart(st, E)
    st.E_prev = E
    st.k += 1


def run_alg2(tau0, op: LCTOperator, p: Params, iters: int, init_iters: int,
             L0_obj: Optional[float] = None, L0_dual: Optional[float] = None):
    """Algorithm 2 warm-started by ``init_iters`` iterations of Algorithm 1
    (remark after Algorithm 2).  Returns (alg1_state, alg2_state)."""
    fwdD = lambda x: apply_A(x, op, masked=True)
    adjD = lambda y: apply_AT(y, op, masked=True)
    fwd = lambda x: apply_A(x, op, masked=False)
    adj = lambda y: apply_AT(y, op, masked=False)
    shape = tau0.shape
    if L0_obj is None:
        L0_obj = p.L0 if p.L0 > 0 else 2.0 * power_norm2(fwdD, adjD, shape, p.power_iters)
    if L0_dual is None:
        L0_dual = p.L0 if p.L0 > 0 else 2.0 * power_norm2(fwd, adj, shape, p.power_iters)
    s1 = alg1_init(shape, p, L0_obj)
    for _ in range(init_iters):
        alg1_step(s1, tau0, fwdD, adjD, p)
    s2 = alg2_init(s1.u, p, L0_dual)
    for _ in range(iters):
        alg2_step(s2, tau0, op.mask, fwd, adj, p)
        if p.eps > 0 and s2.log[-1][5] <= p.eps:
            break
    return s1, s2


# ============================================================================
# Non-confocal model (Section 2), reference only
# ============================================================================
#
# The general model of Section 2 illuminates wall point x_i and detects at
# wall point x_d; light travels d(x_i, x) + d(x, x_d) = t c.  With unit normals
# the direction terms reduce, as in the confocal case, to the volumetric albedo
# weight 1 / (d_i^2 d_d^2).  The oracle discretizes it by direct summation on
# the confocal grid conventions: detector (i, j) at x_i = (i + 1/2) W / n - W/2,
# voxel (p, q, k) at the same lateral positions and depth z_k = (k + 1/2) R / m
# (R = m c dt / 2 as in the confocal model), and time bin b holding path
# lengths in [b, b + 1) c dt.  The illumination point is one fixed wall point
# (the detector grid is scanned).  It is not shift-invariant, so no FFT form
# exists; the midpoint approximation used for the non-confocal experiment of
# Section 5 maps it to the confocal operator (nonconfocal_midpoint_geometry).

@dataclasses.dataclass
class NonConfocalGeometry:
    n: int                 # detector grid n x n (and voxel grid laterally)
    m: int                 # time bins (and depth bins)
    wall: float            # wall extent W (m), square
    bin_ps: float          # time-bin width (ps)
    illum: tuple           # (x, y) of the illumination point on the wall (m)

    def lateral(self) -> np.ndarray:
        return (np.arange(self.n) + 0.5) * self.wall / self.n - self.wall / 2.0

    def depth(self) -> np.ndarray:
        R = range_metres(self.m, self.bin_ps)
        return (np.arange(self.m) + 0.5) * R / self.m

    def bin_length(self) -> float:
        """Path length per time bin, c dt."""
        return C_LIGHT * self.bin_ps * 1e-12


def _nc_paths(g: NonConfocalGeometry, literal: bool = True):
    """For every (detector, voxel): time bin of d_i + d_d (-1 beyond the
    window) and the albedo weight 1 / (d_i^2 d_d^2) (1 when not literal).
    Shapes [n, n, n, n, m] (detector i, j; voxel p, q, k)."""
    x = g.lateral()
    z = g.depth()
    X = x[None, None, :, None, None]
    Y = x[None, None, None, :, None]
    Z = z[None, None, None, None, :]
    di = np.sqrt((X - g.illum[0]) ** 2 + (Y - g.illum[1]) ** 2 + Z ** 2)
    dd = np.sqrt((X - x[:, None, None, None, None]) ** 2
                 + (Y - x[None, :, None, None, None]) ** 2 + Z ** 2)
    L = di + dd
    b = np.floor(L / g.bin_length()).astype(np.int64)
    b = np.where(b < g.m, b, -1)
    w = 1.0 / (di * di * dd * dd) if literal else np.ones_like(L)
    return b, w


def apply_nonconfocal(u: np.ndarray, g: NonConfocalGeometry, literal: bool = True) -> np.ndarray:
    """tau[i, j, b] = sum over voxels of u w, where the voxel's path length
    falls in bin b (direct summation; small grids only)."""
    b, w = _nc_paths(g, literal)
    n, m = g.n, g.m
    tau = np.zeros((n, n, m))
    contrib = w * u[None, None, :, :, :]
    for i in range(n):
        for j in range(n):
            bb = b[i, j].ravel()
            ok = bb >= 0
            tau[i, j] = np.bincount(bb[ok], weights=contrib[i, j].ravel()[ok], minlength=m)[:m]
    return tau


def apply_nonconfocal_T(tau: np.ndarray, g: NonConfocalGeometry, literal: bool = True) -> np.ndarray:
    """The transpose: u[p, q, k] = sum over detectors of w tau[i, j, bin]."""
    b, w = _nc_paths(g, literal)
    n, m = g.n, g.m
    u = np.zeros((n, n, m))
    for i in range(n):
        for j in range(n):
            bb = b[i, j]
            ok = bb >= 0
            u += np.where(ok, w[i, j] * tau[i, j][np.where(ok, bb, 0)], 0.0)
    return u


def nonconfocal_midpoint_geometry(g: NonConfocalGeometry):
    """Midpoint approximation: detector x_d with illumination x_i reads as a
    confocal measurement at x_m = (x_i + x_d) / 2, the path length d_i + d_d
    standing in for 2 d(x_m, x).  The midpoints of a fixed illumination point
    and an n x n detector grid of extent W form an n x n grid of extent W / 2
    centred at (x_i + wall centre) / 2, so the transient array is reused as is
    with the confocal operator of that grid.  Returns (wall extent, (x, y) of
    the grid centre)."""
    return g.wall / 2.0, (g.illum[0] / 2.0, g.illum[1] / 2.0)
