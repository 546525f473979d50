"""Shared helpers of the GPU parity tests (inputs from the seeded generators,
expected values from the oracle only)."""
import os
import sys

import numpy as np
import pytest

from oracle import cnlos_oracle as O
from paper_2301_00406_amd import scenes


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_00406_amd import cnlos
    cnlos.load()   # fails loudly when the HIP library is missing
    return torch


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den > 0 else 1.0))


def max_rel(got, ref):
    """Largest elementwise deviation relative to the reference's largest
    magnitude (catches a wrong block edge that one norm could hide)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.abs(ref).max())
    return float(np.abs(got - ref).max() / (den if den > 0 else 1.0))


def f32(x):
    """The float32 value the GPU receives, as float64 for the oracle."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def to_dev(torch, x):
    return torch.tensor(np.asarray(x, dtype=np.float32), device="cuda").contiguous()


def to_host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def synth_measurement(sc, seed):
    """Raw photon counts of a scene: literal-falloff oracle forward model,
    scaled to the scene's peak, Poisson noise from a seeded generator."""
    opL = O.make_operator(sc.n, sc.n, sc.m, sc.wall_w, sc.wall_h, sc.bin_ps, O.FALLOFF_LITERAL)
    clean = O.apply_A(sc.u_true, opL)
    return scenes.poisson_counts(clean, sc.peak, sc.background,
                                 np.random.Generator(np.random.PCG64(seed)))


def sampled_columns_A(u, n, m, wall_w, wall_h, bin_ps, falloff, cols):
    """A u at the listed scan columns by direct summation of the linear
    convolution (the definition), grouping sources by their kernel offset."""
    S = O.resample_matrix(m)
    dq, Z = O.kernel_offsets(n, n, m, wall_w, wall_h, bin_ps)
    w = O.falloff_weights(m, falloff)
    ut = O.resample(u, S)
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    out = {}
    for (i, j) in cols:
        d = dq[i - I + n - 1, j - J + n - 1]
        g = np.zeros(m)
        for q0 in np.unique(d[d >= 0]):
            s = ut[d == q0].sum(axis=0)
            g[q0:] += s[:m - q0]
        out[(i, j)] = O.resample_T(g / Z, S) * w
    return out


def sampled_columns_AT(y, n, m, wall_w, wall_h, bin_ps, falloff, cols):
    """A^T y at the listed columns by direct summation of the correlation."""
    S = O.resample_matrix(m)
    dq, Z = O.kernel_offsets(n, n, m, wall_w, wall_h, bin_ps)
    w = O.falloff_weights(m, falloff)
    z = O.resample(y * w, S)
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    out = {}
    for (i2, j2) in cols:
        d = dq[I - i2 + n - 1, J - j2 + n - 1]
        g = np.zeros(m)
        for q0 in np.unique(d[d >= 0]):
            s = z[d == q0].sum(axis=0)
            g[:m - q0] += s[q0:]
        out[(i2, j2)] = O.resample_T(g / Z, S)
    return out
