"""Host-side logic of the benchmark script: the image-quality measures of the
curvature-function comparison (Table II's Accuracy, RMSE, PSNR and SSIM), the
roofline figures (flop count, the source-hash gate on measured traffic) and
the one-GPU limit."""
import math

import numpy as np

import bench


def _ssim_direct(x, y, sigma=1.5):
    """SSIM by explicit weighted window sums over a mirror-padded image (the
    padding scipy calls 'reflect': the edge sample repeats)."""
    r = int(3.5 * sigma + 0.5)
    k = np.exp(-0.5 * (np.arange(-r, r + 1) / sigma) ** 2)
    w = np.outer(k, k) / np.outer(k, k).sum()
    xp, yp = np.pad(x, r, mode="symmetric"), np.pad(y, r, mode="symmetric")
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    vals = []
    for i in range(x.shape[0]):
        for j in range(x.shape[1]):
            a, b = xp[i:i + 2 * r + 1, j:j + 2 * r + 1], yp[i:i + 2 * r + 1, j:j + 2 * r + 1]
            mx, my = (w * a).sum(), (w * b).sum()
            vx, vy = (w * (a - mx) ** 2).sum(), (w * (b - my) ** 2).sum()
            cxy = (w * (a - mx) * (b - my)).sum()
            vals.append((2 * mx * my + c1) * (2 * cxy + c2) / ((mx * mx + my * my + c1) * (vx + vy + c2)))
    return float(np.mean(vals))


def test_ssim_matches_direct_window_sums():
    rng = np.random.default_rng(3)
    x = rng.random((17, 13))
    y = np.clip(x + 0.2 * rng.standard_normal(x.shape), 0, 1)
    assert abs(bench._ssim(x, y) - _ssim_direct(x, y)) < 1e-10
    assert abs(bench._ssim(x, x) - 1.0) < 1e-12


def test_image_quality_of_known_images():
    u_true = np.zeros((8, 8, 4))
    u_true[2:5, 3:6, 1] = 2.0
    q = bench.image_quality(3.0 * u_true, u_true)          # any positive scale is exact
    assert q["accuracy"] == 1.0 and q["rmse"] == 0.0 and q["volume_rel_err"] < 1e-15
    assert abs(q["ssim"] - 1.0) < 1e-12
    u = u_true.copy()
    u[0, 0, 0] = 1.0                                        # one stray pixel at half the peak
    q = bench.image_quality(u, u_true)
    assert abs(q["rmse"] - math.sqrt(0.25 / 64)) < 1e-15
    assert abs(q["accuracy"] - (1.0 - 0.5 / 64)) < 1e-15
    assert abs(q["psnr_db"] + 20.0 * math.log10(math.sqrt(0.25 / 64))) < 1e-12


def test_trv_weights_meet_the_other_phis_at_zero_and_infinity():
    pr = dict(a_u=5e-4, b_u=5e-5, a_tau=3e-3, b_tau=5e-4, warm_a=1.5e-4, warm_b=4e-5, mu=0.1,
              lam=200.0)
    t = bench._trv_weights(pr)
    assert t["mu"] == 0.1 and t["lam"] == 200.0
    for a, b in (("a_u", "b_u"), ("a_tau", "b_tau"), ("warm_a", "warm_b")):
        assert math.isclose(math.sqrt(t[a]), pr[a])
        kappa = 1e6
        assert math.isclose(math.sqrt(t[a] + t[b] * kappa ** 2), pr[b] * kappa, rel_tol=1e-6)


def test_more_than_one_gpu_exits_with_a_message():
    """Only one GPU is used: --gpus 2 stops before any device call."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=bench.ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus_requested"] == 2 and "one GPU" in msg["error"]


def test_traffic_is_used_only_for_the_sources_it_was_measured_on(monkeypatch):
    """The counter file carries the hash of the kernel sources it was taken
    with; any other hash, or another workload, gives no traffic figure."""
    import json
    import os
    with open(os.path.join(bench.ROOT, "profiles", "pmc_traffic.json")) as fh:
        d = json.load(fh)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: d["source_hash"])
    got = bench.load_traffic("plane_conv", d["workload"])
    assert got == d["kernels"]["plane_conv"]["bytes_per_launch"]
    assert bench.load_traffic("plane_conv", "large" if d["workload"] != "large" else "medium") is None
    assert bench.load_traffic("no_such_kernel", d["workload"]) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.load_traffic("plane_conv", d["workload"]) is None


def test_plane_pass_flops_count_the_pruned_transforms():
    """Flops of one convolution's plane pass, counted transform by transform:
    per kt plane the padded 2n x 2n transform skips the n zero rows forward
    and the n cropped rows inverse, so n row and 2n column transforms each
    way, 5 L log2 L flops per length-L complex transform, plus 6 flops per
    complex product at the (2n)^2 positions."""
    for n, m in [(8, 16), (16, 128), (64, 512), (128, 1024)]:
        L = 2 * n
        stages = int(round(math.log2(L)))
        per_transform = 0
        for _ in range(stages):          # radix-2: L/2 butterflies of 10 flops per stage
            per_transform += (L // 2) * 10
        schedule = ["row"] * n + ["col"] * L + ["col"] * L + ["row"] * n
        per_plane = len(schedule) * per_transform + 6 * L * L
        assert bench.algorithmic_flops("plane_conv", n, m) == m * per_plane
    assert bench.algorithmic_flops("plane_conv", 64, 512) == 931135488
    assert bench.algorithmic_flops("post", 64, 512) == 0.0


def test_roofline_peaks_and_plane_pass_bytes():
    """The FP32 vector peak is MI355X's published 157.3 TFLOP/s (256 CUs x 4
    SIMDs x 16 lanes x FMA x packed x 2.4 GHz), the non-packed ceiling half of
    it; the plane pass of one convolution at 64x64x512 must move the two
    spectra (m complex planes: the two real planes kt = 0 and kt = m share
    one) plus the quarter of H^ that evenness in kx, ky determines (65 x 65
    per kt plane, kt = 0 .. m), 50.9 MB; the lane-ordered layout reads 4 n^2
    per plane."""
    assert abs(bench.VALU_PEAK_TFLOPS - 157.3) < 0.05
    assert abs(bench.VALU_NONPACKED_TFLOPS - 78.6) < 0.05
    n, m = 64, 512
    assert bench.hq_bytes(n, m) == 65 * 65 * 513 * 8
    assert bench.hq_bytes(n, m, layout=True) == 4 * 64 * 64 * 513 * 8
    b = bench.algorithmic_bytes("plane_conv", n, m, True)
    assert b == 2 * 512 * 4096 * 8 + 65 * 65 * 513 * 8
    assert abs(b / 1e6 - 50.89) < 0.01
