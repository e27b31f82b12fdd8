"""Input generator checks for the robustness protocols: the corrupted
640x480 workload reproduces the standard frames at the standard settings,
masks the requested fraction of pixels and scales its noise with depth."""
import numpy as np

from rlsynth import scene, workloads


def test_default_settings_reproduce_the_standard_frames():
    a = workloads.c2(0, n_adapt=2, n_queries=1)
    b = workloads.c2_corrupted(0, n_adapt=2, n_queries=1)
    for x, y in zip(a.adapt + a.queries, b.adapt + b.queries):
        assert np.array_equal(x.depth, y.depth) and np.array_equal(x.rgb, y.rgb) and np.array_equal(x.pose, y.pose)


def test_missing_depth_fraction_and_depth_dependent_noise():
    clean = workloads.c2_corrupted(0, n_adapt=1, n_queries=0, dropout=0.0)
    f = clean.adapt[0]
    z, _, _ = scene.raycast(clean.room, f.pose, 640, 480, f.K)
    inr = np.isfinite(z) & (z >= scene.DEPTH_MIN) & (z <= scene.DEPTH_MAX)
    for p in (0.3, 0.9):
        m = workloads.c2_corrupted(0, n_adapt=1, n_queries=0, dropout=p).adapt[0]
        lost = np.mean(m.depth[inr] == 0)
        assert abs(lost - p) < 0.01, (p, lost)
    sig = 0.05
    n = workloads.c2_corrupted(0, n_adapt=1, n_queries=0, dropout=0.0, depth_rel_sigma=sig).adapt[0]
    ok = inr & (n.depth > 0)
    rel = (n.depth[ok] - z[ok]) / z[ok]          # includes the 2 mm additive noise
    assert abs(np.std(rel) - sig) < 0.005 and abs(np.mean(rel)) < 0.002
