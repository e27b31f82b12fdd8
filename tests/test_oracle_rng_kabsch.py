"""Oracle pins: the Philox4x32-10 generator and the Kabsch solver.

Philox is checked against rocRAND's independent implementation; Kabsch
(Kabsch 1976, used for the pose hypotheses of Sec. 3.2.3) against exact
recovery of known rigid transforms, the orthonormality and determinant of
its output, least-squares optimality under perturbation, and degenerate
(collinear) inputs.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

HELPER = os.path.join(os.path.dirname(__file__), "helpers", "rocrand_philox_kat.cpp")


@pytest.fixture(scope="module")
def rocrand_kat():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND known-answer helper")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "kat")
    subprocess.run([hipcc, "-O1", "-o", exe, HELPER], check=True, capture_output=True)

    def run(rows):
        inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()],
                        dtype=np.uint64)
    yield run
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(rocrand_kat):
    rng = np.random.default_rng(7)
    rows = [[0, 0, 0, 0, 0, 0], [1, 0, 0, 0, 0, 0], [0, 0, 0, 0, 1, 0]]
    for _ in range(200):
        c = rng.integers(0, 2**32, size=4)
        c[1] = c[1] % (1 << 29)          # the helper encodes counter words 0-1 as offset/4
        k = rng.integers(0, 2**32, size=2)
        rows.append([*c, *k])
    ref = rocrand_kat(rows)
    got = np.array([oracle.philox4x32(r[:4], r[4:]) for r in rows], dtype=np.uint64)
    np.testing.assert_array_equal(got, ref)


def _rand_rot(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a*a+b*b-c*c-d*d, 2*(b*c-a*d), 2*(b*d+a*c)],
                     [2*(b*c+a*d), a*a-b*b+c*c-d*d, 2*(c*d-a*b)],
                     [2*(b*d-a*c), 2*(c*d+a*b), a*a-b*b-c*c+d*d]])


@pytest.mark.parametrize("n", [3, 4, 10, 500])
def test_kabsch_exact_recovery(n):
    rng = np.random.default_rng(n)
    for _ in range(50):
        R = _rand_rot(rng)
        t = rng.uniform(-3, 3, size=3)
        xc = rng.uniform(-2, 2, size=(n, 3)) + np.array([0, 0, 2.0])
        xw = xc @ R.T + t
        ok, R2, t2, sv = oracle.kabsch(xc, xw)
        assert ok
        np.testing.assert_allclose(R2, R, atol=1e-12)
        np.testing.assert_allclose(t2, t, atol=1e-12)


def test_kabsch_orthonormal_det_plus_one_even_for_reflections():
    rng = np.random.default_rng(1)
    for _ in range(200):
        xc = rng.normal(size=(3, 3))
        xw = rng.normal(size=(3, 3))
        if rng.uniform() < 0.5:
            xw = xw * np.array([-1.0, 1.0, 1.0])     # mirrored correspondences
        ok, R, t, sv = oracle.kabsch(xc, xw)
        np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(R) - 1.0) < 1e-12


def test_kabsch_singular_values_are_those_of_the_cross_covariance():
    rng = np.random.default_rng(2)
    for n in (3, 5, 40):
        xc = rng.normal(size=(n, 3))
        xw = rng.normal(size=(n, 3))
        A = (xc - xc.mean(0)).T @ (xw - xw.mean(0))
        _, _, _, sv = oracle.kabsch(xc, xw)
        np.testing.assert_allclose(sv, np.linalg.svd(A, compute_uv=False), rtol=1e-10, atol=1e-12)


def _cost(R, t, xc, xw):
    return float(np.sum((xc @ R.T + t - xw) ** 2))


def test_kabsch_is_least_squares_optimal():
    """No nearby rigid transform has a lower sum of squared residuals."""
    rng = np.random.default_rng(3)
    for n in (3, 8, 100):
        for _ in range(20):
            R0 = _rand_rot(rng)
            xc = rng.uniform(-1, 1, size=(n, 3)) + np.array([0, 0, 2.0])
            xw = xc @ R0.T + rng.uniform(-1, 1, 3) + rng.normal(scale=0.05, size=(n, 3))
            if rng.uniform() < 0.3:
                xw[:, 0] *= -1          # reflected data: best *rotation* still required
            ok, R, t, _ = oracle.kabsch(xc, xw)
            best = _cost(R, t, xc, xw)
            for _ in range(50):
                w = rng.normal(size=3) * rng.choice([1e-3, 1e-2, 1e-1])
                K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
                Rp = R @ (np.eye(3) + np.sin(np.linalg.norm(w)) / max(np.linalg.norm(w), 1e-30) * K
                          + (1 - np.cos(np.linalg.norm(w))) / max(np.linalg.norm(w), 1e-30) ** 2 * K @ K)
                tp = xw.mean(0) - Rp @ xc.mean(0)          # optimal translation for Rp
                assert _cost(Rp, tp, xc, xw) >= best - 1e-9 * max(best, 1.0)
                assert _cost(R, t + rng.normal(scale=1e-3, size=3), xc, xw) >= best - 1e-12


def test_kabsch_point_order_invariance():
    rng = np.random.default_rng(4)
    xc = rng.normal(size=(7, 3))
    xw = rng.normal(size=(7, 3))
    _, R1, t1, _ = oracle.kabsch(xc, xw)
    perm = rng.permutation(7)
    _, R2, t2, _ = oracle.kabsch(xc[perm], xw[perm])
    np.testing.assert_allclose(R1, R2, atol=1e-12)
    np.testing.assert_allclose(t1, t2, atol=1e-12)


def test_kabsch_rejects_collinear_and_coincident():
    xc = np.array([[0, 0, 1.0], [0.3, 0, 1.0], [0.6, 0, 1.0]])
    xw = np.array([[1, 1, 1.0], [1.3, 1, 1.0], [1.6, 1, 1.0]])
    ok, *_ = oracle.kabsch(xc, xw)
    assert not ok
    ok, *_ = oracle.kabsch(np.zeros((3, 3)), np.zeros((3, 3)))
    assert not ok
    # nearly collinear (sigma2/sigma1 ~ 1e-6) rejected, clearly planar accepted
    xc2 = xc.copy()
    xc2[1, 1] = 1e-7
    ok, *_ = oracle.kabsch(xc2, xc2 + 1)
    assert not ok
    xc2[1, 1] = 0.05
    ok, *_ = oracle.kabsch(xc2, xc2 + 1)
    assert ok
