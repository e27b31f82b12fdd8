"""Oracle pins for the Levenberg-Marquardt pose refinement in se(3)
(Sec. 3.2.3, step (ii) of each preemptive-RANSAC iteration): the exponential
map against the matrix exponential, the normal equations' gradient against
finite differences of E, convergence to the generating pose on exact
correspondences (Euclidean and Mahalanobis, with outliers), monotone energy,
and the RANSAC bookkeeping with zero iterations against the incremental
energies."""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle

W, H = 32, 24
K = (np.float32(30.0), np.float32(30.0), np.float32(16.0), np.float32(12.0))
D = 10                      # one leaf per pixel (W * H <= 2^D), one tree
M = 2


def twist(xi):
    w, v = xi[:3], xi[3:]
    X = np.zeros((4, 4))
    X[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    X[:3, 3] = v
    return X


@pytest.mark.parametrize("scale", [0.0, 1e-7, 3e-5, 2e-4, 0.05, 0.7, 2.5])
def test_se3_exp_equals_the_matrix_exponential(scale):
    rng = np.random.default_rng(int(scale * 1e7) % 1000)
    xi = rng.normal(size=6)
    xi[:3] *= scale / max(np.linalg.norm(xi[:3]), 1e-300)
    R, t = oracle.se3_exp(xi)
    E = scipy.linalg.expm(twist(xi))
    np.testing.assert_allclose(R, E[:3, :3], rtol=0, atol=1e-13)
    np.testing.assert_allclose(t, E[:3, 3], rtol=0, atol=1e-13)


def rot(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    return scipy.linalg.expm(ang * np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]],
                                               [-axis[1], axis[0], 0]]))


def scene(seed, outliers=0.0, anisotropic=False, second_mode=False):
    """A frame whose every pixel has its own leaf; the first mode of pixel p is
    H_true x^C(p) (exact up to float32), optionally a far second mode; a
    fraction of pixels gets a wrong first mode."""
    rng = np.random.default_rng(seed)
    depth = rng.uniform(1.0, 3.0, size=(H, W)).astype(np.float32)
    Rt = rot(rng.normal(size=3), rng.uniform(0.2, 1.0))
    tt = rng.normal(size=3)
    P = W * H
    leaves = np.arange(P, dtype=np.uint16).reshape(P, 1)
    nmodes = np.zeros(1 << D, np.uint8)
    nmodes[:P] = 2 if second_mode else 1
    modes = np.zeros((1 << D, M, 16), np.float32)
    fx, fy, cx, cy = [float(v) for v in K]
    bad = rng.uniform(size=P) < outliers
    for p in range(P):
        x, y = p % W, p // W
        d = float(depth[y, x])
        xc = np.array([d * ((x - cx) / fx), d * ((y - cy) / fy), d])
        mu = Rt @ xc + tt
        if bad[p]:
            mu = mu + rng.normal(size=3) * 0.5
        modes[p, 0, 0:3] = mu
        if anisotropic:
            A = rng.normal(size=(3, 3))
            Si = A @ A.T + 0.5 * np.eye(3)
        else:
            Si = np.eye(3)
        modes[p, 0, 4:10] = [Si[0, 0], Si[0, 1], Si[0, 2], Si[1, 1], Si[1, 2], Si[2, 2]]
        modes[p, 1, 0:3] = mu + 5.0
        modes[p, 1, 4:10] = modes[p, 0, 4:10]
    I = rng.integers(0, P, size=300).astype(np.int32)
    return depth, leaves, nmodes, modes.reshape(-1), I, Rt, tt


def perturb(Rt, tt, deg, cm, seed):
    rng = np.random.default_rng(seed)
    R0 = rot(rng.normal(size=3), math.radians(deg)) @ Rt
    t0 = tt + rng.normal(size=3) / np.sqrt(3) * cm / 100
    return np.concatenate([R0.reshape(-1), t0])


def pose_err(p, Rt, tt):
    R = p[:9].reshape(3, 3)
    c = np.clip((np.trace(R.T @ Rt) - 1) / 2, -1, 1)
    return np.linalg.norm(p[9:] - tt), math.degrees(math.acos(c))


@pytest.mark.parametrize("use_cov,aniso", [(0, False), (1, True)])
def test_gradient_of_the_normal_equations_is_the_gradient_of_E(use_cov, aniso):
    depth, leaves, nm, modes, I, Rt, tt = scene(1, anisotropic=aniso, second_mode=True)
    p0 = perturb(Rt, tt, 2.0, 3.0, 7)
    E0, N, g = oracle.lm_linearise(depth, K, leaves, nm, modes, 1, D, M, I, p0, use_cov)
    num = np.zeros(6)
    h = 1e-6
    for i in range(6):
        for sgn in (1, -1):
            xi = np.zeros(6)
            xi[i] = sgn * h
            Rd, td = oracle.se3_exp(xi)
            R = Rd @ p0[:9].reshape(3, 3)
            t = Rd @ p0[9:] + td
            E = oracle.lm_linearise(depth, K, leaves, nm, modes, 1, D, M, I,
                                    np.concatenate([R.reshape(-1), t]), use_cov)[0]
            num[i] += sgn * E / (2 * h)
    np.testing.assert_allclose(g, num, rtol=1e-5, atol=1e-6 * np.abs(num).max())
    np.testing.assert_allclose(N, N.T, rtol=1e-12, atol=1e-9)
    assert np.linalg.eigvalsh(N).min() > 0


@pytest.mark.parametrize("use_cov,aniso,outliers", [(0, False, 0.0), (1, True, 0.0), (1, True, 0.2),
                                                    (0, False, 0.2)])
def test_converges_to_the_generating_pose(use_cov, aniso, outliers):
    depth, leaves, nm, modes, I, Rt, tt = scene(2, outliers, aniso, second_mode=True)
    p0 = perturb(Rt, tt, 3.0, 5.0, 3)
    E0, _, _ = oracle.lm_linearise(depth, K, leaves, nm, modes, 1, D, M, I, p0, use_cov)
    E, p = oracle.lm_refine(depth, K, leaves, nm, modes, 1, D, M, I, p0, use_cov, iters=30)
    dt, dr = pose_err(p, Rt, tt)
    assert E < E0
    assert dt < 1e-4 and dr < 1e-3, (dt, dr)
    np.testing.assert_allclose(p[:9].reshape(3, 3) @ p[:9].reshape(3, 3).T, np.eye(3), atol=1e-12)
    # the returned energy is E at the returned pose
    assert E == oracle.lm_linearise(depth, K, leaves, nm, modes, 1, D, M, I, p, use_cov)[0]


def test_energy_never_increases_and_zero_iterations_keep_the_pose():
    depth, leaves, nm, modes, I, Rt, tt = scene(3, 0.3, True, second_mode=True)
    p0 = perturb(Rt, tt, 8.0, 20.0, 5)
    E0 = oracle.lm_linearise(depth, K, leaves, nm, modes, 1, D, M, I, p0, 1)[0]
    E, p = oracle.lm_refine(depth, K, leaves, nm, modes, 1, D, M, I, p0, 1, iters=0)
    assert E == E0 and np.array_equal(p, p0)
    last = E0
    for it in (1, 2, 3, 5, 8):
        E, _ = oracle.lm_refine(depth, K, leaves, nm, modes, 1, D, M, I, p0, 1, iters=it)
        assert E <= last
        last = E


def _ideal(seed):
    from tests import ideal_scene
    sc = ideal_scene.build(seed=seed)
    return sc, dict(sc["params"], final_refine=0)


def _estimate(sc, p, seed=3):
    return oracle.estimate_pose(sc["depth"], sc["rgb"], sc["K"], sc["leaves"], sc["nmodes"], sc["modes"],
                                sc["T"], sc["D"], sc["M"], p, request_seed=seed)


def test_ransac_with_zero_lm_iterations_matches_the_incremental_energies():
    """With pose_update on and no LM iterations each later round re-scores the
    whole cumulative I at unchanged poses: the same survivors and, up to
    summation order, the same energies as the incremental path."""
    sc, base = _ideal(11)
    a = _estimate(sc, dict(base, pose_update=0))
    b = _estimate(sc, dict(base, pose_update=1, lm_iterations=0))
    assert a["rounds"] == b["rounds"] >= 3
    for ra, rb in zip(a["round_slots"], b["round_slots"]):
        np.testing.assert_array_equal(ra, rb)
    for ea, eb in zip(a["round_energy"], b["round_energy"]):
        np.testing.assert_allclose(ea, eb, rtol=1e-12, atol=0)
    np.testing.assert_array_equal(a["pose"], b["pose"])


def test_ransac_with_lm_returns_the_true_pose_and_lowers_energies():
    """On the ideal forest output every round's refinement can only lower a
    survivor's energy over the same pixels, and the winner is the true pose."""
    sc, base = _ideal(12)
    a = _estimate(sc, dict(base, pose_update=0))
    b = _estimate(sc, dict(base, pose_update=1, lm_iterations=10))
    assert b["status"] == "ok" and b["rounds"] == a["rounds"]
    dt, dr = pose_err(np.concatenate([b["pose"][:3, :3].reshape(-1), b["pose"][:3, 3]]),
                      sc["H"][:3, :3], sc["H"][:3, 3])
    assert dt < 1e-3 and dr < 0.05, (dt, dr)
    # round 0 is the same initial scoring; later energies are over the same
    # cumulative pixels at refined poses, so the best can only be lower
    np.testing.assert_array_equal(a["round_slots"][0], b["round_slots"][0])
    for r in range(1, b["rounds"]):
        assert b["round_energy"][r][0] <= a["round_energy"][r][0] * (1 + 1e-12)
