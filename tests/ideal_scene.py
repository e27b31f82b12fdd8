"""A constructed 'ideal' forest output for pinning pose estimation.

Every valid pixel u of a noise-free frame gets its own leaf whose modes are
the exact world point of u under the true pose (one mode, at a random
position in the leaf's list) plus random distractor points elsewhere in the
room.  Then Eq. 5 vanishes at the true pose up to float32 storage rounding,
every hypothesis built from correct modes equals the true pose, and a correct
relocaliser must return the true pose.
"""
import numpy as np

from rlsynth import scene


def build(seed=0, w=48, h=36, M=4, n_correct=1, dropout=0.0, inv_sigma2=1e4,
          colour_noise=0):
    rng = np.random.default_rng(seed)
    room = scene.make_room(seed)
    H = scene.random_pose(room, rng)
    K = scene.intrinsics(w, h)
    depth, rgb = scene.render(room, H, w, h, seed=seed + 77, noise_sigma=0.0, dropout=dropout)
    D = int(np.ceil(np.log2(w * h + 1)))
    L = 1 << D
    T = 1
    leaves = np.full((w * h, 1), 0xFFFF, dtype=np.uint16)
    nmodes = np.zeros(T * L, dtype=np.uint8)
    modes = np.zeros(T * L * M * 16, dtype=np.float32).reshape(T * L, M, 16)
    fx, fy, cx, cy = [float(v) for v in K]
    truth = {}
    for p in range(w * h):
        d = float(depth.reshape(-1)[p])
        if not d > 0:
            continue
        x, y = p % w, p // w
        xc = np.array([d * (x - cx) / fx, d * (y - cy) / fy, d])
        xw = H[:3, :3] @ xc + H[:3, 3]
        leaves[p, 0] = p
        nmodes[p] = M
        correct = set(rng.choice(M, size=n_correct, replace=False).tolist())
        for m in range(M):
            row = modes[p, m]
            if m in correct:
                row[0:3] = xw
                row[10:13] = np.clip(rgb.reshape(-1, 3)[p].astype(np.float64)
                                     + rng.integers(-colour_noise, colour_noise + 1, size=3), 0, 255)
            else:
                row[0:3] = rng.uniform([0, 0, 0], [4, 4, 3])
                row[10:13] = rng.integers(0, 256, size=3)
            row[3] = 20.0
            row[4] = row[7] = row[9] = inv_sigma2      # isotropic inverse covariance
        truth[p] = xw
    params = dict(max_pose_candidates=64, max_candidate_generation_iterations=2000,
                  max_colour_linf=30.0, min_squared_distance_between_sampled_modes=0.09,
                  max_translation_error_for_correct_pose=0.05, seed=seed,
                  ransac_inliers_per_iteration=50, max_relocalisations_to_output=1,
                  max_pose_candidates_after_cull=64, use_prediction_covariance=1,
                  final_refine=1, inlier_threshold=0.05)
    return dict(room=room, H=H, K=K, depth=depth, rgb=rgb, leaves=leaves, nmodes=nmodes,
                modes=modes.reshape(-1), T=T, D=D, M=M, params=params, truth=truth, w=w, h=h)
