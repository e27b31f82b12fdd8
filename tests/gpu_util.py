"""Helpers shared by the GPU tests: move seeded frames to the device, compare
the HIP path's arrays with the oracle's."""
import numpy as np

import paper_1810_12163_amd as rl


def dev(frame):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(frame.depth)).cuda(),
            torch.from_numpy(np.ascontiguousarray(frame.rgb)).cuda())


def gpu_state(room, T, L, kappa, M):
    seen = room.buffer_np(rl.BUF_SEEN, np.uint32).copy()
    res = room.buffer_np(rl.BUF_RESERVOIR, np.float32).reshape(T * L, kappa, 4)
    nmodes = room.buffer_np(rl.BUF_NMODES, np.uint8).copy()
    modes = room.buffer_np(rl.BUF_MODES, np.float32).reshape(T * L, M, 16)
    return seen, res, nmodes, modes


def reservoir_mismatches(seen, res_gpu, res_oracle_flat, kappa, leaves=None):
    """Count entries (in the filled part of each reservoir) whose bits differ."""
    TL = seen.shape[0]
    ro = res_oracle_flat.reshape(TL, kappa, 4)
    idx = np.arange(TL) if leaves is None else np.asarray(leaves)
    n = np.minimum(seen[idx], kappa)
    mask = np.arange(kappa)[None, :] < n[:, None]
    a = res_gpu[idx].view(np.uint32)
    b = ro[idx].view(np.uint32)
    diff = np.any(a != b, axis=2) & mask
    return int(diff.sum()), int(mask.sum())


def compare_modes(nm_g, modes_g, nm_o, modes_o_flat, M, leaves):
    """Returns (count mismatches, worst relative row error) over the given leaves."""
    mo = modes_o_flat.reshape(-1, M, 16)
    bad_count = 0
    worst = 0.0
    for tl in leaves:
        if nm_g[tl] != nm_o[tl]:
            bad_count += 1
            continue
        k = int(nm_g[tl])
        if k == 0:
            continue
        g = modes_g[tl, :k].astype(np.float64)
        o = mo[tl, :k].astype(np.float64)
        assert np.all(g[:, 3] == o[:, 3]), "cluster sizes differ"
        # mean and colour: absolute float32 resolution; inverse covariance: relative
        worst = max(worst, float(np.max(np.abs(g[:, 0:3] - o[:, 0:3]) / np.maximum(np.abs(o[:, 0:3]), 1.0))))
        worst = max(worst, float(np.max(np.abs(g[:, 10:13] - o[:, 10:13]) / 255.0)))
        sc = np.maximum(np.max(np.abs(o[:, 4:10]), axis=1, keepdims=True), 1e-30)
        worst = max(worst, float(np.max(np.abs(g[:, 4:10] - o[:, 4:10]) / sc)))
    return bad_count, worst


def pose_diff(A, B):
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    return float(np.max(np.abs(A - B)))
