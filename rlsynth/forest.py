"""Randomly generated regression-forest structure (split parameters only).

The paper shows that a forest of complete binary trees with random split
functions works as well as a pre-trained one (Sec. "Is Pre-Training
Necessary?"): for each branch node decide Depth vs DA-RGB with probability p
of choosing Depth, then draw the feature's parameters.  The forest carries no
leaf statistics: those come from online adaptation.

Node record (16 bytes, little endian), one per branch node, per tree
``2**depth - 1`` nodes in implicit complete-tree order (children of i are
2i+1 and 2i+2):

    float32 dx, dy   image offset delta (pixel-metres; divided by depth at use)
    float32 tau      split threshold
    uint32  kind     0 = Depth feature, 1 + c = DA-RGB feature on channel c

Offsets are uniform in +-offset_range (px*m).  The thresholds are uniform in
+-tau_depth (metres) for Depth nodes and +-tau_colour (0..255 scale) for
DA-RGB nodes.
"""
from __future__ import annotations

import numpy as np

NODE_DTYPE = np.dtype([("dx", "<f4"), ("dy", "<f4"), ("tau", "<f4"), ("kind", "<u4")])


def make_forest(seed: int, n_trees: int, depth: int, p_depth: float = 0.4,
                offset_range: float = 130.0, tau_depth: float = 0.2,
                tau_colour: float = 64.0) -> np.ndarray:
    """Returns a (n_trees, 2**depth - 1) array of NODE_DTYPE records."""
    if not (1 <= depth <= 15):
        raise ValueError("depth must be in [1, 15]")
    rng = np.random.default_rng(seed)
    nn = (1 << depth) - 1
    out = np.zeros((n_trees, nn), dtype=NODE_DTYPE)
    for t in range(n_trees):
        is_depth = rng.uniform(size=nn) < p_depth
        chan = rng.integers(0, 3, size=nn)
        out["dx"][t] = rng.uniform(-offset_range, offset_range, size=nn).astype(np.float32)
        out["dy"][t] = rng.uniform(-offset_range, offset_range, size=nn).astype(np.float32)
        tau = np.where(is_depth, rng.uniform(-tau_depth, tau_depth, size=nn),
                       rng.uniform(-tau_colour, tau_colour, size=nn))
        out["tau"][t] = tau.astype(np.float32)
        out["kind"][t] = np.where(is_depth, 0, 1 + chan).astype(np.uint32)
    return out


def zero_threshold(forest: np.ndarray) -> np.ndarray:
    """The paper's own random-forest setting: every threshold fixed to 0."""
    f = forest.copy()
    f["tau"] = 0.0
    return f
