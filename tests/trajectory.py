"""Distances between a trajectory and a reference member, and the FP64 oracle's
own spread under small changes of the rain multiplier: the bar for single-
precision trajectories on ground that sits near h_dry, where each wet/dry
crossing is a branch of the trajectory (one ulp-sized difference can take the
other branch)."""
import numpy as np

TIGHT = np.array([1e-4, 0, 1e-4, 1e-4])   # depth m, cells beyond 1e-4 m, section and edge discharge
PERTURB = (1 + 1e-6, 1 - 1e-6, 1 + 1e-5, 1 - 1e-5)


def divergence(h, qx, qy, ref, dx):
    """[largest depth error, cells beyond 1e-4 m, largest error of the discharge through
    every 4th row / column section, largest error through each edge], the last two
    relative to the largest section discharge of the reference."""
    d = np.abs(h - ref.h)
    sec = lambda a, b: np.concatenate([a[:, ::4].sum(axis=0), b[::4, :].sum(axis=1)]) * dx
    edge = lambda a, b: np.array([b[0].sum(), a[:, -1].sum(), b[-1].sum(), a[:, 0].sum()]) * dx
    sr, er = sec(ref.qx, ref.qy), edge(ref.qx, ref.qy)
    qs = max(np.abs(sr).max(), np.abs(er).max())
    return np.array([d.max(), np.count_nonzero(d > 1e-4), np.abs(sec(qx, qy) - sr).max() / qs,
                     np.abs(edge(qx, qy) - er).max() / qs])


def spread(run, ref, dx):
    """Largest divergence of the reference run's neighbours: run(f) advances the same
    member with its rain multiplier scaled by f."""
    out = np.zeros(4)
    for f in PERTURB:
        p = run(f)
        out = np.maximum(out, divergence(p.h, p.qx, p.qy, ref, dx))
    return out
