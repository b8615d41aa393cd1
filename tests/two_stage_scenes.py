"""Seeded scenes for the reliability-aware refinement tests (data only).

The tiny holistic scene with Huber losses on the observation records and gross
outliers planted in all but two observations of chosen features (seen in exactly
bad_obs + 2 views), so that those features have two active observations, fewer
than the reliability test asks for.
"""
import copy

import numpy as np

from scenegen import make_scene, small_config, OBS_POINT, OBS_LINE, LOSS_HUBER


def outlier_scene(seed=101, n_bad_points=8, n_bad_lines=3, bad_obs=3, shift=40.0):
    s = copy.deepcopy(make_scene(small_config(n_cams=9, n_points=70, n_lines=20), seed=seed))
    s["loss"][OBS_POINT] = (LOSS_HUBER, 2.0, 1.0)
    s["loss"][OBS_LINE] = (LOSS_HUBER, 2.0, 1.0)
    rng = np.random.default_rng(seed + 7)
    cam, pt, meas = (np.array(a) for a in s["obs"][OBS_POINT])
    meas = meas.reshape(-1, 4).copy()
    counts = np.bincount(pt, minlength=len(s["points"]))
    bad_pts = rng.choice(np.nonzero(counts == bad_obs + 2)[0], n_bad_points, replace=False)
    for j in bad_pts:
        rows = np.nonzero(pt == j)[0][:bad_obs]
        meas[rows] += np.array([shift, -0.75 * shift, shift, -0.75 * shift])
    s["obs"][OBS_POINT] = (cam, pt, meas)
    cam, ln, meas = (np.array(a) for a in s["obs"][OBS_LINE])
    meas = meas.reshape(-1, 4).copy()
    counts = np.bincount(ln, minlength=len(s["lines"]))
    bad_lns = rng.choice(np.nonzero(counts == bad_obs + 2)[0], n_bad_lines, replace=False)
    for k in bad_lns:
        rows = np.nonzero(ln == k)[0][:bad_obs]
        meas[rows] += np.array([shift, shift, shift, shift])
    s["obs"][OBS_LINE] = (cam, ln, meas)
    return s, np.sort(bad_pts), np.sort(bad_lns)
