"""CNR / TV / SRR utilities (Sec. 2.5, Eq. (10)) against plain loops and
closed forms (CPU)."""
import numpy as np
import torch

from oracle import metrics_ref
from paper_1201_2450_amd import metrics
from phantom import random_volumes


def test_tv_matches_loops_and_ramp_closed_form():
    h = random_volumes((5, 4, 6), 3)
    assert abs(metrics.tv(torch.from_numpy(h)) - metrics_ref.tv(h)) <= 1e-12 * metrics_ref.tv(h)
    a = 0.37
    ramp = a * np.arange(7.0)[:, None, None] * np.ones((7, 3, 4))
    # |grad| = a wherever a forward difference along x exists
    assert abs(metrics.tv(torch.from_numpy(ramp)) - a * 6 * 3 * 4) <= 1e-12


def test_cnr_matches_definition():
    rng = np.random.default_rng(4)
    vol = rng.normal(0.2, 0.01, size=(8, 8, 8))
    vol[2:5, 2:5, 2:5] += 0.1
    roi = np.zeros(vol.shape, bool)
    roi[2:5, 2:5, 2:5] = True
    bg = np.zeros(vol.shape, bool)
    bg[6:, :, :] = True
    got = metrics.cnr(torch.from_numpy(vol), torch.from_numpy(roi),
                      torch.from_numpy(bg))
    assert abs(got - metrics_ref.cnr(vol, roi, bg)) <= 1e-12


def test_srr_limits():
    t = random_volumes((2, 5, 5, 5), 5)
    fin = t + random_volumes((2, 5, 5, 5), 6, scale=0.1)
    tt, ti = torch.from_numpy(t), torch.from_numpy(fin)
    assert abs(metrics.srr(ti, ti, tt)) <= 1e-12          # nothing removed
    assert abs(metrics.srr(ti, tt, tt) - 1.0) <= 1e-12    # everything removed
    half = 0.5 * (t + fin)
    ref = np.mean([metrics_ref.srr(fin[i], half[i], t[i]) for i in range(2)])
    assert abs(metrics.srr(ti, torch.from_numpy(half), tt) - ref) <= 1e-12


def test_cnr_closed_form_two_level_regions():
    """Regions whose mean and population standard deviation are exact by
    construction: a two-level pattern c +- s with as many + as - voxels has
    mean c and standard deviation s, so CNR = 2|c_roi - c_bg| / (s_roi + s_bg)
    (Sec. 2.5) without evaluating any moment numerically."""
    vol = np.zeros((6, 6, 6))
    roi = np.zeros(vol.shape, bool)
    bg = np.zeros(vol.shape, bool)
    roi[:2] = True          # 72 voxels
    bg[3:] = True           # 108 voxels
    sign = np.where((np.indices(vol.shape).sum(axis=0) % 2) == 0, 1.0, -1.0)
    c_roi, s_roi, c_bg, s_bg = 0.25, 0.0625, 0.125, 0.03125
    vol[roi] = c_roi + s_roi * sign[roi]
    vol[bg] = c_bg + s_bg * sign[bg]
    assert sign[roi].sum() == 0 and sign[bg].sum() == 0
    want = 2 * abs(c_roi - c_bg) / (s_roi + s_bg)   # = 8/3
    assert abs(metrics_ref.cnr(vol, roi, bg) - want) <= 1e-14
    got = metrics.cnr(torch.from_numpy(vol), torch.from_numpy(roi), torch.from_numpy(bg))
    assert abs(got - want) <= 1e-14
    # the sample (n-1) standard deviation would give a different value
    n = roi.sum()
    assert abs(2 * abs(c_roi - c_bg) / (s_roi * np.sqrt(n / (n - 1))
                                        + s_bg * np.sqrt(bg.sum() / (bg.sum() - 1))) - want) > 1e-3
