"""Image-quality metrics of Sec. 2.5, on GPU tensors.

cnr(vol, roi, bg):  contrast-to-noise ratio 2|S - S_b| / (sigma + sigma_b),
                    S, sigma the mean and standard deviation inside the ROI,
                    S_b, sigma_b in a nearby background region.
tv(h):              total-variation semi-norm sum_x |grad h(x)| with forward
                    differences (zero across the far border), per volume.
srr(f_in, f_out, f_true):  streak-reduction ratio of Eq. (10),
                    (TV(f_in - f*) - TV(f_out - f*)) / TV(f_in - f*).
All accept (Nx, Ny, Nz) or (Np, Nx, Ny, Nz) tensors; for a phase stack the
paper averages per-phase values over the phases (Table 1), which is what
`per_phase=True` returns the parts of.
"""
from __future__ import annotations

import torch


def cnr(vol: torch.Tensor, roi: torch.Tensor, bg: torch.Tensor) -> float:
    v = vol.double()
    s, sb = v[roi], v[bg]
    return float(2.0 * (s.mean() - sb.mean()).abs()
                 / (s.std(unbiased=False) + sb.std(unbiased=False)))


def tv(h: torch.Tensor) -> float:
    """sum over voxels of the Euclidean norm of the forward-difference
    gradient of one volume (Nx, Ny, Nz)."""
    h = h.double()
    gx = torch.zeros_like(h)
    gy = torch.zeros_like(h)
    gz = torch.zeros_like(h)
    gx[:-1] = h[1:] - h[:-1]
    gy[:, :-1] = h[:, 1:] - h[:, :-1]
    gz[:, :, :-1] = h[:, :, 1:] - h[:, :, :-1]
    return float(torch.sqrt(gx * gx + gy * gy + gz * gz).sum())


def srr(f_in: torch.Tensor, f_out: torch.Tensor, f_true: torch.Tensor,
        per_phase: bool = False):
    """Eq. (10); for a phase stack the mean over phases (or the list)."""
    if f_in.dim() == 3:
        a = tv(f_in - f_true)
        return (a - tv(f_out - f_true)) / a
    vals = [srr(f_in[i], f_out[i], f_true[i]) for i in range(f_in.shape[0])]
    return vals if per_phase else sum(vals) / len(vals)
