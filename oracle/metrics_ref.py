"""Plain numpy CNR / TV / SRR (Sec. 2.5, Eq. (10)) for checking the GPU
metric utilities. TEST INFRASTRUCTURE ONLY."""
import numpy as np


def cnr(vol, roi, bg):
    s, sb = vol[roi], vol[bg]
    return 2.0 * abs(s.mean() - sb.mean()) / (s.std() + sb.std())


def tv(h):
    """sum_x |grad h(x)|, forward differences, zero beyond the last voxel."""
    tot = 0.0
    nx, ny, nz = h.shape
    for x in range(nx):
        for y in range(ny):
            for z in range(nz):
                gx = h[x + 1, y, z] - h[x, y, z] if x + 1 < nx else 0.0
                gy = h[x, y + 1, z] - h[x, y, z] if y + 1 < ny else 0.0
                gz = h[x, y, z + 1] - h[x, y, z] if z + 1 < nz else 0.0
                tot += (gx * gx + gy * gy + gz * gz) ** 0.5
    return tot


def srr(f_in, f_out, f_true):
    a = tv(f_in - f_true)
    return (a - tv(f_out - f_true)) / a
