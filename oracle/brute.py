"""Brute-force TNLM reference for tiny grids (pure Python + numpy, FP64).

TEST INFRASTRUCTURE ONLY. A second, independent evaluation of the same
definitions as tnlm_oracle.c, written differently on purpose so that the two
can check each other:
  - patches are cut from an edge-padded copy of each phase (np.pad 'edge'),
    i.e. clamp-to-edge extension, and compared as flat vectors;
  - the window is enumerated as the set of grid points whose coordinates
    differ from x by at most M on every axis (no offset loops);
  - with `global_window=True` every grid point of the neighbour phase is a
    candidate: the double integral of Eqs. (2)-(3) over the whole image;
  - gradients come only from central finite differences of the energy.
Paper: Eq. (2) (functional), Eq. (3) (weights), Eq. (8) (Jacobi step),
Sec. 2.4 (patch and search window).
"""
from __future__ import annotations

import itertools

import numpy as np


def patch_matrix(vol3, d):
    """All (2d+1)^3 patches of one phase, clamp-to-edge: (N, P) array."""
    pad = np.pad(vol3, d, mode="edge")
    nx, ny, nz = vol3.shape
    rows = []
    for x, y, z in itertools.product(range(nx), range(ny), range(nz)):
        rows.append(pad[x:x + 2 * d + 1, y:y + 2 * d + 1,
                        z:z + 2 * d + 1].ravel())
    return np.array(rows)


def coords(shape3):
    return np.array(list(itertools.product(*[range(n) for n in shape3])))


def candidate_mask(shape3, M, global_window=False):
    """mask[a, b] = True when grid point b is in the search window of a."""
    c = coords(shape3)
    if global_window:
        return np.ones((len(c), len(c)), dtype=bool)
    diff = np.abs(c[:, None, :] - c[None, :, :]).max(axis=2)
    return diff <= M


def weight_matrices(u, d, M, h, global_window=False):
    """Dense row-normalised weight matrices.

    Returns {(i, j): Wmat} for j in {i+1, i-1} (mod Np) with
    Wmat[a, b] = w_{i->j}(x_a, y_b): exp(-||p_i(x_a) - p_j(y_b)||^2/(2h^2))
    normalised over the candidates b of row a. For Np = 2 both directions
    give the same phase, so the dict is keyed by (i, slot) instead.
    """
    np_ = u.shape[0]
    shape3 = u.shape[1:]
    P = [patch_matrix(u[i], d) for i in range(np_)]
    mask = candidate_mask(shape3, M, global_window)
    out = {}
    for i in range(np_):
        for slot, j in ((0, (i + 1) % np_), (1, (i - 1) % np_)):
            diff = P[i][:, None, :] - P[j][None, :, :]
            ssd = np.einsum("abp,abp->ab", diff, diff)
            logits = np.where(mask, -ssd / (2.0 * h * h), -np.inf)
            mx = logits.max(axis=1, keepdims=True)
            ex = np.exp(logits - mx)
            out[(i, slot)] = ex / ex.sum(axis=1, keepdims=True)
    return out


def jacobi(u, f, g, mu, d, M, h, global_window=False):
    np_ = u.shape[0]
    Wm = weight_matrices(u, d, M, h, global_window)
    out = np.empty_like(f)
    for i in range(np_):
        fp = f[(i + 1) % np_].ravel()
        fm = f[(i - 1) % np_].ravel()
        avg = Wm[(i, 0)] @ fp + Wm[(i, 1)] @ fm
        out[i] = (mu * g[i].ravel() + avg).reshape(f.shape[1:]) / (2.0 + mu)
    return out


def energy(u, f, d, M, h, global_window=False):
    """1/4 sum_i sum_slot sum_{a,b} W[a,b] (f_i(x_a) - f_j(y_b))^2."""
    np_ = u.shape[0]
    Wm = weight_matrices(u, d, M, h, global_window)
    E = 0.0
    for i in range(np_):
        fi = f[i].ravel()
        for slot, j in ((0, (i + 1) % np_), (1, (i - 1) % np_)):
            fj = f[j].ravel()
            R2 = (fi[:, None] - fj[None, :]) ** 2
            E += 0.25 * float((Wm[(i, slot)] * R2).sum())
    return E


def fd_gradients(u, f, d, M, h, eps=1e-6, global_window=False,
                 positions=None):
    """Central differences of energy(): (dE/df, dE/du) at `positions`
    (list of (i, x, y, z); default: every voxel)."""
    if positions is None:
        positions = list(itertools.product(*[range(n) for n in f.shape]))
    gf = np.zeros(len(positions))
    gu = np.zeros(len(positions))
    for k, pos in enumerate(positions):
        for which, out in ((0, gf), (1, gu)):
            a = f.copy() if which == 0 else u.copy()
            a[pos] += eps
            ep = energy(u, a, d, M, h, global_window) if which == 0 else \
                energy(a, f, d, M, h, global_window)
            a[pos] -= 2 * eps
            em = energy(u, a, d, M, h, global_window) if which == 0 else \
                energy(a, f, d, M, h, global_window)
            out[k] = (ep - em) / (2 * eps)
    return gf, gu
