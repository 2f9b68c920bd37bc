"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these compares the oracle with itself: each check is a closed form,
an invariant of the definitions, a special case that reduces to a textbook
routine, or the independent brute force in oracle/brute.py (which evaluates
the double integral of Eqs. (2)-(3) with dense matrices, and gradients only by
finite differences). A plausible slip in the oracle (dropped term, wrong
offset sign, swapped direction slot, wrong normaliser axis, wrong exponent
factor, wrong border rule) fails at least one of them.
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import brute, oracle
from phantom import random_volumes, scaled_phantom

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rnd(shape, seed, scale=0.3):
    return random_volumes(shape, seed, scale=scale)


def valid_count(shape3, M):
    """|V(v)| for every voxel: product over axes of in-grid offsets."""
    out = np.ones(shape3)
    for a, n in enumerate(shape3):
        c = np.arange(n)
        cnt = np.minimum(c + M, n - 1) - np.maximum(c - M, 0) + 1
        sh = [1, 1, 1]
        sh[a] = n
        out = out * cnt.reshape(sh)
    return out


def offsets(M):
    r = range(-M, M + 1)
    return list(itertools.product(r, r, r))


# --------------------------------------------------------------------------
# Weights: Eq. (3) with the per-voxel normaliser, Eq. (9) weight source
# --------------------------------------------------------------------------
@pytest.mark.parametrize("np_,d,M", [(2, 1, 1), (3, 0, 2), (4, 1, 2)])
def test_weights_rows_sum_to_one(np_, d, M):
    u = rnd((np_, 5, 4, 6), 10 + M)
    w, lse = oracle.weights(u, d, M, 0.25)
    s = w.sum(axis=2)
    assert np.abs(s - 1.0).max() <= 1e-14


def test_weights_zero_outside_grid_and_uniform_at_large_h():
    shape = (3, 5, 4, 6)
    M = 2
    u = rnd(shape, 3)
    w, _ = oracle.weights(u, 1, M, 1e6)
    cnt = valid_count(shape[1:], M).ravel()
    offs = offsets(M)
    nx, ny, nz = shape[1:]
    X, Y, Z = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                          indexing="ij")
    for k, (ox, oy, oz) in enumerate(offs):
        inside = ((X + ox >= 0) & (X + ox < nx) & (Y + oy >= 0)
                  & (Y + oy < ny) & (Z + oz >= 0) & (Z + oz < nz)).ravel()
        wk = w[:, :, k, :]
        assert np.all(wk[:, :, ~inside] == 0.0)
        # h -> infinity: every valid candidate gets 1/|V(v)|
        np.testing.assert_allclose(wk[:, :, inside],
                                   np.broadcast_to(1.0 / cnt[inside],
                                                   wk[:, :, inside].shape),
                                   rtol=1e-9, atol=0)


def test_unnormalised_kernel_is_symmetric_between_linked_phases():
    """K_{i,i+1}(v, delta) = K_{i+1,i}(v+delta, -delta) (Sec. 2.4: the
    weight is shared by the two voxels up to the normalisation factors)."""
    shape = (3, 4, 5, 4)
    M = 2
    u = rnd(shape, 7)
    w, lse = oracle.weights(u, 1, M, 0.2)
    logK = np.log(np.maximum(w, 1e-300)) + lse[:, :, None, :]
    nx, ny, nz = shape[1:]
    S = 2 * M + 1
    for i in range(shape[0]):
        j = (i + 1) % shape[0]
        for (ox, oy, oz) in offsets(M):
            k = ((ox + M) * S + (oy + M)) * S + (oz + M)
            kb = ((-ox + M) * S + (-oy + M)) * S + (-oz + M)
            for x, y, z in itertools.product(range(nx), range(ny), range(nz)):
                if not (0 <= x + ox < nx and 0 <= y + oy < ny
                        and 0 <= z + oz < nz):
                    continue
                v = (x * ny + y) * nz + z
                vb = ((x + ox) * ny + (y + oy)) * nz + (z + oz)
                a = logK[i, 0, k, v]
                b = logK[j, 1, kb, vb]
                assert abs(a - b) <= 1e-12 * max(1.0, abs(a))


def test_shifted_copy_makes_weights_one_hot_at_the_shift():
    """f_{i+1}(q) = f_i(q - t): for interior voxels D(v, t) = 0 is the unique
    minimum, so as h -> 0 the weight towards i+1 concentrates on delta = t and
    the one towards i-1 on delta = -t. Pins the offset sign and the slots."""
    rng = np.random.default_rng(5)
    nx, ny, nz, M, d = 9, 9, 9, 2, 1
    t = (1, -2, 1)
    big = rng.uniform(0, 1, size=(nx + 8, ny + 8, nz + 8))
    u = np.empty((2, nx, ny, nz))
    u[0] = big[4:4 + nx, 4:4 + ny, 4:4 + nz]
    u[1] = big[4 - t[0]:4 - t[0] + nx, 4 - t[1]:4 - t[1] + ny,
               4 - t[2]:4 - t[2] + nz]
    # u[1](q) = big(q - t + 4) = u[0](q - t)
    w, _ = oracle.weights(u, d, M, 0.02)
    S = 2 * M + 1
    k_t = ((t[0] + M) * S + (t[1] + M)) * S + (t[2] + M)
    k_mt = ((-t[0] + M) * S + (-t[1] + M)) * S + (-t[2] + M)
    def clean(pt):  # every patch voxel of pt lies inside the grid
        return all(d <= c <= n - 1 - d for c, n in zip(pt, (nx, ny, nz)))

    interior = [(x * ny + y) * nz + z
                for x, y, z in itertools.product(range(nx), range(ny),
                                                 range(nz))
                if clean((x, y, z)) and clean((x + t[0], y + t[1], z + t[2]))]
    assert len(interior) > 20
    interior = np.array(interior)
    # phase 0 -> phase 1 (slot 0) peaks at +t; phase 1 -> phase 0 at -t
    assert np.all(w[0, 0, k_t, interior] > 0.999)
    # Np = 2: slot 1 of phase 0 is also phase 1
    assert np.all(w[0, 1, k_t, interior] > 0.999)
    # from phase 1 the matching voxel of phase 0 sits at q - t
    interior1 = [(x * ny + y) * nz + z
                 for x, y, z in itertools.product(range(nx), range(ny),
                                                  range(nz))
                 if clean((x, y, z)) and clean((x - t[0], y - t[1], z - t[2]))]
    interior1 = np.array(interior1)
    assert np.all(w[1, 0, k_mt, interior1] > 0.999)
    # and the neighbour average then returns the shifted copy exactly
    f = u.copy()
    J = oracle.jacobi(u, f, np.zeros_like(f), 1e-9, d, M, 0.02)
    got = J[0].ravel()[interior] * (2 + 1e-9) / 2
    np.testing.assert_allclose(got, u[0].ravel()[interior], atol=1e-9)


@pytest.mark.parametrize("np_,d", [(2, 1), (3, 0), (3, 1)])
def test_full_window_equals_global_double_integral(np_, d):
    """M >= max(N)-1 makes the window the whole grid: the windowed operator
    must equal the O(N^6) double integral of Eqs. (2)-(3) (brute force)."""
    shape = (np_, 4, 4, 4)
    u, f, g = rnd(shape, 1), rnd(shape, 2), rnd(shape, 3)
    h = 0.35
    E = oracle.energy(u, f, d, 3, h)
    Eb = brute.energy(u, f, d, 3, h, global_window=True)
    assert abs(E - Eb) <= 1e-13 * abs(Eb)
    J = oracle.jacobi(u, f, g, 0.6, d, 3, h)
    Jb = brute.jacobi(u, f, g, 0.6, d, 3, h, global_window=True)
    assert np.abs(J - Jb).max() <= 1e-13


@pytest.mark.parametrize("np_,d,M", list(itertools.product((2, 3, 4), (0, 1),
                                                            (0, 1, 2))))
def test_windowed_against_brute_force(np_, d, M):
    shape = (np_, 4, 4, 4)
    u, f, g = rnd(shape, 11), rnd(shape, 12), rnd(shape, 13)
    h = 0.3
    assert abs(oracle.energy(u, f, d, M, h) - brute.energy(u, f, d, M, h)) \
        <= 1e-13 * brute.energy(u, f, d, M, h)
    J = oracle.jacobi(u, f, g, 0.8, d, M, h)
    assert np.abs(J - brute.jacobi(u, f, g, 0.8, d, M, h)).max() <= 1e-13
    w, _ = oracle.weights(u, d, M, h)
    Wm = brute.weight_matrices(u, d, M, h)
    # row a of the dense matrix restricted to the window equals w[:, :, k, a]
    S = 2 * M + 1
    nx, ny, nz = shape[1:]
    for i, slot in itertools.product(range(np_), range(2)):
        for a, (x, y, z) in enumerate(itertools.product(range(nx), range(ny),
                                                        range(nz))):
            for (ox, oy, oz) in offsets(M):
                k = ((ox + M) * S + (oy + M)) * S + (oz + M)
                if 0 <= x + ox < nx and 0 <= y + oy < ny and 0 <= z + oz < nz:
                    b = ((x + ox) * ny + (y + oy)) * nz + (z + oz)
                    assert abs(w[i, slot, k, a] - Wm[(i, slot)][a, b]) <= 1e-14


# --------------------------------------------------------------------------
# Gauss-Jacobi step, Eq. (8)
# --------------------------------------------------------------------------
def test_constant_volume_is_fixed_point():
    shape = (3, 5, 4, 6)
    c = 0.37
    f = np.full(shape, c)
    for u in (f, rnd(shape, 4)):  # any weight source
        J = oracle.jacobi(u, f, f, 0.5, 1, 2, 0.1)
        assert np.abs(J - c).max() <= 1e-15


def test_jacobi_affine_and_scale_equivariance():
    shape = (3, 4, 5, 4)
    u, f, g = rnd(shape, 21), rnd(shape, 22), rnd(shape, 23)
    d, M, h, mu = 1, 2, 0.2, 0.7
    J = oracle.jacobi(u, f, g, mu, d, M, h)
    c = 1.25
    Jc = oracle.jacobi(u + 0.3, f + c, g + c, mu, d, M, h)
    np.testing.assert_allclose(Jc, J + c, atol=1e-13)
    a = 2.5
    Ja = oracle.jacobi(a * u, a * f, a * g, mu, d, M, a * h)
    np.testing.assert_allclose(Ja, a * J, atol=1e-13)


def test_jacobi_is_a_convex_combination():
    """f+ lies between the min and max of g_i(v) and the neighbour values in
    the window (weights >= 0, mu/(2+mu) + 2/(2+mu) = 1)."""
    shape = (3, 5, 5, 5)
    u, f, g = rnd(shape, 31), rnd(shape, 32), rnd(shape, 33)
    M = 1
    J = oracle.jacobi(u, f, g, 0.4, 1, M, 0.15)
    np_, nx, ny, nz = shape
    for i, x, y, z in itertools.product(range(np_), range(nx), range(ny),
                                        range(nz)):
        vals = [g[i, x, y, z]]
        for j in ((i + 1) % np_, (i - 1) % np_):
            vals.extend(f[j, max(x - M, 0):x + M + 1, max(y - M, 0):y + M + 1,
                          max(z - M, 0):z + M + 1].ravel())
        assert min(vals) - 1e-14 <= J[i, x, y, z] <= max(vals) + 1e-14


def test_jacobi_converges_to_dense_solve_of_optimality_condition():
    """Frozen weights: iterating Eq. (8) converges (Sec. 2.3, any mu > 0) to
    the solution of Eq. (7), ((2+mu) I - W) f = mu g, solved densely; the
    error contracts by 2/(2+mu) per step in the max norm."""
    shape = (3, 4, 4, 4)
    u, g = rnd(shape, 41), rnd(shape, 42)
    d, M, h, mu = 1, 1, 0.2, 0.5
    w, _ = oracle.weights(u, d, M, h)
    np_ = shape[0]
    N = 64
    S = 2 * M + 1
    Wd = np.zeros((np_ * N, np_ * N))
    nx, ny, nz = shape[1:]
    for i, slot in itertools.product(range(np_), range(2)):
        j = (i + 1) % np_ if slot == 0 else (i - 1) % np_
        for a, (x, y, z) in enumerate(itertools.product(range(nx), range(ny),
                                                        range(nz))):
            for (ox, oy, oz) in offsets(M):
                if 0 <= x + ox < nx and 0 <= y + oy < ny and 0 <= z + oz < nz:
                    k = ((ox + M) * S + (oy + M)) * S + (oz + M)
                    b = ((x + ox) * ny + (y + oy)) * nz + (z + oz)
                    Wd[i * N + a, j * N + b] += w[i, slot, k, a]
    fstar = np.linalg.solve((2 + mu) * np.eye(np_ * N) - Wd, mu * g.ravel())
    f = g.copy()
    err_prev = np.abs(f.ravel() - fstar).max()
    for it in range(500):
        f = oracle.jacobi(u, f, g, mu, d, M, h)
        err = np.abs(f.ravel() - fstar).max()
        if it < 20:
            assert err <= 2 / (2 + mu) * err_prev + 1e-15
        err_prev = err
    assert err <= 1e-12


def test_jacobi_equals_eq6_rearranged():
    """Eq. (8) is Eq. (6) set to zero and solved for f_i:
    J(f) = f - (mu (f - g) + G6(f)) / (2 + mu)."""
    shape = (4, 4, 5, 3)
    u, f, g = rnd(shape, 51), rnd(shape, 52), rnd(shape, 53)
    d, M, h, mu = 1, 2, 0.25, 0.9
    J = oracle.jacobi(u, f, g, mu, d, M, h)
    G6 = oracle.grad_eq6(u, f, d, M, h)
    np.testing.assert_allclose(J, f - (mu * (f - g) + G6) / (2 + mu),
                               atol=1e-14)


def test_per_phase_constants_closed_form_golden():
    with open(os.path.join(GOLDEN, "per_phase_constants.json")) as fh:
        gold = json.load(fh)
    shape = tuple(gold["shape"])
    c = np.array(gold["c"])
    cg = np.array(gold["g"])
    f = np.broadcast_to(c[:, None, None, None], shape).copy()
    g = np.broadcast_to(cg[:, None, None, None], shape).copy()
    d, M, h, mu = gold["d"], gold["M"], gold["h"], gold["mu"]
    E = oracle.energy(f, f, d, M, h)
    assert abs(E - gold["energy"]) <= 1e-13
    J = oracle.jacobi(f, f, g, mu, d, M, h)
    np.testing.assert_allclose(J[:, 0, 0, 0], gold["jacobi"], atol=1e-14)
    assert np.abs(J - J[:, :1, :1, :1]).max() <= 1e-14
    gf, gu = oracle.grad_exact_scatter(f, f, d, M, h)
    np.testing.assert_allclose(gf.reshape(shape[0], -1).sum(axis=1),
                               gold["grad_f_phase_sums"], atol=1e-12)
    assert np.abs(gu).max() <= 1e-12


# --------------------------------------------------------------------------
# Energy
# --------------------------------------------------------------------------
def test_energy_zero_for_equal_constants_and_nonnegative():
    shape = (3, 4, 5, 4)
    f = np.full(shape, 0.3)
    assert oracle.energy(f, f, 1, 2, 0.1) == 0.0
    for s in range(3):
        u, f = rnd(shape, 60 + s), rnd(shape, 70 + s)
        assert oracle.energy(u, f, 1, 2, 0.2) > 0.0


def test_energy_invariances():
    shape = (4, 4, 5, 3)
    u, f = rnd(shape, 81), rnd(shape, 82)
    d, M, h = 1, 2, 0.2
    E = oracle.energy(u, f, d, M, h)
    rev = lambda a: a[::-1].copy()
    assert abs(oracle.energy(rev(u), rev(f), d, M, h) - E) <= 1e-13 * E
    cyc = lambda a: np.roll(a, 1, axis=0)
    assert abs(oracle.energy(cyc(u), cyc(f), d, M, h) - E) <= 1e-13 * E
    assert abs(oracle.energy(u + 0.7, f + 0.7, d, M, h) - E) <= 1e-12 * E
    a = 1.7
    assert abs(oracle.energy(a * u, a * f, d, M, a * h) - a * a * E) \
        <= 1e-12 * E
    for ax in (1, 2, 3):
        fl = lambda t: np.flip(t, axis=ax).copy()
        assert abs(oracle.energy(fl(u), fl(f), d, M, h) - E) <= 1e-13 * E


def test_energy_transpose_invariance_on_cubic_grid():
    shape = (3, 4, 4, 4)
    u, f = rnd(shape, 91), rnd(shape, 92)
    E = oracle.energy(u, f, 1, 1, 0.25)
    for perm in ((0, 2, 1, 3), (0, 3, 2, 1), (0, 2, 3, 1)):
        t = lambda a: np.ascontiguousarray(np.transpose(a, perm))
        assert abs(oracle.energy(t(u), t(f), 1, 1, 0.25) - E) <= 1e-13 * E


# --------------------------------------------------------------------------
# Gradients
# --------------------------------------------------------------------------
@pytest.mark.parametrize("np_,d,M", [(2, 1, 1), (3, 0, 2), (3, 1, 1)])
def test_exact_gradient_against_finite_differences(np_, d, M):
    shape = (np_, 4, 3, 4)
    u, f = rnd(shape, 101 + M), rnd(shape, 102 + M)
    h = 0.3
    gf, gu = oracle.grad_exact_scatter(u, f, d, M, h)
    rng = np.random.default_rng(3)
    pos = [tuple(int(rng.integers(0, n)) for n in shape) for _ in range(12)]
    pos += [(0, 0, 0, 0), (np_ - 1, 3, 2, 3)]
    fgf, fgu = brute.fd_gradients(u, f, d, M, h, eps=1e-6, positions=pos)
    a = np.array([gf[p] for p in pos])
    b = np.array([gu[p] for p in pos])
    assert np.abs(a - fgf).max() <= 1e-6 * np.abs(fgf).max()
    assert np.abs(b - fgu).max() <= 1e-6 * np.abs(fgu).max()


def test_gather_gradient_equals_scatter_gradient():
    shape = (3, 5, 4, 4)
    u, f = rnd(shape, 111), rnd(shape, 112)
    d, M, h = 1, 2, 0.25
    gf, gu = oracle.grad_exact_scatter(u, f, d, M, h)
    idx = np.arange(0, u.size, 7)
    af, au = oracle.grad_exact_at(u, f, d, M, h, idx)
    np.testing.assert_allclose(af, gf.ravel()[idx], atol=1e-14)
    np.testing.assert_allclose(au, gu.ravel()[idx], atol=1e-14)


def test_gradient_sums_vanish_and_equivariance():
    shape = (3, 4, 5, 4)
    u, f = rnd(shape, 121), rnd(shape, 122)
    d, M, h = 1, 1, 0.2
    gf, gu = oracle.grad_exact_scatter(u, f, d, M, h)
    scale = np.abs(gf).max() + np.abs(gu).max()
    assert abs(gf.sum()) <= 1e-13 * scale * gf.size
    assert abs(gu.sum()) <= 1e-13 * scale * gu.size
    rf, ru = oracle.grad_exact_scatter(u[::-1].copy(), f[::-1].copy(), d, M, h)
    np.testing.assert_allclose(rf, gf[::-1], atol=1e-13)
    np.testing.assert_allclose(ru, gu[::-1], atol=1e-13)
    fl = lambda a: np.flip(a, axis=2).copy()
    xf, xu = oracle.grad_exact_scatter(fl(u), fl(f), d, M, h)
    np.testing.assert_allclose(xf, fl(gf), atol=1e-13)
    np.testing.assert_allclose(xu, fl(gu), atol=1e-13)


def test_eq6_is_the_frozen_weight_gradient_when_normalisers_match():
    """With uniform weights (h -> inf) and a window covering the whole grid,
    every normaliser is the same, so the exact gradient's image part equals
    the TNLM term of Eq. (6): both are 2 f_i - mean f_{i+1} - mean f_{i-1}."""
    shape = (3, 3, 3, 3)
    u, f = rnd(shape, 131), rnd(shape, 132)
    d, M, h = 1, 2, 1e6  # window = whole 3^3 grid, uniform weights
    gf, _ = oracle.grad_exact_scatter(u, f, d, M, h)
    G6 = oracle.grad_eq6(u, f, d, M, h)
    np.testing.assert_allclose(gf, G6, atol=1e-12)


def test_local_energy_differences_equal_total_energy_differences():
    shape = (3, 6, 5, 5)
    u, f = rnd(shape, 141), rnd(shape, 142)
    d, M, h = 1, 1, 0.25
    eps = 1e-3
    for pos in [(1, 2, 2, 2), (0, 0, 4, 0), (2, 5, 0, 3)]:
        for target in ("f", "u"):
            fp, up = f.copy(), u.copy()
            fm, um = f.copy(), u.copy()
            (fp if target == "f" else up)[pos] += eps
            (fm if target == "f" else um)[pos] -= eps
            dE = oracle.energy(up, fp, d, M, h) - oracle.energy(um, fm, d, M, h)
            dL = (oracle.local_energy(up, fp, d, M, h, *pos)
                  - oracle.local_energy(um, fm, d, M, h, *pos))
            assert abs(dE - dL) <= 1e-12


def test_oracle_on_phantom_is_finite_and_normalised():
    u = scaled_phantom((3, 8, 8, 6), 5)
    w, lse = oracle.weights(u, 1, 2, 0.05)
    assert np.isfinite(w).all() and np.isfinite(lse).all()
    assert np.abs(w.sum(axis=2) - 1).max() <= 1e-13


def test_nan_in_the_data_reaches_exactly_the_outputs_that_read_it():
    """NaN in the volumes is not checked; it propagates. One NaN voxel at
    c of phase 1 (in u, f and g) reaches, in one Eq.-(8) step, the outputs
    of phases 0 and 2 whose windows of candidate patches touch it
    (Chebyshev distance <= M + d) and the outputs of phase 1 whose own patch
    or fidelity term touches it (<= d); every other output stays finite,
    and the energy, which sums all terms, is NaN."""
    d, M = 1, 1
    u = np.random.default_rng(5).random((3, 8, 8, 8))
    u[1, 4, 4, 4] = np.nan
    out = oracle.jacobi(u, u, u, 0.5, d, M, 0.1)
    cheb = np.max(np.abs(np.indices((8, 8, 8)) - 4), axis=0)
    for i, reach in ((0, M + d), (1, d), (2, M + d)):
        assert np.array_equal(np.isnan(out[i]), cheb <= reach), i
        assert np.isfinite(out[i][cheb > reach]).all()
    assert np.isnan(oracle.energy(u, u, d, M, 0.1))
