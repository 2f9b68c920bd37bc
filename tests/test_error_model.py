"""Pins of the rounding-error model that sets the GPU parity tolerances
(oracle.error_model, CPU).

The model writes every output's first-order error as a linear combination
of per-candidate exponent errors. Its correlated part D = sum c_k a_k is the
sensitivity of the output to a common relative change of every exponent,
i.e. of 1/(2h^2): D = d out / d log(1/(2h^2)) = -(1/2) d out / d log h. This
checks D against central differences of the oracle's own outputs in h for
every output the model covers (log-normalisers, neighbour averages through
the Jacobi step, e, both gradient parts), so a wrong coefficient anywhere in
the propagation fails. Independently, the variance proxies must be
non-negative and vanish where every exponent is zero.
"""
import numpy as np
import pytest

from oracle import oracle
from phantom import scaled_phantom

U = 2.0 ** -24


def _fd(fn, h, tau=1e-4):
    """-(1/2) d fn / d log h by central differences in log h."""
    return -(fn(h * np.exp(tau)) - fn(h * np.exp(-tau))) / (4 * tau)


@pytest.mark.parametrize("shape,d,M,h", [
    ((3, 5, 4, 6), 1, 1, 0.05),
    ((2, 4, 5, 4), 1, 2, 0.08),
    ((3, 4, 3, 5), 0, 2, 0.05),
])
def test_correlated_coefficients_equal_the_sensitivity_to_h(shape, d, M, h):
    u = scaled_phantom(shape, 7)
    f = scaled_phantom(shape, 8)
    m = oracle.error_model(u, f, d, M, h, 7, U, 6.0, 3 * U, grad=True)
    N = int(np.prod(shape[1:]))

    def close(got, want, what):
        err = np.abs(got - want).max() / np.abs(want).max()
        assert err <= 1e-6, (what, err)

    close(m["lse_d"], _fd(lambda hh: oracle.weights(u, d, M, hh, want_w=False)[1], h), "lse")
    close(m["e_d"], _fd(lambda hh: oracle.stats(u, f, d, M, hh)[:, :, 1], h), "e")
    mu = 0.5
    jac_d = m["nb_d"].sum(axis=1).reshape(shape) / (2 + mu)
    close(jac_d, _fd(lambda hh: oracle.jacobi(u, f, f, mu, d, M, hh), h), "jacobi")
    close(m["gf_d"], _fd(lambda hh: oracle.grad_exact_scatter(u, f, d, M, hh)[0], h), "dE/df")
    close(m["gu_d"], _fd(lambda hh: oracle.grad_exact_scatter(u, f, d, M, hh)[1], h), "dE/du")
    for k in ("lse_v", "nb_v", "e_v", "gf_v", "gu_v", "w_b"):
        assert np.all(m[k] >= 0) and np.all(np.isfinite(m[k])), k
    assert m["lse_v"].shape == (shape[0], 2, N)


def test_independent_part_scales_with_the_unit_roundoff_squared():
    shape, d, M, h = (2, 4, 4, 5), 1, 1, 0.06
    u = scaled_phantom(shape, 9)
    a = oracle.error_model(u, u, d, M, h, 7, U, 6.0, 0.0, grad=True)
    b = oracle.error_model(u, u, d, M, h, 7, 2 * U, 6.0, 0.0, grad=True)
    for k in ("lse_v", "nb_v", "e_v", "gf_v", "gu_v"):
        assert np.allclose(b[k], 4 * a[k], rtol=1e-12, atol=0), k
    # deeper distance sums can only widen the bound
    c = oracle.error_model(u, u, d, M, h, 27, U, 6.0, 0.0, grad=True)
    for k in ("lse_v", "nb_v", "e_v", "gf_v", "gu_v"):
        assert np.all(c[k] >= a[k] * (1 - 1e-12)), k


def test_constant_volumes_have_no_propagated_error_in_the_averages():
    """Constant phases: every candidate has D = 0 and the averaged values
    are all equal, so the neighbour average, e and both gradient parts have
    zero coefficients (up to the FP64 rounding of the mean, c - cbar ~ 1e-17);
    only the log-normaliser keeps its rounding terms."""
    shape = (3, 4, 4, 4)
    c = np.full(shape, 0.3)
    m = oracle.error_model(c, c, 1, 1, 0.05, 7, U, 6.0, 3 * U, grad=True)
    for k in ("nb_v", "e_v", "gf_v", "gu_v"):
        assert np.abs(m[k]).max() <= 1e-40, k
    for k in ("nb_d", "e_d", "gf_d", "gu_d"):
        assert np.abs(m[k]).max() <= 1e-15, k
    assert m["lse_v"].min() > 0


def test_sampled_model_equals_the_whole_grid_model():
    shape, d, M, h = (3, 6, 5, 7), 1, 2, 0.05
    u = scaled_phantom(shape, 11)
    f = scaled_phantom(shape, 12)
    full = oracle.error_model(u, f, d, M, h, 7, U, 6.0, 3 * U)
    idx = np.array([0, 5, 17, 88, int(np.prod(shape)) - 1], dtype=np.int64)
    at = oracle.error_model_at(u, f, d, M, h, 7, U, 6.0, 3 * U, idx)
    N = int(np.prod(shape[1:]))
    for k in at:
        assert np.array_equal(at[k], full[k][idx // N, :, idx % N]), k
