"""MI355X-native temporal non-local means (TNLM) operator library.

Hand-written HIP kernels for gfx950 behind the C ABI of include/tnlm.h,
with a thin PyTorch binding (device memory and streams only):

  weights(u, d=, M=, h=)                   weights / log-normalisers, Eq. (3)
  jacobi_step(u, f, g, mu, d=, M=, h=)     Gauss-Jacobi step, Eq. (8)
  energy(f, d=, M=, h=, u=)                TNLM energy
  energy_noalloc(f, d=, M=, h=, u=)        same, no workspace (fixed scratch)
  grad(f, d=, M=, h=, u=, mode=)           Eq. (6) operator or exact gradient
  TNLMEnergy / tnlm_energy                 autograd wrapper
  enhance(...), descend(...)               host drivers
  ct.project / ct.backproject / ct.CGLS    cone-beam P, P^T and CGLS, Eqs. (1), (5)
  ct.reconstruct(...)                      the TNLM-R algorithm

The library libtnlm.so is loaded on the first call; that call raises
ImportError if it has not been built: there is no CPU path.
"""
from . import _lib
from ._lib import TNLMError
from .autograd import TNLMEnergy, tnlm_energy
from . import ct, metrics
from .drivers import descend, enhance
from .ops import energy, energy_noalloc, grad, jacobi_step, n_offsets, weights, workspace_bytes

__all__ = ["ct", "TNLMError", "TNLMEnergy", "tnlm_energy", "descend", "enhance", "metrics",
           "energy", "energy_noalloc", "grad", "jacobi_step", "n_offsets", "weights",
           "workspace_bytes"]
