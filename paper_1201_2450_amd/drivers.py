"""Host-side drivers over the kernels.

enhance():  the TNLM enhancement algorithm (Sec. 2.3, TNLM-E): f^0 = g, then
            repeat {weights from the latest images (Eq. (9)); one Gauss-Jacobi
            step (Eq. (8))}. The weight source can be refreshed every step
            (the paper's algorithm), every few steps, or kept at g.
            The iteration state is (f, u, k); a `checkpoint` callable receives
            it after every step and `resume` continues from it, bit for bit
            the same as an uninterrupted run (every step is deterministic).
descend():  plain gradient descent on the TNLM energy, f <- f - tau dE/df,
            with the exact gradient of E(f; f) and the weights recomputed at
            every step (a forward-backward splitting regulariser step).
"""
from __future__ import annotations

import torch

from . import ops


def enhance(g, mu, *, d, M, h, iters, recompute_every=1, weights_from="f",
            step_hook=None, checkpoint=None, resume=None):
    """Returns f after `iters` Gauss-Jacobi steps (same dtype as g).

    weights_from='f': u <- f every `recompute_every` steps (u is f itself when
    recompute_every == 1); weights_from='g': u = g for every step.
    checkpoint(state) is called after every step with state = {"f", "u",
    "k"} (k = steps done; the tensors are the driver's own, copy them to
    keep them); resume=state starts from such a state and runs the steps
    k .. iters-1."""
    if iters < 0 or recompute_every < 1:
        raise ValueError("iters >= 0 and recompute_every >= 1 required")
    k0 = 0
    f = g.clone()
    u = g
    if resume is not None:
        k0 = int(resume["k"])
        if not 0 <= k0 <= iters:
            raise ValueError("resume step k outside [0, iters]")
        f.copy_(resume["f"])
        if weights_from == "f" and recompute_every > 1 and k0 % recompute_every:
            u = resume["u"].clone()  # the snapshot taken at the last refresh
    buf = torch.empty_like(g)
    for k in range(k0, iters):
        if weights_from == "f":
            if recompute_every == 1:
                u = f
            elif k % recompute_every == 0:
                u = f.clone()
        elif weights_from != "g":
            raise ValueError(weights_from)
        ops.jacobi_step(u, f, g, mu, d=d, M=M, h=h, out=buf)
        f, buf = buf, f
        if step_hook is not None:
            step_hook(k, f)
        if checkpoint is not None:
            checkpoint({"f": f, "u": f if u is buf else u, "k": k + 1})
    return f


def descend(f, *, d, M, h, tau, iters):
    """iters steps of f <- f - tau * d/df E(f; f); returns the new f (same
    dtype as the input; the update itself is done in float32)."""
    f = f.clone()
    for _ in range(iters):
        gt = ops.grad(f, d=d, M=M, h=h, mode="exact", total=True)
        f = (f.float() - tau * gt).to(f.dtype)
    return f
