"""Loss and optimiser, FP64 (test infrastructure only).

Loss.  The paper supervises each field with a masked colour term and a masked
depth term summed over the rays of the batch (Sec. 4.3, Eq. 8; un-squared L2
colour norm and L1 depth).  The reading taken for the hot path: squared L2 for
both, averaged over rays,

    L = (1/R) sum_r M_r [ |C_r - C*_r|^2 + lambda_d (D_r - D*_r)^2 ],

with lambda_d = 0 when no depth is supervised; M_r = 1 for synthetic rays.
``eq8_loss`` gives the paper's printed form for reference.

Optimiser (not stated in the paper; Instant-NGP's published choice): Adam with
bias correction, lr 1e-2, beta1 0.9, beta2 0.99, eps 1e-15, no weight decay.
Hash-table entries whose gradient is exactly zero are left untouched (their
moments too).  Mixed precision: gradients arrive multiplied by a static loss
scale S = 2^k; they are divided by S before use; if any is not finite the whole
update is skipped and S is halved.
"""
from __future__ import annotations

import numpy as np


def loss(C, D, C_t, D_t, lambda_d=0.0, mask=None):
    """Returns (L, dC (R,3), dD (R,))."""
    C = np.asarray(C, np.float64)
    D = np.asarray(D, np.float64)
    C_t = np.asarray(C_t, np.float64)
    D_t = np.zeros_like(D) if D_t is None else np.asarray(D_t, np.float64)
    R = C.shape[0]
    m = np.ones(R) if mask is None else np.asarray(mask, np.float64)
    ec = C - C_t
    ed = D - D_t
    L = np.sum(m * (np.sum(ec * ec, 1) + lambda_d * ed * ed)) / R
    dC = 2.0 * m[:, None] * ec / R
    dD = 2.0 * lambda_d * m * ed / R
    return L, dC, dD


def eq8_loss(C, D, C_t, D_t, mask=None):
    """The printed form: sum_r |M(C-C*)|_2 and sum_r |M(D-D*)|_1."""
    C = np.asarray(C, np.float64)
    m = np.ones(C.shape[0]) if mask is None else np.asarray(mask, np.float64)
    lc = np.sum(np.linalg.norm(m[:, None] * (C - C_t), axis=1))
    ld = np.sum(np.abs(m * (np.asarray(D) - np.asarray(D_t))))
    return lc, ld


class Adam:
    """``lr_decay``: update k (1-based) uses lr * lr_decay^(k-1), the exponential
    schedule Instant-NGP applies to its rate; 1 keeps it constant."""

    def __init__(self, lr=1e-2, b1=0.9, b2=0.99, eps=1e-15, lr_decay=1.0):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.lr_decay = lr_decay

    def update(self, p, g, m, v, step, skip_zero=False):
        """One update in place on float64 arrays; ``step`` is the 1-based count."""
        live = (g != 0.0) if skip_zero else np.ones(g.shape, bool)
        m[live] = self.b1 * m[live] + (1.0 - self.b1) * g[live]
        v[live] = self.b2 * v[live] + (1.0 - self.b2) * g[live] * g[live]
        mh = m[live] / (1.0 - self.b1 ** step)
        vh = v[live] / (1.0 - self.b2 ** step)
        lr = self.lr * self.lr_decay ** (step - 1)
        p[live] -= lr * mh / (np.sqrt(vh) + self.eps)


def unscale_and_check(grads, loss_scale):
    """Divide every gradient by S; return (grads, finite)."""
    out = [np.asarray(g, np.float64) / loss_scale for g in grads]
    finite = all(np.all(np.isfinite(g)) for g in out)
    return out, finite
