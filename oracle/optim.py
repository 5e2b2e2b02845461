"""FP64 oracle of the optimizer step on the formation variables.

TEST INFRASTRUCTURE ONLY (imported by ``tests/`` and by nothing in the HIP
package).  Plain numpy in FP64.

Adam as Kingma & Ba (2015) define it (Algorithm 1, bias-corrected moments):
    m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2
    x <- x - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
and the two switches read here from the economical optimizer schedule the
paper adopts (Sec. 4.1): the 45 higher-order SH rows (channels 6-50) can
be left out of a step, and with ``sparse`` a Gaussian whose gradients in the
rows of the step are all exactly zero keeps its values and moments.
"""
from __future__ import annotations

import numpy as np

NCH = 59
SH_REST = np.arange(6, 51)


def adam_vector(x, m, v, g, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, skip=None):
    """One Adam step on arrays of any shape; ``lr`` broadcasts against them.
    ``skip`` (bool, same shape or broadcastable): entries left as they are.
    Returns new (x, m, v) in FP64."""
    x = np.asarray(x, np.float64)
    m = np.asarray(m, np.float64)
    v = np.asarray(v, np.float64)
    g = np.asarray(g, np.float64)
    b1, b2 = float(beta1), float(beta2)
    m1 = b1 * m + (1.0 - b1) * g
    v1 = b2 * v + (1.0 - b2) * g * g
    mh = m1 / (1.0 - b1 ** step)
    vh = v1 / (1.0 - b2 ** step)
    x1 = x - np.asarray(lr, np.float64) * mh / (np.sqrt(vh) + float(eps))
    if skip is not None:
        keep = np.broadcast_to(skip, x.shape)
        x1 = np.where(keep, x, x1)
        m1 = np.where(keep, m, m1)
        v1 = np.where(keep, v, v1)
    return x1, m1, v1


def adam_params(x, m, v, g, lr, step, n, beta1=0.9, beta2=0.999, eps=1e-8, sh_rest=True,
                sparse=False):
    """The parameter block [59][npad] (columns >= n untouched); lr: 59 rates."""
    x = np.asarray(x, np.float64).copy()
    m = np.asarray(m, np.float64).copy()
    v = np.asarray(v, np.float64).copy()
    g = np.asarray(g, np.float64)
    rows = np.ones(NCH, bool)
    if not sh_rest:
        rows[SH_REST] = False
    lr = np.broadcast_to(np.asarray(lr, np.float64), (NCH,))
    skip = None
    if sparse:
        skip = ~np.any(g[rows, :n] != 0.0, axis=0)[None, :]
    r = np.flatnonzero(rows)
    xs, ms, vs = adam_vector(x[r, :n], m[r, :n], v[r, :n], g[r, :n], lr[r, None], step,
                             beta1, beta2, eps, skip)
    x[r, :n], m[r, :n], v[r, :n] = xs, ms, vs
    return x, m, v


def compact(arrays, mask, n):
    """Pruning by the learned mask (the supplement's formation schedule prunes
    with it every 1,000 iterations): the columns i < n with mask[i] != 0 of
    each array ([rows][npad] or [npad]), in index order."""
    keep = np.asarray(mask[:n]) != 0
    return [np.asarray(a)[..., :n][..., keep] for a in arrays]
