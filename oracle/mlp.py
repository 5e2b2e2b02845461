"""FP64 oracle of the learned rate estimator (test infrastructure only).

The MLP and its backward live in ``oracle_mlp.c``; this module marshals
arrays and composes: training targets from the channel-wise fixed-length
coder (Sec. 3.4.1), the in-loop learned rate R = (1/N_hat) sum_i M_i f(x_i)
standing in for L_mask * L_quant (Sec. 3.3.1), and its gradient.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

MI, MH = 64, 128
NCH = 59

P = C.c_void_p
I64 = C.c_int64
F64 = C.c_double


def _declare(L):
    sig = {
        "orc_bf16": (F64, [F64]),
        "orc_mlp_features": (None, [I64, I64, P, P, P, C.c_int, P]),
        "orc_mlp_forward": (None, [I64, P, P, P, P, P, P, P, C.c_int, P]),
        "orc_mlp_backward": (None, [I64, P, P, P, P, P, P, P, C.c_int, P, P, P, P, P, P, P, P]),
        "orc_adam": (None, [I64, P, P, P, P, F64, F64, F64, F64, I64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _lib():
    import oracle
    return oracle.lib()


def _p(a):
    if a is None:
        return None
    assert a.flags.c_contiguous
    return a.ctypes.data


WEIGHT_SHAPES = (("W1", (MI, MH)), ("b1", (MH,)), ("W2", (MH, MH)), ("b2", (MH,)),
                 ("w3", (MH,)), ("b3", (1,)))


def init_weights(seed: int) -> dict:
    """He-uniform initialisation (seeded), float32 master weights."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = {}
    for name, shape in WEIGHT_SHAPES:
        if name.startswith("b"):
            w[name] = np.zeros(shape, np.float32)
        else:
            fan_in = shape[0]
            lim = math.sqrt(6.0 / fan_in)
            w[name] = rng.uniform(-lim, lim, size=shape).astype(np.float32)
    return w


def _wargs(w):
    return [np.ascontiguousarray(w[k], np.float32) for k, _ in WEIGHT_SHAPES]


def bf16(x: float) -> float:
    return float(_lib().orc_bf16(float(x)))


def features(y: np.ndarray, q: np.ndarray, mmin: np.ndarray, n: int, mirror: bool = True):
    """x_ij = log2(1 + (y_ij - m_j) / q_j), 59 channels + 5 zero pads."""
    y = np.ascontiguousarray(y, np.float32)
    X = np.zeros((n, MI))
    _lib().orc_mlp_features(n, y.shape[1], _p(y), _p(np.ascontiguousarray(q, np.float32)),
                            _p(np.ascontiguousarray(mmin, np.float32)), int(mirror), _p(X))
    return X


def forward(X: np.ndarray, w: dict, mirror: bool = True) -> np.ndarray:
    X = np.ascontiguousarray(X, np.float64)
    f = np.zeros(X.shape[0])
    a = _wargs(w)
    _lib().orc_mlp_forward(X.shape[0], _p(X), *[_p(t) for t in a], int(mirror), _p(f))
    return f


def backward(X: np.ndarray, w: dict, c: np.ndarray, mirror: bool = True, want_dx=False):
    """Gradient of sum_i c_i f(x_i) w.r.t. the weights (and X)."""
    X = np.ascontiguousarray(X, np.float64)
    c = np.ascontiguousarray(c, np.float64)
    g = {name: np.zeros(shape) for name, shape in WEIGHT_SHAPES}
    dX = np.zeros(X.shape) if want_dx else None
    a = _wargs(w)
    _lib().orc_mlp_backward(X.shape[0], _p(X), *[_p(t) for t in a], int(mirror), _p(c),
                            _p(g["W1"]), _p(g["b1"]), _p(g["W2"]), _p(g["b2"]), _p(g["w3"]),
                            _p(g["b3"]), _p(dX))
    return g, dX


def mse_grad_weights(f: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Upstream gradient of mean (f - t)^2."""
    return 2.0 * (f - t) / f.size


def adam(w: np.ndarray, m: np.ndarray, v: np.ndarray, g: np.ndarray, lr: float, t: int,
         beta1=0.9, beta2=0.999, eps=1e-8):
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(g, np.float64)
    _lib().orc_adam(w.size, _p(w), _p(m), _p(v), _p(g), lr, beta1, beta2, eps, t)


# --------------------------------------------------------------------------
# Training data: per-kept-Gaussian bits of the channel-wise fixed-length coder
# --------------------------------------------------------------------------

def coder_targets(params, qstep, mhat, n):
    """Sec. 3.4.1 fixed-length coder: total bits B over the kept Gaussians and
    the per-kept-Gaussian target B / N_kept."""
    import oracle
    _, k = oracle.fakequant(params, qstep, n)
    bits, kmin, kmax, width = oracle.fixed_length_bits(k, mhat, n)
    kept = int(mhat.sum())
    return bits, bits / max(kept, 1)


def channel_min(params, n):
    return params[:NCH, :n].min(axis=1).astype(np.float32)


def learned_rate(params, qstep, mhat, n, n_hat, w, mirror=True, weight=1.0):
    """R_learned = (1/N_hat) sum_i M_i f(x_i) and the gradient of weight * R
    w.r.t. the raw parameters, the steps and the hard mask (channel minima
    held fixed).  The weight enters before the BF16 rounding of dz2, as on
    the GPU."""
    params = np.ascontiguousarray(params, np.float32)
    mmin = channel_min(params, n)
    X = features(params, qstep, mmin, n, mirror)
    f = forward(X, w, mirror)
    m = mhat.astype(np.float64)
    R = float((m * f).sum() / n_hat)
    _, dX = backward(X, w, weight * m / n_hat, mirror, want_dx=True)
    u = (params[:NCH, :n].astype(np.float64) - mmin[:, None].astype(np.float64)) \
        / qstep[:, None].astype(np.float64)
    dxdu = 1.0 / ((1.0 + u) * math.log(2.0))
    gx = dX[:, :NCH].T
    gy = np.zeros(params.shape)
    gy[:NCH, :n] = gx * dxdu / qstep[:, None].astype(np.float64)
    gq = -(gx * dxdu * u).sum(axis=1) / qstep.astype(np.float64)
    gm = weight * f / n_hat
    return dict(R=R, f=f, X=X, gy=gy, gq=gq, gm=gm)
