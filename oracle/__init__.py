"""FP64 CPU oracle for the SpeedyGS structural-formation (RD) step.

TEST INFRASTRUCTURE ONLY: this package is imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the CPU-baseline leg of ``bench.py``, and by
nothing else.  It never imports the HIP package, and the HIP package never
imports it.  The arithmetic lives in ``oracle.c`` (plain C, FP64, built with
gcc, no contraction); this module only marshals numpy arrays.  The optimizer
step and pruning are plain FP64 numpy in ``optim.py``, the SSIM term in
``ssim.py``, the rate-proxy variants in ``rate_variants.py``.

Each function names the paper passage it follows; see ``oracle.c`` for the
formulas.  Parity-unpinned constants (near plane 0.2, low-pass dilation 0.3,
3-sigma radius, alpha bounds 1/255 and 0.99, transmittance floor 1e-4, colour
offset 1/2, background 0, field-of-view clamp 1.3) are conventions: the paper
does not state them.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from .optim import adam_params, adam_vector, compact  # noqa: F401
from . import rate_variants, ssim  # noqa: F401

NCH = 59
HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = [os.path.join(HERE, "oracle.c"), os.path.join(HERE, "oracle_mlp.c"),
       os.path.join(HERE, "oracle_coding.c")]

TW_DEFAULT = 16
TH_DEFAULT = 16


LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def build() -> str:
    """Compile liboracle.so with gcc (FP64, no floating-point contraction),
    and the same sources with OpenMP as liboracle_omp.so (only the sampled
    tile step runs its tiles in parallel; results do not depend on the
    thread count)."""
    srcs = [s for s in SRC if os.path.exists(s)]
    base = ["gcc", "-O2", "-std=c11", "-Wall", "-Wno-unknown-pragmas", "-ffp-contract=off",
            "-fno-fast-math", "-fPIC", "-shared"]
    for out, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        subprocess.run([*base, *extra, "-o", out + ".tmp", *srcs, "-lm"], check=True)
        os.replace(out + ".tmp", out)
    return LIB


_lib = None
_lib_omp = None


def _stale(path):
    return (not os.path.exists(path)) or any(
        os.path.exists(s) and os.path.getmtime(s) > os.path.getmtime(path) for s in SRC)


def lib():
    global _lib
    if _lib is None:
        if _stale(LIB) or _stale(LIB_OMP):
            build()
        _lib = C.CDLL(LIB)
        _declare(_lib)
    return _lib


def lib_omp():
    """The OpenMP build (same functions; used for the parallel CPU baseline)."""
    global _lib_omp
    if _lib_omp is None:
        lib()
        _lib_omp = C.CDLL(LIB_OMP)
        _declare(_lib_omp)
    return _lib_omp


P = C.c_void_p
I64 = C.c_int64
I32 = C.c_int32
U64 = C.c_uint64
F32 = C.c_float
F64 = C.c_double


def _declare(L):
    sig = {
        "orc_uniform": (F32, [U64, U64, U64]),
        "orc_exp_dl": (F32, [F32]),
        "orc_fakequant": (None, [I64, I64, P, P, P, P]),
        "orc_mask": (None, [I64, C.c_int, P, P, U64, U64, F64, P, P]),
        "orc_rate_proxy": (None, [I64, I64, P, P, P, I64, F64, P, P, P, P, P, P, P]),
        "orc_fakequant_bwd": (None, [I64, I64, P, P, P, C.c_int, P, F64, P, P, P, P]),
        "orc_decide": (None, [I64, I64, P, I32, P, I32, I32, I32, I32, P, P, P, P, P, P]),
        "orc_bin": (I64, [I64, I32, P, P, P, I32, I32, I32, I32, P, P, P]),
        "orc_forward": (I64, [I64, I64, P, P, I32, P, I32, I32, I32, I32, P, P, P, P,
                              P, P, P, P]),
        "orc_forward_brute": (I64, [I64, I64, P, P, I32, P, I32, I32, P, P, P, P, P]),
        "orc_backward": (None, [I64, I64, P, P, I32, P, I32, I32, I32, I32, P, P, P, P,
                                P, P, P, P]),
        "orc_project64": (None, [I64, I64, P, I32, P, I32, I32, P, P]),
        "orc_tile_counts": (None, [I64, I32, P, P, I32, I32, I32, I32, P]),
        "orc_tile_list": (I64, [I64, I32, I64, P, P, P, I32, I32, I32, P]),
        "orc_pixels_brute": (I64, [I64, I64, P, P, I32, P, I32, I32, P, P, P, I64, P, P, P]),
        "orc_splat_grads_sampled": (I64, [I64, I64, P, P, I32, P, I32, I32, P, P, P, I64, P,
                                          P, P, P, P]),
        "orc_step_tiles_sampled": (I64, [I64, I64, P, P, I32, P, I32, I32, I32, I32, P, P, P,
                                         I64, P, P, P, P]),
        "orc_l1": (F64, [I64, P, P, P]),
        "orc_sh_basis": (None, [I64, P, P]),
        "orc_fixed_length_bits": (I64, [I64, I64, P, P, P, P, P]),
        "orc_fixed_length_pack": (None, [I64, I64, P, P, P, P, P]),
        "orc_fixed_length_unpack": (None, [I64, I64, P, P, P, P, P]),
        "orc_morton3": (U64, [C.c_uint32, C.c_uint32, C.c_uint32, I32]),
        "orc_octree_tokens": (I64, [I64, I64, P, P, P, P, P, P, P, P]),
        "orc_octree_decode": (I64, [P, I64, I32, P, I64]),
        "orc_voxel_positions": (I64, [P, P, I64, I32, P, P, P, I64]),
        "orc_ans_model": (None, [P, I64, I32, I64, P]),
        "orc_ans_ideal_bits": (F64, [P, I64, I32, I64, P]),
        "orc_ans_encode": (I64, [P, I64, I32, I64, P, P, P]),
        "orc_ans_decode": (I64, [P, P, I64, I32, I64, P, P]),
        "orc_morton_order": (I64, [I64, I64, P, P, P, I32, P, P]),
        "orc_attr_planes": (None, [I64, P, P, P, I64, I32, I64, I32, P]),
        "orc_attr_reconstruct": (None, [I64, P, I32, I64, I64, F32, I32, P]),
    }
    for name, (res, args) in sig.items():
        if not hasattr(L, name):
            continue
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    try:
        from . import mlp as _mlp  # noqa: F401  (declares the MLP entry points)
        _mlp._declare(L)
    except ImportError:
        pass


def _p(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags.c_contiguous, "oracle arrays must be C-contiguous"
    return a.ctypes.data


# --------------------------------------------------------------------------
# a1-a3, a12: quantizer, mask, rate proxy
# --------------------------------------------------------------------------

def uniform(seed: int, step: int, i: int) -> float:
    return float(lib().orc_uniform(seed, step, i))


def exp_dl(x: float) -> float:
    return float(lib().orc_exp_dl(np.float32(x)))


def fakequant(y: np.ndarray, q: np.ndarray, n: int):
    """Sec. 3.3.1 uniform quantizer: k = rint(y/q), yhat = fl32(k q)."""
    y = np.ascontiguousarray(y, np.float32)
    q = np.ascontiguousarray(q, np.float32)
    npad = y.shape[1]
    yhat = y.copy()
    k = np.zeros(y.shape, np.int32)
    lib().orc_fakequant(n, npad, _p(y), _p(q), _p(yhat), _p(k))
    return yhat, k


def mask(n: int, mode: int, given: np.ndarray | None, score: np.ndarray | None,
         seed: int = 0, step: int = 0, tau: float = 1.0):
    """Sec. 3.3.1 retention mask. mode 0 given, 1 Gumbel-sigmoid, 2 keep all."""
    given = np.ascontiguousarray(given if given is not None else np.ones(n, np.uint8), np.uint8)
    score = np.ascontiguousarray(score if score is not None else np.zeros(n, np.float32), np.float32)
    mh = np.zeros(n, np.uint8)
    ms = np.zeros(n, np.float64)
    lib().orc_mask(n, mode, _p(given), _p(score), seed, step, tau, _p(mh), _p(ms))
    return mh, ms


def rate_proxy(y: np.ndarray, q: np.ndarray, mhat: np.ndarray, n: int, n_hat: int,
               lam: float = 0.0):
    """Sec. 3.3.1: R_proxy = L_mask * L_quant (and its gradient when lam != 0)."""
    y = np.ascontiguousarray(y, np.float32)
    q = np.ascontiguousarray(q, np.float32)
    mhat = np.ascontiguousarray(mhat, np.uint8)
    npad = y.shape[1]
    out3 = np.zeros(3)
    amin = np.zeros(NCH, np.int32)
    amax = np.zeros(NCH, np.int32)
    cj = np.zeros(NCH)
    gy = np.zeros(y.shape)
    gq = np.zeros(NCH)
    gm = np.zeros(n)
    lib().orc_rate_proxy(n, npad, _p(y), _p(q), _p(mhat), n_hat, lam, _p(out3), _p(amin),
                         _p(amax), _p(cj), _p(gy), _p(gq), _p(gm))
    return dict(R=out3[0], Lq=out3[1], Lm=out3[2], argmin=amin, argmax=amax, c=cj,
                gy=gy, gq=gq, gm=gm)


def fakequant_bwd(y, q, gyhat, mode, msoft, tau, gmhat, n):
    y = np.ascontiguousarray(y, np.float32)
    q = np.ascontiguousarray(q, np.float32)
    gyhat = np.ascontiguousarray(gyhat, np.float64)
    msoft = np.ascontiguousarray(msoft, np.float64)
    gmhat = np.ascontiguousarray(gmhat, np.float64)
    gy = np.zeros(y.shape)
    gq = np.zeros(NCH)
    gs = np.zeros(n)
    lib().orc_fakequant_bwd(n, y.shape[1], _p(y), _p(q), _p(gyhat), mode, _p(msoft), tau,
                            _p(gmhat), _p(gy), _p(gq), _p(gs))
    return gy, gq, gs


# --------------------------------------------------------------------------
# a4-a7: decision layer, binning, sort order, ranges
# --------------------------------------------------------------------------

@dataclass
class Structure:
    valid: np.ndarray   # int32 [V][n]
    tz: np.ndarray      # float32 [V][n]
    pxy: np.ndarray     # float32 [V][n][2]
    span: np.ndarray    # int32 [V][n][4]  x0, x1, y0, y1 (inclusive)
    radius: np.ndarray  # int32 [V][n]
    tiles: np.ndarray   # int32 [V][n]
    keys: np.ndarray    # uint64 [P]  (global tile << 32) | bits(t_z)
    vals: np.ndarray    # uint32 [P]  Gaussian index
    ranges: np.ndarray  # uint32 [V*tiles][2]
    TW: int
    TH: int


def decide(yhat: np.ndarray, n: int, cams: np.ndarray, W: int, H: int,
           TW: int = TW_DEFAULT, TH: int = TH_DEFAULT, bin_pairs: bool = True) -> Structure:
    """Decision layer for every (view, Gaussian); with bin_pairs the sorted
    (tile, depth, index) pair list too (skip it where it would not fit)."""
    yhat = np.ascontiguousarray(yhat, np.float32)
    cams = np.ascontiguousarray(cams, np.float32)
    V = cams.shape[0]
    valid = np.zeros((V, n), np.int32)
    tz = np.zeros((V, n), np.float32)
    pxy = np.zeros((V, n, 2), np.float32)
    span = np.zeros((V, n, 4), np.int32)
    radius = np.zeros((V, n), np.int32)
    tiles = np.zeros((V, n), np.int32)
    L = lib()
    L.orc_decide(n, yhat.shape[1], _p(yhat), V, _p(cams), W, H, TW, TH, _p(valid), _p(tz),
                 _p(pxy), _p(span), _p(radius), _p(tiles))
    Pn = L.orc_bin(n, V, _p(valid), _p(tz), _p(span), W, H, TW, TH, None, None, None)
    GW, GH = (W + TW - 1) // TW, (H + TH - 1) // TH
    if not bin_pairs:
        e = np.zeros(0, np.uint32)
        st = Structure(valid, tz, pxy, span, radius, tiles, e.astype(np.uint64), e,
                       np.zeros((0, 2), np.uint32), TW, TH)
        st.pairs = int(Pn)
        return st
    keys = np.zeros(max(Pn, 1), np.uint64)
    vals = np.zeros(max(Pn, 1), np.uint32)
    ranges = np.zeros((V * GW * GH, 2), np.uint32)
    L.orc_bin(n, V, _p(valid), _p(tz), _p(span), W, H, TW, TH, _p(keys), _p(vals), _p(ranges))
    return Structure(valid, tz, pxy, span, radius, tiles, keys[:Pn], vals[:Pn], ranges, TW, TH)


# --------------------------------------------------------------------------
# a8-a11: render forward / backward, L1
# --------------------------------------------------------------------------

def forward(p64: np.ndarray, mask64: np.ndarray, n: int, cams: np.ndarray, W: int, H: int,
            st: Structure):
    """Sec. 3.1 compositing over the (tile, depth) lists. FP64."""
    p64 = np.ascontiguousarray(p64, np.float64)
    mask64 = np.ascontiguousarray(mask64, np.float64)
    cams = np.ascontiguousarray(cams, np.float32)
    V = cams.shape[0]
    img = np.zeros((V, 3, H, W))
    T = np.zeros((V, H, W))
    last = np.zeros((V, H, W), np.int32)
    margin = np.zeros((V, H, W), np.uint8)
    vals = st.vals if st.vals.size else np.zeros(1, np.uint32)
    E = lib().orc_forward(n, p64.shape[1], _p(p64), _p(mask64), V, _p(cams), W, H, st.TW, st.TH,
                          _p(st.valid), _p(st.span), _p(vals), _p(st.ranges), _p(img), _p(T),
                          _p(last), _p(margin))
    return dict(image=img, T=T, last=last, margin=margin, evals=int(E))


def forward_brute(p64, mask64, n, cams, W, H, st: Structure):
    """Definition: every pixel composites ALL splats in global depth order."""
    p64 = np.ascontiguousarray(p64, np.float64)
    mask64 = np.ascontiguousarray(mask64, np.float64)
    cams = np.ascontiguousarray(cams, np.float32)
    V = cams.shape[0]
    img = np.zeros((V, 3, H, W))
    T = np.zeros((V, H, W))
    E = lib().orc_forward_brute(n, p64.shape[1], _p(p64), _p(mask64), V, _p(cams), W, H,
                                _p(st.valid), _p(st.tz), _p(st.span), _p(img), _p(T))
    return dict(image=img, T=T, evals=int(E))


def backward(p64, mask64, n, cams, W, H, st: Structure, dimage, want_splat: bool = False):
    p64 = np.ascontiguousarray(p64, np.float64)
    mask64 = np.ascontiguousarray(mask64, np.float64)
    cams = np.ascontiguousarray(cams, np.float32)
    dimage = np.ascontiguousarray(dimage, np.float64)
    V = cams.shape[0]
    gp = np.zeros(p64.shape)
    gm = np.zeros(n)
    gs = np.zeros((V, n, 10)) if want_splat else None
    vals = st.vals if st.vals.size else np.zeros(1, np.uint32)
    lib().orc_backward(n, p64.shape[1], _p(p64), _p(mask64), V, _p(cams), W, H, st.TW, st.TH,
                       _p(st.valid), _p(st.span), _p(vals), _p(st.ranges), _p(dimage), _p(gp),
                       _p(gm), _p(gs))
    return gp, gm, gs


def project64(p64, n, cams, W, H, st: Structure):
    p64 = np.ascontiguousarray(p64, np.float64)
    cams = np.ascontiguousarray(cams, np.float32)
    V = cams.shape[0]
    out = np.zeros((V, n, 9))
    lib().orc_project64(n, p64.shape[1], _p(p64), V, _p(cams), W, H, _p(st.valid), _p(out))
    return out


def l1(image: np.ndarray, target: np.ndarray):
    image = np.ascontiguousarray(image, np.float64)
    target = np.ascontiguousarray(target, np.float32)
    d = np.zeros(image.shape)
    D = lib().orc_l1(image.size, _p(image), _p(target), _p(d))
    return float(D), d


def tile_counts(st: Structure, n: int, V: int, W: int, H: int) -> np.ndarray:
    """Pairs per tile from the spans (orc_bin's rule, no pair list)."""
    GW, GH = (W + st.TW - 1) // st.TW, (H + st.TH - 1) // st.TH
    out = np.zeros(V * GW * GH, np.int64)
    lib().orc_tile_counts(n, V, _p(st.valid), _p(st.span), W, H, st.TW, st.TH, _p(out))
    return out


def tile_list(st: Structure, n: int, view: int, tile_in_view: int, W: int) -> np.ndarray:
    """Gaussians of one tile in (depth, index) order."""
    L = lib()
    cnt = L.orc_tile_list(n, view, tile_in_view, _p(st.valid), _p(st.tz), _p(st.span), W,
                          st.TW, st.TH, None)
    out = np.zeros(max(cnt, 1), np.uint32)
    L.orc_tile_list(n, view, tile_in_view, _p(st.valid), _p(st.tz), _p(st.span), W, st.TW,
                    st.TH, _p(out))
    return out[:cnt]


def pixels_brute(p64, mask64, n, cams, W, H, st: Structure, pix: np.ndarray):
    """Colour and T of sampled pixels pix [k][3] = (view, u, v) by brute force."""
    p64 = np.ascontiguousarray(p64, np.float64)
    mask64 = np.ascontiguousarray(mask64, np.float64)
    cams = np.ascontiguousarray(cams, np.float32)
    pix = np.ascontiguousarray(pix, np.int32)
    if pix.size and not ((pix[:, 0] >= 0).all() and (pix[:, 0] < cams.shape[0]).all()
                         and (pix[:, 1] >= 0).all() and (pix[:, 1] < W).all()
                         and (pix[:, 2] >= 0).all() and (pix[:, 2] < H).all()):
        raise ValueError("sampled pixel outside the views")
    out = np.zeros((pix.shape[0], 4))
    margin = np.zeros(pix.shape[0], np.uint8)
    E = lib().orc_pixels_brute(n, p64.shape[1], _p(p64), _p(mask64), cams.shape[0], _p(cams), W,
                               H, _p(st.valid), _p(st.tz), _p(st.span), pix.shape[0], _p(pix),
                               _p(out), _p(margin))
    return out, margin, int(E)


def splat_grads_sampled(p64, mask64, n, cams, W, H, st: Structure, sel, dimage=None):
    """Gradients of chosen Gaussians by brute force over their span pixels:
    (gsplat [k][V][10], gparam [k][59], margin [V][H][W] uint8).  Without
    dimage only the margin flags of the span pixels are produced."""
    p64 = np.ascontiguousarray(p64, np.float64)
    mask64 = np.ascontiguousarray(mask64, np.float64)
    cams = np.ascontiguousarray(cams, np.float32)
    sel = np.ascontiguousarray(sel, np.int64)
    if sel.size and not ((sel >= 0).all() and (sel < n).all()):
        raise ValueError("chosen Gaussian outside the scene")
    V = cams.shape[0]
    if dimage is not None:
        dimage = np.ascontiguousarray(dimage, np.float64)
        assert dimage.shape == (V, 3, H, W)
    gs = np.zeros((sel.size, V, 10))
    gp = np.zeros((sel.size, NCH))
    margin = np.zeros((V, H, W), np.uint8)
    lib().orc_splat_grads_sampled(n, p64.shape[1], _p(p64), _p(mask64), V, _p(cams), W, H,
                                  _p(st.valid), _p(st.tz), _p(st.span), sel.size, _p(sel),
                                  _p(dimage), _p(gs), _p(gp), _p(margin))
    return gs, gp, margin


def step_tiles_sampled(p64, mask64, n, cams, W, H, st: Structure, tiles, dimage,
                       parallel: bool = False):
    """Render forward and backward over the chosen global tile ids only (the
    rest of the image has zero dL/dC): (evals, image [k][3][TH][TW],
    gparams [59][npad]).  parallel: the OpenMP build."""
    p64 = np.ascontiguousarray(p64, np.float64)
    mask64 = np.ascontiguousarray(mask64, np.float64)
    cams = np.ascontiguousarray(cams, np.float32)
    tiles = np.ascontiguousarray(tiles, np.int64)
    V = cams.shape[0]
    GW, GH = (W + st.TW - 1) // st.TW, (H + st.TH - 1) // st.TH
    if tiles.size and not ((tiles >= 0).all() and (tiles < V * GW * GH).all()):
        raise ValueError("tile id outside the views")
    if np.unique(tiles).size != tiles.size:
        raise ValueError("repeated tile id")
    dimage = np.ascontiguousarray(dimage, np.float64)
    assert dimage.shape == (V, 3, H, W)
    img = np.zeros((tiles.size, 3, st.TH, st.TW))
    gp = np.zeros(p64.shape)
    L = lib_omp() if parallel else lib()
    E = L.orc_step_tiles_sampled(n, p64.shape[1], _p(p64), _p(mask64), V, _p(cams), W, H,
                                 st.TW, st.TH, _p(st.valid), _p(st.tz), _p(st.span), tiles.size,
                                 _p(tiles), _p(dimage), _p(img), _p(gp))
    return int(E), img, gp


def sh_basis(dirs: np.ndarray) -> np.ndarray:
    dirs = np.ascontiguousarray(dirs, np.float64)
    Y = np.zeros((dirs.shape[0], 16))
    lib().orc_sh_basis(dirs.shape[0], _p(dirs), _p(Y))
    return Y


# --------------------------------------------------------------------------
# Sec. 3.4.1: channel-wise fixed-length code length
# --------------------------------------------------------------------------

def fixed_length_bits(k: np.ndarray, mhat: np.ndarray, n: int):
    k = np.ascontiguousarray(k, np.int32)
    mhat = np.ascontiguousarray(mhat, np.uint8)
    kmin = np.zeros(NCH, np.int32)
    kmax = np.zeros(NCH, np.int32)
    width = np.zeros(NCH, np.int32)
    bits = lib().orc_fixed_length_bits(n, k.shape[1], _p(k), _p(mhat), _p(kmin), _p(kmax),
                                       _p(width))
    return int(bits), kmin, kmax, width


def fixed_length_roundtrip(k: np.ndarray, mhat: np.ndarray, n: int):
    bits, kmin, kmax, width = fixed_length_bits(k, mhat, n)
    payload = bits - NCH * 72
    buf = np.zeros((payload + 7) // 8 + 1, np.uint8)
    L = lib()
    L.orc_fixed_length_pack(n, k.shape[1], _p(np.ascontiguousarray(k, np.int32)),
                            _p(np.ascontiguousarray(mhat, np.uint8)), _p(kmin), _p(width), _p(buf))
    out = np.zeros_like(k, dtype=np.int32)
    L.orc_fixed_length_unpack(n, k.shape[1], _p(buf), _p(np.ascontiguousarray(mhat, np.uint8)),
                              _p(kmin), _p(width), _p(out))
    return out, buf, bits


# --------------------------------------------------------------------------
# One whole RD step (plain rate proxy): loss = L1(render) + lam * R_proxy
# --------------------------------------------------------------------------

def rd_forward(params, qstep, score, given_mask, cams, W, H, target, n, n_hat, lam,
               mask_mode=0, seed=0, step=0, tau=1.0, TW=TW_DEFAULT, TH=TH_DEFAULT):
    """Forward of D_render + lam * R_proxy [Sec. 3.3.2 total loss]."""
    yhat, k = fakequant(params, qstep, n)
    mh, ms = mask(n, mask_mode, given_mask, score, seed, step, tau)
    rp = rate_proxy(params, qstep, mh, n, n_hat, lam)
    st = decide(yhat, n, cams, W, H, TW, TH)
    p64 = yhat.astype(np.float64)
    m64 = mh.astype(np.float64)
    fw = forward(p64, m64, n, cams, W, H, st)
    D, d_img = l1(fw["image"], target)
    return dict(params=params, qstep=qstep, cams=cams, W=W, H=H, n=n, lam=lam,
                mask_mode=mask_mode, tau=tau, yhat=yhat, k=k, mhat=mh, msoft=ms, rate=rp,
                st=st, p64=p64, m64=m64, fw=fw, D=D, loss=D + lam * rp["R"], dimage=d_img)


def rd_backward(s, dimage=None):
    """Backward of rd_forward's loss; ``dimage`` overrides dL/dimage (to feed
    both sides the same upstream gradient)."""
    d_img = s["dimage"] if dimage is None else np.asarray(dimage, np.float64)
    n = s["n"]
    gyhat, gmh, _ = backward(s["p64"], s["m64"], n, s["cams"], s["W"], s["H"], s["st"], d_img)
    rp = s["rate"]
    gmh_total = gmh + rp["gm"]
    gy, gq, gs = fakequant_bwd(s["params"], s["qstep"], gyhat, s["mask_mode"], s["msoft"],
                               s["tau"], gmh_total, n)
    out = dict(s)
    out.update(dimage=d_img, gyhat=gyhat, gmhat=gmh, gmhat_total=gmh_total,
               gy=gy + rp["gy"], gq=gq + rp["gq"], gs=gs)
    return out


def rd_step(params, qstep, score, given_mask, cams, W, H, target, n, n_hat, lam,
            mask_mode=0, seed=0, step=0, tau=1.0, TW=TW_DEFAULT, TH=TH_DEFAULT,
            dimage=None):
    """Forward and backward of D_render + lam * R_proxy [Sec. 3.3.2 total loss]."""
    s = rd_forward(params, qstep, score, given_mask, cams, W, H, target, n, n_hat, lam,
                   mask_mode, seed, step, tau, TW, TH)
    return rd_backward(s, dimage)


# --------------------------------------------------------------------------
# Learned-coding stage, lossless parts [Sec. 3.4.2]: octree tokens of the
# quantized geometry and the interleaved rANS coder (see oracle_coding.c)
# --------------------------------------------------------------------------

ANS_M = 4096
ANS_CTX = 257


def morton3(ux: int, uy: int, uz: int, depth: int) -> int:
    return int(lib().orc_morton3(ux, uy, uz, depth))


def octree_tokens(y: np.ndarray, q: np.ndarray, mhat: np.ndarray, n: int):
    """Sec. 3.4.2 geometry occupancy coding: the kept Gaussians' position
    codes voxelized, merged and written as 8-bit octree tokens, level by
    level from the root, Morton order within a level."""
    y = np.ascontiguousarray(y, np.float32)
    q = np.ascontiguousarray(q[:3], np.float32)
    mhat = np.ascontiguousarray(mhat[:n], np.uint8)
    npad = y.shape[1]
    kept = max(int(mhat.sum()), 1)
    hdr = np.zeros(8, np.int64)
    codes = np.zeros(kept, np.uint64)
    dup = np.zeros(kept, np.uint32)
    tokens = np.zeros(21 * kept, np.uint8)
    level = np.zeros(22, np.int64)
    nt = lib().orc_octree_tokens(n, npad, _p(y), _p(q), _p(mhat), _p(hdr), _p(codes), _p(dup),
                                 _p(tokens), _p(level))
    m = int(hdr[5])
    return dict(depth=int(hdr[0]), kmin=hdr[1:4].copy(), kept=int(hdr[4]), unique=m,
                flags=int(hdr[7]), codes=codes[:m].copy(), dup=dup[:m].copy(),
                tokens=tokens[:nt].copy(), level_size=level[:int(hdr[0])].copy())


def octree_decode(tokens: np.ndarray, depth: int, cap: int):
    """The unique voxel codes a token stream describes (None if malformed)."""
    tokens = np.ascontiguousarray(tokens, np.uint8)
    codes = np.zeros(max(cap, 1), np.uint64)
    m = lib().orc_octree_decode(_p(tokens), tokens.size, depth, _p(codes), cap)
    return None if m < 0 else codes[:m].copy()


def voxel_positions(codes, dup, depth: int, kmin, q):
    codes = np.ascontiguousarray(codes, np.uint64)
    dup = np.ascontiguousarray(dup, np.uint32)
    kmin = np.ascontiguousarray(kmin, np.int64)
    q = np.ascontiguousarray(q[:3], np.float32)
    total = int(dup.astype(np.int64).sum()) + codes.size
    xyz = np.zeros((3, max(total, 1)), np.float32)
    lib().orc_voxel_positions(_p(codes), _p(dup), codes.size, depth, _p(kmin), _p(q), _p(xyz),
                              total)
    return xyz[:, :total].copy()


def ans_model(sym: np.ndarray, order: int, lane_len: int):
    sym = np.ascontiguousarray(sym, np.uint8)
    freq = np.zeros((ANS_CTX, 256), np.uint16)
    lib().orc_ans_model(_p(sym), sym.size, order, lane_len, _p(freq))
    return freq


def ans_ideal_bits(sym: np.ndarray, order: int, lane_len: int, freq: np.ndarray) -> float:
    sym = np.ascontiguousarray(sym, np.uint8)
    freq = np.ascontiguousarray(freq, np.uint16)
    return float(lib().orc_ans_ideal_bits(_p(sym), sym.size, order, lane_len, _p(freq)))


def ans_encode(sym: np.ndarray, order: int, lane_len: int, freq: np.ndarray):
    """Returns (words uint16, block offsets int64) or None if a symbol has
    frequency 0."""
    sym = np.ascontiguousarray(sym, np.uint8)
    freq = np.ascontiguousarray(freq, np.uint16)
    nb = (sym.size + 64 * lane_len - 1) // (64 * lane_len)
    words = np.zeros(128 * nb + sym.size + 1, np.uint16)
    off = np.zeros(nb + 1, np.int64)
    r = lib().orc_ans_encode(_p(sym), sym.size, order, lane_len, _p(freq), _p(words), _p(off))
    return None if r < 0 else (words[:r].copy(), off)


def ans_decode(words, block_off, n: int, order: int, lane_len: int, freq):
    """Returns the n symbols, or None if the stream is malformed."""
    words = np.ascontiguousarray(words, np.uint16)
    block_off = np.ascontiguousarray(block_off, np.int64)
    freq = np.ascontiguousarray(freq, np.uint16)
    sym = np.zeros(max(n, 1), np.uint8)
    r = lib().orc_ans_decode(_p(words), _p(block_off), n, order, lane_len, _p(freq), _p(sym))
    return None if r < 0 else sym[:n].copy()


# attributes [Sec. 3.4.2, autoregressive attribute coding]
ATTR_CHANNELS = tuple(range(3, NCH))   # colour (DC and higher SH), opacity, scale, rotation


def morton_order(y, q, mhat, n, depth, kmin):
    """Indices of the kept Gaussians in the Morton order of their voxels
    (ties by index)."""
    y = np.ascontiguousarray(y, np.float32)
    q = np.ascontiguousarray(q[:3], np.float32)
    mhat = np.ascontiguousarray(mhat[:n], np.uint8)
    kmin = np.ascontiguousarray(kmin, np.int64)
    perm = np.zeros(max(n, 1), np.int64)
    kept = lib().orc_morton_order(n, y.shape[1], _p(y), _p(q), _p(mhat), depth, _p(kmin),
                                  _p(perm))
    return perm[:kept].copy()


def attr_plane_count(width: int, predictor: int = 1) -> int:
    """Byte planes of a channel whose values take `width` bits: the values
    themselves (predictor 0) take width bits, the residual of two of them
    zigzag-mapped (predictor 1) width + 1; none for width 0."""
    if width == 0:
        return 0
    return (width + 7) // 8 if predictor == 0 else (width + 1 + 7) // 8


def attr_planes(y_row, q_c, perm, kmin: int, width: int, S: int, predictor: int = 1):
    """Byte planes [planes][kept] of one channel along perm (predictor 1:
    zigzag residual against the group's previous value; 0: the value)."""
    y_row = np.ascontiguousarray(y_row, np.float32)
    perm = np.ascontiguousarray(perm, np.int64)
    P = attr_plane_count(width, predictor)
    out = np.zeros((max(P, 1), perm.size), np.uint8)
    qc = np.array([q_c], np.float32)
    lib().orc_attr_planes(perm.size, _p(y_row), _p(qc), _p(perm), int(kmin), P, S, predictor,
                          _p(out))
    return out[:P].copy()


def attr_reconstruct(planes, kmin: int, q_c: float, S: int, kept: int, predictor: int = 1):
    planes = np.ascontiguousarray(planes, np.uint8)
    P = planes.shape[0] if planes.ndim == 2 else 0
    out = np.zeros(max(kept, 1), np.float32)
    if P == 0:
        out[:] = np.float32(np.float32(kmin) * np.float32(q_c))
        return out[:kept]
    lib().orc_attr_reconstruct(kept, _p(planes), P, S, int(kmin), np.float32(q_c), predictor,
                               _p(out))
    return out[:kept].copy()


def fourier_features(mu, L: int = 12):
    """phi(mu) = [mu; sin(2 pi F mu); cos(2 pi F mu)], F = (2^0 .. 2^(L-1)),
    per Gaussian: [n][3 + 6L] in FP64 (sin block: band-major, axis-minor)."""
    mu = np.asarray(mu, np.float64).reshape(-1, 3)
    F = 2.0 ** np.arange(L)
    ang = 2.0 * np.pi * mu[:, None, :] * F[None, :, None]          # [n][L][3]
    return np.concatenate([mu, np.sin(ang).reshape(len(mu), -1),
                           np.cos(ang).reshape(len(mu), -1)], axis=1)


def positional_embedding(mu, W, b, L: int = 12):
    """PE(mu) = W phi(mu) + b (W [d][3 + 6L], b [d]) in FP64."""
    return fourier_features(mu, L) @ np.asarray(W, np.float64).T + np.asarray(b, np.float64)
