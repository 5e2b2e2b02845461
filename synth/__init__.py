"""Seeded synthetic inputs for the SpeedyGS structural-formation (RD) step.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic. Both the FP64 oracle (``oracle/``) and the HIP path
(``paper_2607_12656_amd``) are fed from here, so the two sides see the same
float32 arrays.

Parameter layout (59 channels per Gaussian, SoA ``[59][npad]`` float32,
``npad`` = N rounded up to a multiple of 64), following the channel counts of
the vanilla 3DGS representation (paper, Supplementary "Bitstream Composition":
3 geometry + 48 colour + 1 opacity + 3 scale + 4 rotation):

====== =========================================================
0-2    mean mu (x, y, z), world units
3-5    SH DC coefficients (r, g, b)
6-50   SH coefficients k = 1..15, coefficient-major: 6 + 3*(k-1) + c
51     opacity logit (opacity = sigmoid)
52-54  log-scale (scale = exp)
55-58  rotation quaternion (w, x, y, z), not necessarily unit
====== =========================================================

Camera record (float32[19]): world->camera rotation R (row-major, 9),
translation t (3), fx, fy, cx, cy, camera centre in world coordinates (3).
OpenCV axes: x right, y down, z forward. A pixel (u, v) has its centre at image
coordinate (u, v).

Workloads (the paper's scenes are real captures, Mip-NeRF360 / Tanks&Temples /
DeepBlending; these synthetic scenes stand in for them with the paper's
Gaussian counts, 3DGS attribute statistics and the image sizes of the
measured configurations):

* ``c1``: 4,096 Gaussians, means U[-1,1]^3, 128x128 camera at distance 3.
* ``c2``: 1,000,000 Gaussians, means from a 3-component mixture (clustered),
  one 1297x840 camera on a ring of radius 4, 20 % pruned.
* ``c3``: 3,000,000 Gaussians, 8 views of 1600x1060 on the ring.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NCH = 59
CH_MU, CH_DC, CH_REST, CH_OPA, CH_SCALE, CH_ROT = 0, 3, 6, 51, 52, 55


def pad64(n: int) -> int:
    return max(64, (n + 63) // 64 * 64)


@dataclass
class Scene:
    n: int
    npad: int
    params: np.ndarray          # float32 [59][npad]
    qstep: np.ndarray           # float32 [59]
    score: np.ndarray           # float32 [n] mask scores s_i
    given_mask: np.ndarray      # uint8 [n]
    cams: np.ndarray            # float32 [V][19]
    width: int
    height: int
    target: np.ndarray          # float32 [V][3][H][W]
    lam: float = 2.5e-5
    n_hat: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def views(self) -> int:
        return int(self.cams.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def camera_axis(width: int, height: int, dist: float, fov_deg: float = 60.0) -> np.ndarray:
    """Camera at (0, 0, -dist) looking along +z with camera axes = world axes."""
    f = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    cam = np.zeros(19, np.float64)
    cam[0:9] = np.eye(3).reshape(-1)
    cam[9:12] = (0.0, 0.0, dist)
    cam[12:16] = (f, f, width / 2.0, height / 2.0)
    cam[16:19] = (0.0, 0.0, -dist)
    return cam.astype(np.float32)


def camera_ring(width: int, height: int, radius: float, theta: float,
                fov_deg: float = 60.0) -> np.ndarray:
    """Camera at radius*(sin th, 0, -cos th) looking at the origin, image y down."""
    pos = np.array([radius * math.sin(theta), 0.0, -radius * math.cos(theta)])
    fwd = -pos / np.linalg.norm(pos)
    down = np.array([0.0, 1.0, 0.0])
    right = np.cross(down, fwd)
    right /= np.linalg.norm(right)
    dn = np.cross(fwd, right)
    R = np.stack([right, dn, fwd])
    t = -R @ pos
    f = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    cam = np.zeros(19, np.float64)
    cam[0:9] = R.reshape(-1)
    cam[9:12] = t
    cam[12:16] = (f, f, width / 2.0, height / 2.0)
    cam[16:19] = pos
    return cam.astype(np.float32)


def _attributes(rng: np.random.Generator, n: int, means: np.ndarray,
                logscale_mu: float = -4.0, logscale_sd: float = 0.5,
                sh_sd: float = 0.3) -> np.ndarray:
    npad = pad64(n)
    p = np.zeros((NCH, npad), np.float32)
    p[0:3, :n] = means.T
    p[CH_DC:CH_OPA, :n] = rng.normal(0.0, sh_sd, size=(48, n))
    p[CH_OPA, :n] = rng.normal(0.0, 1.0, size=n)
    p[CH_SCALE:CH_ROT, :n] = rng.normal(logscale_mu, logscale_sd, size=(3, n))
    q = rng.normal(0.0, 1.0, size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    p[CH_ROT:NCH, :n] = q
    return p


def _prune_mask(n: int, frac: float, seed: int) -> np.ndarray:
    m = np.ones(n, np.uint8)
    k = int(math.floor(frac * n))
    if k:
        m[_rng(seed).permutation(n)[:k]] = 0
    return m


def make_scene(name: str, n: int | None = None, width: int | None = None,
               height: int | None = None, views: int | None = None,
               seed: int | None = None) -> Scene:
    """Build one of the named synthetic workloads (optionally resized)."""
    if name == "c1":
        n = 4096 if n is None else n
        seed = 1 if seed is None else seed
        W = 128 if width is None else width
        H = 128 if height is None else height
        rng = _rng(seed)
        means = rng.uniform(-1.0, 1.0, size=(n, 3))
        params = _attributes(rng, n, means)
        cams = np.stack([camera_axis(W, H, 3.0)])
        mask = _prune_mask(n, 0.10, seed + 1)
        tseed = seed + 2
        qinit = 2.0 ** -6
    elif name in ("c2", "c3"):
        big = name == "c3"
        n = (3_000_000 if big else 1_000_000) if n is None else n
        seed = (21 if big else 11) if seed is None else seed
        W = (1600 if big else 1297) if width is None else width
        H = (1060 if big else 840) if height is None else height
        V = (8 if big else 1) if views is None else views
        rng = _rng(seed)
        centres = rng.uniform(-0.6, 0.6, size=(3, 3))
        comp = rng.integers(0, 3, size=n)
        means = centres[comp] + rng.normal(0.0, 0.2, size=(n, 3))
        params = _attributes(rng, n, means)
        cams = np.stack([camera_ring(W, H, 4.0, 2 * math.pi * k / V) for k in range(V)])
        mask = _prune_mask(n, 0.20, seed + 1)
        tseed = seed + 2
        qinit = 2.0 ** -6
    else:
        raise ValueError(f"unknown workload {name!r}")
    V = cams.shape[0]
    srng = _rng(seed + 3)
    score = srng.normal(1.5, 1.0, size=n).astype(np.float32)
    target = _rng(tseed).random(size=(V, 3, H, W), dtype=np.float32)
    return Scene(n=n, npad=params.shape[1], params=params,
                 qstep=np.full(NCH, qinit, np.float32), score=score,
                 given_mask=mask, cams=cams, width=W, height=H, target=target,
                 n_hat=n, name=name)


def make_tiny(n: int, width: int, height: int, views: int = 1, seed: int = 0,
              logscale_mu: float = -2.5, dist: float = 3.0, spread: float = 0.6,
              prune: float = 0.2, qstep: float = 2.0 ** -8) -> Scene:
    """Small scene for oracle self-tests and element-by-element parity.

    Larger splats than the c1 statistics (log-scale N(-2.5, 0.5)) so that a few
    dozen Gaussians cover a small image with overlaps, terminations and ties.
    """
    rng = _rng(seed)
    means = rng.uniform(-spread, spread, size=(n, 3))
    params = _attributes(rng, n, means, logscale_mu=logscale_mu)
    if views == 1:
        cams = np.stack([camera_axis(width, height, dist)])
    else:
        cams = np.stack([camera_ring(width, height, dist, 2 * math.pi * k / views)
                         for k in range(views)])
    mask = _prune_mask(n, prune, seed + 1)
    score = _rng(seed + 3).normal(1.5, 1.0, size=n).astype(np.float32)
    target = _rng(seed + 2).random(size=(views, 3, height, width), dtype=np.float32)
    return Scene(n=n, npad=params.shape[1], params=params,
                 qstep=np.full(NCH, qstep, np.float32), score=score,
                 given_mask=mask, cams=cams, width=width, height=height,
                 target=target, n_hat=n, name=f"tiny{n}x{width}x{height}v{views}")


def learnable_qsteps(seed: int, lo_exp: float = -9.0, hi_exp: float = -3.0) -> np.ndarray:
    """Per-channel step sizes 2^U[lo,hi] (training data for the learned rate)."""
    return (2.0 ** _rng(seed).uniform(lo_exp, hi_exp, size=NCH)).astype(np.float32)
