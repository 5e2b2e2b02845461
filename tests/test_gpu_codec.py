"""GPU channel-wise fixed-length coder (paper Sec. 3.4.1) against the oracle's
coder on the same codes: header (kmin, width), payload bytes and bit count
bit-exact; decoding returns the fake quantizer's values of the kept
Gaussians bit-exact.  Edge cases: nothing kept, constant channels, a ragged
chunk, a payload buffer that is too small, codes outside int32."""
import sys

import numpy as np
import pytest

import synth
from synth import NCH

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


@pytest.fixture(scope="module")
def gctx(dev):
    from paper_2607_12656_amd import Context
    return Context(0)


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def encode(gctx, dev, sc, params, q, mask, words=None):
    gctx.set_scene(sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    if words is None:
        words = NCH * sc.n + 2   # 32 bits per value at most
    hdr = torch.zeros(NCH, 3, dtype=torch.int32, device=dev)
    payload = torch.full((words + 64,), 0x5A5A5A5A, dtype=torch.int32, device=dev)
    info = torch.zeros(3, dtype=torch.int64, device=dev)
    gctx.fl_encode(T(params, dev), T(q, dev), T(mask, dev), hdr, payload, words, info)
    torch.cuda.synchronize()
    return hdr.cpu().numpy(), payload.cpu().numpy().view(np.uint32), info.cpu().numpy()


def check_against_oracle(orc, gctx, dev, sc, params, q, mask, name):
    _say(f"[gpu] codec {name} n={sc.n}")
    hdr, payload, info = encode(gctx, dev, sc, params, q, mask)
    yhat, k = orc.fakequant(params, q, sc.n)
    bits, kmin, kmax, width = orc.fixed_length_bits(k, mask, sc.n)
    kept = int(mask[:sc.n].astype(bool).sum())
    assert info[2] == 0, f"flags {info[2]}"
    assert info[1] == kept
    assert info[0] == bits - NCH * 72, f"payload bits {info[0]} vs {bits - NCH * 72}"
    assert np.array_equal(hdr[:, 0].view(np.float32), q.astype(np.float32)), "header q"
    assert np.array_equal(hdr[:, 1], kmin), "header kmin"
    assert np.array_equal(hdr[:, 2], width), "header width"
    _, buf, _ = orc.fixed_length_roundtrip(k, mask, sc.n)
    nbytes = (int(info[0]) + 7) // 8
    gbytes = payload.view(np.uint8)
    assert np.array_equal(gbytes[:nbytes], buf[:nbytes]), "payload bytes"
    nwords = (int(info[0]) + 31) // 32
    tail = int(info[0]) % 32
    if tail:
        assert payload[nwords - 1] >> tail == 0, "bits past the payload"
    assert (payload[-64:] == 0x5A5A5A5A).all(), "write past the payload buffer"
    # decode
    pad = max(64, -(-kept // 64) * 64)
    out = torch.zeros(NCH, pad, dtype=torch.float32, device=dev)
    gctx.fl_decode(T(hdr, dev), T(payload[:nwords + 1].view(np.int32), dev), nwords + 1, kept,
                   pad, out)
    torch.cuda.synchronize()
    idx = np.flatnonzero(mask[:sc.n])
    assert np.array_equal(out.cpu().numpy()[:, :kept], yhat[:, idx]), "decoded values"
    return info


@pytest.mark.parametrize("cfg", [dict(n=300, W=64, H=48, seed=1), dict(n=5000, W=64, H=48, seed=2),
                                 dict(n=9000, W=64, H=48, seed=3)])
def test_tiny_scenes(orc, gctx, dev, cfg):
    sc = synth.make_tiny(cfg["n"], cfg["W"], cfg["H"], seed=cfg["seed"])
    check_against_oracle(orc, gctx, dev, sc, sc.params, sc.qstep, sc.given_mask, "tiny")


def test_c1_and_learnable_steps(orc, gctx, dev):
    sc = synth.make_scene("c1")
    check_against_oracle(orc, gctx, dev, sc, sc.params, sc.qstep, sc.given_mask, "c1")
    q = synth.learnable_qsteps(5)
    check_against_oracle(orc, gctx, dev, sc, sc.params, q, sc.given_mask, "c1 steps")


def test_edge_cases(orc, gctx, dev):
    sc = synth.make_tiny(4100, 64, 48, seed=4)      # one full chunk and a ragged one
    params = sc.params.copy()
    params[7, :sc.n] = 0.3                          # a constant channel -> width 0
    check_against_oracle(orc, gctx, dev, sc, params, sc.qstep, sc.given_mask, "constant channel")
    none = np.zeros_like(sc.given_mask)
    info = check_against_oracle(orc, gctx, dev, sc, params, sc.qstep, none, "nothing kept")
    assert info[0] == 0 and info[1] == 0
    one = np.zeros_like(sc.given_mask)
    one[4099] = 1                                   # the last Gaussian of the ragged chunk
    check_against_oracle(orc, gctx, dev, sc, params, sc.qstep, one, "one kept")


def test_small_payload_buffer_is_flagged(orc, gctx, dev):
    sc = synth.make_tiny(3000, 64, 48, seed=6)
    hdr, payload, info = encode(gctx, dev, sc, sc.params, sc.qstep, sc.given_mask, words=100)
    assert info[2] & 2, "capacity flag"
    assert (payload[100:] == 0x5A5A5A5A).all(), "nothing written past the given words"
    # the words that were written are the stream's first words
    yhat, k = orc.fakequant(sc.params, sc.qstep, sc.n)
    _, buf, _ = orc.fixed_length_roundtrip(k, sc.given_mask, sc.n)
    assert np.array_equal(payload[:100].view(np.uint8), buf[:400])


def test_code_outside_int32_is_flagged(gctx, dev):
    sc = synth.make_tiny(500, 64, 48, seed=7)
    q = sc.qstep.copy()
    q[3] = 1e-30
    _, _, info = encode(gctx, dev, sc, sc.params, q, sc.given_mask)
    assert info[2] & 1


def test_full_size_1m(orc, gctx, dev):
    """The measured workload (1M Gaussians, 20 % pruned): every byte."""
    sc = synth.make_scene("c2")
    info = check_against_oracle(orc, gctx, dev, sc, sc.params, sc.qstep, sc.given_mask, "c2")
    _say(f"c2 codec: {info[0]} payload bits for {info[1]} kept Gaussians "
         f"({info[0] / max(info[1], 1):.1f} bits each)")


def test_near_ties_and_awkward_steps(orc, gctx, dev):
    """Codes decided near half-integers (exact ties and a few ulps either
    side), near and past |y/q| = 2^19 and 2^23, with steps that are not powers
    of two, a negative step, a step whose reciprocal is subnormal and a
    subnormal step whose reciprocal overflows: every code equal to
    rint(fl32(y / q)) as the oracle's quantizer takes it."""
    sc = synth.make_tiny(8192 + 77, 64, 48, seed=11)
    rng = np.random.default_rng(12)
    n = sc.n
    q = synth.learnable_qsteps(9).astype(np.float32).copy()
    params = sc.params.copy()

    def around(x):  # each value, and 1..3 ulps below and above it
        x = np.asarray(x, np.float32)
        outs = [x]
        lo, hi = x.copy(), x.copy()
        for _ in range(3):
            lo = np.nextafter(lo, np.float32(-np.inf)).astype(np.float32)
            hi = np.nextafter(hi, np.float32(np.inf)).astype(np.float32)
            outs += [lo, hi]
        return np.concatenate(outs)

    def fill(j, vals):
        vals = np.resize(vals.astype(np.float32), n)
        params[j, :n] = vals[rng.permutation(n)]

    awkward = [0.0137, 1.0 / 3.0, 0.1, 7.3e-3, 2.0 ** -6, 1e-3, 0.77, 3.1, -0.05]
    for j, qq in enumerate(awkward):
        q[j] = np.float32(qq)
        m = rng.integers(-1000, 1000, 1200)
        fill(j, around((m + 0.5).astype(np.float32) * q[j]))
    for j, mag in ((10, 2 ** 19), (11, 2 ** 19 - 3), (12, 2 ** 20), (13, 2 ** 22), (14, 2 ** 23)):
        q[j] = np.float32(0.37)
        m = mag + rng.integers(-6, 6, 1200)
        sgn = np.where(rng.random(1200) < 0.5, -1.0, 1.0)
        fill(j, around((sgn * (m + 0.5)).astype(np.float32) * q[j]))
    q[15] = np.float32(3e38)                                 # 1/q subnormal
    fill(15, around(np.array([1.5e38, -1.5e38, 4.5e38 / 2, 3e38, 0.0, 1e30], np.float32)))
    q[16] = np.float32(2.0 ** -140)                          # subnormal step, 1/q overflows
    m = rng.integers(-5000, 5000, 1200)
    fill(16, around((m + 0.5).astype(np.float32) * q[16]))
    mask = sc.given_mask.copy()
    with np.errstate(over="ignore", invalid="ignore"):
        k = np.rint(params[:, :n] / q[:, None])
    assert np.isfinite(k).all() and np.abs(k).max() < 2 ** 31
    check_against_oracle(orc, gctx, dev, sc, params, q, mask, "near ties")
