"""Pins of the coding oracle (paper Sec. 3.4.2: octree occupancy tokens of the
quantized geometry, and the entropy coder standing in for the arithmetic
coder).  Each check ties the oracle to something outside itself: hand-built
octrees and hand-run rANS steps (Duda's range-ANS map C(s, x) = floor(x / f)
M + cum + x mod f), the set of distinct quantized positions from the
quantizer (pinned elsewhere), round trips through independently written
decoders, closed-form code lengths of dyadic models, and the entropy bound."""
import numpy as np
import pytest

import synth

L16 = 1 << 16


def one_point_cloud(points, q=1.0, npad=None):
    """params [59][npad] with the given integer voxel positions (times q)."""
    pts = np.asarray(points, np.float64)
    n = len(pts)
    npad = npad or synth.pad64(n)
    y = np.zeros((59, npad), np.float32)
    y[:3, :n] = (pts * q).T
    qs = np.full(59, q, np.float32)
    return y, qs, np.ones(n, np.uint8), n


# ---------------------------------------------------------------------------
# Morton codes and octree tokens
# ---------------------------------------------------------------------------
def test_morton_bit_layout(orc):
    # x bit b -> code bit 3b+2, y -> 3b+1, z -> 3b
    assert orc.morton3(1, 0, 0, 1) == 4
    assert orc.morton3(0, 1, 0, 1) == 2
    assert orc.morton3(0, 0, 1, 1) == 1
    assert orc.morton3(7, 7, 7, 3) == 511
    assert orc.morton3(2, 0, 0, 2) == 32
    assert orc.morton3(3, 1, 2, 2) == 0b101110   # level 1: x1 z1; level 0: x0 y0
    # bits above the depth are ignored
    assert orc.morton3(5, 0, 0, 2) == orc.morton3(1, 0, 0, 2)
    # Z order of the unit cube: z fastest, then y, then x
    order = sorted(((x, y, z) for x in range(2) for y in range(2) for z in range(2)),
                   key=lambda p: orc.morton3(*p, 1))
    assert order == [(x, y, z) for x in range(2) for y in range(2) for z in range(2)]


def test_octree_hand_example(orc):
    # voxels (0,0,0), (1,0,0), (3,3,3): depth 2.  Root: children (0,0,0)-prefix
    # (bit 0) and (1,1,1)-prefix (bit 7) -> 0x81.  Level 1, node 0: children
    # (0,0,0) (bit 0) and (1,0,0) (bit 4) -> 0x11; node 7: child 7 -> 0x80.
    y, q, m, n = one_point_cloud([(0, 0, 0), (1, 0, 0), (3, 3, 3)])
    r = orc.octree_tokens(y, q, m, n)
    assert r["depth"] == 2 and r["flags"] == 0
    assert list(r["tokens"]) == [0x81, 0x11, 0x80]
    assert list(r["level_size"]) == [1, 2]
    assert list(r["codes"]) == [0, 4, 63]
    assert list(r["kmin"]) == [0, 0, 0]
    # shifted by (5, -3, 2) with a duplicate of the second point: same tokens
    y, q, m, n = one_point_cloud([(5, -3, 2), (6, -3, 2), (8, 0, 5), (6, -3, 2)])
    r = orc.octree_tokens(y, q, m, n)
    assert list(r["tokens"]) == [0x81, 0x11, 0x80]
    assert list(r["kmin"]) == [5, -3, 2]
    assert r["kept"] == 4 and r["unique"] == 3
    assert list(r["dup"]) == [0, 1, 0]


def test_octree_depth_rule(orc):
    for rng_, depth in ((0, 1), (1, 1), (2, 2), (3, 2), (7, 3), (8, 4), (1000, 10)):
        y, q, m, n = one_point_cloud([(0, 0, 0), (0, rng_, 0)])
        r = orc.octree_tokens(y, q, m, n)
        assert r["depth"] == depth, (rng_, r["depth"])
        assert r["tokens"].size == sum(r["level_size"])


def test_octree_single_and_empty(orc):
    y, q, m, n = one_point_cloud([(4, 4, 4)])
    r = orc.octree_tokens(y, q, m, n)
    assert r["depth"] == 1 and list(r["tokens"]) == [1] and list(r["codes"]) == [0]
    r = orc.octree_tokens(y, q, np.zeros(1, np.uint8), n)
    assert r["kept"] == 0 and r["unique"] == 0 and r["tokens"].size == 0
    assert list(r["kmin"]) == [0, 0, 0]


def test_octree_flags_wide_range(orc):
    y, q, m, n = one_point_cloud([(0, 0, 0), (1 << 21, 0, 0)])
    assert orc.octree_tokens(y, q, m, n)["flags"] & 1
    y, q, m, n = one_point_cloud([(0, 0, 0), ((1 << 21) - 1, 0, 0)])
    r = orc.octree_tokens(y, q, m, n)
    assert r["flags"] == 0 and r["depth"] == 21


@pytest.mark.parametrize("seed,qv,frac", [(0, 0.01, 0.8), (1, 0.05, 1.0), (2, 0.002, 0.5)])
def test_octree_against_quantizer(orc, seed, qv, frac):
    """Structure and content against the (pinned) quantizer: the decoded
    voxels are exactly the distinct quantized positions of the kept
    Gaussians, and the decoded positions with copies are their dequantized
    positions, as multisets."""
    rng = np.random.default_rng(seed)
    n = 4000
    npad = synth.pad64(n)
    y = np.zeros((59, npad), np.float32)
    centers = rng.normal(0, 1, (8, 3))
    y[:3, :n] = (centers[rng.integers(0, 8, n)] + rng.normal(0, 0.2, (n, 3))).T
    q = np.full(59, qv, np.float32)
    m = (rng.random(n) < frac).astype(np.uint8)
    r = orc.octree_tokens(y, q, m, n)
    assert r["flags"] == 0
    tok, ls = r["tokens"], r["level_size"]
    # level structure: one root; each level's children are the next level
    assert ls[0] == 1 and np.all(tok != 0)
    starts = np.concatenate([[0], np.cumsum(ls)])
    pop = np.array([bin(int(t)).count("1") for t in tok])
    for l in range(r["depth"] - 1):
        assert pop[starts[l]:starts[l + 1]].sum() == ls[l + 1]
    assert pop[starts[-2]:].sum() == r["unique"]
    # decode (an independent routine) gives back the codes
    codes = orc.octree_decode(tok, r["depth"], r["unique"])
    assert np.array_equal(codes, r["codes"])
    assert np.all(np.diff(codes.astype(np.uint64)) > 0)
    # distinct voxels = distinct quantized positions
    yhat, k = orc.fakequant(y, q, n)
    kk = k[:3, :n][:, m.astype(bool)].T.astype(np.int64)
    uniq = np.unique(kk, axis=0)
    assert r["unique"] == len(uniq) and r["kept"] == len(kk)
    assert np.array_equal(r["kmin"], kk.min(axis=0))
    xyz = orc.voxel_positions(r["codes"], r["dup"], r["depth"], r["kmin"], q)
    got = np.unique(np.rint(xyz.astype(np.float64) / qv).astype(np.int64).T, axis=0)
    assert np.array_equal(got, uniq)
    # with copies: the multiset of dequantized kept positions
    want = yhat[:3, :n][:, m.astype(bool)]
    key = lambda a: a[:, np.lexsort(a[::-1])]
    assert np.array_equal(key(xyz), key(want))
    assert r["dup"].sum() == len(kk) - len(uniq)


def test_octree_decode_rejects_truncation(orc):
    y, q, m, n = one_point_cloud([(0, 0, 0), (1, 0, 0), (3, 3, 3)])
    r = orc.octree_tokens(y, q, m, n)
    assert orc.octree_decode(r["tokens"][:2], r["depth"], 8) is None


# ---------------------------------------------------------------------------
# Entropy coder
# ---------------------------------------------------------------------------
def test_model_hand_normalization(orc):
    # counts a:3, b:1 -> K = 2, N = 4: f_a = 1 + 3*4094//4 = 3071, f_b = 1024,
    # remainder 1 to a -> exactly 3/4 and 1/4 of 4096
    f = orc.ans_model(np.array([0, 0, 0, 1], np.uint8), 0, 64)
    assert f[0, 0] == 3072 and f[0, 1] == 1024 and f[0].sum() == 4096
    assert f[1:].sum() == 0
    # dyadic counts that sum to 4096 reproduce themselves
    sym = np.repeat(np.arange(4, dtype=np.uint8), [2048, 1024, 512, 512])
    f = orc.ans_model(sym, 0, 1 << 20)
    assert list(f[0, :4]) == [2048, 1024, 512, 512]
    # ties go to the lowest symbol
    f = orc.ans_model(np.array([5, 9, 5, 9, 2], np.uint8), 0, 64)
    assert f[0].sum() == 4096 and f[0, 5] == f[0, 9] + 1
    # order 1: contexts are the previous symbol of the lane, 256 at its start
    f = orc.ans_model(np.array([1, 2, 1, 2, 1, 2], np.uint8), 1, 2)
    assert f[256, 1] == 4096 and f[1, 2] == 4096 and f[2].sum() == 0


def test_model_rows_valid_random(orc):
    rng = np.random.default_rng(3)
    sym = (rng.geometric(0.3, 50000) % 256).astype(np.uint8)
    for order in (0, 1):
        f = orc.ans_model(sym, order, 100).astype(np.int64)
        used = f.sum(axis=1) > 0
        assert np.all(f.sum(axis=1)[used] == 4096)
        # every symbol that occurs in a context has a nonzero frequency there
        ctx = np.zeros(sym.size, np.int64)
        if order:
            ctx = np.where(np.arange(sym.size) % 100 == 0, 256,
                           np.roll(sym, 1).astype(np.int64))
        assert np.all(f[ctx, sym] > 0)


def test_single_symbol_stream_costs_nothing(orc):
    sym = np.full(1000, 7, np.uint8)
    f = orc.ans_model(sym, 0, 4)
    assert f[0, 7] == 4096
    w, off = orc.ans_encode(sym, 0, 4, f)
    nb = len(off) - 1
    assert nb == 4 and w.size == 128 * nb
    assert np.all(w[0::2] == 1) and np.all(w[1::2] == 0)   # every state still 2^16
    assert np.array_equal(orc.ans_decode(w, off, sym.size, 0, 4, f), sym)
    assert orc.ans_ideal_bits(sym, 0, 4, f) == 0.0


def test_hand_encoded_block(orc):
    """64 lanes of two symbols each under a hand-made model: symbol 0 has
    frequency 4032, symbols 1..64 frequency 1 (cum_s = 4031 + s).  Lane l
    codes (c_l, b_l) = (64 - l, l + 1).  Backwards from x = 2^16: b_l gives
    x = 2^28 + cum(b_l) (no renormalization: 2^16 < 2^20 f); c_l first pushes
    the low half cum(b_l) (x >= 2^20), then x = 2^24 + cum(c_l).  So the
    states read (256, cum(c_l)) and the renormalization words, in decoding
    order (step 0, lanes ascending), are cum(b_0) .. cum(b_63)."""
    freq = np.zeros((257, 256), np.uint16)
    freq[0, 0] = 4032
    freq[0, 1:65] = 1
    cum = lambda s: 4031 + s
    sym = np.zeros(128, np.uint8)
    for l in range(64):
        sym[2 * l] = 64 - l
        sym[2 * l + 1] = l + 1
    w, off = orc.ans_encode(sym, 0, 2, freq)
    want = []
    for l in range(64):
        want += [256, cum(64 - l)]
    want += [cum(l + 1) for l in range(64)]
    assert list(off) == [0, 192]
    assert list(w) == want
    assert np.array_equal(orc.ans_decode(w, off, 128, 0, 2, freq), sym)


def test_one_symbol_state(orc):
    # one lane, one symbol s = 1 with f = 1024, cum = 3072: from x = 2^16,
    # C = (2^16 // 1024) * 4096 + 3072 + 0 = 265216 = 4 * 2^16 + 3072
    freq = np.zeros((257, 256), np.uint16)
    freq[0, 0], freq[0, 1] = 3072, 1024
    w, off = orc.ans_encode(np.array([1], np.uint8), 0, 1, freq)
    assert list(w[:2]) == [4, 3072]
    assert np.all(w[2::2] == 1) and np.all(w[3::2] == 0) and w.size == 128


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("lane_len", [1, 3, 64, 512])
@pytest.mark.parametrize("n", [0, 1, 63, 65, 5000, 70001])
def test_round_trip(orc, order, lane_len, n):
    rng = np.random.default_rng(n * 7 + lane_len + order)
    # a Markov source: the next symbol depends on the previous one
    sym = np.zeros(n, np.uint8)
    for i in range(1, n):
        sym[i] = (sym[i - 1] * 5 + rng.geometric(0.4)) % 37
    f = orc.ans_model(sym, order, lane_len)
    w, off = orc.ans_encode(sym, order, lane_len, f)
    out = orc.ans_decode(w, off, n, order, lane_len, f)
    assert out is not None and np.array_equal(out, sym)


def test_code_length_tracks_ideal(orc):
    """Renormalization words plus the final states carry the ideal code
    length -sum log2(f / M) up to the rANS rounding loss: per symbol at most
    log2(1 + f / x) <= log2(17 / 16) (x >= 16 f before each step), far less in
    practice; and never less than the ideal minus the states' 32 bits."""
    rng = np.random.default_rng(11)
    n = 200000
    sym = np.minimum(rng.geometric(0.2, n) - 1, 255).astype(np.uint8)
    for order, S in ((0, 256), (1, 512)):
        f = orc.ans_model(sym, order, S)
        ideal = orc.ans_ideal_bits(sym, order, S, f)
        w, off = orc.ans_encode(sym, order, S, f)
        nb = len(off) - 1
        total = 16.0 * w.size
        assert total >= ideal - 1e-6
        assert total <= ideal + 32 * 64 * nb + 0.0875 * n
        # in practice the loss is tiny
        assert total - 32 * 64 * nb <= ideal * 1.001


def test_dyadic_ideal_bits_closed_form(orc):
    sym = np.repeat(np.arange(4, dtype=np.uint8), [2048, 1024, 512, 512])
    f = orc.ans_model(sym, 0, 64)
    want = 2048 * 1 + 1024 * 2 + 512 * 3 + 512 * 3
    assert orc.ans_ideal_bits(sym, 0, 64, f) == pytest.approx(want, abs=1e-9)


def test_decode_rejects_damage(orc):
    rng = np.random.default_rng(5)
    sym = rng.integers(0, 9, 20000).astype(np.uint8)
    f = orc.ans_model(sym, 1, 64)
    w, off = orc.ans_encode(sym, 1, 64, f)
    short = off.copy()
    short[-1] -= 1
    assert orc.ans_decode(w, short, sym.size, 1, 64, f) is None
    # a model without the stream's symbols fails
    g = np.zeros_like(f)
    g[:, 200] = 4096
    assert orc.ans_decode(w, off, sym.size, 1, 64, g) is None


# ---------------------------------------------------------------------------
# attributes: Morton order, DPCM byte planes, Fourier positional embedding
# ---------------------------------------------------------------------------
def test_morton_order_hand_example(orc):
    y, q, m, n = one_point_cloud([(3, 3, 3), (0, 0, 0), (1, 0, 0), (0, 0, 0), (2, 2, 2)])
    m[4] = 0                                   # not kept
    r = orc.octree_tokens(y, q, m, n)
    perm = orc.morton_order(y, q, m, n, r["depth"], r["kmin"])
    # codes 63, 0, 4, 0: by code, then index
    assert list(perm) == [1, 3, 2, 0]


def test_morton_order_matches_octree(orc):
    rng = np.random.default_rng(21)
    n = 6000
    y = np.zeros((59, synth.pad64(n)), np.float32)
    y[:3, :n] = rng.normal(0, 0.3, (3, n))
    q = np.full(59, 0.05, np.float32)
    m = (rng.random(n) < 0.7).astype(np.uint8)
    r = orc.octree_tokens(y, q, m, n)
    perm = orc.morton_order(y, q, m, n, r["depth"], r["kmin"])
    assert sorted(perm) == list(np.nonzero(m)[0])
    # voxels along the order: the octree's distinct codes with their copies
    yhat, k = orc.fakequant(y, q, n)
    got = np.unique(k[:3, perm].T, axis=0, return_index=True)[1]
    assert len(got) == r["unique"]
    xyz = orc.voxel_positions(r["codes"], r["dup"], r["depth"], r["kmin"], q)
    assert np.array_equal(xyz, yhat[:3, perm])
    # ties (copies of one voxel) by index
    kk = [tuple(k[:3, i]) for i in perm]
    for a in range(1, len(perm)):
        if kk[a] == kk[a - 1]:
            assert perm[a] > perm[a - 1]


def test_attr_planes_hand_example(orc):
    # values v = k - kmin = [5, 7, 6, 6 | 2], groups of 4: residuals 5, 2, -1,
    # 0 | 2 -> zigzag 10, 4, 1, 0 | 4; width 3 -> one plane
    y = np.array([5, 7, 6, 6, 2], np.float32)
    perm = np.arange(5)
    pl = orc.attr_planes(y, 1.0, perm, 0, 3, 4)
    assert pl.shape == (1, 5) and list(pl[0]) == [10, 4, 1, 0, 4]
    # width 8 -> two planes, most significant first; kmin shifts the values
    y = np.array([300, 40, 299], np.float32)
    pl = orc.attr_planes(y, 1.0, np.arange(3), 40, 8, 64)
    z = [2 * 260, 2 * 260 - 1, 2 * 259]          # 260, then -260, then +259
    assert list(pl[0]) == [v >> 8 for v in z] and list(pl[1]) == [v & 255 for v in z]
    assert orc.attr_plane_count(0) == 0 and orc.attr_plane_count(7) == 1
    assert orc.attr_plane_count(8) == 2 and orc.attr_plane_count(32) == 5


@pytest.mark.parametrize("S", [1, 7, 256])
def test_attr_round_trip_equals_quantizer(orc, S):
    sc = synth.make_tiny(3000, 32, 32, seed=4)
    q = synth.learnable_qsteps(5)
    m = sc.given_mask
    n = sc.n
    yhat, k = orc.fakequant(sc.params, q, n)
    bits, kmin, kmax, width = orc.fixed_length_bits(k, m, n)
    r = orc.octree_tokens(sc.params, q, m, n)
    perm = orc.morton_order(sc.params, q, m, n, r["depth"], r["kmin"])
    for c in orc.ATTR_CHANNELS:
        pl = orc.attr_planes(sc.params[c], q[c], perm, kmin[c], width[c], S)
        assert pl.shape[0] == orc.attr_plane_count(int(width[c]))
        back = orc.attr_reconstruct(pl, kmin[c], q[c], S, perm.size)
        assert np.array_equal(back, yhat[c, perm]), c


def test_fourier_features_closed_form(orc):
    L = 12
    phi = orc.fourier_features(np.array([[0.0, 0.25, -0.5]]), L)
    assert phi.shape == (1, 3 + 6 * L)
    s = phi[0, 3:3 + 3 * L].reshape(L, 3)
    c = phi[0, 3 + 3 * L:].reshape(L, 3)
    # x = 0: sin 0, cos 1 in every band
    assert np.allclose(s[:, 0], 0, atol=1e-15) and np.allclose(c[:, 0], 1, atol=1e-15)
    # y = 1/4: band 0 at pi/2, band 1 at pi, then whole turns
    assert np.isclose(s[0, 1], 1) and np.isclose(c[1, 1], -1)
    assert np.allclose(s[1:, 1], 0, atol=1e-12) and np.allclose(c[2:, 1], 1, atol=1e-12)
    # z = -1/2: band 0 at -pi
    assert np.isclose(c[0, 2], -1) and np.allclose(c[1:, 2], 1, atol=1e-12)
    # the linear map picks features: PE = W phi + b
    W = np.zeros((32, 3 + 6 * L))
    W[0, 0] = 2.0           # 2 mu_x
    W[1, 3 + 3 * 0 + 1] = 1.0   # sin band 0 of y
    W[2, 3 + 3 * L + 3 * 1 + 1] = -1.0  # -cos band 1 of y
    b = np.arange(32, dtype=np.float64)
    pe = orc.positional_embedding(np.array([[0.5, 0.25, 0.0]]), W, b, L)
    assert np.allclose(pe[0, :3], [1.0 + 0, 1.0 + 1, 1.0 + 2])
    assert np.allclose(pe[0, 3:], b[3:])


def test_attr_planes_without_prediction(orc):
    # predictor 0: the values themselves, width bits -> ceil(width / 8) planes
    y = np.array([5, 7, 6, 6, 2], np.float32)
    pl = orc.attr_planes(y, 1.0, np.arange(5), 0, 3, 4, predictor=0)
    assert pl.shape == (1, 5) and list(pl[0]) == [5, 7, 6, 6, 2]
    y = np.array([300, 40, 299], np.float32)
    pl = orc.attr_planes(y, 1.0, np.arange(3), 40, 9, 64, predictor=0)
    assert list(pl[0]) == [1, 0, 1] and list(pl[1]) == [4, 0, 3]
    assert orc.attr_plane_count(8, 0) == 1 and orc.attr_plane_count(9, 0) == 2
    sc = synth.make_tiny(2000, 32, 32, seed=6)
    q = synth.learnable_qsteps(7)
    yhat, k = orc.fakequant(sc.params, q, sc.n)
    bits, kmin, kmax, width = orc.fixed_length_bits(k, sc.given_mask, sc.n)
    perm = np.nonzero(sc.given_mask)[0]
    for c in orc.ATTR_CHANNELS:
        pl = orc.attr_planes(sc.params[c], q[c], perm, kmin[c], width[c], 16, predictor=0)
        back = orc.attr_reconstruct(pl, kmin[c], q[c], 16, perm.size, predictor=0)
        assert np.array_equal(back, yhat[c, perm]), c


# ---------------------------------------------------------------------------
# stream container marshalling (host code, no GPU)
# ---------------------------------------------------------------------------
def test_container_model_and_stream_round_trip(orc):
    from paper_2607_12656_amd import coding
    rng = np.random.default_rng(9)
    sym = rng.integers(0, 40, 20000).astype(np.uint8)
    for order in (0, 1):
        f = orc.ans_model(sym, order, 64)
        b = coding.pack_model(f, order)
        g, o, pos = coding.unpack_model(b, 0)
        assert o == order and pos == len(b) and np.array_equal(f, g)
        used = (f.sum(axis=1) > 0).sum()
        nz = int((f > 0).sum())
        assert len(b) == 1 + (33 if order else 0) + 2 * used + 3 * nz
        w, off = orc.ans_encode(sym, order, 64, f)
        s = coding.pack_stream(w, off)
        w2, off2, pos = coding.unpack_stream(s, 0)
        assert pos == len(s) and np.array_equal(w, w2) and np.array_equal(off, off2)
        # the unpacked pieces decode
        assert np.array_equal(orc.ans_decode(w2, off2, sym.size, order, 64, g), sym)
