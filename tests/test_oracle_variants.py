"""Pins of the decoder-variant oracle (oracle/variants.py), CPU only.

- The transposed AAN flowgraph, in exact arithmetic, is the orthonormal
  8-point IDCT once its inputs carry the 1 / (sqrt(8) s(k)) scale: every
  unit input reproduces one DCT basis vector (a swapped constant, sign or
  index fails).
- The float method against the FP64 IDCT (T.81 A.3.3): off by at most one
  level, on random blocks of the whole input domain.
- The ifast method against the FP64 IDCT: within its fixed-point error.
- DC-only blocks: every method gives round(c * q / 8) + 128 exactly.
- Samplings: the vertical filter is the pinned horizontal one transposed;
  the variants decode equals the main oracle on the samplings both cover;
  grayscale equals the luma channel of a 4:4:4 image with neutral chroma.
"""
import math

import numpy as np
import pytest

import oracle
import oracle.variants as V
from oracle.upsample import fancy_h2v1

# x = C @ F @ C.T for the orthonormal DCT (T.81 A.3.3 normalisation)
C = np.array([[(math.sqrt(0.125) if k == 0 else 0.5) * math.cos((2 * m + 1) * k * math.pi / 16)
               for k in range(8)] for m in range(8)])


def exact_idct(coef, q):
    F = np.asarray(coef, dtype=np.float64).reshape(-1, 8, 8) * np.asarray(q, np.float64).reshape(8, 8)
    return np.einsum("mu,nuv,kv->nmk", C, F, C)


def test_aan_flowgraph_is_the_scaled_orthonormal_idct():
    for k in range(8):
        Y = [0.0] * 8
        Y[k] = 1.0 / (math.sqrt(8.0) * V.S[k])
        out = np.array(V.aan_1d(Y, lambda v, name: v * {"r": V.C_R, "c5": V.C_5, "c2": V.C_2, "c4": V.C_4}[name]))
        assert np.allclose(out, C[:, k], atol=1e-14), k
    # the scale factors in closed form
    assert V.S[0] == 1.0
    for k in range(1, 8):
        assert math.isclose(V.S[k], math.sqrt(2) * math.cos(k * math.pi / 16), rel_tol=1e-15)


def _blocks(rng, n, q):
    """Random blocks on the documented domain |c * q| <= 1155: dense, sparse
    and extreme-sign blocks."""
    lim = 1155 // q
    out = rng.integers(-lim, lim + 1, (n, 64))
    sparse = rng.random((n, 64)) < 0.8
    out[n // 3: 2 * n // 3][sparse[n // 3: 2 * n // 3]] = 0
    out[2 * n // 3:] = rng.choice([-lim, lim], (n - 2 * n // 3, 64))
    return out.astype(np.int16)


@pytest.mark.parametrize("qv", [1, 2, 5, 16])
def test_float_within_one_level_of_fp64(qv):
    rng = np.random.default_rng(qv)
    q = np.full(64, qv, np.uint16)
    coef = _blocks(rng, 600, qv)
    ref = np.clip(np.floor(exact_idct(coef, q) + 128.5), 0, 255)
    got = V.idct_float(coef, q).astype(np.float64)
    d = np.abs(got - ref)
    assert d.max() <= 1
    assert (d == 0).mean() > 0.995


# measured bounds of the fixed-point design on the whole domain, extreme
# blocks included (the multipliers' six fraction bits dominate at small q)
@pytest.mark.parametrize("qv,max_err,mean_err", [(1, 22, 0.4), (2, 14, 0.25), (8, 3, 0.06), (30, 2, 0.04)])
def test_ifast_within_its_fixed_point_error(qv, max_err, mean_err):
    rng = np.random.default_rng(100 + qv)
    q = np.full(64, qv, np.uint16)
    coef = _blocks(rng, 600, qv)
    ref = np.clip(np.floor(exact_idct(coef, q) + 128.5), 0, 255)
    d = np.abs(V.idct_ifast(coef, q).astype(np.float64) - ref)
    assert d.max() <= max_err
    assert d.mean() <= mean_err


def test_ifast_on_encoded_photographic_blocks():
    # blocks of a textured image through the encoder at quality 75
    from synth import encode, images
    frame, coef, qt = encode.encode_rgb(images.texture_rgb(96, 64, 21, sigma=12), "444", 75)
    c = np.asarray(coef).reshape(-1, 3, 64)
    for comp in range(3):
        q = qt[frame["qsel"][comp]]
        ref = np.clip(np.floor(exact_idct(c[:, comp], q) + 128.5), 0, 255)
        d = np.abs(V.idct_ifast(c[:, comp], q).astype(np.float64) - ref)
        assert d.max() <= 2 and d.mean() < 0.05


def test_ifast_stays_in_int32_on_the_domain():
    # the sign patterns of every output's basis product drive each output to
    # its largest magnitude; random extreme signs cover the inner nodes
    T = np.einsum("mu,kv->mkuv", C, C).reshape(64, 64)
    q = np.ones(64, np.uint16)
    V.idct_ifast((np.sign(T) * 1155).astype(np.int16), q)
    V.idct_ifast(np.random.default_rng(3).choice([-1155, 1155], (4000, 64)).astype(np.int16), q)


@pytest.mark.parametrize("method", V.IDCT_METHODS)
def test_dc_only_blocks_are_exact(method):
    rng = np.random.default_rng(7)
    for qv in (1, 3, 8, 16, 99):
        q = rng.integers(1, 256, 64).astype(np.uint16)
        q[0] = qv
        dc = np.arange(-1155 // qv, 1155 // qv + 1)
        coef = np.zeros((len(dc), 64), np.int16)
        coef[:, 0] = dc
        want = np.clip(np.floor(dc * qv / 8 + 0.5) + 128, 0, 255)
        got = V.idct(coef, q, method)
        assert np.array_equal(got, np.broadcast_to(want[:, None, None], got.shape)), (method, qv)


def test_vertical_filter_is_the_horizontal_one_transposed():
    rng = np.random.default_rng(11)
    for h, w in ((1, 5), (7, 3), (16, 9)):
        c = rng.integers(0, 256, (h, w)).astype(np.uint8)
        assert np.array_equal(V.fancy_h1v2(c), fancy_h2v1(c.T).T)
    assert np.array_equal(V.fancy_h1v2(np.full((4, 4), 77, np.uint8)), np.full((8, 4), 77))


def _frame(w, h, hy, vy):
    return {"width": w, "height": h, "h": (hy, 1, 1), "v": (vy, 1, 1), "qsel": (0, 1, 1)}


def _coef(rng, frame):
    n = V.variant_geometry(frame)["n_blocks"]
    c = rng.integers(-20, 21, (n, 64))
    c[:, 0] = rng.integers(-100, 101, n)
    return c.astype(np.int16)


def test_variants_equal_the_main_oracle_where_both_apply():
    rng = np.random.default_rng(5)
    qt = rng.integers(1, 12, (4, 64)).astype(np.uint16)
    for hy, vy in ((1, 1), (2, 1), (2, 2)):
        for w, h in ((37, 21), (64, 48)):
            fr = _frame(w, h, hy, vy)
            c = _coef(rng, fr)
            for mode in ("simple", "fancy"):
                assert np.array_equal(V.decode_variant(fr, c, qt, "islow", mode), oracle.decode(fr, c, qt, mode))


def test_new_samplings_compose_from_their_planes():
    # (1,2) and (4,1): colour conversion of the luma plane and the chroma
    # planes upsampled by the pinned filters
    rng = np.random.default_rng(9)
    qt = rng.integers(1, 12, (4, 64)).astype(np.uint16)
    for hy, vy, mode in ((1, 2, "fancy"), (1, 2, "simple"), (4, 1, "fancy"), (4, 1, "simple")):
        fr = _frame(45, 35, hy, vy)
        c = _coef(rng, fr)
        p = V.planes(fr, c, qt, "islow")
        if (hy, vy) == (1, 2) and mode == "fancy":
            cb, cr = fancy_h2v1(p[1].T).T, fancy_h2v1(p[2].T).T
        else:
            cb, cr = (np.repeat(np.repeat(x.astype(np.int64), vy, 0), hy, 1) for x in p[1:])
        want = oracle.ycc_to_rgb(p[0][:35, :45], cb[:35, :45], cr[:35, :45])
        assert np.array_equal(V.decode_variant(fr, c, qt, "islow", mode), want)


@pytest.mark.parametrize("method", V.IDCT_METHODS)
def test_grayscale_is_the_luma_of_neutral_chroma(method):
    rng = np.random.default_rng(13)
    qt = rng.integers(1, 12, (4, 64)).astype(np.uint16)
    w, h = 29, 19
    gray = {"width": w, "height": h, "ncomp": 1, "h": (1, 1, 1), "v": (1, 1, 1), "qsel": (2, 0, 0)}
    cg = _coef(rng, gray)
    fr = {"width": w, "height": h, "h": (1, 1, 1), "v": (1, 1, 1), "qsel": (2, 0, 0)}
    c3 = np.zeros((cg.shape[0] * 3, 64), np.int16)
    c3[0::3] = cg              # chroma blocks all zero: Cb = Cr = 128
    rgb = V.decode_variant(fr, c3, qt, method, "fancy")
    g = V.decode_variant(gray, cg, qt, method, "fancy")
    assert g.shape == (h, w)
    for ch in range(3):
        assert np.array_equal(rgb[..., ch], g)


def test_rejects_unknown_variants():
    with pytest.raises(ValueError):
        V.variant_geometry(_frame(8, 8, 4, 2))
    with pytest.raises(ValueError):
        V.idct(np.zeros((1, 64), np.int16), np.ones(64, np.uint16), "aan")


# ---- scaled decoding ----------------------------------------------------------------------


def _exact_reduced(coef, q, n):
    Cn = np.array([[(math.sqrt(0.5) if u == 0 else 1.0) * math.cos((2 * m + 1) * u * math.pi / (2 * n))
                    for u in range(n)] for m in range(n)])
    F = (np.asarray(coef, np.float64).reshape(-1, 8, 8) * np.asarray(q, np.float64).reshape(8, 8))[:, :n, :n]
    return 0.25 * np.einsum("mu,kuv,nv->kmn", Cn, F, Cn)


@pytest.mark.parametrize("n", [4, 2, 1])
def test_reduced_idct_within_one_level_of_fp64(n):
    rng = np.random.default_rng(40 + n)
    for qv in (1, 3, 12):
        q = np.full(64, qv, np.uint16)
        coef = _blocks(rng, 500, qv)
        ref = np.clip(np.floor(_exact_reduced(coef, q, n) + 128.5), 0, 255)
        d = np.abs(V.idct_reduced(coef, q, n).astype(np.float64) - ref)
        assert d.max() <= 1 and (d == 0).mean() > 0.95


@pytest.mark.parametrize("n", [4, 2, 1])
def test_reduced_dc_only_is_exact(n):
    for qv in (1, 5, 16):
        q = np.full(64, 7, np.uint16)
        q[0] = qv
        dc = np.arange(-1155 // qv, 1155 // qv + 1)
        coef = np.zeros((len(dc), 64), np.int16)
        coef[:, 0] = dc
        want = np.clip(np.floor(dc * qv / 8 + 0.5) + 128, 0, 255)
        got = V.idct_reduced(coef, q, n)
        assert np.array_equal(got, np.broadcast_to(want[:, None, None], got.shape))


def test_reduced_2x2_is_the_exact_haar_average():
    # N = 2: sqrt(2) cos(pi/4) = 1, so the transform is exact integer
    # arithmetic: x(m, n) = round((F00 + sm F10 + sn F01 + sm sn F11) / 8) + 128
    rng = np.random.default_rng(8)
    q = rng.integers(1, 9, 64).astype(np.uint16)
    coef = rng.integers(-100, 101, (300, 64)).astype(np.int16)
    F = coef.reshape(-1, 8, 8).astype(np.int64) * q.reshape(8, 8).astype(np.int64)
    got = V.idct_reduced(coef, q, 2)
    for m, sm in ((0, 1), (1, -1)):
        for n, sn in ((0, 1), (1, -1)):
            s = F[:, 0, 0] + sm * F[:, 1, 0] + sn * F[:, 0, 1] + sm * sn * F[:, 1, 1]
            want = np.clip(np.floor(s / 8 + 0.5) + 128, 0, 255)
            assert np.array_equal(got[:, m, n], want)


@pytest.mark.parametrize("samp,scale", [("444", 2), ("444", 4), ("420", 2), ("420", 8), ("422", 4)])
def test_scaled_decode_is_close_to_a_box_downscale(samp, scale):
    # a smooth image: the scaled decode against the full-size decode averaged
    # over scale x scale boxes
    from synth import encode, images
    w, h = 128, 96
    frame, coef, qt = encode.encode_rgb(images.texture_rgb(w, h, 5, sigma=2), samp, 95)
    full = V.decode_variant(frame, coef, qt, "islow", "fancy").astype(np.float64)
    box = full.reshape(h // scale, scale, w // scale, scale, 3).mean(axis=(1, 3))
    got = V.decode_variant(frame, coef, qt, "islow", "fancy", scale).astype(np.float64)
    assert got.shape == (h // scale, w // scale, 3)
    # chroma upsampled at the reduced size differs from averaged full-size
    # chroma by a few levels; a one-pixel shift costs several times more
    err = np.abs(got - box).mean()
    assert err < (2.5 if samp == "444" else 5.0)
    assert np.abs(got[:, 1:] - box[:, :-1]).mean() > 2 * err
    assert np.abs(got[1:] - box[:-1]).mean() > 2 * err


def test_scaled_output_sizes():
    rng = np.random.default_rng(2)
    qt = np.ones((4, 64), np.uint16)
    for w, h, hy, vy in ((37, 21, 2, 2), (1, 1, 4, 1), (17, 9, 1, 2), (65, 33, 2, 1)):
        fr = {"width": w, "height": h, "h": (hy, 1, 1), "v": (vy, 1, 1), "qsel": (0, 1, 1)}
        c = _coef(rng, fr)
        for s in (2, 4, 8):
            assert V.decode_variant(fr, c, qt, "islow", "fancy", s).shape == (-(-h // s), -(-w // s), 3)
            p = V.planes(fr, c, qt, "islow", s)
            assert p[1].shape == (-(-h // (vy * s)), -(-w // (hy * s)))
    with pytest.raises(ValueError):
        V.planes(fr, c, qt, "ifast", 2)
    with pytest.raises(ValueError):
        V.planes(fr, c, qt, "islow", 3)


# ---- ifast: constants, multipliers and bias ----------------------------------------------


def _graph_response(mul, amplitude):
    """8x8 matrix E[n][k]: the 1-D graph's output n for an impulse of the
    given amplitude at input k, divided by the amplitude."""
    E = np.zeros((8, 8))
    for k in range(8):
        Y = [np.array([0], dtype=np.int64) for _ in range(8)]
        Y[k] = np.array([amplitude], dtype=np.int64)
        out = V.aan_1d(Y, mul, V._ifast_add, V._ifast_sub)
        E[:, k] = [int(o[0]) / amplitude for o in out]
    return E


def test_ifast_graph_constants_are_the_nearest_9_bit_roundings():
    # Every path of the transposed AAN graph crosses at most one constant
    # multiply, so its impulse response is M0 + sum_j (K_j / 2^9) M_j with
    # integer structure matrices.  Recover the four K_j from the fixed-point
    # graph's behaviour at a large amplitude (truncation below 2^-10) and
    # check each against the real constant: only the correctly rounded
    # integer lies within 1/2, so a constant one LSB off fails.
    names = ("r", "c5", "c2", "c4")
    real = {"r": V.C_R, "c5": V.C_5, "c2": V.C_2, "c4": V.C_4}
    structure = {}
    for j in names + (None,):
        structure[j] = np.array([[float(v) for v in col] for col in
                                 [V.aan_1d([1.0 if i == k else 0.0 for i in range(8)],
                                           lambda v, name, j=j: v if name == j else 0.0) for k in range(8)]]).T
    M0 = structure[None]
    for j in names:
        structure[j] = structure[j] - M0   # the terms through constant j alone
    E = _graph_response(V._ifast_mul, 1 << 20)
    A = np.stack([structure[j].ravel() for j in names], axis=1)
    k, *_ = np.linalg.lstsq(A, (E - M0).ravel(), rcond=None)
    K = k * (1 << V.IFAST_CONST_BITS)
    resid = np.abs(A @ k - (E - M0).ravel()).max()
    assert resid < 1e-5
    for j, kj in zip(names, K):
        assert abs(kj - round(kj)) < 1e-3, (j, kj)
        assert abs(round(kj) - real[j] * (1 << V.IFAST_CONST_BITS)) < 0.5, (j, kj)


def test_ifast_multipliers_round_the_scaled_table():
    # M(u, v) approximates q * 2^6 / (s(u) s(v)) through two roundings (the
    # 14-bit table entry, then the product to 6 fraction bits); at q = 256
    # the second is exact, so M is the table entry itself
    exact = np.array([[(1 << 14) / (V.S[u] * V.S[v]) for v in range(8)] for u in range(8)])
    a = V.ifast_multipliers(np.full(64, 256, np.uint16)).reshape(8, 8)
    assert np.all(np.abs(a - exact) <= 0.5)
    for qv in (1, 7, 99, 255):
        m = V.ifast_multipliers(np.full(64, qv, np.uint16)).reshape(8, 8)
        assert np.all(np.abs(m - qv * exact / 256) <= 0.5 + qv * 0.5 / 256 + 1e-9)
    # the DC multiplier is exact: q * 2^6
    for qv in range(1, 256):
        assert V.ifast_multipliers(np.full(64, qv, np.uint16)).reshape(64)[0] == qv << 6


def test_ifast_per_position_error_is_unbiased_on_photographic_blocks():
    # IEEE-1180-style statistics against the FP64 IDCT on encoded texture
    # blocks (quality 50, 75, 90), over samples away from the clamp: per
    # position, the mean signed error and the mean squared error stay small
    # (a wrong rounding bias shifts every mean by about 1/2)
    from synth import encode, images
    errs = []
    for seed, qual in ((21, 75), (22, 50), (23, 90)):
        frame, coef, qt = encode.encode_rgb(images.texture_rgb(256, 192, seed, sigma=12), "444", qual)
        c = np.asarray(coef).reshape(-1, 3, 64)
        for comp in range(3):
            q = qt[frame["qsel"][comp]]
            ex = exact_idct(c[:, comp], q) + 128
            e = V.idct_ifast(c[:, comp], q).astype(np.float64) - np.clip(np.floor(ex + 0.5), 0, 255)
            e[(ex < 0.5) | (ex > 254.5)] = np.nan
            errs.append(e)
    e = np.concatenate(errs)
    assert np.nanmax(np.abs(np.nanmean(e, axis=0))) < 0.05
    assert np.nanmax(np.nanmean(e * e, axis=0)) < 0.06
