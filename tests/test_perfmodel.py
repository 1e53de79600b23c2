"""The performance model of the paper's Sec. 5.1 (CPU only: host code).

The oracle (oracle/perfmodel.py) is pinned first:
- numpy's own polynomial routines (polyfit, polyval, polyval2d);
- exact recovery of known polynomials;
- the AIC's closed form;
- AIC degree choice on data of known degree.
The library's fits, Horner evaluation and predictions (include/mjd.h) then
match the oracle's."""
import math

import numpy as np
import pytest
from numpy.polynomial import polynomial as P

import oracle.perfmodel as O


@pytest.fixture(scope="module")
def M():
    import paper_1311_5304_amd as mod
    return mod


def _grid2(rng, n, lo=0.1, hi=6.0):
    return rng.uniform(lo, hi, n), rng.uniform(lo, hi, n)


# ---- the oracle against numpy and the mathematics ---------------------------------------

def test_oracle_fit1_equals_numpy_polyfit_at_its_degree():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 3, 80)
    y = np.sin(x) + 0.01 * rng.standard_normal(80)
    deg, coef, _ = O.fit1(x, y)
    assert np.allclose(coef, P.polyfit(x, y, deg), rtol=1e-8, atol=1e-10)


def test_oracle_recovers_exact_polynomials_with_fewest_terms():
    rng = np.random.default_rng(4)
    x = rng.uniform(-2, 2, 50)
    true = [0.25, -1.5, 0.0, 0.75]
    deg, coef, a = O.fit1(x, P.polyval(x, true))
    assert deg == 3 and np.allclose(coef, true, atol=1e-10)
    y = P.polyval(x, true)
    assert math.isclose(a, 50 * math.log(O.EXACT_FLOOR * float(y @ y) / 50) + 2 * 4)
    a2, b2 = _grid2(rng, 70)
    c = np.zeros((3, 3))
    c[0, 0], c[1, 1], c[2, 0], c[0, 1] = 2.0, 1.0, 0.3, -0.5  # 2 + ab + 0.3a^2 - 0.5b
    deg, coef, _ = O.fit2(a2, b2, P.polyval2d(a2, b2, c))
    assert deg == 2
    for cf, (i, j) in zip(coef, O.terms2(deg)):
        assert math.isclose(cf, c[i, j], abs_tol=1e-9)


def test_oracle_eval_equals_numpy_polyval():
    rng = np.random.default_rng(5)
    for deg in range(8):
        coef = rng.standard_normal(deg + 1)
        for x in rng.uniform(-2, 2, 5):
            assert math.isclose(O.eval1(deg, coef, x), P.polyval(x, coef), rel_tol=1e-12, abs_tol=1e-12)
        t = O.terms2(deg)
        cf = rng.standard_normal(len(t))
        c = np.zeros((deg + 1, deg + 1))
        for v, (i, j) in zip(cf, t):
            c[i, j] = v
        for a, b in zip(*_grid2(rng, 5, 0.0, 3.0)):
            assert math.isclose(O.eval2(deg, cf, a, b), P.polyval2d(a, b, c), rel_tol=1e-10, abs_tol=1e-10)


def test_oracle_aic_picks_the_true_degree_of_noisy_data():
    rng = np.random.default_rng(6)
    x = rng.uniform(0, 2, 300)
    y = 1.0 + 0.5 * x - 0.8 * x * x + 1e-3 * rng.standard_normal(300)
    assert O.fit1(x, y)[0] == 2
    a, b = _grid2(rng, 400)
    z = 3.0 + a * b + 1e-3 * rng.standard_normal(400)
    assert O.fit2(a, b, z)[0] == 2


def test_oracle_predict_composes_the_equations():
    model = {"huff_per_pixel": (1, [2e-9, 4e-9]), "o_w": (0, [1e-4]), "t_kernel": (1, [1e-5, 2e-5, 3e-5]),
             "o_r": (0, [2e-4])}
    p = O.predict(model, 2048, 1024, 2048 * 1024 // 2)
    assert math.isclose(p["d"], 0.5)
    assert math.isclose(p["t_huff"], (2e-9 + 4e-9 * 0.5) * 2048 * 1024)
    # t_kernel terms in (i, j) order (0,0), (0,1), (1,0): c00 + c01 * b + c10 * a, a = 2, b = 1
    assert math.isclose(p["t_kernel"], 1e-5 + 2e-5 * 1 + 3e-5 * 2)
    assert math.isclose(p["total"], p["t_huff"] + 1e-4 + p["t_kernel"] + 2e-4)


# ---- the library against the oracle ------------------------------------------------------

def _as_list1(p):
    return [p.c[i] for i in range(p.degree + 1)]


def _cases1():
    rng = np.random.default_rng(7)
    x = rng.uniform(0.05, 2.0, 120)
    yield x, 3e-9 + 2e-9 * x + 1e-9 * x * x                         # exact quadratic
    yield x, 1e-9 * (1 + x) + 1e-11 * rng.standard_normal(120)       # noisy line
    yield x, np.exp(-x) + 1e-4 * rng.standard_normal(120)           # smooth, not polynomial
    x2 = rng.uniform(0, 1, 12)
    yield x2, np.cos(3 * x2)                                          # few samples


def _cases2():
    rng = np.random.default_rng(8)
    a, b = _grid2(rng, 150, 0.25, 6.0)
    yield a, b, 2e-5 + 1e-4 * a * b                                  # exact: linear in pixels
    yield a, b, 1e-5 + 8e-5 * a * b + 1e-6 * rng.standard_normal(150)  # noisy
    yield a, b, 1e-3 * np.sqrt(a * b + 1)                            # smooth, not polynomial


def test_fit1_matches_oracle(M):
    for x, y in _cases1():
        p, aic = M.mjd_poly1_fit(x, y)
        deg, coef, oaic = O.fit1(x, y)
        assert p.degree == deg
        assert math.isclose(aic, oaic, rel_tol=1e-6, abs_tol=1e-6)
        for v in np.linspace(x.min(), x.max(), 9):
            assert math.isclose(M.mjd_poly1_eval(p, v), O.eval1(deg, coef, v), rel_tol=1e-7,
                                abs_tol=1e-9 * float(np.abs(y).max()))


def test_fit2_matches_oracle(M):
    for a, b, y in _cases2():
        p, aic = M.mjd_poly2_fit(a, b, y)
        deg, coef, oaic = O.fit2(a, b, y)
        assert p.degree == deg
        assert math.isclose(aic, oaic, rel_tol=1e-6, abs_tol=1e-6)
        rng = np.random.default_rng(9)
        for u, v in zip(*_grid2(rng, 9, 0.25, 6.0)):
            assert math.isclose(M.mjd_poly2_eval(p, u, v), O.eval2(deg, coef, u, v), rel_tol=1e-7,
                                abs_tol=1e-9 * float(np.abs(y).max()))


def test_horner_evaluation_equals_the_term_sum(M):
    rng = np.random.default_rng(10)
    for deg in range(8):
        p1 = M.mjd_poly1()
        p1.degree = deg
        coef = rng.standard_normal(deg + 1)
        for i, c in enumerate(coef):
            p1.c[i] = c
        p2 = M.mjd_poly2()
        p2.degree = deg
        cf = rng.standard_normal(len(O.terms2(deg)))
        for i, c in enumerate(cf):
            p2.c[i] = c
        for x, y in zip(*_grid2(rng, 6, -1.5, 1.5)):
            assert math.isclose(M.mjd_poly1_eval(p1, x), O.eval1(deg, coef, x), rel_tol=1e-12, abs_tol=1e-12)
            assert math.isclose(M.mjd_poly2_eval(p2, x, y), O.eval2(deg, cf, x, y), rel_tol=1e-10, abs_tol=1e-10)


def test_predict_matches_oracle(M):
    rng = np.random.default_rng(11)
    d = rng.uniform(0.05, 1.5, 60)
    hp, _ = M.mjd_poly1_fit(d, 2e-9 + 3e-9 * d + 1e-11 * rng.standard_normal(60))
    a, b = _grid2(rng, 120, 0.25, 6.0)
    parts = {}
    model = M.mjd_model()
    model.huff_per_pixel = hp
    omodel = {"huff_per_pixel": (hp.degree, _as_list1(hp))}
    for name, scale in (("o_w", 4e-5), ("t_kernel", 3e-6), ("o_r", 6e-5)):
        y = 5e-6 + scale * a * b + 1e-7 * rng.standard_normal(120)
        p, _ = M.mjd_poly2_fit(a, b, y)
        setattr(model, name, p)
        parts[name] = p
        omodel[name] = (p.degree, [p.c[i] for i in range(len(O.terms2(p.degree)))])
    for w, h, nbytes in ((4096, 3072, 4_000_000), (640, 480, 90_000), (6000, 4000, 9_500_000)):
        got = M.mjd_model_predict(model, w, h, nbytes)
        exp = O.predict(omodel, w, h, nbytes)
        for k in ("d", "t_huff", "o_w", "t_kernel", "o_r", "p_gpu", "total"):
            assert math.isclose(got[k], exp[k], rel_tol=1e-9, abs_tol=1e-15), k


def test_fit_errors(M):
    with pytest.raises(M.MjdError) as ei:
        M.mjd_poly1_fit([1.0, 2.0, 3.0], [1.0, 2.0, 3.0], max_degree=8)
    assert ei.value.code == -1
    with pytest.raises(M.MjdError) as ei:
        M.mjd_poly1_fit([1.0], [1.0])
    assert ei.value.code == -1
    # every x equal: only the constant is determined
    p, _ = M.mjd_poly1_fit([2.0] * 10, [5.0] * 10)
    assert p.degree == 0 and math.isclose(p.c[0], 5.0)
    with pytest.raises(M.MjdError) as ei:
        M.mjd_model_predict(M.mjd_model(), 0, 10, 100)
    assert ei.value.code == -1


# ---- CPU-GPU partitioning (Sec. 5.2) ------------------------------------------------------

def _model_pair(M, cpu_rate, gpu_rate, dispatch, hpp):
    """A library model and the oracle's copy: P_cpu and P_gpu linear in the
    pixels (seconds per 1024^2 pixels), a constant dispatch, a constant
    Huffman rate."""
    m = M.mjd_model()
    m.huff_per_pixel.degree = 0
    m.huff_per_pixel.c[0] = hpp
    o = {"huff_per_pixel": (0, [hpp])}
    for name, val in (("o_w", 0.0), ("t_kernel", gpu_rate), ("o_r", 0.0), ("p_cpu", cpu_rate),
                      ("t_dispatch", 0.0)):
        p = getattr(m, name)
        p.degree = 2
        c = [0.0] * 6
        c[4] = val  # the a*b term: t(1, 1) = 1 * (2*2 + 3 - 1) / 2 + 1 = 4
        if name == "t_dispatch":
            c[0] = dispatch
        for i, v in enumerate(c):
            p.c[i] = v
        o[name] = (2, c)
    return m, o


SCHEMES = ["sps", "overlap", "pps"]


def _code(M, scheme):
    return {"sps": M.MJD_PART_SPS, "overlap": M.MJD_PART_OVERLAP, "pps": M.MJD_PART_PPS}[scheme]


@pytest.mark.parametrize("scheme", SCHEMES)
def test_newton_partition_matches_brute_force(M, scheme):
    code = _code(M, scheme)
    cases = [(2e-3, 2e-3, 1e-5, 5e-10), (4e-3, 1e-3, 2e-5, 1e-9), (1e-3, 3e-3, 1e-5, 2e-9), (1e-3, 4e-3, 1e-5, 1e-10)]
    for cpu_rate, gpu_rate, dispatch, hpp in cases:
        m, o = _model_pair(M, cpu_rate, gpu_rate, dispatch, hpp)
        for w, h, mh in ((4096, 3072, 16), (1000, 777, 16), (640, 480, 8)):
            nbytes = w * h // 3
            chunk = 4 * mh if scheme == "pps" else 0
            got = M.mjd_partition_rows(m, code, w, h, mh, nbytes, 4.0, chunk)
            t_best, x_best = O.best_partition(o, scheme, w, h, mh, nbytes, 4.0, chunk)
            assert abs(got["cpu_rows"] - x_best) <= mh, (cpu_rate, gpu_rate, w, h)
            # the continuous root balances both sides
            if 0 < got["x"] < h:
                cpu, gpu = O.sides(o, scheme, w, h, nbytes, 4.0, got["x"], chunk)
                assert math.isclose(cpu, gpu, rel_tol=1e-6)
            assert got["iterations"] >= 1 or got["x"] in (0.0, float(h))
            cpu, gpu = O.sides(o, scheme, w, h, nbytes, 4.0, got["cpu_rows"], chunk)
            assert math.isclose(got["t_gpu"], gpu if got["cpu_rows"] < h else 0.0, rel_tol=1e-9)
            if got["cpu_rows"]:
                assert math.isclose(got["t_cpu"], cpu, rel_tol=1e-9)


def test_repartition_matches_brute_force(M):
    m, o = _model_pair(M, 1e-3, 3e-3, 1e-5, 2e-9)
    w, h, mh = 4096, 3072, 16
    nbytes = w * h // 3
    est = 2e-9 * w * h / 4.0
    for r, u, t_done, busy in ((1024, 1008, 0.5 * est, 0.0), (1024, 1008, 0.9 * est, 1e-3), (512, 500, 0.2 * est, 0.0),
                               (3072, 3072, 0.0, 0.0), (200, 0, est, 5e-4), (1024, 1008, 2.0 * est, 0.0)):
        got = M.mjd_repartition_rows(m, w, h, r, mh, nbytes, 4.0, u, t_done, busy)
        _, x_best = O.best_repartition(o, w, h, r, mh, nbytes, 4.0, u, t_done, busy)
        assert abs(got["cpu_rows"] - x_best) <= mh, (r, u, t_done, busy)
        assert 0 <= got["cpu_rows"] <= r
        if 0 < got["x"] < r:
            cpu, gpu = O.repartition_sides(o, w, h, r, nbytes, 4.0, u, t_done, busy, got["x"])
            assert math.isclose(cpu, gpu, rel_tol=1e-6)
    with pytest.raises(M.MjdError):
        M.mjd_repartition_rows(m, w, h, 0, mh, nbytes, 4.0, 0, 0.0, 0.0)
    with pytest.raises(M.MjdError):
        M.mjd_repartition_rows(m, w, h, 100, mh, nbytes, 4.0, 100, -1.0, 0.0)


def test_oracle_repartition_density_closed_form():
    # Huffman on schedule (t_done the decoded rows' share of the estimate)
    # keeps d' = d; behind schedule the rest is sparser; past the estimate, zero
    o = {"huff_per_pixel": (1, [0.0, 1e-9]), "p_cpu": (0, [0.0]), "t_dispatch": (0, [0.0]),
         "o_w": (0, [0.0]), "t_kernel": (0, [0.0]), "o_r": (0, [0.0])}
    w, h, nbytes, n = 1000, 1000, 400_000, 2.0
    d = nbytes / (w * h)
    est = 1e-9 * d * w * h / n
    u = 250
    cpu, _ = O.repartition_sides(o, w, h, 300, nbytes, n, u, est * (1 - u / h), 0.0, 0.0)
    assert math.isclose(cpu, 1e-9 * d * w * u / n, rel_tol=1e-12)
    cpu, _ = O.repartition_sides(o, w, h, 300, nbytes, n, u, est * (1 - u / h) + 0.5 * est * u / h, 0.0, 0.0)
    assert math.isclose(cpu, 0.5 * 1e-9 * d * w * u / n, rel_tol=1e-12)
    cpu, _ = O.repartition_sides(o, w, h, 300, nbytes, n, u, 2 * est, 0.0, 0.0)
    assert cpu == 0.0


def test_partition_ends(M):
    # a GPU far faster than the CPU keeps every row; a GPU far slower gives them all away
    m, _ = _model_pair(M, 1.0, 1e-6, 1e-4, 1e-9)
    assert M.mjd_partition_rows(m, M.MJD_PART_SPS, 4096, 3072, 16, 10 ** 6)["cpu_rows"] == 0
    m, _ = _model_pair(M, 1e-6, 1.0, 0.0, 1e-9)
    assert M.mjd_partition_rows(m, M.MJD_PART_SPS, 4096, 3072, 16, 10 ** 6)["cpu_rows"] == 3072
    # heights off the MCU grid: the GPU's share may end in the partial MCU row
    for h, mh in ((121, 8), (777, 16), (3000, 16)):
        m, _ = _model_pair(M, 1.0, 1e-6, 1e-4, 1e-9)
        assert M.mjd_partition_rows(m, M.MJD_PART_SPS, 4096, h, mh, 10 ** 6)["cpu_rows"] == 0
        assert M.mjd_repartition_rows(m, 4096, h, h - mh, mh, 10 ** 6, 1.0, 0, 0.0, 0.0)["cpu_rows"] == 0
        m, _ = _model_pair(M, 1e-6, 1.0, 0.0, 1e-9)
        assert M.mjd_partition_rows(m, M.MJD_PART_SPS, 4096, h, mh, 10 ** 6)["cpu_rows"] == h
    with pytest.raises(M.MjdError):
        M.mjd_partition_rows(m, 7, 4096, 3072, 16, 10 ** 6)
    with pytest.raises(M.MjdError):
        M.mjd_partition_rows(m, M.MJD_PART_SPS, 4096, 3072, 12, 10 ** 6)
    with pytest.raises(M.MjdError):  # PPS needs its chunk height
        M.mjd_partition_rows(m, M.MJD_PART_PPS, 4096, 3072, 16, 10 ** 6)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_oracle_sides_balance_at_the_linear_closed_form(scheme):
    # linear costs: CPU = D + c*A*x + H(x), GPU = g*A*(h - x), A = w / 1024^2,
    # H(x) = 0 (SPS), hpp*w*x/n (overlap), hpp*w*(h - chunk)/n (PPS, chunk
    # below the GPU's rows), so the sides meet at x = (g*A*h - D - H0) / slope
    cpu_rate, gpu_rate, dispatch, hpp, n = 3e-3, 1e-3, 2e-4, 1e-9, 4.0
    o = {"huff_per_pixel": (0, [hpp])}
    for name, val in (("o_w", 0.0), ("t_kernel", gpu_rate), ("o_r", 0.0), ("p_cpu", cpu_rate),
                      ("t_dispatch", 0.0)):
        c = [0.0] * 6
        c[4] = val  # a*b
        if name == "t_dispatch":
            c[0] = dispatch
        o[name] = (2, c)
    w, h, mh, chunk = 4096, 3072, 16, 128
    A = w / 1024.0 ** 2
    slope = cpu_rate * A + gpu_rate * A + (hpp * w / n if scheme == "overlap" else 0.0)
    h0 = hpp * w * (h - chunk) / n if scheme == "pps" else 0.0
    x = (gpu_rate * A * h - dispatch - h0) / slope
    assert 0 < x < h - chunk
    cpu, gpu = O.sides(o, scheme, w, h, w * h // 3, n, x, chunk)
    assert math.isclose(cpu, gpu, rel_tol=1e-12)
    assert math.isclose(gpu, gpu_rate * A * (h - x), rel_tol=1e-12)
    # the brute force's split is the MCU-row boundary on either side of the root
    t, xb = O.best_partition(o, scheme, w, h, mh, w * h // 3, n, chunk)
    assert abs(xb - x) < mh
    assert t >= gpu - 1e-15


def test_fit_recovers_host_parts_against_rows(M):
    # samples carrying host-part points at (width, rows): a bilinear truth is
    # recovered and evaluated where the partition needs it
    from paper_1311_5304_amd import perfmodel
    rng = np.random.default_rng(5)
    samples = []
    for _ in range(30):
        w = int(rng.integers(1024, 6000))
        h = int(rng.integers(768, 4000))
        s = {"width": w, "height": h, "bytes": w * h // 4, "t_huff": 2e-9 * w * h,
             "o_w": 1e-4 + 1e-3 * w * h / 2 ** 20, "t_kernel": 2e-5 * w * h / 2 ** 20, "o_r": 1e-3 * w * h / 2 ** 20}
        host = []
        for x in (h // 4, h // 2, h):
            host.append(("p_cpu", w, x, 3e-4 + 4e-3 * w * x / 2 ** 20))
            host.append(("t_dispatch", w, h - x + 1, 5e-5))
        s["host"] = host
        samples.append(s)
    model, info = perfmodel.fit(samples)
    assert set(info) == {"huff_per_pixel", "o_w", "t_kernel", "o_r", "p_cpu", "t_dispatch"}
    assert info["p_cpu"][0] == 2 and info["t_dispatch"][0] == 0
    for w, x in ((2000, 100), (5000, 3000)):
        got = M.mjd_poly2_eval(model.p_cpu, w / 1024.0, x / 1024.0)
        assert math.isclose(got, 3e-4 + 4e-3 * w * x / 2 ** 20, rel_tol=1e-8)
    back = perfmodel.from_dict(perfmodel.to_dict(model))
    assert back.p_cpu.degree == 2 and math.isclose(back.t_dispatch.c[0], 5e-5, rel_tol=1e-9)


def test_host_parts_are_capped_and_never_fall_with_rows(M):
    # host times with a dip between their row counts (t = u^3 - 1.5 u^2 +
    # 0.6 u + 1 in u = rows / 4096, falling for u in (0.28, 0.72)): the
    # unconstrained degree-3 surface follows the dip; the fit used for the
    # host parts stays at degree 3 or below and picks one that does not fall
    # as rows grow.  Exact bilinear data are predicted with no error.
    from paper_1311_5304_amd import perfmodel
    rng = np.random.default_rng(9)

    def dip(x):
        u = x / 4096.0
        return 1e-3 * (u ** 3 - 1.5 * u ** 2 + 0.6 * u + 1.0)

    samples = []
    for _ in range(40):
        w = int(rng.integers(1024, 6000))
        h = int(rng.integers(768, 4096))
        s = {"width": w, "height": h, "bytes": w * h // 4, "t_huff": 2e-9 * w * h,
             "o_w": 1e-4 + 1e-3 * w * h / 2 ** 20, "t_kernel": 2e-5 * w * h / 2 ** 20, "o_r": 1e-3 * w * h / 2 ** 20}
        host = []
        for x in (h // 4, h // 2, 3 * h // 4, h):
            host.append(("p_cpu", w, x, dip(x)))
            host.append(("t_dispatch", w, h - x + 1, 5e-5))
        s["host"] = host
        samples.append(s)
    pts = np.array([x[1:] for s in samples for x in s["host"] if x[0] == "p_cpu"], np.float64)
    free, _ = M.mjd_poly2_fit(pts[:, 0] / 1024.0, pts[:, 1] / 1024.0, pts[:, 2], 3)
    assert free.degree == 3 and not perfmodel.rows_monotone(free, 1.0, 6000 / 1024.0, 4.0)
    model, info = perfmodel.fit(samples)
    assert info["p_cpu"][0] < 3
    assert perfmodel.rows_monotone(model.p_cpu, 1.0, 6000 / 1024.0, 4.0)
    exact = [dict(s, host=[(k, w, x, 3e-4 + 4e-3 * w * x / 2 ** 20) if k == "p_cpu" else (k, w, x, t)
                           for k, w, x, t in s["host"]]) for s in samples]
    m2, info2 = perfmodel.fit(exact)
    assert info2["p_cpu"][0] == 2
    errs = perfmodel.host_errors(m2, exact)
    assert max(errs["p_cpu"]) < 1e-8 and max(errs["t_dispatch"]) < 1e-8


def test_pps_with_a_whole_image_chunk_is_the_overlapped_scheme(M):
    # c = min(chunk, h - x) = h - x when chunk >= h, so the CPU's Huffman term
    # T_huff(w, h - c) becomes T_huff(w, x): exactly the overlapped scheme
    for rates in ((2e-3, 2e-3, 1e-5, 5e-10), (1e-3, 3e-3, 1e-5, 2e-9), (4e-3, 1e-3, 2e-5, 1e-9)):
        m, o = _model_pair(M, *rates)
        for w, h, mh in ((4096, 3072, 16), (1000, 777, 16)):
            a = M.mjd_partition_rows(m, M.MJD_PART_PPS, w, h, mh, w * h // 3, 4.0, h)
            b = M.mjd_partition_rows(m, M.MJD_PART_OVERLAP, w, h, mh, w * h // 3, 4.0)
            assert a["cpu_rows"] == b["cpu_rows"] and math.isclose(a["x"], b["x"], rel_tol=1e-9, abs_tol=1e-9)
            for x in (0.0, h / 3, h - 1.0):
                assert all(math.isclose(p, q, rel_tol=1e-12, abs_tol=1e-15) for p, q in
                           zip(O.sides(o, "pps", w, h, w * h // 3, 4.0, x, h), O.sides(o, "overlap", w, h, w * h // 3, 4.0, x)))


def test_repartition_with_nothing_left_to_decode_is_sps_on_the_remainder(M):
    # no Huffman data left (u = 0) and an idle GPU: Eq. 16 is Eq. 10 on the
    # remaining rows
    for rates in ((2e-3, 2e-3, 1e-5, 5e-10), (1e-3, 3e-3, 1e-5, 2e-9)):
        m, _ = _model_pair(M, *rates)
        for r in (3072, 1000, 480):
            a = M.mjd_repartition_rows(m, 4096, 3072, r, 16, 4096 * 3072 // 3, 4.0, 0, 0.0, 0.0)
            b = M.mjd_partition_rows(m, M.MJD_PART_SPS, 4096, r, 16, 4096 * r // 3, 4.0)
            assert a["cpu_rows"] == b["cpu_rows"] and math.isclose(a["x"], b["x"], rel_tol=1e-9, abs_tol=1e-9)
            assert math.isclose(a["t_cpu"], b["t_cpu"], rel_tol=1e-12) and math.isclose(a["t_gpu"], b["t_gpu"], rel_tol=1e-12)
