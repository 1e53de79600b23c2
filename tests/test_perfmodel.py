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
