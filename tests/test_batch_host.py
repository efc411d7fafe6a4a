"""Host logic of the batch executor: the depth cost model and its accuracy
constraint (no device work; the library is only loaded)."""
import math

import pytest

import paper_1201_5430_amd as LH


def _k(r, a):
    # Gaussian-core factor K(r; a) of eq. vem1, written from the closed form
    return math.erf(r / (a * math.sqrt(2))) - math.sqrt(2 / math.pi) * (r / a) * math.exp(-r * r / (2 * a * a))


def _tune(t_box, t_pair):
    t = LH.Tune()
    t.p, t.precision, t.t_box_ns, t.t_pair_ns = 10, LH.FP32, t_box, t_pair
    return t


def test_depth_grows_with_near_field_cost():
    # dearer pairs push towards smaller leaves (deeper trees), dearer boxes the other way
    n = 200000
    ds = [LH.choose_depth(_tune(10.0, tp), n)[0] for tp in (1e-4, 1e-3, 1e-2, 1e-1, 1.0)]
    assert ds == sorted(ds) and ds[0] < ds[-1]
    db = [LH.choose_depth(_tune(tb, 1e-2), n)[0] for tb in (0.1, 1.0, 10.0, 100.0, 1000.0)]
    assert db == sorted(db, reverse=True) and db[0] > db[-1]


def test_depth_balances_the_model_at_the_optimum():
    # the chosen depth's modelled cost is not above that of its neighbours
    t = _tune(8.0, 0.003)
    for n in (5000, 60000, 1 << 20):
        d, _ = LH.choose_depth(t, n)

        def cost(dd):
            boxes = sum((8.0 ** l) * -math.expm1(n * math.log1p(-(8.0 ** -l))) for l in range(2, dd + 1))
            m = 2.0 ** dd
            f = (3 * m - 2) / (m * m)
            return t.t_box_ns * boxes + t.t_pair_ns * n * (n - 1) * f ** 3

        for dd in (d - 1, d + 1):
            if 2 <= dd <= 8:
                assert cost(d) <= cost(dd) * (1 + 1e-12)


def test_core_split_limits_depth():
    # with a = 0.5 N^(-1/3) and tol = 1e-6 the leaf side must keep 1 - K(h; a) <= tol
    t = _tune(1.0, 1.0)  # costly pairs: the model alone would go deep
    for n in (4096, 65536):
        a = 0.5 * n ** (-1 / 3)
        d, warn = LH.choose_depth(t, n, 1.0, a, 1e-6)
        assert not warn
        assert 1 - _k(2.0 ** -d, a) <= 1e-6
        assert 1 - _k(2.0 ** -(d + 1), a) > 1e-6


def test_core_split_unsatisfiable_warns():
    # 1024 elements: even depth 2 (h = 1/4) is below the needed ~5.7 a with a = 0.05
    d, warn = LH.choose_depth(_tune(1.0, 1.0), 1024, 1.0, 0.5 * 1024 ** (-1 / 3), 1e-6)
    assert warn and d == 2


def test_choose_depth_rejects_bad_arguments():
    t = _tune(1.0, 1.0)
    with pytest.raises(LH.LhfError):
        LH.choose_depth(t, -1)
    with pytest.raises(LH.LhfError):
        LH.choose_depth(t, 10, L=0.0)
    with pytest.raises(LH.LhfError):
        LH.choose_depth(_tune(0.0, 1.0), 10)


def test_tune_default_scales_with_p():
    a, b = LH.tune_default(8, LH.FP32), LH.tune_default(16, LH.FP32)
    assert b.t_box_ns > a.t_box_ns > 0 and a.t_pair_ns > 0
