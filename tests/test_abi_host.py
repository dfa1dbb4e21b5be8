"""C ABI checks that need no GPU: the library loads, exports every declared
function, and rejects invalid arguments on the host before any GPU work."""
import ctypes

import pytest

import paper_1601_05904_amd as aidw


@pytest.fixture(scope="module")
def L():
    return aidw.load()


def test_every_declared_function_is_exported(L):
    names = aidw.exported_functions()
    assert {"aidw_build_grid", "aidw_knn", "aidw_interpolate", "aidw_run"} <= set(names)
    for n in names:
        assert hasattr(L, n), n


def test_status_strings_and_version(L):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.aidw_status_string(code).decode() != "unknown status"
    assert b"gfx950" in L.aidw_version()


def test_params_default(L):
    p = aidw._Params()
    L.aidw_params_default(ctypes.byref(p))
    assert p.k == 10 and list(p.alpha) == [1, 2, 3, 4, 5]
    assert (p.r_min, p.r_max, p.area, p.cell_width, p.occupancy) == (0.0, 2.0, 0.0, 0.0, 2.0)


def _p(**kw):
    p = aidw.Params(**kw)._c()
    return ctypes.byref(p)


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails host validation first


@pytest.mark.parametrize("case", [
    dict(n=0), dict(x=None), dict(m=-1), dict(qx=None), dict(z=None), dict(qz=None),
    dict(p=dict(k=0)), dict(p=dict(k=65)), dict(p=dict(k=11), n=10),
    dict(p=dict(r_min=2.0, r_max=1.0)), dict(p=dict(r_min=-1.0)), dict(p=dict(levels=(1, 2, float("nan"), 4, 5))),
    dict(p=dict(levels=(1, 2, 0, 4, 5))), dict(p=dict(area=float("inf"))), dict(p=dict(occupancy=0.0)),
])
def test_run_rejects_invalid_arguments(L, case):
    args = dict(x=FAKE, y=FAKE, z=FAKE, n=100, qx=FAKE, qy=FAKE, m=10, qz=FAKE, p={})
    args.update({k: v for k, v in case.items() if k != "p"})
    p = _p(**case.get("p", {}))
    st = L.aidw_run(args["x"], args["y"], args["z"], args["n"], args["qx"], args["qy"], args["m"], p, args["qz"],
                    None, None, None)
    assert st == aidw.EINVAL
    assert L.aidw_last_error_detail().decode() != ""


def test_sizes_beyond_int32_are_capacity_errors(L):
    st = L.aidw_run(FAKE, FAKE, FAKE, 1 << 31, FAKE, FAKE, 10, _p(), FAKE, None, None, None)
    assert st == aidw.ECAPACITY


def test_empty_query_set_is_a_no_op(L):
    st = L.aidw_run(FAKE, FAKE, FAKE, 100, None, None, 0, _p(), None, None, None, None)
    assert st == aidw.OK


def test_other_entry_points_validate(L):
    assert L.aidw_knn(None, FAKE, FAKE, 10, 5, FAKE, None, None, None) == aidw.EINVAL
    assert L.aidw_build_grid(None, FAKE, 10, None, None, 0, _p(), None, None) == aidw.EINVAL
    out = ctypes.c_void_p()
    assert L.aidw_build_grid(FAKE, FAKE, 0, None, None, 0, _p(), None, ctypes.byref(out)) == aidw.EINVAL
    assert L.aidw_interpolate(FAKE, FAKE, FAKE, 10, FAKE, FAKE, 5, None, FAKE, _p(), None, FAKE, None,
                              None) == aidw.EINVAL
    assert L.aidw_grid_describe(None, None) == aidw.EINVAL
    assert L.aidw_grid_info(None, None, None, None, None, None) == aidw.EINVAL
    assert L.aidw_set_interp_config(3, 0, -1) == aidw.EINVAL
    assert L.aidw_set_interp_config(0, 0, 2) == aidw.EINVAL
    assert L.aidw_set_interp_config(0, 0, -1) == aidw.OK
    t = aidw._Timing()
    assert L.aidw_last_timing(ctypes.byref(t)) == aidw.EINVAL
    L.aidw_grid_destroy(None)


def _jobs(count=2, **over):
    arr = (aidw._Job * count)()
    for j in range(count):
        a = arr[j]
        a.x = a.y = a.z = a.qx = a.qy = a.qz = FAKE
        a.n, a.m = 100, 10
        a.params = aidw.Params(k=10)._c()
        for k, v in over.items():
            if k == "p":
                a.params = aidw.Params(**v)._c()
            else:
                setattr(a, k, v)
    return arr


def test_batch_config_default(L):
    c = aidw._BatchConfig()
    L.aidw_batch_config_default(ctypes.byref(c))
    assert (c.q, c.split_points, c.workers_per_cu, c.integer_powers, c.use_graph) == (1, 0, 8, 1, 0)


@pytest.mark.parametrize("case", [
    dict(n=0), dict(m=-1), dict(x=None), dict(z=None), dict(qx=None), dict(qz=None), dict(p=dict(k=0)),
    dict(p=dict(k=101)), dict(p=dict(k=65)), dict(p=dict(r_min=3.0)), dict(p=dict(occupancy=-1.0)),
])
def test_batch_create_rejects_invalid_jobs(L, case):
    out = ctypes.c_void_p()
    st = L.aidw_batch_create(_jobs(3, **case), 3, None, ctypes.byref(out))
    assert st == aidw.EINVAL and not out.value
    assert "job 0" in L.aidw_last_error_detail().decode()


@pytest.mark.parametrize("cfg", [dict(q=3), dict(q=0), dict(split_points=-8), dict(workers_per_cu=0),
                                 dict(workers_per_cu=33), dict(integer_powers=2), dict(use_graph=-1)])
def test_batch_create_rejects_invalid_config(L, cfg):
    c = aidw._BatchConfig()
    L.aidw_batch_config_default(ctypes.byref(c))
    for k, v in cfg.items():
        setattr(c, k, v)
    out = ctypes.c_void_p()
    assert L.aidw_batch_create(_jobs(), 2, ctypes.byref(c), ctypes.byref(out)) == aidw.EINVAL
    if "use_graph" not in cfg:  # the one-shot form ignores use_graph
        assert L.aidw_run_batch(_jobs(), 2, ctypes.byref(c), None, None) == aidw.EINVAL


def test_batch_other_entry_points_validate(L):
    out = ctypes.c_void_p()
    assert L.aidw_batch_create(None, 2, None, ctypes.byref(out)) == aidw.EINVAL
    assert L.aidw_batch_create(_jobs(), 0, None, ctypes.byref(out)) == aidw.EINVAL
    assert L.aidw_batch_create(_jobs(), 2, None, None) == aidw.EINVAL
    assert L.aidw_batch_run(None, None) == aidw.EINVAL
    assert L.aidw_batch_job_status(None, None, None) == aidw.EINVAL
    assert L.aidw_batch_describe(None, None) == aidw.EINVAL
    assert L.aidw_batch_set_timing(None, 1) == aidw.EINVAL
    assert L.aidw_batch_last_timing(None, None) == aidw.EINVAL
    L.aidw_batch_destroy(None)
    ms = (ctypes.c_float * 1)()
    assert L.aidw_batch_tune(_jobs(), 2, None, 1, 1, ms, None) == aidw.EINVAL
    bad = (aidw._BatchConfig * 1)()
    bad[0].q = 5
    assert L.aidw_batch_tune(_jobs(), 2, bad, 1, 1, ms, None) == aidw.EINVAL


def test_batch_totals_beyond_int32_are_capacity_errors(L):
    out = ctypes.c_void_p()
    st = L.aidw_batch_create(_jobs(3, n=600_000_000, m=600_000_000), 3, None, ctypes.byref(out))
    assert st == aidw.ECAPACITY


def test_baseline_entry_points_validate(L):
    assert L.aidw_knn_bruteforce(None, FAKE, 10, FAKE, FAKE, 5, 3, FAKE, None, None, None) == aidw.EINVAL
    assert L.aidw_knn_bruteforce(FAKE, FAKE, 0, FAKE, FAKE, 5, 3, FAKE, None, None, None) == aidw.EINVAL
    assert L.aidw_knn_bruteforce(FAKE, FAKE, 10, FAKE, FAKE, 5, 11, FAKE, None, None, None) == aidw.EINVAL
    assert L.aidw_knn_bruteforce(FAKE, FAKE, 10, None, None, 0, 3, None, None, None, None) == aidw.OK
    assert L.aidw_knn_bruteforce(FAKE, FAKE, 1 << 31, FAKE, FAKE, 5, 3, FAKE, None, None, None) == aidw.ECAPACITY
    assert L.aidw_interpolate_naive(FAKE, FAKE, None, 10, FAKE, FAKE, 5, FAKE, FAKE, _p(), None, FAKE, None,
                                    None) == aidw.EINVAL
    assert L.aidw_knn_paper(None, FAKE, FAKE, 10, 5, FAKE, None, None, None) == aidw.EINVAL


def test_nn_statistic_validates(L):
    # null grid, negative m, k out of range and NaN clip are rejected on the host
    assert L.aidw_nn_statistic(None, FAKE, FAKE, 10, 5, 3.0, FAKE, None) == aidw.EINVAL
    assert L.aidw_nn_statistic(FAKE, FAKE, FAKE, -1, 5, 3.0, FAKE, None) == aidw.EINVAL


@pytest.mark.parametrize("case", [dict(n=0), dict(z=None), dict(qz=None), dict(p=dict(k=0)),
                                  dict(p=dict(cell_width=0.01)), dict(p=dict(occupancy=0.0))])
def test_run_noalloc_rejects_invalid_arguments(L, case):
    """The no-allocation run checks its arguments as aidw_run does, and refuses an explicit cell
    side (its grid is sized by occupancy), all before any GPU work."""
    args = dict(x=FAKE, y=FAKE, z=FAKE, n=100, qx=FAKE, qy=FAKE, m=10, qz=FAKE)
    args.update({k: v for k, v in case.items() if k != "p"})
    st = L.aidw_run_noalloc(args["x"], args["y"], args["z"], args["n"], args["qx"], args["qy"], args["m"],
                            _p(**case.get("p", {})), args["qz"], None, None, None)
    assert st == aidw.EINVAL
    assert L.aidw_last_error_detail().decode() != ""


@pytest.mark.parametrize("n,m,occ", [(1 << 22, 1 << 22, 2.0), (1 << 20, 1 << 23, 2.0), (1 << 21, 16, 0.25)])
def test_run_noalloc_rejects_sizes_beyond_its_scratch(L, n, m, occ):
    """Sizes whose temporaries exceed the fixed scratch array (or whose grid exceeds the banded
    build's cell limit) are capacity errors, raised before any GPU work."""
    st = L.aidw_run_noalloc(FAKE, FAKE, FAKE, n, FAKE, FAKE, m, _p(occupancy=occ), FAKE, None, None, None)
    assert st == aidw.ECAPACITY
    assert L.aidw_last_error_detail().decode() != ""


def test_run_noalloc_empty_query_set_is_a_no_op(L):
    assert L.aidw_run_noalloc(FAKE, FAKE, FAKE, 100, None, None, 0, _p(), None, None, None, None) == aidw.OK
