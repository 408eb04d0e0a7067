"""The C ABI without a GPU: the library loads, exports every declared symbol, and
rejects invalid arguments before doing any device work (CPU only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def api():
    from paper_1808_06992_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1808_06992_amd import build
        build.build()
    _lib.load()
    return _lib


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "uoi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(uoi_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(api):
    names = _declared_functions()
    assert len(names) >= 12
    lib = api.load()
    for n in names:
        assert hasattr(lib, n), n
    assert set(api.EXPORTS) == set(names)


def test_default_opts(api):
    o = api.Opts()
    api.load().uoi_default_opts(C.byref(o))
    assert (o.rho, o.kkt_tol, o.max_iter, o.check_every) == (1.0, 1e-6, 20000, 10)
    assert (o.train_num, o.train_den, o.precision, o.solver) == (4, 5, 0, 0)


def _fit(api, lam, **kw):
    o, keep = api.make_opts(lam, B1=kw.pop("B1", 2), B2=kw.pop("B2", 2), stream=None, **kw)
    d = api.Diag()
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    code = api.load().uoi_lasso_fit(10, 3, fake, fake, C.byref(o), fake, fake, fake, C.byref(d))
    return code, api.load().uoi_last_error().decode()


@pytest.mark.parametrize("lam,kw,msg", [
    ([1.0, 2.0], {}, "decreasing"),
    ([1.0, 1.0], {}, "decreasing"),
    ([1.0, -0.5], {}, ">= 0"),
    ([float("nan")], {}, "finite"),
    ([1.0], {"B1": 0}, "B1"),
    ([1.0], {"B2": 0}, "B2"),
    ([1.0], {"rho": -1.0}, "rho"),
    ([1.0], {"rho": float("nan")}, "rho"),
    ([1.0], {"kkt_tol": -1.0}, "kkt_tol"),
    ([1.0], {"max_iter": 0}, "max_iter"),
    ([1.0], {"check_every": 0}, "check_every"),
    ([1.0], {"train": (5, 5)}, "train"),
])
def test_invalid_options_rejected_before_device_work(api, lam, kw, msg):
    code, err = _fit(api, lam, **kw)
    assert code == api.UOI_EINVAL
    assert msg in err


def test_data_scaled_rho_not_allocation_free(api):
    """rho = 0 reads the data's scale back through pinned host memory, so the
    allocation-free entry point refuses it before any device work."""
    o, keep = api.make_opts([1.0], rho=0.0, stream=None)
    fake = C.c_void_p(0x1000)
    lib = api.load()
    code = lib.uoi_lasso_solve_batch_noalloc(2, 3, fake, fake, C.byref(o), None, None, fake, None, None, None)
    assert code == api.UOI_EINVAL
    assert "rho > 0" in lib.uoi_last_error().decode()


def test_empty_lambda_grid_rejected(api):
    o, keep = api.make_opts([1.0], stream=None)
    o.q = 0
    fake = C.c_void_p(0x1000)
    code = api.load().uoi_lasso_fit(10, 3, fake, fake, C.byref(o), fake, fake, fake, None)
    assert code == api.UOI_EINVAL


def test_var_order_and_length_checked(api):
    o, keep = api.make_opts([1.0], B1=1, B2=1, stream=None)
    fake = C.c_void_p(0x1000)
    lib = api.load()
    code = lib.uoi_var_fit(100, 3, 0, fake, 0, C.byref(o), fake, fake, fake, fake, None)
    assert code == api.UOI_EINVAL
    assert "order d must be >= 1" in lib.uoi_last_error().decode()
    code = lib.uoi_var_fit(5, 3, 4, fake, 0, C.byref(o), fake, fake, fake, fake, None)
    assert code == api.UOI_EINVAL
    assert "T >= d + 2" in lib.uoi_last_error().decode()


def test_intercept_flag_is_for_var(api):
    o, keep = api.make_opts([1.0], B1=1, B2=1, stream=None)
    o.flags |= api.UOI_FLAG_INTERCEPT
    fake = C.c_void_p(0x1000)
    lib = api.load()
    assert lib.uoi_lasso_fit(10, 3, fake, fake, C.byref(o), fake, fake, fake, None) == api.UOI_EINVAL
    assert "UoI_VAR" in lib.uoi_last_error().decode()


def test_null_pointers_rejected(api):
    o, keep = api.make_opts([1.0], B1=1, B2=1, stream=None)
    code = api.load().uoi_lasso_fit(10, 3, None, None, C.byref(o), None, None, None, None)
    assert code == api.UOI_EINVAL


def test_bad_sizes_rejected(api):
    o, keep = api.make_opts([1.0], B1=1, B2=1, stream=None)
    fake = C.c_void_p(0x1000)
    lib = api.load()
    assert lib.uoi_lasso_fit(1, 3, fake, fake, C.byref(o), fake, fake, fake, None) == api.UOI_EINVAL
    # a split of 4 rows at 1/5 leaves an empty training side
    o2, keep2 = api.make_opts([1.0], B1=1, B2=1, stream=None, train=(1, 5))
    assert lib.uoi_lasso_fit(4, 3, fake, fake, C.byref(o2), fake, fake, fake, None) == api.UOI_EINVAL
    assert lib.uoi_gram(0, 5, fake, 3, fake, 3, 0, None, 0, fake, None, None) == api.UOI_EINVAL
    assert lib.uoi_bootstrap_rows(0, 0, 5, fake, None) == api.UOI_EINVAL
    assert lib.uoi_spd_inverse(1, 3, fake, -1.0, fake, None) == api.UOI_EINVAL


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1808_06992_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        _lib.load()


def test_no_alloc_rejects_oversize_before_device_work(api):
    """The allocation-free entry point checks the problem's scratch against its
    static array before touching the device (fake pointers are never used)."""
    o, keep = api.make_opts([1.0, 0.5], stream=None)
    fake = C.c_void_p(0x1000)
    lib = api.load()
    code = lib.uoi_lasso_solve_batch_noalloc(40, 1000, fake, fake, C.byref(o), None, None, fake,
                                             None, None, None)
    assert code == api.UOI_EINVAL
    msg = lib.uoi_last_error().decode()
    assert "static buffer" in msg and str(64 << 20) in msg
