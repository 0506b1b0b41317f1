"""CPU-side checks of the C ABI: the library loads, exports every declared symbol, and
rejects invalid arguments before touching a device.  No compute call is made here."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfe.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1602_06621_amd import _ffi
    from paper_1602_06621_amd import build as b

    if not os.path.exists(_ffi.library_path()):
        b.build()
    return _ffi._lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(mfe_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mfe_equilibrate", "mfe_lsqr", "mfe_default_alpha_beta", "mfe_plan_create",
                     "mfe_plan_equilibrate", "mfe_plan_destroy", "mfe_residual", "mfe_draw_signs",
                     "mfe_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []


def test_default_alpha_beta(lib):
    a, b = C.c_double(), C.c_double()
    assert lib.mfe_default_alpha_beta(200, 100, C.byref(a), C.byref(b)) == 0
    assert a.value == pytest.approx(0.5 ** 0.25, rel=1e-15)
    assert b.value == pytest.approx(2.0 ** 0.25, rel=1e-15)
    assert lib.mfe_default_alpha_beta(0, 5, C.byref(a), C.byref(b)) == -1
    assert "positive" in lib.mfe_last_error().decode()


def _params(**kw):
    from paper_1602_06621_amd._ffi import _Params

    p = _Params()
    p.alpha, p.beta, p.gamma, p.box_M = 1.0, 1.0, 0.1, 10.0
    p.steps, p.probes, p.seed, p.t0, p.batch = 10, 4, 1, 0, 0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _csr_struct(m=4, n=3):
    from paper_1602_06621_amd._ffi import _Matrix

    s = _Matrix()
    s.kind, s.m, s.n, s.nnz = 2, m, n, 0
    return s


@pytest.mark.parametrize("bad,code", [
    (dict(alpha=0.0), -1), (dict(beta=-1.0), -1), (dict(gamma=0.0), -1), (dict(box_M=0.0), -1),
    (dict(alpha=float("nan")), -1), (dict(steps=-1), -1), (dict(probes=0), -1), (dict(probes=257), -1),
    (dict(t0=-2), -1), (dict(batch=-1), -1),
])
def test_invalid_parameters_rejected_on_host(lib, bad, code):
    s = _csr_struct()
    p = _params(**bad)
    dummy = C.c_void_p(16)
    assert lib.mfe_equilibrate(C.byref(s), C.byref(p), dummy, dummy, None, None) == code
    assert lib.mfe_last_error().decode() != ""


def test_missing_outputs_and_dims_rejected(lib):
    s = _csr_struct()
    p = _params()
    assert lib.mfe_equilibrate(C.byref(s), C.byref(p), None, None, None, None) == -1
    s.m = 0
    dummy = C.c_void_p(16)
    assert lib.mfe_equilibrate(C.byref(s), C.byref(p), dummy, dummy, None, None) == -2
    assert lib.mfe_equilibrate(None, C.byref(p), dummy, dummy, None, None) == -1


def test_bf16_limits_rejected_on_host(lib):
    """The bf16 path refuses more than 64 probes and a box beyond the bf16 range of e^x
    (EUNSUPPORTED) and a leading dimension below n (EDIM) before any device work."""
    s = _csr_struct(40, 30)
    s.kind, s.ld, s.data = 1, 30, C.c_void_p(16)
    dummy = C.c_void_p(16)
    assert lib.mfe_equilibrate(C.byref(s), C.byref(_params(probes=65)), dummy, dummy, None, None) == -6
    assert lib.mfe_equilibrate(C.byref(s), C.byref(_params(box_M=81.0)), dummy, dummy, None, None) == -6
    assert "M <= 80" in lib.mfe_last_error().decode()
    s.ld = 29
    assert lib.mfe_equilibrate(C.byref(s), C.byref(_params()), dummy, dummy, None, None) == -2


def test_draw_signs_argument_checks(lib):
    assert lib.mfe_draw_signs(1, -1, 1, 0, 4, C.c_void_p(16), None) == -1
    assert lib.mfe_draw_signs(1, 0, 2**32, 0, 4, C.c_void_p(16), None) == -1
    assert lib.mfe_draw_signs(1, 0, 1, 4, 4, C.c_void_p(16), None) == -1
    assert lib.mfe_draw_signs(1, 0, 1, 0, 0, None, None) == 0


def test_plan_rejects_bad_probe_counts(lib):
    s = _csr_struct()
    h = C.c_void_p()
    assert lib.mfe_plan_create(C.byref(s), 1, 65, None, C.byref(h)) == -6
    assert lib.mfe_plan_create(C.byref(s), 0, 4, None, C.byref(h)) == -1


def test_autotune_argument_checks(lib):
    p = _params()
    assert lib.mfe_plan_autotune(None, C.byref(p), None, None, 10, None, None, None) == -1
    assert lib.mfe_plan_autotune(C.c_void_p(16), None, None, None, 10, None, None, None) == -1


def test_set_tuning_argument_checks(lib):
    assert lib.mfe_plan_set_tuning(None, 8, 0, 0, -1, -1, 0) == -1


def test_probe_argument_checks(lib):
    """The ceiling probes refuse sizes, load counts and row lengths they do not support
    before allocating anything."""
    ms = C.c_double()
    assert lib.mfe_probe_gather(4, 10, 1, 1, C.byref(ms), None) == -1
    assert lib.mfe_probe_gather(1024, 10, 3, 1, C.byref(ms), None) == -1
    assert lib.mfe_probe_gather_sorted(1024, 10, 7, 1, C.byref(ms), None) == -1
    assert lib.mfe_probe_gather_sorted(1024, 0, 10, 1, C.byref(ms), None) == -1
    assert lib.mfe_probe_gather_sorted(8 << 32, 10, 10, 1, C.byref(ms), None) == -1
    assert lib.mfe_probe_gather_sorted(1024, 10, 10, 1, None, None) == -1
    assert lib.mfe_probe_stream(8, 1, C.byref(ms), None) == -1


def test_variant_argument_checks(lib):
    """Section 6 entry points reject NULL plans, non-square symmetric requests and other
    kinds before any device work."""
    assert lib.mfe_plan_set_targets(None, None, None, None) == -1
    assert lib.mfe_plan_set_blocks(None, None, 0, None, 0) == -1
    h = C.c_void_p()
    assert lib.mfe_plan_create_symmetric(None, 4, None, C.byref(h)) == -1
    assert lib.mfe_plan_create_symmetric(None, 4, None, None) == -1
    s = _csr_struct()   # 4 x 3
    assert lib.mfe_plan_create_symmetric(C.byref(s), 4, None, C.byref(h)) == -2
    s.kind = 0          # dense FP64
    assert lib.mfe_plan_create_symmetric(C.byref(s), 4, None, C.byref(h)) == -6


def test_ccp_argument_checks(lib):
    nrm, it = C.c_double(), C.c_int32()
    assert lib.mfe_plan_op_norm(None, None, None, 10, 1e-6, C.byref(nrm), C.byref(it), None) == -1
    assert lib.mfe_plan_ccp_lasso(None, None, None, None, 1.0, 0.0, 10, 0, None, None, None, None) == -1
    fake = C.c_void_p(16)   # rejected before the plan is touched
    buf = (C.c_double * 4)()
    assert lib.mfe_plan_op_norm(fake, None, None, 0, 1e-6, C.byref(nrm), None, None) == -1
    assert lib.mfe_plan_ccp_lasso(fake, buf, None, None, 0.0, 0.0, 10, 0, None, buf, None, None) == -1
    assert lib.mfe_plan_ccp_lasso(fake, buf, None, None, 1.0, 0.0, -1, 0, None, buf, None, None) == -1
    assert lib.mfe_plan_ccp_lasso(fake, buf, None, None, 1.0, 0.0, 10, 0, buf, buf, None, None) == -1


def test_version(lib):
    assert "gfx950" in lib.mfe_version().decode()


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1602_06621_amd import _ffi

    monkeypatch.setattr(_ffi, "_LIB", None)
    monkeypatch.setenv("MFE_LIBRARY", str(tmp_path / "absent.so"))
    with pytest.raises(_ffi.LibraryMissing):
        _ffi.default_alpha_beta(2, 2)


def test_target_relation_check_warns_without_failing(lib):
    """Section 1: m alpha^2 = n beta^2 is needed for exact equilibration.  The host-only
    check returns OK either way and leaves a warning when the relation fails."""
    rel = C.c_double()
    a = (100 / 200) ** 0.25
    assert lib.mfe_check_targets(200, 100, a, 1 / a, C.byref(rel)) == 0
    assert rel.value < 1e-15
    assert lib.mfe_last_error().decode() == ""
    assert lib.mfe_check_targets(200, 100, 1.0, 1.0, C.byref(rel)) == 0
    assert rel.value == pytest.approx(0.5, rel=1e-15)     # |200 - 100| / 200
    msg = lib.mfe_last_error().decode()
    assert msg.startswith("warning:") and "Section 1" in msg
    assert lib.mfe_check_targets(0, 100, 1.0, 1.0, C.byref(rel)) == -1
    assert lib.mfe_check_targets(10, 10, float("nan"), 1.0, None) == -1
    from paper_1602_06621_amd import check_targets

    r, w = check_targets(3, 12, 2.0, 1.0)      # 3 * 4 = 12 * 1
    assert r == 0.0 and w == ""


def test_csr_f64_kind_declared_and_refused(lib):
    """MFE_CSR_F64 is named in the header and refused with EUNSUPPORTED before any
    device work."""
    text = open(HEADER).read()
    assert "MFE_CSR_F64 = 4" in text
    s = _csr_struct()
    s.kind = 4
    dummy = C.c_void_p(16)
    assert lib.mfe_equilibrate(C.byref(s), C.byref(_params()), dummy, dummy, None, None) == -6
    assert "FP64 values" in lib.mfe_last_error().decode()
    h = C.c_void_p()
    assert lib.mfe_plan_create(C.byref(s), 1, 4, None, C.byref(h)) == -6


def test_training_set_argument_checks(lib):
    cnt = C.c_int64()
    buf = C.c_void_p(16)
    assert lib.mfe_plan_training_set(None, 1, 4, None, None, 0.1, 10.0, buf, buf, 8, 0, None, None, None,
                                     C.byref(cnt), None) == -1
    assert lib.mfe_plan_training_set(buf, 1, 4, None, None, 0.1, 10.0, buf, buf, 0, 0, None, None, None,
                                     C.byref(cnt), None) == -1


def test_noalloc_entry_point_refuses_on_host(lib):
    """The allocation-free entry point takes dense FP64 only and refuses a run that needs
    more than its 8 MiB scratch before any device work."""
    s = _csr_struct(300000, 10)
    dummy = C.c_void_p(16)
    assert lib.mfe_equilibrate_noalloc(C.byref(s), C.byref(_params(alpha=(10 / 300000) ** 0.25,
                                                                    beta=(300000 / 10) ** 0.25)),
                                       dummy, dummy, None, None) == -6
    s.kind, s.ld, s.data = 0, 10, C.c_void_p(16)
    p = _params(alpha=(10 / 300000) ** 0.25, beta=(300000 / 10) ** 0.25)
    assert lib.mfe_equilibrate_noalloc(C.byref(s), C.byref(p), dummy, dummy, None, None) == -2
    assert "scratch" in lib.mfe_last_error().decode()
    assert lib.mfe_equilibrate_noalloc(C.byref(s), C.byref(p), None, None, None, None) == -1
