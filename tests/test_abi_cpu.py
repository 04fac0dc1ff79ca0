"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/wombat_weno.h, and rejects invalid
configurations before touching a device."""
import ctypes as C
import os
import re

import pytest

from paper_1808_10633_amd import wombat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(wombat_\w+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(wombat.LIB_PATH):
        pytest.fail("libwombat_weno.so is not built (run paper_1808_10633_amd.build.build())")
    return wombat.lib()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 14, names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_abi_version(lib):
    assert lib.wombat_weno_abi_version() == 6 == wombat.ABI_VERSION


def _cfg(**kw):
    cfg = wombat.Config()
    assert wombat.lib().wombat_weno_config_default(C.byref(cfg)) == 0
    for k, v in kw.items():
        if k == "bc":
            for i in range(6):
                cfg.bc[i] = v[i]
        else:
            setattr(cfg, k, v)
    return cfg


def test_default_config_is_valid(lib):
    cfg = _cfg()
    assert lib.wombat_weno_validate_config(C.byref(cfg)) == 0
    assert lib.wombat_weno_state_elems(C.byref(cfg)) == 8 * 38 ** 3
    cfg2 = _cfg(ny=1, dy=1.0)
    assert lib.wombat_weno_state_elems(C.byref(cfg2)) == 8 * 38 * 1 * 38


@pytest.mark.parametrize("kw,frag", [
    (dict(nx=0), "cell counts"),
    (dict(ny=2), "at least 3"),
    (dict(nx=1, ny=1, nz=1), "more than one cell"),
    (dict(ng=2), "ng must be 3"),
    (dict(gamma=1.0), "gamma"),
    (dict(cfl=1.5), "cfl"),
    (dict(cfl=0.0), "cfl"),
    (dict(eps=0.0), "eps"),
    (dict(dx=-1.0), "widths"),
    (dict(dz=float("nan")), "widths"),
    (dict(precision=7), "precision"),
    (dict(weights=2), "weights"),
    (dict(weights=-1), "weights"),
    (dict(integrator=2), "integrator"),
    (dict(lf_speed=3), "lf_speed"),
    (dict(bc=(0, 1, 0, 0, 0, 0)), "both faces"),
    (dict(bc=(2, 2, 0, 0, 0, 0)), "user_bc"),
    (dict(bc=(5, 5, 0, 0, 0, 0)), "unknown boundary"),
])
def test_invalid_configs_rejected(lib, kw, frag):
    cfg = _cfg(**kw)
    assert lib.wombat_weno_validate_config(C.byref(cfg)) == wombat.WW_ERR_INVALID_ARG
    assert frag in wombat.last_error()
    h = C.c_void_p(1234)
    assert lib.wombat_weno_init(C.byref(cfg), C.byref(h)) == wombat.WW_ERR_INVALID_ARG
    assert h.value == 1234      # out untouched on failure


def test_null_arguments(lib):
    assert lib.wombat_weno_validate_config(None) == wombat.WW_ERR_INVALID_ARG
    assert lib.wombat_weno_init(None, None) == wombat.WW_ERR_INVALID_ARG
    lib.wombat_weno_destroy(None)   # NULL-safe
    assert lib.wombat_weno_fill_ghosts(None, None) == wombat.WW_ERR_INVALID_ARG
    d = C.c_double()
    assert lib.wombat_weno_cfl_dt(None, None, C.byref(d)) == wombat.WW_ERR_INVALID_ARG
    assert lib.wombat_weno_step(None, None, 0.0, None) == wombat.WW_ERR_INVALID_ARG
    assert lib.wombat_weno_stage(None, 0, 0.1, None, None, None, None) == wombat.WW_ERR_INVALID_ARG


def test_product_path_fails_loudly_without_library(monkeypatch, tmp_path):
    # No silent fallback: a missing library is an error, not a CPU path.
    monkeypatch.setattr(wombat, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(wombat, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        wombat.lib()


def test_weights_default_and_batched_rejects_z(lib):
    cfg = _cfg()
    assert cfg.weights == wombat.WEIGHTS_JS
    cfg.weights = wombat.WEIGHTS_Z
    assert lib.wombat_weno_validate_config(C.byref(cfg)) == 0
    # the batched form is JS-only: refused before any device work
    dims = (C.c_int32 * 3)(16, 16, 16)
    h = C.c_void_p(1234)
    assert lib.wombat_weno_batch_init(C.byref(cfg), 1, dims, C.byref(h)) == wombat.WW_ERR_UNSUPPORTED
    assert "WENO-JS" in lib.wombat_weno_batch_last_error(None).decode()
    assert h.value == 1234


def test_integrator_default_and_batched_rejects_ssprk3(lib):
    cfg = _cfg()
    assert cfg.integrator == wombat.RK4
    cfg.integrator = wombat.SSPRK3
    assert lib.wombat_weno_validate_config(C.byref(cfg)) == 0
    dims = (C.c_int32 * 3)(16, 16, 16)
    h = C.c_void_p(1234)
    assert lib.wombat_weno_batch_init(C.byref(cfg), 1, dims, C.byref(h)) == wombat.WW_ERR_UNSUPPORTED
    assert "RK4" in lib.wombat_weno_batch_last_error(None).decode()
    assert h.value == 1234


def test_lf_speed_default_and_batched_rejects_global(lib):
    cfg = _cfg()
    assert cfg.lf_speed == wombat.LF_LOCAL
    cfg.lf_speed = wombat.LF_GLOBAL
    assert lib.wombat_weno_validate_config(C.byref(cfg)) == 0
    dims = (C.c_int32 * 3)(16, 16, 16)
    h = C.c_void_p(1234)
    assert lib.wombat_weno_batch_init(C.byref(cfg), 1, dims, C.byref(h)) == wombat.WW_ERR_UNSUPPORTED
    assert "LF" in lib.wombat_weno_batch_last_error(None).decode()
    assert h.value == 1234


def test_learned_field_default_and_checks(lib):
    cfg = _cfg()
    assert cfg.learned == 0
    cfg.learned = 2
    assert lib.wombat_weno_validate_config(C.byref(cfg)) == wombat.WW_ERR_INVALID_ARG
    assert "learned" in wombat.last_error()
    # the learned form's buffers are for FP32 contexts of the paper's scheme:
    # refused before any device work
    h = C.c_void_p(1234)
    for kw in (dict(learned=1), dict(learned=1, precision=wombat.WW_FP32_MIXED, weights=wombat.WEIGHTS_Z),
               dict(learned=1, precision=wombat.WW_FP32_MIXED, integrator=wombat.SSPRK3),
               dict(learned=1, precision=wombat.WW_FP32_MIXED, lf_speed=wombat.LF_GLOBAL)):
        c2 = _cfg(**kw)
        assert lib.wombat_weno_validate_config(C.byref(c2)) == 0
        assert lib.wombat_weno_init(C.byref(c2), C.byref(h)) == wombat.WW_ERR_UNSUPPORTED
        assert h.value == 1234


def test_alloc_count_is_exported(lib):
    n0 = wombat.alloc_count()
    assert n0 >= 0
    # refused configurations allocate nothing
    cfg = _cfg(nx=0)
    h = C.c_void_p()
    assert lib.wombat_weno_init(C.byref(cfg), C.byref(h)) == wombat.WW_ERR_INVALID_ARG
    assert wombat.alloc_count() == n0


def test_slab_planes_checks(lib):
    assert _cfg().slab_planes == 0
    for kw, frag in ((dict(slab_planes=2), "slab_planes"), (dict(slab_planes=-1), "slab_planes"),
                     (dict(slab_planes=8, nz=1, dz=1.0), "z axis")):
        cfg = _cfg(**kw)
        assert lib.wombat_weno_validate_config(C.byref(cfg)) == wombat.WW_ERR_INVALID_ARG
        assert frag in wombat.last_error()
    h = C.c_void_p(1234)
    for kw in (dict(slab_planes=8, integrator=wombat.SSPRK3), dict(slab_planes=8, lf_speed=wombat.LF_GLOBAL),
               dict(slab_planes=8, learned=1, precision=wombat.WW_FP32_MIXED)):
        cfg = _cfg(**kw)
        assert lib.wombat_weno_validate_config(C.byref(cfg)) == 0
        assert lib.wombat_weno_init(C.byref(cfg), C.byref(h)) == wombat.WW_ERR_UNSUPPORTED
        assert h.value == 1234


def test_b_storage_checks(lib):
    assert _cfg().b_storage == wombat.B_CELL
    cfg = _cfg(b_storage=2)
    assert lib.wombat_weno_validate_config(C.byref(cfg)) == wombat.WW_ERR_INVALID_ARG
    assert "b_storage" in wombat.last_error()
    h = C.c_void_p(1234)
    for kw in (dict(b_storage=1, bc=(1, 1, 0, 0, 0, 0)), dict(b_storage=1, slab_planes=8),
               dict(b_storage=1, learned=1, precision=wombat.WW_FP32_MIXED)):
        c2 = _cfg(**kw)
        assert lib.wombat_weno_validate_config(C.byref(c2)) == 0
        assert lib.wombat_weno_init(C.byref(c2), C.byref(h)) == wombat.WW_ERR_UNSUPPORTED
        assert h.value == 1234
    dims = (C.c_int32 * 3)(16, 16, 16)
    assert lib.wombat_weno_batch_init(C.byref(_cfg(b_storage=1)), 1, dims, C.byref(h)) == wombat.WW_ERR_UNSUPPORTED
