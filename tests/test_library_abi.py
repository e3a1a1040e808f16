"""The C-ABI library loads and exports every symbol include/psatd.h declares.

No compute call is made: validation errors are reported on the host before
any HIP call, so they can be checked without a GPU.
"""

import ctypes
import os
import re

import pytest

import paper_1608_05739_amd as pk
from paper_1608_05739_amd import _binding as b

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "psatd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(psatd_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pk.LIBRARY_PATH):
        pytest.fail("libpsatd.so is not built; run __graft_entry__.build()")
    return pk.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("psatd_plan", "psatd_push", "psatd_destroy", "psatd_workspace_size",
                 "psatd_set_workspace", "psatd_status_string", "psatd_last_error"):
        assert must in names
    assert set(names) == set(b.EXPORTED_SYMBOLS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code, name in b.STATUS_NAMES.items():
        assert lib.psatd_status_string(code).decode() == name


def _desc(n=(8, 1, 8), d=(1.0, 1.0, 1.0), dt=0.5, ndim=2, offset=0):
    pd = b.PatchDesc()
    pd.ndim = ndim
    pd.n = (ctypes.c_int64 * 3)(*n)
    pd.d = (ctypes.c_double * 3)(*d)
    pd.dt = dt
    pd.offset = offset
    return pd


def _cfg(**kw):
    c = b.Config()
    c.precision, c.source_mode, c.path, c.order = 0, 0, 0, 0
    c.c, c.eps0, c.flags = 1.0, 1.0, 0
    for k, v in kw.items():
        setattr(c, k, v)
    return c


@pytest.mark.parametrize("desc,cfg,expect", [
    (_desc(n=(10, 1, 8)), _cfg(), -2),          # 10 = 2 * 5: radix 5 unsupported
    (_desc(n=(7, 1, 8)), _cfg(), -2),           # odd x length
    (_desc(n=(8, 1, 8192)), _cfg(), -2),        # longer than 4096
    (_desc(n=(8, 2, 8)), _cfg(), -1),           # 2D with ny != 1
    (_desc(dt=0.0), _cfg(), -1),                # dt must be > 0
    (_desc(d=(1.0, 1.0, -1.0)), _cfg(), -1),    # spacing must be > 0
    (_desc(offset=3), _cfg(), -1),              # odd offset
    (_desc(), _cfg(precision=5), -1),
    (_desc(), _cfg(source_mode=9), -1),
    (_desc(), _cfg(order=3), -1),               # odd order
    (_desc(), _cfg(c=0.0), -1),
    (_desc(), _cfg(flags=0x100), -1),
])
def test_plan_validation_on_host(lib, desc, cfg, expect):
    out = ctypes.c_void_p()
    st = lib.psatd_plan(ctypes.byref(cfg), ctypes.byref(desc), 1, 0, ctypes.byref(out))
    assert st == expect, lib.psatd_last_error().decode()
    assert out.value is None
    assert lib.psatd_last_error().decode() != ""


def test_overlapping_patches_rejected(lib):
    descs = (b.PatchDesc * 2)(_desc(offset=0), _desc(offset=32))
    out = ctypes.c_void_p()
    st = lib.psatd_plan(ctypes.byref(_cfg()), descs, 2, 0, ctypes.byref(out))
    assert st == -1 and "overlap" in lib.psatd_last_error().decode()


def test_null_arguments(lib):
    out = ctypes.c_void_p()
    assert lib.psatd_plan(None, ctypes.byref(_desc()), 1, 0, ctypes.byref(out)) == -1
    assert lib.psatd_plan(ctypes.byref(_cfg()), None, 1, 0, ctypes.byref(out)) == -1
    assert lib.psatd_plan(ctypes.byref(_cfg()), ctypes.byref(_desc()), 0, 0, ctypes.byref(out)) == -1
    assert lib.psatd_push(None, None, 1, None) == -1
    assert lib.psatd_destroy(None) == 0
    n = ctypes.c_size_t()
    assert lib.psatd_workspace_size(None, ctypes.byref(n)) == -1


def test_package_fails_loudly_without_library(tmp_path):
    with pytest.raises(RuntimeError, match="not built"):
        b.load_library(str(tmp_path / "missing.so"))


def _dom(n=(128, 1, 128), parts=(2, 1, 2), guard=(16, 0, 16), ndim=2):
    dd = b.DomainDesc()
    dd.ndim = ndim
    dd.n = (ctypes.c_int64 * 3)(*n)
    dd.parts = (ctypes.c_int32 * 3)(*parts)
    dd.guard = (ctypes.c_int32 * 3)(*guard)
    dd.d = (ctypes.c_double * 3)(0.1, 0.1, 0.1)
    dd.dt = 0.05
    return dd


@pytest.mark.parametrize("dom,expect", [
    (_dom(guard=(5, 0, 16)), -2),            # 64 + 2 * 5 = 74 = 2 * 37: unsupported length
    (_dom(parts=(3, 1, 2)), -1),             # 128 does not split into 3 equal boxes
    (_dom(guard=(-1, 0, 16)), -1),           # negative guard
    (_dom(guard=(49, 0, 16)), -1),           # 64 + 2 * 49 = 162 is supported, but the x guard is odd
    (_dom(n=(128, 2, 128)), -1),             # 2D with ny != 1
    (_dom(ndim=4), -1),
])
def test_domain_validation_on_host(lib, dom, expect):
    h = ctypes.c_void_p()
    st = lib.psatd_domain_create(ctypes.byref(_cfg()), ctypes.byref(dom), 0, ctypes.byref(h))
    assert st == expect
    assert h.value is None
    assert lib.psatd_last_error().decode()


def test_plan_flags_match_the_header():
    # every PSATD_FLAG_* of include/psatd.h has the binding's value, and the
    # planner accepts each of them (fails only at the device query without a GPU)
    import re
    text = open(HEADER).read()
    flags = dict(re.findall(r"#define PSATD_FLAG_(\w+) (0x[0-9a-f]+)u", text))
    assert "RADIX4_LINES" in flags
    for name, val in flags.items():
        assert getattr(b, "FLAG_" + name) == int(val, 16), name


@pytest.mark.parametrize("flag", ["RADIX4_LINES", "GENERIC_KERNELS"])
def test_known_flags_pass_host_validation(lib, flag):
    out = ctypes.c_void_p()
    st = lib.psatd_plan(ctypes.byref(_cfg(flags=getattr(b, "FLAG_" + flag))), ctypes.byref(_desc()),
                        1, 0, ctypes.byref(out))
    assert st in (0, -4), lib.psatd_last_error().decode()
    if st == 0:
        lib.psatd_destroy(out)
    st = lib.psatd_plan(ctypes.byref(_cfg(flags=0x80)), ctypes.byref(_desc()), 1, 0, ctypes.byref(out))
    assert st == -1 and "flag" in lib.psatd_last_error().decode()


@pytest.mark.parametrize("desc,cfg,expect", [
    (_desc(), _cfg(flags=b.FLAG_PSTD, source_mode=1), -1),   # PSTD takes J only
    (_desc(dt=0.7), _cfg(flags=b.FLAG_PSTD), -1),            # c dt |k|max / 2 = 1.18 > 1
    (_desc(dt=0.6), _cfg(flags=b.FLAG_PSTD), None),          # 0.5 * 0.6 * 2 pi 3/8 sqrt 2 = 0.9996
])
def test_pstd_validation_on_host(lib, desc, cfg, expect):
    out = ctypes.c_void_p()
    st = lib.psatd_plan(ctypes.byref(cfg), ctypes.byref(desc), 1, 0, ctypes.byref(out))
    if expect is None:
        # valid: fails only at the device query without a GPU
        assert st in (0, -4), lib.psatd_last_error().decode()
        if st == 0:
            lib.psatd_destroy(out)
    else:
        assert st == expect, lib.psatd_last_error().decode()
        assert out.value is None


@pytest.mark.parametrize("scheme,desc,cfg,expect", [
    (5, _desc(), _cfg(), -1),                                   # unknown scheme
    (0, _desc(), _cfg(source_mode=1), -1),                      # rho form: FDTD takes J only
    (0, _desc(), _cfg(order=3), -1),                            # odd order
    (0, _desc(), _cfg(order=34), -1),                           # beyond 32
    (0, _desc(), _cfg(flags=b.FLAG_GRAPH), -1),                 # flags must be 0
    (1, _desc(), _cfg(order=4), -1),                            # CKC is second order
    (1, _desc(n=(8, 8, 8), ndim=3), _cfg(), -2),                # CKC in 3D
    (1, _desc(d=(1.0, 1.0, 0.5), dt=0.4), _cfg(), -1),          # CKC needs dx = dz
    (0, _desc(dt=0.75), _cfg(), -1),                            # Yee 2D: c dt <= dx / sqrt 2
    (0, _desc(n=(8, 1, 8), dt=0.1), _cfg(order=16), -2),        # n < p
    (0, _desc(n=(8, 1, 8), dt=0.1, offset=-1), _cfg(), -1),
    (1, _desc(dt=1.0), _cfg(), None),                           # CKC at c dt = dx: allowed
    (0, _desc(dt=0.7071), _cfg(), None),                        # Yee just below 1/sqrt 2
    (0, _desc(n=(5, 1, 7), dt=0.3), _cfg(), None),              # any length
])
def test_fdtd_validation_on_host(lib, scheme, desc, cfg, expect):
    out = ctypes.c_void_p()
    st = lib.psatd_fdtd_plan(ctypes.byref(cfg), scheme, ctypes.byref(desc), 0, ctypes.byref(out))
    if expect is None:
        assert st in (0, -4), lib.psatd_last_error().decode()
        if st == 0:
            lib.psatd_fdtd_destroy(out)
    else:
        assert st == expect, lib.psatd_last_error().decode()
        assert out.value is None
        assert lib.psatd_last_error().decode()
    assert lib.psatd_fdtd_push(None, None, 1, None) == -1
    assert lib.psatd_fdtd_destroy(None) == 0


# ---- host-only planning (psatd_plan_describe): no GPU needed
def _spec_elems(n, nin, ndim):
    # k-space elements of one patch: nx/2 * ny * nz per input, padded to 64
    m = n[0] // 2 * (n[1] if ndim == 3 else 1) * n[2]
    return (m * nin + 63) // 64 * 64


@pytest.mark.parametrize("shape,precision,source,nin", [
    ((4096, 1, 4096), "fp32", "rho", 11),
    ((512, 512, 512), "fp32", "vacuum", 6),
    ((1024, 1024, 512), "fp32", "rho", 11),
    ((256, 1, 384), "fp64", "j", 9),
])
def test_describe_workspace_matches_the_layout(lib, shape, precision, source, nin):
    ndim = 3 if shape[1] > 1 else 2
    p = pk.Patch(ndim, shape, (1.0, 1.0, 1.0), 0.3)
    ws, info = pk.describe_plan([p], precision=precision, source_mode=source)
    elem = 4 if precision == "fp32" else 8
    blocks = 2 if ndim == 3 else 1  # 3D: a second block for the y passes
    assert ws == _spec_elems(shape, nin, ndim) * blocks * 2 * elem
    assert info.startswith(f"ndim={ndim} patches=1") and f"ws={ws}" in info


def test_describe_batched_patches_workload(lib):
    ps = [pk.Patch(2, (128, 1, 128), (1.0, 1.0, 1.0), 0.5) for _ in range(256)]
    ws, info = pk.describe_plan(ps)
    assert ws == 256 * _spec_elems((128, 1, 128), 6, 2) * 2 * 4
    names = [ln.split()[0] for ln in info.splitlines()[1:]]
    assert names[0].startswith("x") and names[-1].startswith("x") and len(names) == 3


def test_describe_long_z_lines_fall_back_to_plain_z_passes(lib):
    # FP64 2D holds at most 2048 modes per workgroup in the fused pass: the
    # plan runs the plain z passes (transform, update, transform) instead
    p = pk.Patch(2, (256, 1, 4096), (1.0, 1.0, 1.0), 0.5)
    _, fused = pk.describe_plan([p], precision="fp64", path="fused")
    _, plain = pk.describe_plan([p], precision="fp64", path="plain")
    names = lambda s: [ln.split()[0] for ln in s.splitlines()[1:]]  # noqa: E731
    assert names(fused) == names(plain) and "update" in names(fused)
    _, short = pk.describe_plan([pk.Patch(2, (256, 1, 2048), (1.0, 1.0, 1.0), 0.5)], precision="fp64")
    assert "update" not in names(short)


def test_describe_reports_the_same_errors_as_plan(lib):
    with pytest.raises(pk.PsatdError) as e:
        pk.describe_plan([pk.Patch(2, (10, 1, 8), (1.0, 1.0, 1.0), 0.5)])
    assert e.value.status == -2
    with pytest.raises(pk.PsatdError) as e:
        pk.describe_plan([pk.Patch(2, (64, 1, 64), (1.0, 1.0, 1.0), 0.9)], pstd=True)
    assert e.value.status == -1 and "Courant" in str(e.value)


@pytest.mark.parametrize("tuning", [
    b"",                                  # no version tag
    b"psatd-tuning-1",                    # no choices
    b"psatd-tuning-2;1,0,8,0,8,-1",       # unknown version
    b"psatd-tuning-1;1,0,8,0,8",          # five fields
    b"psatd-tuning-1;1,0,8,0,8,-1;",      # trailing separator
    b"psatd-tuning-1;1,0,8,0,8,-1 junk",  # trailing text
])
def test_tuned_plan_rejects_malformed_tuning_on_host(lib, tuning):
    # the string is parsed before any device is touched
    out = ctypes.c_void_p()
    st = lib.psatd_plan_tuned(ctypes.byref(_cfg()), ctypes.byref(_desc()), 1, 0, tuning,
                              ctypes.byref(out))
    assert st == -1 and "tuning" in lib.psatd_last_error().decode()
    assert out.value is None


def test_tuned_plan_null_arguments(lib):
    out = ctypes.c_void_p()
    assert lib.psatd_plan_tuned(ctypes.byref(_cfg()), ctypes.byref(_desc()), 1, 0, None,
                                ctypes.byref(out)) == -1
    n = ctypes.c_size_t()
    assert lib.psatd_plan_tuning(None, None, 0, ctypes.byref(n)) == -1
