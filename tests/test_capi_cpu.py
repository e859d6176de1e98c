"""CPU checks of the C ABI: the library loads, exports every function of include/fde.h, its struct
layout matches the Python binding, and argument validation fails cleanly before any device work."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1706_06844_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fde.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fde_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return L.load()


def test_every_declared_function_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and every exported binding signature refers to a declared function
    assert set(n for n in L.SIGNATURES if hasattr(lib, n)) >= set(names)


def test_struct_layout_matches_c(tmp_path):
    exe = tmp_path / "abi_layout"
    src = os.path.join(ROOT, "tests", "abi_layout.c")
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    c = dict(line.rsplit(" ", 1) for line in out if line.strip())
    assert int(c["fde_problem"]) == ctypes.sizeof(L.fde_problem)
    assert int(c["fde_stats"]) == ctypes.sizeof(L.fde_stats)
    for key, val in c.items():
        if "." in key:
            struct, field = key.split(".")
            cls = getattr(L, struct)
            assert getattr(cls, field).offset == int(val), key


def test_problem_default(lib):
    p = L.fde_problem()
    lib.fde_problem_default(ctypes.byref(p), 1.5, 1.6, 63, 31, 0.01)
    assert (p.alpha, p.beta, p.n1, p.n2, p.tau) == (1.5, 1.6, 63, 31, 0.01)
    assert (p.a1, p.b1, p.a2, p.b2) == (0.0, 1.0, 0.0, 1.0)
    assert p.omega == 0.7 and p.nu_pre == 1 and p.nu_post == 1 and p.coarsest_n == 7
    assert p.restart == 20 and p.maxit == 5000 and p.rtol == 1e-10


@pytest.mark.parametrize("field,value,needle", [
    ("alpha", 2.0, "alpha"), ("alpha", 1.0, "alpha"), ("beta", 0.5, "alpha and beta"),
    ("n1", 10, "2^l - 1"), ("n2", 3, "2^l - 1"), ("n1", 4, "2^l - 1"), ("n1", 4095, "2048"),
    ("n1", 4096, "2048"),
    ("tau", 0.0, "tau"), ("tau", -1.0, "tau"), ("restart", 40, "restart"),
    ("omega", 1.5, "omega"), ("b1", -1.0, "a < b"), ("precision", 7, "precision"),
    ("precision", 5, "precision"),
])
def test_setup_rejects_invalid_problems(lib, field, value, needle):
    p = L.fde_problem()
    lib.fde_problem_default(ctypes.byref(p), 1.5, 1.5, 63, 63, 0.01)
    setattr(p, field, value)
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    rc = lib.fde_setup(ctypes.byref(p), fake, fake, fake, fake, None, ctypes.byref(out))
    assert rc == L.FDE_EINVAL and out.value is None
    assert needle in lib.fde_last_error(None).decode()


def test_even_sides_default_to_the_8x8_coarsest_grid_and_geometric_only(lib):
    p = L.fde_problem()
    lib.fde_problem_default(ctypes.byref(p), 1.8, 1.6, 64, 64, 1 / 64)
    assert p.coarsest_n == 8
    lib.fde_problem_default(ctypes.byref(p), 1.8, 1.6, 63, 64, 1 / 64)
    assert p.coarsest_n == 7
    fake = ctypes.c_void_p(0x1000)
    out = ctypes.c_void_p()
    for field, value, needle in (("mg_variant", L.FDE_MG_GALERKIN, "geometric"),
                                 ("mg_variant", L.FDE_MG_BAND, "geometric"),
                                 ("precision", L.FDE_MIXED_BF16GEMM, "2^l - 1")):
        lib.fde_problem_default(ctypes.byref(p), 1.8, 1.6, 64, 64, 1 / 64)
        setattr(p, field, value)
        rc = lib.fde_setup(ctypes.byref(p), fake, fake, fake, fake, None, ctypes.byref(out))
        assert rc == L.FDE_EINVAL and out.value is None
        assert needle in lib.fde_last_error(None).decode()


@pytest.mark.parametrize("prec", [L.FDE_MIXED_FP32_CYCLE, L.FDE_MIXED_CYCLE_BF16])
def test_fp32_cycles_need_a_rediscretised_fine_level(lib, prec):
    p = L.fde_problem()
    lib.fde_problem_default(ctypes.byref(p), 1.5, 1.5, 63, 63, 0.01)
    p.precision = prec
    p.mg_variant = L.FDE_MG_BAND
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    assert lib.fde_setup(ctypes.byref(p), fake, fake, fake, fake, None, ctypes.byref(out)) == L.FDE_EINVAL
    assert "band" in lib.fde_last_error(None).decode()
    assert lib.fde_footprint(ctypes.byref(p)) == 0


def test_fp32_cycles_halve_the_basis_footprint():
    from paper_1706_06844_amd import fde

    q = {}
    for prec in (L.FDE_MIXED_FP32, L.FDE_MIXED_FP32_CYCLE, L.FDE_MIXED_CYCLE_BF16):
        p = fde.fde_problem_default(1.5, 1.5, 2047, 2047, 0.01)
        p.precision = prec
        q[prec] = fde.fde_footprint(p)
    ld = 2047 * 2047 + 63 - (2047 * 2047 + 63) % 64
    # 21 basis columns of FP64 become one FP64 column plus 21 FP32 columns (the estimate carries a
    # 5% margin)
    saved = 21 * ld * 8 - (ld * 8 + 21 * ld * 4)
    assert q[L.FDE_MIXED_FP32] - q[L.FDE_MIXED_FP32_CYCLE] == pytest.approx(1.05 * saved, abs=2)
    # BF16 storage: 21 BF16 columns plus one FP32 work vector in place of 21 FP32 columns
    saved16 = 21 * ld * 4 - (ld * 4 + 21 * ld * 2)
    assert q[L.FDE_MIXED_FP32_CYCLE] - q[L.FDE_MIXED_CYCLE_BF16] == pytest.approx(1.05 * saved16, abs=2)


def test_setup_rejects_null_arguments(lib):
    p = L.fde_problem()
    lib.fde_problem_default(ctypes.byref(p), 1.5, 1.5, 63, 63, 0.01)
    out = ctypes.c_void_p()
    assert lib.fde_setup(ctypes.byref(p), None, None, None, None, None, ctypes.byref(out)) == L.FDE_EINVAL
    assert lib.fde_setup(None, None, None, None, None, None, ctypes.byref(out)) == L.FDE_EINVAL
    assert lib.fde_setup(ctypes.byref(p), None, None, None, None, None, None) == L.FDE_EINVAL


def test_null_handle_calls_fail_cleanly(lib):
    assert lib.fde_solve(None, None, None, None) == L.FDE_EINVAL
    assert lib.fde_step(None, None, None, None, None) == L.FDE_EINVAL
    assert lib.fde_num_levels(None) == L.FDE_EINVAL
    lib.fde_destroy(None)


def test_footprint_and_budget_admission_on_host():
    import ctypes

    from paper_1706_06844_amd import _lib as L
    from paper_1706_06844_amd import fde

    lib = L.load()
    small = fde.fde_problem_default(1.5, 1.5, 127, 127, 0.01)
    big = fde.fde_problem_default(1.5, 1.5, 2047, 2047, 0.01)
    fs, fb = fde.fde_footprint(small), fde.fde_footprint(big)
    assert 0 < fs < fb
    # FP64 C3: outer fields, 21 basis vectors, 20 FP64 preconditioned vectors, hierarchy
    assert 1.0e9 < fb < 4.0e9
    bad = fde.fde_problem_default(2.5, 1.5, 127, 127, 0.01)
    assert fde.fde_footprint(bad) == 0
    # a request that does not fit is refused before any device memory is touched
    out = ctypes.c_void_p()
    assert lib.fde_batch_create(ctypes.c_size_t(fs // 2), None, ctypes.byref(out)) == 0
    fake = ctypes.c_void_p(0x1000)
    rc = lib.fde_batch_admit(out, ctypes.byref(small), fake, fake, fake, fake, fake, 4, 0.0, 0, None, None, None)
    assert rc == L.FDE_EAGAIN
    active, used = ctypes.c_int32(), ctypes.c_size_t()
    assert lib.fde_batch_info(out, ctypes.byref(active), ctypes.byref(used)) == 0
    assert active.value == 0 and used.value == 0
    lib.fde_batch_destroy(out)


def test_batch_settings_are_validated_on_host():
    # grouping, scheduling and lane settings check their arguments before touching the device
    import ctypes

    from paper_1706_06844_amd import _lib as L

    lib = L.load()
    out = ctypes.c_void_p()
    assert lib.fde_batch_create(ctypes.c_size_t(1 << 30), None, ctypes.byref(out)) == 0
    assert lib.fde_batch_set_grouping(out, 127, 0) == L.FDE_EINVAL
    assert lib.fde_batch_set_grouping(out, 127, 2000) == L.FDE_EINVAL
    assert lib.fde_batch_set_grouping(out, -1, 4) == L.FDE_EINVAL
    assert lib.fde_batch_set_grouping(out, 511, 16) == 0
    assert lib.fde_batch_set_grouping(out, 0, 0) == 0
    assert lib.fde_batch_set_policy(out, -1, 0, -1) == L.FDE_EINVAL
    assert lib.fde_batch_set_policy(out, 2, -1, -1) == L.FDE_EINVAL
    assert lib.fde_batch_set_policy(out, 2, 5, -2) == L.FDE_EINVAL
    assert lib.fde_batch_set_policy(out, 2, 5, 1) == 0
    assert lib.fde_batch_set_policy(out, 0, 0, -1) == 0
    assert lib.fde_batch_set_lanes(out, 1) == L.FDE_EINVAL
    assert lib.fde_batch_set_lanes(out, 17) == L.FDE_EINVAL
    assert lib.fde_batch_set_lanes(out, 0) == 0
    assert lib.fde_batch_set_grouping(None, 127, 4) == L.FDE_EINVAL
    assert lib.fde_batch_set_policy(None, 0, 0, -1) == L.FDE_EINVAL
    assert lib.fde_batch_set_lanes(None, 0) == L.FDE_EINVAL
    lib.fde_batch_destroy(out)
