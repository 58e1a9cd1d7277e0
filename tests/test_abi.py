"""CPU checks of the C ABI: the library loads, exports everything the header
declares, and its host-only logic (push count, validation, workspace sizes)
behaves as documented.  No GPU work is launched."""
import ctypes as C
import math
import os

import pytest

from paper_2112_14944_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libpprviz.so is not built (run __graft_entry__.build())")
    return L.lib()


def test_exports_every_declared_symbol(lib):
    names = L.header_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), name
    # and the binding's signature table covers the same set
    assert set(names) == set(L._SIGS)


def test_version_and_status_strings(lib):
    assert lib.pprviz_version().startswith(b"pprviz")
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.pprviz_status_string(code) != b"unknown status"
    assert lib.pprviz_status_string(42) == b"unknown status"


@pytest.mark.parametrize("alpha,tol", [(0.15, 1e-6), (0.15, 1e-7), (0.15, 1e-10), (0.1, 1e-9), (0.2, 3e-5),
                                       (0.5, 0.3), (0.99, 1e-12)])
def test_pushes_for_tolerance(lib, alpha, tol):
    T = C.c_int32()
    cv = C.c_int32()
    assert lib.pprviz_pushes_for_tolerance(alpha, tol, 100000, C.byref(T), C.byref(cv)) == 0
    q = 1.0 - float(C.c_float(alpha).value)
    # smallest t with (1-alpha)^t <= tol, from the closed form of the residue norm
    assert q ** T.value <= tol
    assert T.value == 0 or q ** (T.value - 1) > tol
    assert cv.value == 1


def test_pushes_for_tolerance_edges(lib):
    T = C.c_int32()
    cv = C.c_int32()
    assert lib.pprviz_pushes_for_tolerance(0.15, 1e-6, 10, C.byref(T), C.byref(cv)) == 0
    assert (T.value, cv.value) == (10, 0)          # capped: not converged
    assert lib.pprviz_pushes_for_tolerance(0.15, 0.0, 37, C.byref(T), C.byref(cv)) == 0
    assert (T.value, cv.value) == (37, 1)          # tol <= 0: fixed T
    assert lib.pprviz_pushes_for_tolerance(0.15, 1.5, 37, C.byref(T), C.byref(cv)) == 0
    assert T.value == 0
    for a in (0.0, 1.0, -0.1, float("nan")):
        assert lib.pprviz_pushes_for_tolerance(a, 1e-6, 10, C.byref(T), C.byref(cv)) == L.PPR_EINVAL
    assert lib.pprviz_pushes_for_tolerance(0.15, 1e-6, -1, C.byref(T), C.byref(cv)) == L.PPR_EINVAL
    assert lib.pprviz_pushes_for_tolerance(0.15, 1e-6, 5, None, None) == L.PPR_EINVAL


def test_argument_validation_before_any_gpu_work(lib):
    g = L.ppr_csr(10, 20, C.c_void_p(16), C.c_void_p(16), None)
    ws = C.c_void_p(256)
    f = lib.ppr_matrix
    # NULL graph, bad alpha, missing sources, tgt/n_tgt mismatch
    assert f(None, None, 0, None, 0, 0.15, 1e-6, 10, None, None, None, None, ws, 1 << 20, None) == L.PPR_EINVAL
    assert f(C.byref(g), C.c_void_p(16), 1, None, 10, 1.5, 1e-6, 10, None, None, None, None, ws, 1 << 20,
             None) == L.PPR_EINVAL
    assert f(C.byref(g), None, 3, None, 10, 0.15, 1e-6, 10, None, None, None, None, ws, 1 << 20,
             None) == L.PPR_EINVAL
    assert f(C.byref(g), C.c_void_p(16), 3, None, 9, 0.15, 1e-6, 10, None, None, None, None, ws, 1 << 20,
             None) == L.PPR_EINVAL
    # workspace too small
    assert f(C.byref(g), C.c_void_p(16), 3, None, 10, 0.15, 1e-6, 10, None, None, None, None, ws, 8,
             None) == L.PPR_EWORKSPACE
    bad = L.ppr_csr(0, 0, C.c_void_p(16), None, None)
    assert f(C.byref(bad), None, 0, None, 0, 0.15, 1e-6, 10, None, None, None, None, ws, 1 << 20,
             None) == L.PPR_EINVAL
    assert lib.pdist(None, 4, 4, C.c_void_p(16), None) == L.PPR_EINVAL
    assert lib.pdist(C.c_void_p(16), 4, 4, C.c_void_p(16), None) == L.PPR_EINVAL  # aliasing
    assert lib.layout_step(C.c_void_p(16), 4, C.c_void_p(32), C.c_void_p(32), None, None, 0, None) == L.PPR_EINVAL
    assert lib.stress_eval(C.c_void_p(16), 4, C.c_void_p(32), C.c_void_p(64), None, 0, None) == L.PPR_EWORKSPACE
    assert lib.stress_backward(C.c_void_p(16), 4, C.c_void_p(32), 1.0, None, None, None) == L.PPR_EINVAL
    assert lib.ppr_matrix_backward(None, 0.15, 10, None, None, None, None, 0, None) == L.PPR_EINVAL


def test_validation_of_the_level_and_layout_entry_points(lib):
    # every case returns before any GPU work
    p = C.c_void_p(64)
    ws = C.c_void_p(256)
    g = L.ppr_csr(100, 400, p, p, None)
    r = C.c_int32()
    gfp = lib.gfp_level_dppr
    assert gfp(C.byref(g), None, p, 3, 10, 0.15, 1e-6, 100, p, None, None, C.byref(r), ws, 1 << 30,
               None) == L.PPR_EINVAL  # no leaf_ptr
    assert gfp(C.byref(g), p, p, 0, 10, 0.15, 1e-6, 100, p, None, None, C.byref(r), ws, 1 << 30,
               None) == L.PPR_EINVAL  # k < 1
    assert gfp(C.byref(g), p, p, 3, 2, 0.15, 1e-6, 100, p, None, None, C.byref(r), ws, 1 << 30,
               None) == L.PPR_EINVAL  # fewer leaves than sets
    assert gfp(C.byref(g), p, p, 3, 10, 1.0, 1e-6, 100, p, None, None, C.byref(r), ws, 1 << 30,
               None) == L.PPR_EINVAL  # alpha
    assert gfp(C.byref(g), p, p, 3, 10, 0.15, -1.0, 100, p, None, None, C.byref(r), ws, 1 << 30,
               None) == L.PPR_EINVAL  # r_max < 0
    assert gfp(C.byref(g), p, p, 3, 10, 0.15, float("nan"), 100, p, None, None, C.byref(r), ws, 1 << 30,
               None) == L.PPR_EINVAL
    assert gfp(C.byref(g), p, p, 3, 10, 0.15, 1e-6, 0, p, None, None, C.byref(r), ws, 1 << 30,
               None) == L.PPR_EINVAL  # max_rounds
    assert gfp(C.byref(g), p, p, 3, 10, 0.15, 1e-6, 100, p, None, None, C.byref(r), ws, 16,
               None) == L.PPR_EWORKSPACE
    gbp = lib.gbp_level_dppr
    assert gbp(C.byref(g), p, p, 3, 10, None, 2, p, 0.15, 100, p, None, None, C.byref(r), ws, 1 << 30,
               None) == L.PPR_EINVAL  # no targets
    assert gbp(C.byref(g), p, p, 3, 10, p, 4, p, 0.15, 100, p, None, None, C.byref(r), ws, 1 << 30,
               None) == L.PPR_EINVAL  # more targets than sets
    tau = lib.tau_push_level_dppr
    for eps, delta in ((0.0, 0.1), (0.5, 0.0), (float("inf"), 0.1)):
        assert tau(C.byref(g), p, p, 3, 10, 0.15, eps, delta, 0.0, 100, p, None, None, ws, 1 << 30,
                   None) == L.PPR_EINVAL
    assert lib.gfp_workspace(C.byref(g), 40, 100) > lib.gfp_workspace(C.byref(g), 3, 100) > 0
    huge = L.ppr_csr((1 << 24) + 1, 400, p, p, None)  # beyond the 32-bit slab gather offsets
    assert gfp(C.byref(huge), p, p, 3, 10, 0.15, 1e-6, 100, p, None, None, C.byref(r), ws, 1 << 62,
               None) == L.PPR_EUNSUPPORTED
    # exact majorization step and metrics
    it = C.c_int32()
    ex = lib.layout_step_exact
    assert ex(p, 8, C.c_void_p(128), C.c_void_p(128), 1e-6, 10, C.byref(it), ws, 1 << 20, None) == L.PPR_EINVAL
    assert ex(p, 8, C.c_void_p(128), C.c_void_p(256), -1.0, 10, C.byref(it), ws, 1 << 20, None) == L.PPR_EINVAL
    assert ex(p, 8, C.c_void_p(128), C.c_void_p(256), 1e-6, -1, C.byref(it), ws, 1 << 20, None) == L.PPR_EINVAL
    assert ex(p, 8, C.c_void_p(128), C.c_void_p(256), 1e-6, 10, C.byref(it), ws, 8, None) == L.PPR_EWORKSPACE
    assert lib.layout_exact_workspace(4096) > lib.layout_exact_workspace(64) > 0
    nd = C.c_double()
    ul = C.c_double()
    lm = lib.layout_metrics
    assert lm(p, 8, None, None, None, ws, 1 << 20, None) == L.PPR_EINVAL  # nothing asked
    assert lm(p, 8, None, C.byref(nd), C.byref(ul), ws, 1 << 20, None) == L.PPR_EINVAL  # ULCV needs a graph
    g8 = L.ppr_csr(9, 4, p, p, None)
    assert lm(p, 8, C.byref(g8), C.byref(nd), C.byref(ul), ws, 1 << 20, None) == L.PPR_EINVAL  # n != k
    assert lm(p, 8, None, C.byref(nd), None, ws, 8, None) == L.PPR_EWORKSPACE
    assert lib.layout_metrics_workspace(4096) > lib.layout_metrics_workspace(64) > 0


def test_plain_c_client(lib, tmp_path):
    # the header compiles as C99 and a C program links and calls the library
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    exe = str(tmp_path / "c_abi_check")
    libdir = os.path.dirname(L.LIB_PATH)
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_abi_check.c"), "-o", exe, "-L", libdir, "-lpprviz",
                    "-Wl,-rpath," + libdir, "-lm"], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.startswith("c abi ok")


def test_batch_validation_and_limits(lib):
    assert lib.pprviz_batch_max_n() == 2304
    p = C.c_void_p(64)
    big = L.ppr_batch(2, 5000, 10, 2305, 5000 * 2305, p, p, p, p)
    ws_big = lib.pprviz_batch_workspace(C.byref(big))
    assert ws_big > 0
    assert lib.pprviz_batch(C.byref(big), 0.15, 1e-6, 100, 10, p, C.c_void_p(128), p, p, None, p, ws_big,
                            None) == L.PPR_EUNSUPPORTED
    ok = L.ppr_batch(2, 5000, 10, 100, 5000 * 100, p, p, p, p)
    assert lib.pprviz_batch(C.byref(ok), 0.15, 1e-6, 100, 10, p, p, p, p, None, p, 1 << 30,
                            None) == L.PPR_EINVAL  # x0 aliases x_out
    assert lib.pprviz_batch(C.byref(ok), 0.15, 1e-6, 100, 10, p, C.c_void_p(128), p, p, None, p, 16,
                            None) == L.PPR_EWORKSPACE
    h = C.c_void_p()
    assert lib.pprviz_batch_plan_create(C.byref(ok), 0.15, 1e-6, 100, -1, p, C.c_void_p(128), p, p, None, p,
                                        1 << 30, None, C.byref(h)) == L.PPR_EINVAL
    assert lib.pprviz_batch_plan_launch(None, None) == L.PPR_EINVAL
    lib.pprviz_batch_plan_destroy(None)


def test_workspace_queries_grow_with_size(lib):
    small = L.ppr_csr(500, 4000, None, None, None)
    mid = L.ppr_csr(20000, 400000, None, None, None)
    large = L.ppr_csr(50000, 1000000, None, None, None)
    assert 0 < lib.ppr_matrix_workspace(C.byref(small), 500, 500) < (1 << 20)
    # the mid-size kernel keeps the iterate in LDS: its workspace is the
    # padded 16-bit arc copy (bounded by 17 slices of the longest row, nnz
    # entries and a group per slice) and small tables, independent of the
    # source count
    ws_mid = lib.ppr_matrix_workspace(C.byref(mid), 20000, 20000)
    assert 2 * (64 * 17 * 20000 + 400000) <= ws_mid < (64 << 20)
    assert ws_mid - lib.ppr_matrix_workspace(C.byref(mid), 2, 2) <= 8 * 20000 + 512  # FP64 residual per source
    # the streaming path holds two node-major iterates of n x round64(S) floats
    ws = lib.ppr_matrix_workspace(C.byref(large), 20000, 20000)
    assert ws >= 2 * 50000 * 20032 * 4
    assert lib.layout_workspace(20000) >= 8 * math.ceil(20000 / 16)
    assert lib.ppr_backward_workspace(C.byref(large), 1) > lib.ppr_backward_workspace(C.byref(large), 0)


def test_no_oracle_in_product_sources():
    pkg = os.path.join(ROOT, "paper_2112_14944_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
