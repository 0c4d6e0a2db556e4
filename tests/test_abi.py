"""Host-only checks of the C-ABI (no GPU needed): the library loads, exports
every function include/farpca.h declares, the binding's struct layouts match
what a C compiler makes of the header, and farpca_plan validates parameters
and applies the paper's default rules (Sections 5.1, 5.2, 5.4)."""
import ctypes
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "farpca.h")


@pytest.fixture(scope="module")
def fp():
    from paper_2506_03859_amd import farpca as fpm
    if not os.path.exists(fpm.LIB_PATH):
        from paper_2506_03859_amd import build
        build.build()
    fpm.load_library()
    return fpm


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(farpca_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(fp):
    lib = fp.load_library()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(fp.EXPORTED) == names


def test_struct_layout_matches_c(fp, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "farpca.h"\n'
        "int main(void){\n"
        'printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(farpca_params), offsetof(farpca_params, tol),'
        " offsetof(farpca_params, max_blocks), offsetof(farpca_params, seed), sizeof(farpca_info),"
        " offsetof(farpca_info, eig_sweeps));\n"
        'printf("%zu %zu %zu %zu %zu\\n", sizeof(farpca_result), offsetof(farpca_result, info),'
        " offsetof(farpca_result, t_done), offsetof(farpca_result, dV), offsetof(farpca_result, n));\n"
        "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    got = [int(x) for x in out]
    P, I, R = fp.FarpcaParams, fp.FarpcaInfo, fp.FarpcaResult
    assert got == [ctypes.sizeof(P), P.tol.offset, P.max_blocks.offset, P.seed.offset,
                   ctypes.sizeof(I), I.eig_sweeps.offset,
                   ctypes.sizeof(R), R.info.offset, R.t_done.offset, R.dV.offset, R.n.offset]


def plan_or_rc(fp, **kw):
    m = kw.pop("m", 2000)
    n = kw.pop("n", 1500)
    prm = fp.make_params(m, n, kw.pop("lda", None), **kw)
    lib = fp.load_library()
    h = ctypes.c_void_p()
    lmax = ctypes.c_int64()
    ws = ctypes.c_size_t()
    rc = lib.farpca_plan(ctypes.byref(prm), ctypes.byref(h), ctypes.byref(lmax), ctypes.byref(ws))
    if rc == 0:
        lib.farpca_free(h)
    return rc, lmax.value, ws.value


@pytest.mark.parametrize("kw", [
    dict(tol=0.0), dict(tol=-1.0), dict(tol=float("nan")), dict(tol=0.1, block=65),
    dict(tol=0.1, block=-1), dict(tol=0.1, power=-1), dict(tol=0.1, sketch_zeta=9, block=8),
    dict(tol=0.1, p=1.0), dict(tol=0.1, p=-0.5), dict(tol=0.1, lda=100), dict(tol=0.1, m=0),
    dict(tol=0.1, rank=-3), dict(tol=0.1, sketch="bernoulli", p=1e-12),
])
def test_plan_rejects_invalid(fp, kw):
    kw = dict(kw)
    if "sketch_zeta" in kw:
        kw["zeta"] = kw.pop("sketch_zeta")
    kw.setdefault("sketch", "sparse_sign")
    rc, _, _ = plan_or_rc(fp, **kw)
    assert rc == -1


def test_column_major_layout_rules(fp):
    # column-major A: lda >= m (not n), FP32 only, layout codes 0 and 1 only
    ok, _, ws_col = plan_or_rc(fp, m=2000, n=1500, tol=0.1, layout="col")
    assert ok == 0
    assert plan_or_rc(fp, m=2000, n=1500, lda=1500, tol=0.1, layout="col")[0] == -1
    assert plan_or_rc(fp, m=1500, n=2000, lda=1500, tol=0.1, layout="col")[0] == 0
    assert plan_or_rc(fp, m=2000, n=1500, tol=0.1, layout="col", a_dtype="bf16")[0] == -1
    prm = fp.make_params(2000, 1500, tol=0.1, sketch="sparse_sign")
    prm.a_layout = 2
    lib = fp.load_library()
    h, lmax, ws = ctypes.c_void_p(), ctypes.c_int64(), ctypes.c_size_t()
    assert lib.farpca_plan(ctypes.byref(prm), ctypes.byref(h), ctypes.byref(lmax), ctypes.byref(ws)) == -1
    # the per-column lists (b x n entries of 8 bytes) come on top of the row-major
    # workspace, less the transposed skinny operand of its split A^T Y passes
    # (max(m, n) rounded up to 192, times 64 floats)
    _, _, ws_row = plan_or_rc(fp, m=2000, n=1500, tol=0.1)
    pack = -(-2000 // 192) * 192 * 64 * 4
    assert ws_col >= ws_row - pack + 20 * 1500 * 8


def test_step_entry_points_need_begin(fp):
    # host-side checks only (no device work): step and finish before begin
    plan = fp.farpca_plan(fp.make_params(2000, 1500, tol=0.1, sketch="sparse_sign"))
    lib = fp.load_library()
    try:
        assert lib.farpca_step(plan.handle, None) == -1
        assert lib.farpca_finish(plan.handle, ctypes.c_void_p(16), ctypes.c_void_p(16),
                                 ctypes.c_void_p(16), None, None) == -1
        assert lib.farpca_begin(plan.handle, None, None, 0, None, None) == -1
        assert lib.farpca_step(None, None) == -1
        # the two halves of a step: nothing to enqueue or poll before begin
        assert lib.farpca_step_async(plan.handle, None) == -1
        assert lib.farpca_step_poll(plan.handle, 0) == -1
        assert lib.farpca_step_async(None, None) == -1
        assert lib.farpca_step_poll(None, 1) == -1
    finally:
        plan.free()


def test_default_rules(fp):
    # b = min(max(20, floor(min(m,n)/100)), 50); cap ceil(min(m,n)/(2b)) blocks
    for m, n in [(2000, 1500), (20000, 15000), (9504, 4752), (300, 500), (5000, 5000)]:
        rc, lmax, ws = plan_or_rc(fp, m=m, n=n, tol=1e-3, sketch="sparse_sign", zeta=4)
        assert rc == 0
        mn = min(m, n)
        b = min(max(20, mn // 100), 50)
        blocks = min(math.ceil(mn / (2 * b)), mn // b)
        assert lmax == blocks * b
        assert ws > 0
    # fixed rank: ceil(k / b) blocks
    rc, lmax, _ = plan_or_rc(fp, m=200000, n=4000, rank=200, block=50, sketch="bernoulli")
    assert rc == 0 and lmax == 200
    rc, lmax, _ = plan_or_rc(fp, m=2000, n=1500, rank=45, block=20, sketch="gaussian")
    assert rc == 0 and lmax == 60
    # explicit cap, and l never exceeds min(m, n)
    rc, lmax, _ = plan_or_rc(fp, m=100, n=64, tol=1e-9, block=20, max_blocks=50, sketch="gaussian")
    assert rc == 0 and lmax == 60


def test_status_strings(fp):
    lib = fp.load_library()
    for code in (0, 1, -1, -2, -3, -4):
        assert lib.farpca_status_str(code)


def test_request_footprint(fp):
    # workspace + U (m x l_max FP32) + S (l_max FP64) + V (n x l_max FP32), each
    # rounded up to 256 bytes; 0 for invalid parameters
    def up(x):
        return (x + 255) // 256 * 256
    for m, n, b, dt in ((1000, 700, 32, "f32"), (333, 2000, 7, "bf16"), (8000, 4000, 50, "f32")):
        prm = fp.make_params(m, n, tol=1e-3, block=b, power=1, a_dtype=dt)
        rc, lmax, ws = plan_or_rc(fp, m=m, n=n, tol=1e-3, block=b, power=1, a_dtype=dt)
        assert rc == 0
        assert fp.farpca_request_footprint(prm) == up(ws) + up(m * lmax * 4) + up(lmax * 8) + up(n * lmax * 4)
    assert fp.farpca_request_footprint(fp.make_params(10, 10, tol=0.0)) == 0
