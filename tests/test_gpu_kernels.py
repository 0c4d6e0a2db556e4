"""GPU parity of the individual kernels, called through the C-ABI:
Omega generation (bit-exact against the oracle's independent generator),
the sparse sketch (bit-exact on integer-valued A), the matrix-core products
(bit-exact on small integers, FP32 error bound otherwise) and the FP64
eigensolver."""
import math

import numpy as np
import pytest

from oracle import omega as om
from paper_2506_03859_amd import synth

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def fp():
    import torch  # noqa: F401
    from paper_2506_03859_amd import farpca as fpm
    fpm.load_library()
    return fpm


def dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


OMEGA_CASES = [
    ("sparse_sign", 0.0, 8, 64), ("sparse_sign", 0.0, 4, 50), ("sparse_sign", 0.0, 1, 20),
    ("sparse_sign", 0.05, 0, 64), ("std_bernoulli", 0.5, 0, 20), ("std_bernoulli", 0.003, 0, 64),
    ("sparse_gaussian", 0.05, 0, 64), ("bernoulli", 0.02, 0, 33), ("gaussian", 0.0, 0, 64),
    ("gaussian", 0.0, 0, 7),
]


@pytest.mark.parametrize("sketch,p,zeta,b", OMEGA_CASES)
def test_omega_bit_exact(fp, sketch, p, zeta, b):
    import torch
    n, seed = 1000, 1234
    prm = fp.make_params(500, n, tol=0.1, block=b, power=1, sketch=sketch, p=p, zeta=zeta, seed=seed)
    plan = fp.farpca_plan(prm)
    try:
        work, *_ = fp.alloc_outputs(plan)
        mask = torch.zeros(n, dtype=torch.int64, device="cuda")
        neg = torch.zeros(n, dtype=torch.int64, device="cuda")
        dense = torch.zeros((n, 64), dtype=torch.float32, device="cuda")
        for j in (0, 3):
            print(f"omega {sketch} p={p} zeta={zeta} b={b} block={j}", flush=True)
            fp.farpca_omega(plan, j, work, mask, neg, dense)
            gm = host(mask).view(np.uint64)
            gn = host(neg).view(np.uint64)
            gd = host(dense)
            ref = om.omega_dense(n, b, j, sketch, seed, p, zeta)
            bits = (np.uint64(1) << np.arange(b, dtype=np.uint64))
            gmask = (gm[:, None] & bits[None, :]) != 0
            gneg = (gn[:, None] & bits[None, :]) != 0
            if sketch == "gaussian":
                assert gmask.all()
            elif sketch == "std_bernoulli":
                assert np.array_equal(gmask, ref > 0)
            else:
                assert np.array_equal(gmask, ref != 0)
            assert np.array_equal(gneg, ref < 0)
            assert np.all(gd[:, b:] == 0)
            if sketch == "std_bernoulli":
                expect = gmask.astype(np.float64) - p       # Algorithm 2's unscaled B - p
            else:
                expect = ref
            if sketch in ("gaussian", "sparse_gaussian"):
                # Box-Muller through the device math library: FP64 rounding, then FP32
                assert np.allclose(gd[:, :b], expect, rtol=2 * U32, atol=1e-12)
            else:
                assert np.array_equal(gd[:, :b], expect.astype(np.float32))
    finally:
        plan.free()


SKETCH_CASES = [
    # (sketch, p, zeta, b, m, n)  scales chosen exact in binary for bit-exact sums
    ("sparse_sign", 0.0, 4, 64, 1000, 700),
    ("sparse_sign", 0.0, 16, 50, 3000, 1300),
    ("sparse_sign", 0.25, 0, 20, 257, 64),
    ("std_bernoulli", 0.5, 0, 64, 2000, 777),
    ("bernoulli", 0.125, 0, 33, 1500, 1000),
    ("sparse_sign", 0.0, 1, 8, 100, 12),
    # about 3600 list entries per chunk: several LDS pieces
    ("bernoulli", 0.875, 0, 64, 600, 300),
    # second row block of a workgroup mostly past m; three chunks (prefetch clamps)
    ("sparse_sign", 0.0, 4, 64, 130, 192),
    # many row tiles and K splits
    ("sparse_sign", 0.0, 16, 64, 12000, 4096),
]


# column-major A (the column gather): the same cases plus the paper's p near
# 1e-3 (a few entries per column of Omega, many columns without any) and
# row counts that are not multiples of 4 (no 16-byte loads).  p is a power of
# two, so that the scale 1 / sqrt(p) and z = p A 1 stay exact.
SKETCH_CASES_COL = SKETCH_CASES + [
    ("sparse_sign", 2.0 ** -10, 0, 64, 3000, 5000),
    ("std_bernoulli", 2.0 ** -9, 0, 50, 1001, 3333),
    ("bernoulli", 1e-3, 0, 64, 513, 9000),
    ("sparse_sign", 2.0 ** -8, 0, 64, 255, 700),
]


@pytest.mark.parametrize("layout,sketch,p,zeta,b,m,n",
                         [("row",) + c for c in SKETCH_CASES] + [("col",) + c for c in SKETCH_CASES_COL])
def test_sketch_bit_exact_integer_A(fp, layout, sketch, p, zeta, b, m, n):
    import torch
    a = synth.integer_matrix(m, n, seed=m + n, amax=1000)
    prm = fp.make_params(m, n, tol=0.1, block=b, power=1, sketch=sketch, p=p, zeta=zeta, seed=77,
                         layout=layout)
    plan = fp.farpca_plan(prm)
    try:
        work, *_ = fp.alloc_outputs(plan)
        S = torch.full((m, 64), float("nan"), dtype=torch.float32, device="cuda")
        # column-major: the buffer holds A^T row-major (lda = m)
        A = dev(a if layout == "row" else a.T, torch.float32)
        for j in (0, 5):
            print(f"sketch {layout} {sketch} p={p} zeta={zeta} b={b} m={m} n={n} block={j}", flush=True)
            fp.farpca_sketch(plan, A, j, work, S)
            got = host(S)
            if sketch == "std_bernoulli":
                bm = om.bernoulli_mask(n, b, j, 77, p).astype(np.float64)
                ref = a @ bm - (a @ (p * np.ones(n)))[:, None]     # Algorithm 2: A B_j - z
            else:
                ref = a @ om.omega_dense(n, b, j, sketch, 77, p, zeta)
            assert np.array_equal(got[:, :b], ref.astype(np.float32))
            assert np.all(got[:, b:] == 0)
    finally:
        plan.free()


@pytest.mark.parametrize("layout", ["row", "col"])
@pytest.mark.parametrize("sketch,p,zeta,b", [("sparse_gaussian", 0.05, 0, 64), ("sparse_sign", 0.0, 8, 64),
                                             ("gaussian", 0.0, 0, 50), ("std_bernoulli", 0.01, 0, 64),
                                             ("sparse_gaussian", 1e-3, 0, 64)])
def test_sketch_real_A(fp, sketch, p, zeta, b, layout):
    import torch
    m, n = 4000, 2500
    a = synth.gaussian_matrix(m, n, seed=5).astype(np.float32)
    prm = fp.make_params(m, n, tol=0.1, block=b, power=1, sketch=sketch, p=p, zeta=zeta, seed=91,
                         layout=layout)
    plan = fp.farpca_plan(prm)
    try:
        work, *_ = fp.alloc_outputs(plan)
        S = torch.zeros((m, 64), dtype=torch.float32, device="cuda")
        print(f"sketch real {layout} {sketch} p={p} zeta={zeta} b={b}", flush=True)
        fp.farpca_sketch(plan, dev(a if layout == "row" else a.T), 2, work, S)
        got = host(S)[:, :b].astype(np.float64)
        a64 = a.astype(np.float64)
        if sketch == "std_bernoulli":
            bm = om.bernoulli_mask(n, b, 2, 91, p).astype(np.float64)
            ref = a64 @ bm - (a64 @ (p * np.ones(n)))[:, None]
            absref = np.abs(a64) @ bm + np.abs(a64 @ (p * np.ones(n)))[:, None]
        else:
            o = om.omega_dense(n, b, 2, sketch, 91, p, zeta)
            ref = a64 @ o
            absref = np.abs(a64) @ np.abs(o)
        nnz_row = max(1, int(np.ceil(n * (zeta / b if zeta else (p if sketch != "gaussian" else 1)))))
        bound = 4 * U32 * math.sqrt(nnz_row) * absref + 4 * U32 * np.abs(ref)
        assert np.all(np.abs(got - ref) <= bound + 1e-30)
    finally:
        plan.free()


# small-M layout (one output tile per workgroup, K interleaved over its waves)
# and large-M layout (M >= 8192: 4 tiles per workgroup), aligned and ragged
GEMM_SHAPES = [(1000, 777, 50), (130, 3000, 64), (64, 64, 1), (5000, 20000, 64), (1, 300, 7),
               (257, 1500, 33), (3000, 64, 64), (9001, 3001, 64), (20000, 1000, 64),
               (8192, 4000, 50), (12000, 2048, 64), (8200, 40, 64),
               # short K (the basis products Q r, K = l <= 384) and just past it
               (20000, 320, 64), (7001, 130, 7), (5000, 384, 33), (300, 385, 64), (129, 3, 64),
               # tall A: short output (4000 or 2500 columns of A) over a long K
               (4000, 100000, 50), (2500, 30000, 64),
               # short K over many rows (the basis product Q r of a tall A)
               (131072, 200, 50)]


@pytest.mark.parametrize("M,K,N", GEMM_SHAPES)
@pytest.mark.parametrize("kind", ["nn", "tn"])
def test_gemm_integer_exact(fp, M, K, N, kind):
    import torch
    rng = np.random.default_rng(M * 7 + K)
    amax = 8 if K <= 20000 else 2
    if kind == "nn":
        a = rng.integers(-amax, amax + 1, size=(M, K)).astype(np.float32)
    else:
        a = rng.integers(-amax, amax + 1, size=(K, M)).astype(np.float32)
    x = rng.integers(-amax, amax + 1, size=(K, N)).astype(np.float32)
    C = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    part = torch.empty(fp.farpca_gemm_scratch_bytes(M) // 4 + 1, dtype=torch.float32, device="cuda")
    print(f"gemm {kind} M={M} K={K} N={N}", flush=True)
    # |entries| <= amax^2 K < 2^24: every partial sum is exact in FP32, and
    # the FP64 reference is exact in any order
    if kind == "nn":
        fp.farpca_gemm_nn(dev(a), dev(x), C, M, N, K, part)
        ref = a.astype(np.float64) @ x.astype(np.float64)
    else:
        fp.farpca_gemm_tn(dev(a), dev(x), C, M, N, K, part)
        ref = a.astype(np.float64).T @ x.astype(np.float64)
    assert np.array_equal(host(C), ref.astype(np.float32))


@pytest.mark.parametrize("M,K,N", [(4000, 20000, 50), (1000, 777, 50), (9001, 3001, 33), (8200, 40, 1)])
@pytest.mark.parametrize("kind", ["nn", "tn"])
def test_gemm_skinny_in_wide_buffer(fp, M, K, N, kind):
    # the library's own skinny operands are N < 64 columns of K x 64 buffers:
    # rows are read 64 wide and the columns >= N (here NaN) must not reach C
    import torch
    rng = np.random.default_rng(M + 3 * K + N)
    a = rng.integers(-4, 5, size=(M, K) if kind == "nn" else (K, M)).astype(np.float32)
    x = rng.integers(-4, 5, size=(K, N)).astype(np.float32)
    xb = torch.full((K, 64), float("nan"), dtype=torch.float32, device="cuda")
    xb[:, :N] = dev(x)
    C = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    part = torch.empty(fp.farpca_gemm_scratch_bytes(M) // 4 + 1, dtype=torch.float32, device="cuda")
    print(f"gemm {kind} M={M} K={K} N={N} ldx=64", flush=True)
    if kind == "nn":
        fp.farpca_gemm_nn(dev(a), xb, C, M, N, K, part, ldx=64)
        ref = a.astype(np.float64) @ x.astype(np.float64)
    else:
        fp.farpca_gemm_tn(dev(a), xb, C, M, N, K, part, ldy=64)
        ref = a.astype(np.float64).T @ x.astype(np.float64)
    assert np.array_equal(host(C), ref.astype(np.float32))


@pytest.mark.parametrize("M,K,N", [(2000, 15000, 64), (15000, 2000, 64), (333, 4000, 50), (4000, 100000, 50)])
@pytest.mark.parametrize("kind", ["nn", "tn"])
def test_gemm_float_error_bound(fp, M, K, N, kind):
    import torch
    rng = np.random.default_rng(3)
    a = rng.standard_normal((M, K) if kind == "nn" else (K, M)).astype(np.float32)
    x = rng.standard_normal((K, N)).astype(np.float32)
    C = torch.zeros((M, N), dtype=torch.float32, device="cuda")
    part = torch.empty(fp.farpca_gemm_scratch_bytes(M) // 4 + 1, dtype=torch.float32, device="cuda")
    print(f"gemm float {kind} M={M} K={K} N={N}", flush=True)
    a64, x64 = a.astype(np.float64), x.astype(np.float64)
    if kind == "nn":
        fp.farpca_gemm_nn(dev(a), dev(x), C, M, N, K, part)
        ref, absref = a64 @ x64, np.abs(a64) @ np.abs(x64)
    else:
        fp.farpca_gemm_tn(dev(a), dev(x), C, M, N, K, part)
        ref, absref = a64.T @ x64, np.abs(a64).T @ np.abs(x64)
    err = np.abs(host(C) - ref)
    # probabilistic bound of FP32 summation: a few u sqrt(K) |A||X| per entry
    assert np.all(err <= 6 * U32 * math.sqrt(K) * absref)


# ---------------------------------------------------------------- BF16 form
def bf16_dev(a32):
    """BF16 storage of an FP32 matrix on the GPU (int16 bit patterns) and the
    exact values it holds (float64)."""
    import torch
    bits = synth.bf16_bits(a32)
    return (torch.from_numpy(bits.view(np.int16)).cuda(),
            synth.bf16_value(bits).astype(np.float64))


def bf16_scratch(fp, M, K):
    import torch
    n = fp.farpca_gemm_bf16_scratch_bytes(M, K)
    buf = torch.empty(n + 256, dtype=torch.uint8, device="cuda")
    off = (-buf.data_ptr()) % 256
    return buf[off:off + n]


# NN vector loads need K % 8 == 0, TN vector loads M % 4 == 0: both paths occur
BF16_GEMM_SHAPES = [(1000, 777, 50), (130, 3000, 64), (64, 64, 1), (5000, 20000, 64), (1, 300, 7),
                    (257, 1500, 33), (3000, 64, 64), (9001, 3001, 64), (20000, 1000, 64),
                    (8200, 40, 64), (1024, 4096, 64), (700, 5, 3)]


def bf16_gemm(fp, kind, A, x, M, N, K):
    import torch
    C = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    scratch = bf16_scratch(fp, M, K)
    if kind == "nn":
        fp.farpca_gemm_bf16_nn(A, dev(x), C, M, N, K, scratch)
    else:
        fp.farpca_gemm_bf16_tn(A, dev(x), C, M, N, K, scratch)
    return host(C)


@pytest.mark.parametrize("M,K,N", BF16_GEMM_SHAPES)
@pytest.mark.parametrize("kind", ["nn", "tn"])
def test_gemm_bf16_integer_exact(fp, M, K, N, kind):
    rng = np.random.default_rng(M * 11 + K)
    # A in [-4, 4] (exact in BF16); X up to 2^11 in magnitude, so that the
    # split of X uses two BF16 terms; |sums| < 2^24: every order is exact
    xmax = min(2048, (2 ** 24 - 1) // (4 * max(K, 1)))
    shape = (M, K) if kind == "nn" else (K, M)
    a = rng.integers(-4, 5, size=shape).astype(np.float32)
    x = rng.integers(-xmax, xmax + 1, size=(K, N)).astype(np.float32)
    A, a64 = bf16_dev(a)
    assert np.array_equal(a64, a)
    print(f"gemm bf16 {kind} M={M} K={K} N={N}", flush=True)
    got = bf16_gemm(fp, kind, A, x, M, N, K)
    ref = (a64 @ x.astype(np.float64)) if kind == "nn" else (a64.T @ x.astype(np.float64))
    assert np.array_equal(got, ref.astype(np.float32))


@pytest.mark.parametrize("M,K,N", [(1000, 777, 50), (1003, 2430, 64), (337, 345, 64), (9001, 3001, 33)])
@pytest.mark.parametrize("kind", ["nn", "tn"])
def test_gemm_bf16_padded_rows(fp, M, K, N, kind):
    # rows padded to a multiple of 8 BF16 (the vector paths for any width):
    # the padding holds NaN patterns, which must reach no stored output
    import torch
    rng = np.random.default_rng(M * 5 + K)
    rows, cols = (M, K) if kind == "nn" else (K, M)
    a = rng.integers(-4, 5, size=(rows, cols)).astype(np.float32)
    xmax = min(2048, (2 ** 24 - 1) // (4 * K))          # |sums| < 2^24: exact in any order
    x = rng.integers(-xmax, xmax + 1, size=(K, N)).astype(np.float32)
    ld = (cols + 7) // 8 * 8
    bits = np.full((rows, ld), 0x7FC0, dtype=np.uint16)
    bits[:, :cols] = synth.bf16_bits(a)
    A = torch.from_numpy(bits.view(np.int16)).cuda()
    C = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    scratch = bf16_scratch(fp, M, K)
    print(f"gemm bf16 {kind} M={M} K={K} N={N} lda={ld}", flush=True)
    if kind == "nn":
        fp.farpca_gemm_bf16_nn(A, dev(x), C, M, N, K, scratch, lda=ld)
        ref = a.astype(np.float64) @ x.astype(np.float64)
    else:
        fp.farpca_gemm_bf16_tn(A, dev(x), C, M, N, K, scratch, lda=ld)
        ref = a.astype(np.float64).T @ x.astype(np.float64)
    assert np.array_equal(host(C), ref.astype(np.float32))


@pytest.mark.parametrize("M,K,N", [(1000, 2048, 64), (3000, 777, 50), (9001, 3001, 64)])
@pytest.mark.parametrize("kind", ["nn", "tn"])
def test_gemm_bf16_split_exact(fp, M, K, N, kind):
    # one nonzero +-2^e per output row of A's product, X with full 24-bit
    # significands: every output is a single product, exact only if the
    # three-term split of X is exact
    rng = np.random.default_rng(K)
    shape = (M, K) if kind == "nn" else (K, M)
    a = np.zeros(shape, dtype=np.float32)
    pick = rng.integers(0, K, size=M)
    val = rng.choice([-1.0, 1.0], size=M) * 2.0 ** rng.integers(-3, 4, size=M)
    if kind == "nn":
        a[np.arange(M), pick] = val
    else:
        a[pick, np.arange(M)] = val
    x = (rng.standard_normal((K, N)) * 2.0 ** rng.integers(-20, 20, size=(K, N))).astype(np.float32)
    A, a64 = bf16_dev(a)
    print(f"gemm bf16 split {kind} M={M} K={K} N={N}", flush=True)
    got = bf16_gemm(fp, kind, A, x, M, N, K)
    ref = (a64 @ x.astype(np.float64)) if kind == "nn" else (a64.T @ x.astype(np.float64))
    assert np.array_equal(got, ref.astype(np.float32))


@pytest.mark.parametrize("M,K,N", [(2000, 15000, 64), (15000, 2000, 64), (333, 4000, 50),
                                   (20000, 15000, 64)])
@pytest.mark.parametrize("kind", ["nn", "tn"])
def test_gemm_bf16_float_error_bound(fp, M, K, N, kind):
    rng = np.random.default_rng(5)
    a = rng.standard_normal((M, K) if kind == "nn" else (K, M)).astype(np.float32)
    x = rng.standard_normal((K, N)).astype(np.float32)
    A, a64 = bf16_dev(a)
    print(f"gemm bf16 float {kind} M={M} K={K} N={N}", flush=True)
    got = bf16_gemm(fp, kind, A, x, M, N, K)
    x64 = x.astype(np.float64)
    if kind == "nn":
        ref, absref = a64 @ x64, np.abs(a64) @ np.abs(x64)
    else:
        ref, absref = a64.T @ x64, np.abs(a64).T @ np.abs(x64)
    # the products are exact; only the FP32 accumulation rounds
    assert np.all(np.abs(got - ref) <= 6 * U32 * math.sqrt(K) * absref)


# ------------------------------------------- FP32 A on the BF16 matrix cores
def f32s_gemm(fp, kind, a, x, M, N, K, lda=None):
    import torch
    C = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    scratch = bf16_scratch(fp, M, K)
    A = a if isinstance(a, torch.Tensor) else dev(a)
    if kind == "nn":
        fp.farpca_gemm_f32s_nn(A, dev(x), C, M, N, K, scratch, lda=lda)
    else:
        fp.farpca_gemm_f32s_tn(A, dev(x), C, M, N, K, scratch, lda=lda)
    return host(C)


# NN vector loads need K % 4 == 0, TN vector loads M % 4 == 0: both paths occur
@pytest.mark.parametrize("M,K,N", BF16_GEMM_SHAPES)
@pytest.mark.parametrize("kind", ["nn", "tn"])
def test_gemm_f32s_integer_exact(fp, M, K, N, kind):
    # |a| <= 255 (one BF16 term), X up to 2^11 (two terms): every term product
    # that is formed is exact and the left-out ones are zero; |sums| < 2^24
    rng = np.random.default_rng(M * 13 + K)
    xmax = max(1, min(2048, (2 ** 24 - 1) // (255 * max(K, 1))))
    shape = (M, K) if kind == "nn" else (K, M)
    a = rng.integers(-255, 256, size=shape).astype(np.float32)
    x = rng.integers(-xmax, xmax + 1, size=(K, N)).astype(np.float32)
    print(f"gemm f32s {kind} M={M} K={K} N={N}", flush=True)
    got = f32s_gemm(fp, kind, a, x, M, N, K)
    a64, x64 = a.astype(np.float64), x.astype(np.float64)
    ref = (a64 @ x64) if kind == "nn" else (a64.T @ x64)
    assert np.array_equal(got, ref.astype(np.float32))


@pytest.mark.parametrize("M,K,N", [(1000, 777, 50), (1003, 2430, 64), (337, 345, 64), (9001, 3001, 33)])
@pytest.mark.parametrize("kind", ["nn", "tn"])
def test_gemm_f32s_padded_rows(fp, M, K, N, kind):
    # rows padded to a multiple of 4 floats (the vector paths for any width),
    # NaN in the padding: it must reach no stored output
    import torch
    rng = np.random.default_rng(M * 7 + K)
    rows, cols = (M, K) if kind == "nn" else (K, M)
    a = rng.integers(-255, 256, size=(rows, cols)).astype(np.float32)
    xmax = max(1, min(2048, (2 ** 24 - 1) // (255 * K)))
    x = rng.integers(-xmax, xmax + 1, size=(K, N)).astype(np.float32)
    ld = (cols + 3) // 4 * 4
    buf = np.full((rows, ld), np.nan, dtype=np.float32)
    buf[:, :cols] = a
    A = torch.from_numpy(buf).cuda()
    print(f"gemm f32s {kind} M={M} K={K} N={N} lda={ld}", flush=True)
    got = f32s_gemm(fp, kind, A, x, M, N, K, lda=ld)
    a64, x64 = a.astype(np.float64), x.astype(np.float64)
    ref = (a64 @ x64) if kind == "nn" else (a64.T @ x64)
    assert np.array_equal(got, ref.astype(np.float32))


@pytest.mark.parametrize("M,K,N", [(2000, 15000, 64), (15000, 2000, 64), (333, 4000, 50),
                                   (4000, 100000, 50), (20000, 15000, 64)])
@pytest.mark.parametrize("kind", ["nn", "tn"])
def test_gemm_f32s_float_error_bound(fp, M, K, N, kind):
    rng = np.random.default_rng(7)
    a = rng.standard_normal((M, K) if kind == "nn" else (K, M)).astype(np.float32)
    x = rng.standard_normal((K, N)).astype(np.float32)
    print(f"gemm f32s float {kind} M={M} K={K} N={N}", flush=True)
    got = f32s_gemm(fp, kind, a, x, M, N, K)
    a64, x64 = a.astype(np.float64), x.astype(np.float64)
    if kind == "nn":
        ref, absref = a64 @ x64, np.abs(a64) @ np.abs(x64)
    else:
        ref, absref = a64.T @ x64, np.abs(a64).T @ np.abs(x64)
    # the three term products left out are below 2^-23 |a x| per product
    # together; six FP32 accumulations per product
    err = np.abs(got - ref)
    assert np.all(err <= (6 * U32 * math.sqrt(6 * K) + 2.0 ** -23) * absref)
    # and the typical error is FP32's, not BF16's
    assert np.median(err / absref) < 4 * U32 * math.sqrt(K)


@pytest.mark.parametrize("kind", ["nn", "tn"])
def test_gemm_f32s_sum_of_squares_unbiased(fp, kind):
    # the indicator subtracts sum ||C_j||^2 from ||A||^2: a one-signed error of
    # the left-out term products (truncated splits: about 1e-7 of every
    # product) would shift the sum of squares by about 2e-7 relative; splits
    # rounded to nearest keep it at the level of random FP32 rounding
    M, K, N = 3000, 20000, 64
    rng = np.random.default_rng(11)
    a = rng.standard_normal((M, K) if kind == "nn" else (K, M)).astype(np.float32)
    x = rng.standard_normal((K, N)).astype(np.float32)
    print(f"gemm f32s sum of squares {kind}", flush=True)
    got = f32s_gemm(fp, kind, a, x, M, N, K).astype(np.float64)
    a64, x64 = a.astype(np.float64), x.astype(np.float64)
    ref = (a64 @ x64) if kind == "nn" else (a64.T @ x64)
    rel = abs(np.sum(got * got) - np.sum(ref * ref)) / np.sum(ref * ref)
    assert rel < 3e-8, rel


@pytest.mark.parametrize("sketch,p,zeta,b,m,n", SKETCH_CASES[:6] + SKETCH_CASES[-3:])
def test_sketch_bf16_bit_exact_integer_A(fp, sketch, p, zeta, b, m, n):
    import torch
    # integers up to 256 are exact in BF16
    a = synth.integer_matrix(m, n, seed=m + 3 * n, amax=256)
    A, a64 = bf16_dev(a.astype(np.float32))
    assert np.array_equal(a64, a)
    prm = fp.make_params(m, n, tol=0.1, block=b, power=1, sketch=sketch, p=p, zeta=zeta, seed=78,
                         a_dtype="bf16")
    plan = fp.farpca_plan(prm)
    try:
        work, *_ = fp.alloc_outputs(plan)
        S = torch.full((m, 64), float("nan"), dtype=torch.float32, device="cuda")
        for j in (0, 4):
            print(f"sketch bf16 {sketch} p={p} zeta={zeta} b={b} m={m} n={n} block={j}", flush=True)
            fp.farpca_sketch(plan, A, j, work, S)
            got = host(S)
            if sketch == "std_bernoulli":
                bm = om.bernoulli_mask(n, b, j, 78, p).astype(np.float64)
                ref = a @ bm - (a @ (p * np.ones(n)))[:, None]
            else:
                ref = a @ om.omega_dense(n, b, j, sketch, 78, p, zeta)
            assert np.array_equal(got[:, :b], ref.astype(np.float32))
            assert np.all(got[:, b:] == 0)
    finally:
        plan.free()


EIG_CASES = ([(l, 0.0) for l in (5, 20, 64, 65, 100, 250)] +
             [(l, 1e-8) for l in (20, 65, 250, 384, 1024, 2000)])


@pytest.mark.parametrize("l,rel", EIG_CASES)
@pytest.mark.parametrize("spectrum", ["uniform", "graded", "method", "clustered"])
def test_eig_vs_lapack(fp, l, rel, spectrum):
    # uniform: eigenvalues in [0.1, 10]; graded: 1e8 .. 1e-2 (logarithmic);
    # method: the squared singular values of the 20000 x 15000 workload,
    # exp(-2i/50) (1 down to 2e-7 at i = 384), in a K that is block diagonal up
    # to a coupling of 1e-3 between its 64-wide blocks (as the final Gram of the
    # method: each block of Q sees mostly its own singular directions);
    # clustered: eigenvalues repeated 8 times (exact ties).  rel = 0: the
    # solver's default relative test 1e-14; 1e-8: the value of the method's
    # final step.
    import torch
    rng = np.random.default_rng(l)
    q = synth.haar_columns(l, l, rng)
    if spectrum == "uniform":
        lam = rng.uniform(0.1, 10.0, l)
    elif spectrum == "graded":
        lam = np.logspace(8, -2, l)
    elif spectrum == "clustered":
        lam = np.repeat(np.linspace(1.0, 2.0, (l + 7) // 8), 8)[:l]
    else:
        lam = np.exp(-2.0 * np.arange(1, l + 1) / 50.0)
        blocks = [synth.haar_columns(min(64, l - i), min(64, l - i), rng) for i in range(0, l, 64)]
        qb = np.zeros((l, l))
        for i, blk in zip(range(0, l, 64), blocks):
            qb[i:i + blk.shape[0], i:i + blk.shape[0]] = blk
        e = 1e-3 * rng.standard_normal((l, l))
        q, _ = np.linalg.qr(qb + e)
    k = (q * lam) @ q.T
    k = (k + k.T) / 2
    W = torch.zeros(l, dtype=torch.float64, device="cuda")
    V = torch.zeros((l, l), dtype=torch.float64, device="cuda")
    work = torch.zeros(fp.farpca_eig_scratch_bytes(l) // 8 + 64, dtype=torch.float64, device="cuda")
    print(f"eig l={l} rel={rel} {spectrum}", flush=True)
    sweeps, converged = fp.farpca_eig(dev(k), W, V, work, rel=rel)
    w, v = host(W), host(V)
    ref = np.sort(np.linalg.eigvalsh(k))[::-1]
    lmax = np.abs(ref).max()
    eps = np.finfo(np.float64).eps
    # the solver's own contract on D = V^T K V (formed here in FP64): every
    # off-diagonal entry below rel sqrt(|d_pp d_qq|), below 4e-15 max |d_ii|,
    # or - once the sweeps stalled at the rounding level - below 1e-11
    # sqrt(|d_pp d_qq|) or 1e-12 max |d_ii|; the eigenvectors are orthonormal
    # and the eigenvalues carry the backward error of the rotations, a few
    # l u64 max|lambda| (LAPACK's order)
    d = v.T @ k @ v
    dd = np.abs(np.diag(d))
    off = np.abs(d - np.diag(np.diag(d)))
    relt = max(rel if rel > 0 else 1e-14, 1e-11)
    # rounding of the FP64 product V^T K V itself: gamma_2l |V|^T |K| |V|
    slack = 2 * l * eps * (np.abs(v).T @ np.abs(k) @ np.abs(v))
    bad = off > np.maximum(relt * np.sqrt(np.outer(dd, dd)), 1e-12 * dd.max()) + slack
    # the pairs that still fail the solver's own tests (no stall allowance, no slack)
    sq = np.sqrt(np.outer(dd, dd))
    fail = off > np.maximum((rel if rel > 0 else 1e-14) * sq, 4e-15 * dd.max())
    np.fill_diagonal(fail, False)
    worst = np.unravel_index(np.argmax(np.where(fail, off / np.maximum(sq, 1e-300), 0)), off.shape)
    print(f"  sweeps={sweeps} converged={converged} max|w-ref|/lmax={np.max(np.abs(w - ref)) / lmax:.2e} "
          f"orth={np.abs(v.T @ v - np.eye(l)).max():.2e} max off/lmax={off.max() / lmax:.2e} "
          f"violations={int(bad.sum())} failing pairs={int(fail.sum()) // 2} "
          f"worst ratio {off[worst] / max(sq[worst], 1e-300):.2e} (|d_pq|/lmax {off[worst] / lmax:.2e}, "
          f"d_pp {dd[worst[0]]:.2e}, d_qq {dd[worst[1]]:.2e})", flush=True)
    assert converged and 0 <= sweeps < 40
    assert np.all(np.diff(w) <= 0)
    assert not bad.any()
    # eigenvalues: Weyl's bound for the remaining off-diagonal part E of D
    # (|lambda_p - d_pp| <= ||E||_2) plus the rounding of the rotations
    weyl = np.linalg.norm(d - np.diag(np.diag(d)), 2)
    assert np.allclose(w, ref, rtol=0, atol=weyl + max(1e-13 * math.sqrt(l), 32 * l * eps) * lmax)
    assert np.abs(v.T @ v - np.eye(l)).max() < 1e-12 * l
