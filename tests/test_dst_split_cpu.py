"""The arithmetic of the FP32 plans' matrix-core DST-I, emulated in NumPy (CPU, no GPU).

The Poisson passes of FP32 plans form each DST-I (App. C.2, eq. DST_delta) as a product with
the sine matrix in FP16 with FP32 accumulation: every FP32 operand v is scaled by a power of
two per block (the block maximum lands in [2^12, 2^13)) and split into hi = fp16(v) and
lo = fp16(v - hi); the sine matrix is split the same way, and hi*hi + hi*lo + lo*hi are
accumulated in FP32.  These tests check, on the CPU, that this recipe reaches FP32-level
accuracy (the GPU parity tests then hold the kernels to the oracle), and that the pieces
it rests on hold: v - hi is exact in FP32, the split keeps 22 significant bits, and the
dropped lo*lo term is what separates it from the exact product.
"""
import numpy as np


def pow2_scale(m):
    """2^(13 - e) for m = f 2^e, f in [0.5, 1); 1 for m = 0."""
    if m <= 0:
        return np.float32(1.0)
    e = int(np.frexp(np.float32(m))[1])
    e = min(max(e, -100), 100)
    return np.float32(np.ldexp(1.0, 13 - e))


def split(v):
    v = np.asarray(v, dtype=np.float32)
    hi = v.astype(np.float16)
    lo = (v - hi.astype(np.float32)).astype(np.float16)
    return hi, lo


def sine_matrix(M):
    j = np.arange(1, M)
    return np.sin(np.pi * np.outer(j, j) / M)


def split_product(S, Y):
    """S @ Y the way the kernels form it: FP16 halves, products exact in FP32, FP32 sums
    (the sums are taken term by term in FP32; the matrix unit's internal order differs
    only by FP32 rounding)."""
    s = pow2_scale(np.abs(Y).max())
    yh, yl = split(Y * s)
    sh, sl = split(S.astype(np.float32))
    f = lambda a, b: a.astype(np.float32) @ b.astype(np.float32)
    out = f(sh, yh) + f(sh, yl) + f(sl, yh)
    return out.astype(np.float32) / s


def test_split_is_exact_in_fp32_and_keeps_22_bits():
    rng = np.random.default_rng(1)
    v = (rng.standard_normal(100000) * 2.0 ** rng.integers(-8, 13, 100000)).astype(np.float32)
    v = v[np.abs(v) < 2.0 ** 13]
    hi, lo = split(v)
    r = v - hi.astype(np.float32)
    # the remainder is exact in FP32: hi + r reproduces v bit for bit
    assert np.array_equal(hi.astype(np.float32) + r, v)
    # hi + lo carries 22 significant bits where both halves are normal FP16 numbers
    normal = np.abs(v) >= 2.0 ** -2
    err = np.abs(hi.astype(np.float64) + lo.astype(np.float64) - v.astype(np.float64))
    assert (err[normal] <= 2.0 ** -23 * np.abs(v[normal]) * 1.0001).all()


def test_split_dst_reaches_fp32_accuracy():
    rng = np.random.default_rng(2)
    for M in (16, 48, 64, 96, 128):
        S = sine_matrix(M)
        # a density-contrast-like plane: mostly O(1), a few large nodes
        Y = rng.standard_normal((M - 1, M - 1)).astype(np.float32)
        Y[rng.integers(0, M - 1, 5), rng.integers(0, M - 1, 5)] = 900.0
        exact = S @ Y.astype(np.float64)
        got = split_product(S, Y)
        rel = np.abs(got - exact).max() / np.abs(exact).max()
        # the same product with FP32 operands and FP32 sums
        f32 = S.astype(np.float32) @ Y
        rel32 = np.abs(f32 - exact).max() / np.abs(exact).max()
        # as accurate as FP32 arithmetic itself (within a factor 2), below 1e-6 of the maximum
        assert rel < 2 * rel32 + 1e-8 and rel < 1e-6, (M, rel, rel32)


def test_dropping_the_lo_lo_term_is_what_is_left():
    rng = np.random.default_rng(3)
    M = 64
    S = sine_matrix(M)
    Y = rng.standard_normal((M - 1, 8)).astype(np.float32)
    s = pow2_scale(np.abs(Y).max())
    yh, yl = split(Y * s)
    sh, sl = split(S.astype(np.float32))
    d = lambda a: a.astype(np.float64)
    three = d(sh) @ d(yh) + d(sh) @ d(yl) + d(sl) @ d(yh)
    four = three + d(sl) @ d(yl)
    exact = S @ (d(Y) * float(s))
    # with all four products (in FP64) only the representation error of the halves remains
    assert np.abs(four - exact).max() <= 2.0 ** -21 * np.abs(exact).max()
    # the fourth product is below 2^-22 of the result's scale
    assert np.abs(d(sl) @ d(yl)).max() <= 2.0 ** -22 * np.abs(exact).max()


def test_power_of_two_scaling_is_exact_and_bounded():
    for m in (1e-30, 3.7e-5, 1.0, 2047.9, 4096.0, 1.3e7):
        s = pow2_scale(m)
        assert 2.0 ** 12 <= m * float(s) < 2.0 ** 13 + 1e-9
        # a power of two: scaling and unscaling are exact
        assert np.frexp(float(s))[0] == 0.5
    assert pow2_scale(0.0) == 1.0
