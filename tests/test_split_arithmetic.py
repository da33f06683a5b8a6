"""The arithmetic of the mixed-precision M2L products, emulated on the CPU.

The products run on the fp16 matrix instruction with FP32 accumulation, each
operand carried as two fp16 terms x1 = fp16(x), x2 = fp16(x - x1) after a
power-of-two scale that puts its largest entry in [2^14, 2^15), and three
cross products x1 y1 + x1 y2 + x2 y1 per product.  numpy's float16 rounds to
nearest even like the conversion instruction, so these checks pin the
scheme's error bounds (about 2^-22 per operand, a few 2^-22 per product term
relative to the sum of magnitudes) and show why the scales are needed.  They
check the scheme, not the kernel: the GPU parity tests compare the kernel's
products with the oracle."""

import numpy as np

TOP = 14  # scaled operands' largest entries lie in [2^TOP, 2^(TOP+1))


def split2(x):
    x = np.asarray(x, dtype=np.float32)
    h = x.astype(np.float16)
    lo = (x - h.astype(np.float32)).astype(np.float16)
    return h, lo


def scale_exponent(v):
    m = float(np.max(np.abs(v)))
    return TOP - int(np.floor(np.log2(m))) if m > 0 else 0


def split_dot(T, M):
    """sum_k T[:, k] M[k, :] by the three cross products of the two-term
    splits, products exact and sums in float64 (isolating the split error)."""
    t1, t2 = (a.astype(np.float64) for a in split2(T))
    m1, m2 = (a.astype(np.float64) for a in split2(M))
    return t2 @ m1 + t1 @ m2 + t1 @ m1


def test_two_term_split_holds_twenty_two_bits():
    rng = np.random.default_rng(1)
    # scaled values: the largest of a vector in [2^14, 2^15), the rest over the 40 binades below
    x = (2.0 ** rng.uniform(TOP - 40, TOP + 1, 100000) * rng.choice([-1, 1], 100000)).astype(np.float32)
    h, lo = split2(x)
    err = np.abs(x.astype(np.float64) - h.astype(np.float64) - lo.astype(np.float64))
    assert np.all(np.isfinite(h.astype(np.float64)))
    # 2^-22 relative, or half of fp16's subnormal spacing 2^-24 once the second
    # term is subnormal: at most 2^-39 of a largest entry of at least 2^14
    assert np.all(err <= np.maximum(2.0 ** -22 * np.abs(x), 2.0 ** -25) * 1.0001)
    big = np.abs(x) >= 2.0 ** -3  # both terms normal: the relative bound alone
    assert np.all(err[big] <= 2.0 ** -22 * np.abs(x[big]) * 1.0001)


def test_products_within_a_few_units_of_twenty_two_bits():
    rng = np.random.default_rng(2)
    P, K, n = 165, 168, 64
    T = rng.standard_normal((P, K)) * 2.0 ** rng.uniform(-12, 0, (P, K))  # entries over 12 binades
    M = rng.standard_normal((K, n)) * 2.0 ** rng.uniform(-12, 0, (K, 1))
    T = T.astype(np.float32)
    M = M.astype(np.float32)
    et, em = scale_exponent(T), np.array([scale_exponent(M[:, j]) for j in range(n)])
    Ts = (T * np.float32(2.0 ** et)).astype(np.float32)
    Ms = (M * (2.0 ** em).astype(np.float32)).astype(np.float32)
    got = split_dot(Ts, Ms) * 2.0 ** -et * 2.0 ** -em  # scales undone (exact powers of two)
    ref = T.astype(np.float64) @ M.astype(np.float64)
    mag = np.abs(T.astype(np.float64)) @ np.abs(M.astype(np.float64))
    assert np.max(np.abs(got - ref) / mag) < 4 * 2.0 ** -22


def test_without_scales_small_operands_lose_their_precision():
    rng = np.random.default_rng(3)
    T = (rng.standard_normal((16, 32)) * 1e-6).astype(np.float32)  # below fp16's normal range
    M = (rng.standard_normal((32, 8)) * 1e-3).astype(np.float32)
    ref = T.astype(np.float64) @ M.astype(np.float64)
    mag = np.abs(T.astype(np.float64)) @ np.abs(M.astype(np.float64))
    unscaled = np.max(np.abs(split_dot(T, M) - ref) / mag)
    et, em = scale_exponent(T), scale_exponent(M)
    scaled = split_dot(T * np.float32(2.0 ** et), M * np.float32(2.0 ** em)) * 2.0 ** -(et + em)
    assert unscaled > 1e-4
    assert np.max(np.abs(scaled - ref) / mag) < 4 * 2.0 ** -22


def test_large_operands_overflow_without_scales():
    x = np.float32(7.0e4)  # above fp16's largest finite value
    with np.errstate(over="ignore"):
        h, _ = split2(x)
    assert not np.isfinite(float(h))
    e = scale_exponent(np.array([x]))
    h, lo = split2(x * np.float32(2.0 ** e))
    assert np.isfinite(float(h)) and abs(float(h) + float(lo) - x * 2.0 ** e) <= 2.0 ** -22 * x * 2.0 ** e
