"""The narrow storage formats the BF16 / FP8 inputs are prepared in, checked
against their definitions (no GPU)."""
import numpy as np

import synth


def test_bf16_round_to_nearest_even():
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -7)
    x = np.array([one, one + ulp / 2, one + 3 * ulp / 2, one + ulp / 2 + 2 ** -20,
                  -2.5, 3.0e38], dtype=np.float32)
    v = synth.bf16_value(synth.bf16_bits(x))
    # a tie goes to the even significand, anything above the tie rounds up
    assert v[0] == 1.0 and v[1] == 1.0 and v[2] == 1.0 + 2 * float(ulp)
    assert v[3] == 1.0 + float(ulp)
    assert v[4] == -2.5
    # every BF16 value survives the round trip
    bits = np.arange(0, 0x7F80, 7, dtype=np.uint16)
    vals = synth.bf16_value(bits).astype(np.float32)
    assert np.array_equal(synth.bf16_bits(vals), bits)


def test_e4m3_table_matches_the_format():
    t = synth.E4M3_VALUES
    assert len(t) == 127 and t[0] == 0.0
    assert t[1] == 2.0 ** -9          # smallest subnormal
    assert t[7] == 7 * 2.0 ** -9      # largest subnormal
    assert t[8] == 2.0 ** -6          # smallest normal
    assert t[-1] == 448.0             # largest finite (0x7E); 0x7F is NaN
    assert np.all(np.diff(t) > 0)
    codes = np.arange(256, dtype=np.uint8)
    finite = (codes & 0x7F) != 0x7F
    v = synth.e4m3_value(codes)
    assert np.all(np.isnan(v[~finite]))
    rt = synth.e4m3_encode(v[finite])
    # +0 and -0 both encode to 0x00; everything else round-trips
    assert np.array_equal(rt[codes[finite] != 0x80], codes[finite][codes[finite] != 0x80])


def test_e4m3_rounding_and_saturation():
    enc = synth.e4m3_encode
    val = synth.e4m3_value
    assert val(enc(np.array([1.0625])))[0] == 1.0        # tie -> even code 0x38
    assert val(enc(np.array([1.0626])))[0] == 1.125
    assert val(enc(np.array([232.0])))[0] == 224.0        # tie -> even code 0x76
    assert val(enc(np.array([1e6, -1e6])))[0] == 448.0    # saturating
    assert val(enc(np.array([-1e6])))[0] == -448.0
    assert val(enc(np.array([2.0 ** -10])))[0] == 0.0     # tie with zero -> 0
    rng = np.random.default_rng(0)
    x = rng.standard_normal((64, 8)) * np.exp(rng.standard_normal(8))[None, :]
    s = synth.fp8_column_scales(x)
    q = synth.fp8_dequantize(synth.fp8_quantize(x, s), s)
    # 3-bit mantissa: relative error <= 2^-4 above the subnormal range
    big = np.abs(x) > 2.0 ** -6 * s[None, :]
    assert np.all(np.abs(q - x)[big] <= 2.0 ** -4 * np.abs(x)[big] + 1e-300)
    assert np.allclose(np.abs(x).max(axis=0), np.abs(q).max(axis=0))


def test_fast_orthogonal_mixing_is_orthogonal_and_planted():
    """The O(d^2) orthogonal factor equals its definition (scipy's orthonormal
    DCT-II of a signed permutation, then two reflections), is orthogonal, and
    the fast general instance keeps A v = lam B v exactly for the planted
    top-k (checked against the exact solver)."""
    from scipy.fft import dct

    import oracle
    from oracle import targets
    f = synth._FastOrth(np.random.default_rng(4), 29)
    P = np.zeros((29, 29))
    P[f.perm, np.arange(29)] = f.sign
    M = dct(P, type=2, norm="ortho", axis=0)
    for u in f.u:
        M -= 2.0 * np.outer(u, u @ M)
    Q = f.dense()
    assert np.abs(M - Q).max() < 1e-13
    assert np.abs(Q.T @ Q - np.eye(29)).max() < 1e-13
    g = synth.GeneralPlanted(48, k=8, seed=5, mixing="fast")
    A, B = targets.general_population_AB(g)
    lam, V = targets.general_planted_topk(g, 8)
    assert np.allclose(lam, np.geomspace(10.0, 0.1, 8))
    assert np.abs(A @ V - (B @ V) * lam[None, :]).max() < 1e-12
    lam2, V2 = oracle.gep_topk(A, B, 8)
    assert np.abs(lam2 - lam).max() < 1e-11
    assert oracle.subspace_error(V, V2, B) < 1e-12
    # the sample covariances approach A and B
    X, Y = g.sample(100000, np.random.default_rng(1))
    assert np.abs(X.T @ X / 1e5 + 1e-3 * np.eye(48) - B).max() < 0.05 * np.abs(B).max()
    assert np.abs(Y.T @ Y / 1e5 - A).max() < 0.05 * np.abs(A).max()
