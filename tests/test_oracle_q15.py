"""Pins of the oracle's fixed-point (Q15 / Q30-sum) form of the proposed
inversion, against facts fixed outside it:

* diagonal inputs whose entries are powers of four have exact Q15 square
  roots and exactly representable inverses: the result must be exact;
* on MIMO-like inputs (and random Hermitian ones of every order up to 16) the
  dequantized inverse must agree with the FP64 oracle's inverse of the same
  quantized matrix to 4 kappa n 2^-15: every rounding is absolute (half a
  Q15 unit, two per entry and step), the inputs are scaled so that their
  largest entry is at least 1/2, so the backward error relative to ||A||_2 is
  at most 2 * 2 n 2^-16 / (1/2), amplified by the condition number;
* the output is Hermitian bit for bit; a clearly indefinite input fails at the
  pivot the FP64 factorisation names; a hand-worked 2 x 2 case saturates its
  off-diagonal factor entry and the saturation is counted.
"""
import numpy as np
import pytest

import oracle as O
from paper_1111_4144_amd import inputs as G
from tests.helpers import kappas


def _values(q):
    return (q[..., 0] + 1j * q[..., 1]).astype(np.complex128) / 2.0 ** 15


def test_q15_diagonal_powers_of_four_exact():
    n = 7
    q = np.zeros((1, n, n, 2), np.int16)
    pw = [13, 11, 9, 7, 5, 13, 3]
    for i, p in enumerate(pw):
        q[0, i, i, 0] = 1 << p                   # a_ii = 2^(p - 15), an even power of two
    x, xe, sat, info = O.inv_q15(q)
    assert info[0] == 0 and sat[0] == 0
    got = O.dequant_q15(x, xe)[0]
    want = np.diag([2.0 ** (15 - p) for p in pw])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n", [8, 16])
def test_q15_mimo_within_fixed_point_bound(n):
    a = G.mimo(n, 300, seed=77)
    q, _ = G.quantize_q15(a)
    x, xe, sat, info = O.inv_q15(q)
    assert (info == 0).all()
    at = _values(q)
    ref = np.stack([O.inv_prop(m)[0] for m in at])
    got = O.dequant_q15(x, xe)
    err = np.linalg.norm(got - ref, axis=(1, 2)) / np.linalg.norm(ref, axis=(1, 2))
    bound = 4 * kappas(at) * n * 2.0 ** -15
    assert (err <= bound).all(), (err / bound).max()


def test_q15_random_orders_within_bound():
    rng = np.random.default_rng(3)
    for n in range(1, 17):
        a = G.random_hpd(rng, 20, n, shift=0.3 * n)
        q, _ = G.quantize_q15(a)
        x, xe, sat, info = O.inv_q15(q)
        assert (info == 0).all()
        at = _values(q)
        ref = np.stack([O.inv_prop(m)[0] for m in at])
        got = O.dequant_q15(x, xe)
        err = np.linalg.norm(got - ref, axis=(1, 2)) / np.linalg.norm(ref, axis=(1, 2))
        assert (err <= 4 * kappas(at) * n * 2.0 ** -15).all(), n


def test_q15_output_hermitian_bitwise():
    q, _ = G.quantize_q15(G.mimo(12, 40, seed=5))
    x, _, _, _ = O.inv_q15(q)
    xt = np.swapaxes(x, 1, 2)
    assert np.array_equal(x[..., 0], xt[..., 0])
    assert np.array_equal(x[..., 1], -xt[..., 1])
    assert (np.diagonal(x[..., 1], axis1=1, axis2=2) == 0).all()


def test_q15_indefinite_fails_at_the_fp64_pivot():
    a = G.random_hpd(np.random.default_rng(9), 1, 6, shift=1.0)[0]
    a[3, 3] = -a[3, 3]                            # row 4's radicand is clearly negative
    q, _ = G.quantize_q15(a)
    _, info64 = O.chol(_values(q)[0])
    x, xe, sat, info = O.inv_q15(q)
    assert info64 == 4 and info[0] == 4
    assert (x == 0).all()


def test_q15_saturation_is_counted():
    # a = [[32766, 32766], [32766, 32767]] / 2^15 (real):
    # r_00 = floor(sqrt(32766 * 2^15)) = 32766 since 32767^2 = 32766 * 2^15 + 1;
    # r_01 = round(32766 * 2^15 / 32766) = 32768, one above the Q15 range;
    # r_11 = floor(sqrt(32767 * 2^15 - 32767^2)) = floor(sqrt(32767)) = 181
    q = np.zeros((1, 2, 2, 2), np.int16)
    q[0, :, :, 0] = [[32766, 32766], [32766, 32767]]
    x, xe, sat, info = O.inv_q15(q)
    assert info[0] == 0
    assert sat[0] >= 1
    # the inverse's (1, 1) entry is 1 / r_11^2 (in units of 2^-30 / 2^-30)
    got = O.dequant_q15(x, xe)[0]
    assert abs(got[1, 1].real - (2.0 ** 15 / 181) ** 2) <= 1e-3 * (2.0 ** 15 / 181) ** 2


def test_q15_negative_tie_rounds_away_from_zero():
    """A hand-worked 2 x 2 real case whose output rounding meets an exact
    negative half, so halves-away-from-zero (-12683) differs from half-up and
    from half-to-even (both -12682).  a = [[27752, 21162], [21162, 24209]]:
      r00 = floor(sqrt(27752 * 2^15 = 909377536)) = 30155   (30155^2 = 909324025)
      r01 = round(21162 * 2^15 / 30155) = round(22995 + 22191/30155) = 22996
      r11 = floor(sqrt(24209 * 2^15 - 22996^2 = 264464496)) = 16262
      F   = 2 floor(log2 16262) - ceil(log2 2) = 2 * 13 - 1 = 25
      t1  = round(2^55 / 16262) = 2215520662831          (remainder 6246)
      y11 = round(t1 / 16262) = 136239126                (136239125 rem 12081)
      y01 = round(-22996 * y11 / 30155) = -103895040     (|.| = 103895040 rem 10296)
      t0  = round(2^55 / 30155) = 1194786835316          (remainder 9988)
      y00 = round((t0 + 22996 * 103895040) / 30155) = 118851175
      shift s = 13: round(136239126 / 2^13) = 16631 <= 32767, s = 12 gives 33262
      x00 = round(118851175 / 8192) = 14508, x11 = 16631,
      x01 = round(-103895040 / 8192) = round(-12682.5) = -12683, xexp = s - F = -12."""
    q = np.zeros((1, 2, 2, 2), np.int16)
    q[0, :, :, 0] = [[27752, 21162], [21162, 24209]]
    x, xe, sat, info = O.inv_q15(q)
    assert info[0] == 0 and sat[0] == 0
    assert xe[0] == -12
    assert x[0, :, :, 0].tolist() == [[14508, -12683], [-12683, 16631]]
    assert (x[0, :, :, 1] == 0).all()


def test_q15_y_saturation_and_shift_search():
    """The 10 x 10 matrix A = R^T R with R = (I - N) / 4 (N: ones strictly above
    the diagonal) has an exact Q15 factor: a_ii = 2048 (i + 1), a_ij =
    2048 (i - 1) (i < j) in Q15 units, so every radicand is 2^26 and every
    division exact: r_ii = 8192, r_ij = -8192.  Then F = 2 * 13 - ceil(log2 10)
    = 22.  The true inverse 16 U^{-1} U^{-T} (U^{-1}_ij = 2^(j-i-1)) has
    x_00 = 16 (1 + (4^9 - 1)/3) = 1398112, and x_00 2^F = 5.9e12 is beyond the
    Y range 2^40 - 1, so Y saturates (counted) and the largest |y| is exactly
    2^40 - 1.  The smallest shift that fits: round((2^40 - 1) / 2^25) = 32768
    does not fit, s = 26 gives 16384.  So x_00 = 16384 and xexp = 26 - 22 = 4,
    while the last diagonal entry, y_99 = 2^(F + 30) / 8192^2 = 2^26 (x_99 = 16,
    exact), gives x_99 = round(2^26 / 2^26) = 1."""
    n = 10
    q = np.zeros((1, n, n, 2), np.int16)
    for i in range(n):
        for j in range(n):
            lo = min(i, j)
            q[0, i, j, 0] = 2048 * (i + 1) if i == j else 2048 * (lo - 1)
    x, xe, sat, info = O.inv_q15(q)
    assert info[0] == 0
    assert sat[0] >= 1
    assert xe[0] == 4
    assert x[0, 0, 0, 0] == 16384
    assert x[0, n - 1, n - 1, 0] == 1
    assert np.abs(x[0, ..., 0].astype(np.int64)).max() == 16384


# ---- the Section III methods in the same fixed-point format ------------------
VARIANTS = ["III.A", "III.B"]


@pytest.mark.parametrize("variant", VARIANTS)
def test_q15_compare_diagonal_powers_of_four_exact(variant):
    """Diagonal inputs with power-of-four entries: the factor, the forward
    solutions of III.A, M = R^{-1} of III.B and the inverse are all exact."""
    n = 7
    q = np.zeros((1, n, n, 2), np.int16)
    pw = [13, 11, 9, 7, 5, 13, 3]
    for i, p in enumerate(pw):
        q[0, i, i, 0] = 1 << p
    x, xe, sat, info = O.inv_q15(q, variant)
    assert info[0] == 0 and sat[0] == 0
    assert np.array_equal(O.dequant_q15(x, xe)[0], np.diag([2.0 ** (15 - p) for p in pw]))


@pytest.mark.parametrize("variant", VARIANTS)
def test_q15_compare_hand_worked_2x2(variant):
    """A = [[1/4, 1/8], [1/8, 5/16]] (mantissas 8192, 4096, 10240) = R^T R with
    R = [[1/2, 1/4], [0, 1/2]], exact in Q15 (16384, 8192, 16384; both radicands
    are 2^28).  min r_ii = 2^14, so F = 2 * 14 - 1 = 27 and G = 14 + 13 - 1 = 26.
      III.B: M = R^{-1} = [[2, -1], [0, 2]]: w00 = w11 = 2^41 / 2^14 = 2^27,
             w01 = -(8192 * 2^27) / 16384 = -2^26; X = M M^T with 2G - F = 25:
             y00 = (2^54 + 2^52) / 2^25 = 5 * 2^27, y01 = -2^53 / 2^25 = -2^28,
             y11 = 2^54 / 2^25 = 2^29.
      III.A: column 1: w1 = 2^27, y11 = 2^27 * 2^(27+15-26) / 2^14 = 2^29,
             y01 = -8192 * 2^29 / 16384 = -2^28; column 0: w0 = 2^27,
             y00 = (2^27 * 2^16 + 8192 * 2^28) / 16384 = 5 * 2^27.
    Output: 5 * 2^27 / 2^15 = 20480 fits and 2^14 would not, so the mantissas
    are (20480, -8192, 16384) with xexp = 15 - 27 = -12: X = [[5, -2], [-2, 4]]."""
    q = np.zeros((1, 2, 2, 2), np.int16)
    q[0, :, :, 0] = [[8192, 4096], [4096, 10240]]
    x, xe, sat, info = O.inv_q15(q, variant)
    assert info[0] == 0 and sat[0] == 0 and xe[0] == -12
    assert x[0, :, :, 0].tolist() == [[20480, -8192], [-8192, 16384]]
    assert (x[0, :, :, 1] == 0).all()


@pytest.mark.parametrize("variant", VARIANTS)
def test_q15_compare_within_fixed_point_bound(variant):
    """Every order 1..16 (random Hermitian) and the MIMO matrices: the same
    4 kappa n 2^-15 bound against the FP64 inverse of the quantized matrix as
    the proposed route (reading and derivation in the module docstring)."""
    rng = np.random.default_rng(13)
    cases = [G.random_hpd(rng, 20, n, shift=0.3 * n) for n in range(1, 17)]
    cases += [G.mimo(8, 200, seed=81), G.mimo(16, 200, seed=82)]
    for a in cases:
        n = a.shape[-1]
        q, _ = G.quantize_q15(a)
        x, xe, sat, info = O.inv_q15(q, variant)
        assert (info == 0).all()
        at = _values(q)
        ref = np.stack([O.inv_prop(m)[0] for m in at])
        got = O.dequant_q15(x, xe)
        err = np.linalg.norm(got - ref, axis=(1, 2)) / np.linalg.norm(ref, axis=(1, 2))
        assert (err <= 4 * kappas(at) * n * 2.0 ** -15).all(), (variant, n)


@pytest.mark.parametrize("variant", VARIANTS)
def test_q15_compare_hermitian_and_failing_pivot(variant):
    q, _ = G.quantize_q15(G.mimo(12, 40, seed=6))
    x, _, _, _ = O.inv_q15(q, variant)
    xt = np.swapaxes(x, 1, 2)
    assert np.array_equal(x[..., 0], xt[..., 0]) and np.array_equal(x[..., 1], -xt[..., 1])
    a = G.random_hpd(np.random.default_rng(9), 1, 6, shift=1.0)[0]
    a[3, 3] = -a[3, 3]
    q, _ = G.quantize_q15(a)
    x, xe, sat, info = O.inv_q15(q, variant)
    assert info[0] == 4 and (x == 0).all() and xe[0] == 0


def test_q15_routes_agree_to_one_unit():
    """All routes invert the same quantized factor with wide intermediates, so
    their int16 results agree to one unit of the output mantissa (same
    exponent) -- an invariant of the method, not of any one implementation."""
    for n in (4, 8, 16):
        q, _ = G.quantize_q15(G.mimo(n, 300, seed=90 + n))
        x0, e0, _, _ = O.inv_q15(q, "IV.A")
        for v in VARIANTS:
            x1, e1, _, _ = O.inv_q15(q, v)
            assert np.array_equal(e0, e1), (n, v)
            assert np.abs(x1.astype(np.int32) - x0.astype(np.int32)).max() <= 1, (n, v)
