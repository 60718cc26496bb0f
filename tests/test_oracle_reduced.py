"""Pins for the oracle's reduced-precision emulation (oracle/reduced.py).

The BF16 Gram-factor apply (the multi-right-hand-side extension of the BRAS
inverse, eq. mhatinvbras_def, with M_K^-1 = L_K^-T L_K^-1 and the factor
Gt_K = L_K^-1 D_K^-1 stored in bfloat16) is the only checker of the BF16
matrix-core path, so each of its rounding steps is pinned here by values
that follow from the bfloat16 format alone (8 significand bits, round to
nearest, ties to even), worked out by hand in the comments:

    w = bf16(f32(x[pi_K]))          gathered input, rounded twice
    U = bf16(Gt_K w)                intermediate, one rounding
    Z = Gt_K^T U                    not rounded (float32 or wider on the device)
    y = P^T sum_K Z_K

Dropping or moving any one rounding changes at least one literal below.
"""
import numpy as np

from oracle import reduced


# ---------------------------------------------------------------------------
# round_bf16 against torch's float32 -> bfloat16 conversion (RNE)
# ---------------------------------------------------------------------------
def _torch_bf16(f32):
    import torch
    return torch.from_numpy(f32).to(torch.bfloat16).to(torch.float64).numpy()


def test_round_bf16_matches_torch_on_random_bit_patterns():
    rng = np.random.default_rng(0x2607)
    bits = rng.integers(0, 2**32, size=1_000_000, dtype=np.uint64).astype(np.uint32)
    # every exponent, both signs; NaN patterns (exponent all ones, mantissa
    # non-zero) are outside the domain of the apply and are replaced by +-inf
    expo = (bits >> 23) & 0xFF
    man = bits & 0x7FFFFF
    bits = np.where((expo == 0xFF) & (man != 0), bits & np.uint32(0xFF800000), bits)
    f = bits.view(np.float32)
    got = reduced.round_bf16(f.astype(np.float64))
    want = _torch_bf16(f)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def test_round_bf16_ties_subnormals_and_overflow():
    rng = np.random.default_rng(0x2608)
    hi = rng.integers(0, 2**16, size=200_000, dtype=np.uint64).astype(np.uint32)
    hi = hi[((hi >> 7) & 0xFF) != 0xFF]                       # finite high halves
    ties = (hi << 16) | np.uint32(0x8000)                     # exactly half-way
    sub = rng.integers(1, 2**23, size=200_000, dtype=np.uint64).astype(np.uint32)   # float32 subnormals
    sub = np.concatenate([sub, sub | np.uint32(0x80000000)])
    big = np.array([0x7F7FFFFF, 0x7F7F8000, 0x7F7F7FFF, 0xFF7FFFFF, 0x00000001, 0x80000001,
                    0x00008000, 0x00018000, 0x3F808000, 0x3F818000], dtype=np.uint32)
    for bits in (ties, sub, big):
        f = bits.view(np.float32)
        got = reduced.round_bf16(f.astype(np.float64))
        assert np.array_equal(got.view(np.uint64), _torch_bf16(f).view(np.uint64))
    # ties go to the even neighbour: 1 + 2^-8 -> 1, 1 + 3 * 2^-8 -> 1 + 2^-6
    assert reduced.round_bf16(np.array([1 + 2**-8, 1 + 3 * 2**-8])).tolist() == [1.0, 1 + 2**-6]
    # the largest finite float32 rounds past the largest bfloat16 to infinity
    assert np.isinf(reduced.round_bf16(np.array([np.float64(np.finfo(np.float32).max)]))[0])


def test_round_bf16_rounds_through_float32():
    """Reading of the storage conversion: float64 -> float32 -> bfloat16, each
    to nearest even.  1 + 2^-8 + 2^-30 lies just above the bfloat16 tie
    1 + 2^-8; float32 (24 bits) first rounds it onto the tie, which then goes
    to the even neighbour 1 (a direct float64 -> bfloat16 rounding gives
    1 + 2^-7)."""
    v = np.array([1 + 2**-8 + 2**-30, -(1 + 2**-8 + 2**-30)])
    assert reduced.round_bf16(v).tolist() == [1.0, -1.0]


# ---------------------------------------------------------------------------
# bras_apply_bf16_emulated on hand-worked one- and two-element cases
# ---------------------------------------------------------------------------
def _mass_from_gram(G):
    """M = (G^T G)^-1, so that Cholesky M = L L^T gives L^-1 = G (G lower
    triangular with a positive diagonal)."""
    return np.linalg.inv(G.T @ G)


def test_one_element_every_rounding_step():
    """One element, n_loc = 2, P = I, d = (1, 1), Gt = [[1, 0], [1, 1]]
    (bfloat16-exact), x = (1 + 3 * 2^-9, 1 + 2^-8 + 2^-30):
      w = (1 + 2^-7, 1)         x_0 above the half-way point 1 + 2^-8 rounds up;
                                x_1 reaches the tie 1 + 2^-8 in float32 and
                                goes to the even 1
      Gt w = (1 + 2^-7, 2 + 2^-7)
      U = (1 + 2^-7, 2)         2 + 2^-7 is the tie between 2 and 2 + 2^-6: even 2
      Z = Gt^T U = (U_0 + U_1, U_1) = (3 + 2^-7, 2)
    Without the rounding of w: U = (1 + 2^-7, 2 + 2^-6), Z_0 = 3 + 3 * 2^-7;
    without the rounding of U: Z = (3 + 2^-6, 2 + 2^-7); rounding Z as well
    gives Z_0 = 3 (3 + 2^-7 is a tie, even 3)."""
    G = np.array([[1.0, 0.0], [1.0, 1.0]])
    M = _mass_from_gram(G)[None]
    pi = np.array([[0, 1]])
    d = np.array([1, 1])
    x = np.array([1 + 3 * 2**-9, 1 + 2**-8 + 2**-30])
    y = reduced.bras_apply_bf16_emulated(pi, M, d, x)
    assert y.tolist() == [3.0078125, 2.0]
    # several columns: each column as in the one-column case (the second is -x)
    y2 = reduced.bras_apply_bf16_emulated(pi, M, d, np.stack([x, -x], axis=1))
    assert y2.tolist() == [[3.0078125, -3.0078125], [2.0, -2.0]]


def test_two_elements_factor_rounding_and_multiplicity():
    """Two elements sharing DOF 1 (d = (1, 2, 1)), L_0^-1 = [[1, 0], [1 + 3 * 2^-9, 1]],
    L_1^-1 = [[2, 0], [1/2, 3/2]], x = (1, 0, 1).
    Folded factors Gt_K = L_K^-1 D_K^-1:
      Gt_0 = [[1, 0], [1 + 3 * 2^-9, 1/2]] -> bf16 [[1, 0], [1 + 2^-7, 1/2]]
      Gt_1 = [[1, 0], [1/4, 3/2]]           (exact)
    Element 0: w = (1, 0), U = (1, 1 + 2^-7), Z = (1 + (1 + 2^-7)^2, (1 + 2^-7)/2)
             = (2 + 2^-6 + 2^-14, 1/2 + 2^-8)
    Element 1: w = (0, 1), U = (0, 3/2), Z = (3/8, 9/4)
    y = (2 + 2^-6 + 2^-14, 1/2 + 2^-8 + 3/8, 9/4).
    An unrounded factor gives y_0 = 1 + (1 + 3 * 2^-9)(1 + 2^-7); D applied on
    one side only, or not at all, changes y_1 and y_2."""
    G0 = np.array([[1.0, 0.0], [1 + 3 * 2**-9, 1.0]])
    G1 = np.array([[2.0, 0.0], [0.5, 1.5]])
    mats = np.stack([_mass_from_gram(G0), _mass_from_gram(G1)])
    pi = np.array([[0, 1], [1, 2]])
    d = np.array([1, 2, 1])
    y = reduced.bras_apply_bf16_emulated(pi, mats, d, np.array([1.0, 0.0, 1.0]))
    assert y.tolist() == [2 + 2**-6 + 2**-14, 0.5 + 2**-8 + 0.375, 2.25]


def test_gram_factors_fold_multiplicities():
    """Gt_K^T Gt_K = D_K^-1 M_K^-1 D_K^-1 (the folded BRAS block), to rounding."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((4, 5, 5))
    mats = A @ A.transpose(0, 2, 1) + 5 * np.eye(5)
    pi = np.array([[0, 1, 2, 3, 4], [2, 3, 4, 5, 6], [4, 5, 6, 7, 8], [0, 2, 4, 6, 8]])
    d = np.bincount(pi.ravel())
    G = reduced.gram_factors(mats, pi, d)
    Dinv = 1.0 / d[pi]
    want = Dinv[:, :, None] * np.linalg.inv(mats) * Dinv[:, None, :]
    assert np.allclose(G.transpose(0, 2, 1) @ G, want, rtol=1e-13, atol=0)
    assert np.all(np.triu(G, 1) == 0)
