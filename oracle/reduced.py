"""Emulation of reduced-precision storage (round to nearest, ties to even).

Used to predict the error of applying a BRAS operator whose element inverses
are stored in FP32 or BF16 (parity unpinned: these are extensions the paper
does not discuss; they state errors against the float64 operator).
"""
import numpy as np


def round_fp32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(a):
    """float64 -> float32 (RNE) -> bfloat16 (RNE on the top 16 bits) -> float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gram_factors(mats, pi, d):
    """G_K = L_K^-1 D_K^-1 with M_K = L_K L_K^T (so D_K^-1 M_K^-1 D_K^-1 = G_K^T G_K)."""
    L = np.linalg.cholesky(mats)
    Linv = np.linalg.inv(L)
    return Linv / np.asarray(d, dtype=float)[pi][:, None, :]


def bras_apply_bf16_emulated(pi, mats, d, x):
    """BRAS apply with the Gram factors stored in BF16 (float64 -> float32 ->
    bfloat16, round to nearest even), the gathered input rounded to BF16, the
    intermediate U = G_K w rounded to BF16 and exact accumulation otherwise:
        y = P^T sum_K G_K^T bf16(G_K bf16(x[pi_K]))
    (parity unpinned: an extension outside the paper; used to bound the error
    of the MFMA path, which accumulates in float32)."""
    G = round_bf16(gram_factors(mats, pi, d))
    x = np.asarray(x, dtype=float)
    w = round_bf16(x[pi])                                   # [E, nl(, R)]
    n = len(d)
    if x.ndim == 1:
        U = round_bf16(np.einsum("kij,kj->ki", G, w))
        Z = np.einsum("kji,kj->ki", G, U)
        return np.bincount(pi.ravel(), weights=Z.ravel(), minlength=n)
    U = round_bf16(np.einsum("kij,kjr->kir", G, w))
    Z = np.einsum("kji,kjr->kir", G, U)
    y = np.zeros((n, x.shape[1]))
    np.add.at(y, pi.ravel(), Z.reshape(-1, x.shape[1]))
    return y
