"""bras_apply_noalloc (the BRAS apply for callers that cannot allocate: its
broken-vector workspace is a fixed device array) against bras_apply, bit for
bit: the same kernels in the same order.  Two calls in a row on one handle,
the second with fewer columns, then a call on a smaller mesh (the array keeps
the previous call's contents, which the element pass overwrites), and the
size limit, which is checked on the host before any device work."""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [
    # family, dim, degree, N, jitter, precision, max_rhs
    ("N1curl", 3, 2, 6, 0.2, "f32", 3),   # per-lane packed float32 inverses
    ("P", 3, 3, 6, 0.2, "f64", 3),        # scaled H1
    ("RT", 3, 3, 4, 0.2, "f64", 3),       # per-lane packed float64 (n_loc 36)
    ("N1curl", 3, 3, 4, 0.2, "f64", 2),   # n_loc 45: matrix cores
    ("RT", 3, 2, 4, 0.2, "bf16", 3),      # BF16 Gram factors
]


def ids(c):
    return "%s%d-%s" % (c[0], c[2], c[5])


def check_pair(gpu, R, seed):
    import torch
    from paper_2607_12138_amd import _lib as L
    X = torch.from_numpy(np.ascontiguousarray(workloads.rhs(gpu.n, R, seed))).cuda()
    y0 = gpu.vec(R)
    y1 = gpu.vec(R)
    y1.fill_(float("nan"))
    L.bras_apply(gpu.h, X, y0)
    L.bras_apply_noalloc(gpu.h, X, y1)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    assert torch.isfinite(y1).all()


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_noalloc_matches_bras_apply(case):
    from paper_2607_12138_amd.problem import MassProblem
    fam, dim, deg, N, jit, prec, R = case
    say("noalloc %s" % (case,))
    big = MassProblem(fam, dim, deg, N, jitter=jit, seed=3, prec=prec, max_rhs=R)
    check_pair(big, R, 11)          # all columns
    check_pair(big, 1, 12)          # a smaller input on the same handle
    small = MassProblem(fam, dim, deg, max(N - 2, 1), jitter=jit, seed=4, prec=prec, max_rhs=1)
    check_pair(small, 1, 13)        # a smaller mesh after a larger one
    small.close()
    big.close()


def test_noalloc_rejects_workspace_above_the_limit():
    import torch
    from paper_2607_12138_amd import _lib as L
    from paper_2607_12138_amd.problem import MassProblem
    # 16^3 N1curl2 in float64: 24576 elements x 20 copies x 8 bytes x 16 columns > 32 MiB
    gpu = MassProblem("N1curl", 3, 2, 16, prec="f64", max_rhs=16)
    R = 16
    assert 8 * gpu.E * gpu.n_loc * R > L.NOALLOC_SCRATCH_BYTES
    X = torch.zeros((gpu.n, R), dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(X)
    with pytest.raises(L.BrasError) as ei:
        L.bras_apply_noalloc(gpu.h, X, Y)
    assert ei.value.code == L.BRAS_EINVAL
    # one column fits and matches
    check_pair(gpu, 1, 14)
    gpu.close()
