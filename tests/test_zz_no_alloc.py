"""The allocation-free Riccati entry point (dme_riccati_noalloc, temporaries in
the library's static device scratch) gives the result of dme_riccati on two
calls in a row, the second smaller than the first (the scratch keeps the first
call's contents), and refuses sizes beyond its scratch."""
import numpy as np
import pytest

from paper_1805_08990_amd import _binding as b
from tests.gpu_common import announce, rel_fro, to_np

pytestmark = pytest.mark.gpu


def _case(n, r, m, seed):
    rng = np.random.default_rng(seed)
    L = rng.standard_normal((n, r)) / np.sqrt(n)
    F = rng.standard_normal((r, r))
    D = F @ F.T
    B = rng.standard_normal((n, m))
    G = rng.standard_normal((m, m))
    R = G @ G.T + m * np.eye(m)
    return L, B, R, D


def test_noalloc_matches_riccati_twice(ctx):
    for n, r, m, seed in [(16384, 122, 4, 1), (1000, 37, 3, 2)]:
        announce("riccati_noalloc", n, r, m)
        L, B, R, D = _case(n, r, m, seed)
        ref = to_np(ctx.riccati(L, B, R, 1e-3, D))
        got = to_np(ctx.riccati_noalloc(L, B, R, 1e-3, D))
        err = rel_fro(got, ref)
        print(f"  rel diff to dme_riccati {err:.2e}", flush=True)
        assert err < 1e-14


def test_noalloc_refuses_oversized(ctx):
    announce("riccati_noalloc oversized")
    L, B, R, D = _case(16384, 512, 64, 3)  # 64-way split of L^T B: 16 MiB of partial sums
    with pytest.raises(b.DmeError) as e:
        ctx.riccati_noalloc(L, B, R, 1e-3, D)
    assert e.value.code == b.DME_EINVAL
