"""mehdg_dot_noalloc (no context, no device allocation) against mehdg_dot on
the same vectors: identical results (same kernel, same summation order), on
two calls in a row, the second smaller than the first, so that the shared
per-GPU partial-sum array is reused with fewer active elements."""
import numpy as np
import pytest

from paper_2507_22195_amd import workloads as W
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu


def test_dot_noalloc_matches_dot_on_two_calls():
    import torch
    from paper_2507_22195_amd import mehdg
    w = W.workload(1)
    ctx = mehdg.Context(w.p, w.mesh.h, w.params)
    g = torch.Generator(device="cuda").manual_seed(1234)
    try:
        for n in (3_000_017, 1_001):
            banner(f"dot_noalloc: n = {n}")
            x = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
            y = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
            got = mehdg.dot_noalloc(x, y)
            ref = ctx.dot(x, y)
            exact = float(torch.dot(x.cpu(), y.cpu()))
            banner(f"  noalloc {got!r} dot {ref!r} |diff| {abs(got - ref):.1e}")
            assert got == ref
            assert abs(got - exact) <= 1e-12 * float(x.norm() * y.norm())
        assert mehdg.dot_noalloc(x[:0], y[:0]) == 0.0
    finally:
        ctx.close()
