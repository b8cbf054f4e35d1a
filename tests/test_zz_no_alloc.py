"""cmg_apply_noalloc (the operator product with its intermediates in the
library's fixed per-device scratch array) against cmg_apply, through the C
ABI: bit for bit, two calls in a row with the second on a smaller level (the
array keeps the first call's contents), in FP64 and FP32; a level beyond the
array's size is refused without a launch.

Every case prints its name first so that a failing GPU run can be located."""
import numpy as np
import pytest

import workloads as W

try:  # import at collection time: the first import on a fresh machine is slow
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

pytestmark = pytest.mark.gpu

SCRATCH = 32 << 20


@pytest.mark.parametrize("w", [W.ball_q2().with_levels(5), W.offcentre_disc(3, 4), W.ball_union(2, 3)],
                         ids=lambda w: w.name)
def test_noalloc_apply_equals_apply(w):
    import torch
    from paper_2508_11608_amd import CutmgError, Problem

    print(f"\n[case] {w.name} dim={w.dim} k={w.k} levels={w.n_levels} (allocation-free operator)", flush=True)
    P = Problem(w)
    try:
        L = w.n_levels - 1
        fits = [l for l in range(L + 1) if 2 * (P.counts(l)["nodes_per_dir"] ** w.dim) * 8 < SCRATCH // 2]
        big = [l for l in range(L + 1) if 2 * (P.counts(l)["nodes_per_dir"] ** w.dim) * 8 > SCRATCH]
        seq = sorted(fits)[-2:][::-1]  # the largest level that fits, then a smaller one
        assert len(seq) == 2
        for fp32 in (False, True):
            P.set_precision(fp32)
            for l in seq:
                x = torch.from_numpy(W.random_vector(P.ndofs(l), seed=700 + l)).cuda()
                y0 = P.apply(l, x)
                y1 = torch.full_like(y0, float("nan"))
                P.apply_noalloc(l, x, y1)
                torch.cuda.synchronize()
                print(f"  fp32={fp32} level {l}: max |diff| {float((y1 - y0).abs().max()):.3e}", flush=True)
                assert torch.equal(y0, y1), (fp32, l)
        P.set_precision(False)
        for l in big:
            x = torch.zeros(P.ndofs(l), dtype=torch.float64, device="cuda")
            y = torch.zeros_like(x)
            with pytest.raises(CutmgError) as e:
                P.apply_noalloc(l, x, y)
            assert e.value.status == -1 and "scratch" in str(e.value)
    finally:
        P.close()
        torch.cuda.synchronize()
