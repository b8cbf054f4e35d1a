"""The Fourier load vector assembled on the device (cmg_rhs_fourier_device)
through the C ABI against the CPU oracle's load vector (and the library's host
assembly), on 2-D and 3-D domains, single shapes and unions, k = 1..3; the
result is the same bit for bit in every call and on every stream.

Every case prints its name first so that a failing GPU run can be located."""
import numpy as np
import pytest

import oracle_cache
import workloads as W

try:  # import at collection time: the first import on a fresh machine is slow
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

pytestmark = pytest.mark.gpu

CASES = [W.disc_q2(), W.offcentre_disc(3, 3), W.offcentre_disc(1, 4), W.offcentre_ball(2, 3),
         W.offcentre_ball(1, 3), W.ball_union(2, 3), W.disc_union(3, 3), W.offcentre_ball(3, 2)]


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_device_load_vector_matches_oracle(w):
    import torch
    from oracle import problem as OP
    from paper_2508_11608_amd import Problem

    print(f"\n[case] {w.name} dim={w.dim} k={w.k} levels={w.n_levels} (device load vector)", flush=True)
    levels, *_ = oracle_cache.build(w)
    P = Problem(w)
    try:
        for seed in (1000, 1013):
            modes = W.fourier_modes(w.dim, seed)
            bd = P.rhs_fourier_device(*modes).cpu().numpy()
            bo = OP.rhs_fourier(w, levels[-1], *modes)
            bh = P.rhs_fourier(*modes)
            scale = np.abs(bo).max()
            d_or, d_host = np.abs(bd - bo).max() / scale, np.abs(bd - bh).max() / scale
            print(f"  seed {seed}: vs oracle {d_or:.2e}, vs host assembly {d_host:.2e}", flush=True)
            assert d_or < 1e-12 and d_host < 1e-13
    finally:
        P.close()
        torch.cuda.synchronize()


def test_device_load_vector_is_deterministic():
    import torch
    from paper_2508_11608_amd import Problem

    w = W.ball_union(2, 3)
    print(f"\n[case] {w.name} (device load vector, repeat and other stream)", flush=True)
    P = Problem(w)
    try:
        modes = W.fourier_modes(3, 1001)
        b0 = P.rhs_fourier_device(*modes)
        b1 = P.rhs_fourier_device(*modes)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            b2 = P.rhs_fourier_device(*modes)
        s.synchronize()
        assert torch.equal(b0, b1) and torch.equal(b0, b2)
    finally:
        P.close()
        torch.cuda.synchronize()
