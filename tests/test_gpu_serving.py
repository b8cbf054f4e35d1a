"""The solve server: every result is the same alone and in the mix (bitwise),
and equals a direct solve of the same problem through cmg_solve."""
import time

import numpy as np
import pytest

import workloads as W

try:
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

pytestmark = pytest.mark.gpu


def _mix():
    """Eight geometries / degrees / precisions, plus six more requests of one
    geometry with their own right-hand sides, so that batches form."""
    ws = [W.offcentre_disc(2, 4), W.offcentre_ball(2, 3), W.ellipse(3, 3), W.offcentre_disc(1, 4),
          W.offcentre_ball(1, 3), W.disc_union(2, 3)]
    out = []
    for i, w in enumerate(ws + ws[:2]):
        out.append((w, W.fourier_modes(w.dim, 1000 + i), bool(i % 2)))
    for i in range(6):
        out.append((ws[0], W.fourier_modes(2, 2000 + i), True))
    return out


def _run(server, reqs):
    from paper_2508_11608_amd import footprint

    tickets = [server.submit(w, fourier=f, fp32=fp32) for w, f, fp32 in reqs]
    sizes = {}
    results = []
    for (w, f, fp32), t in zip(reqs, tickets):
        if w.name not in sizes:
            sizes[w.name] = footprint(w)[1]
        while True:
            r = server.poll(t, sizes[w.name])
            if r is not None:
                break
            time.sleep(0.001)
        results.append(r)
    return results


def test_results_alone_equal_results_in_the_mix():
    """Every request of a mix (three slots, batches of one geometry) gives the
    same iterations and the same solution, bit for bit, as the same request
    alone on a fresh server."""
    from paper_2508_11608_amd import Server

    reqs = _mix()
    print(f"\n[case] serving mix of {len(reqs)} requests", flush=True)
    mix = Server(8 << 30, 3)
    in_mix = _run(mix, reqs)
    mix.close()
    print("  batch sizes in the mix:", [r["batch"] for r, _ in in_mix], flush=True)
    for i, ((w, f, fp32), (res, x)) in enumerate(zip(reqs, in_mix)):
        print(f"  mix request {i} {w.name} fp32={fp32}: status {res['status']}, {res['iterations']} its, "
              f"rel residual {res['rel_residual']:.2e}, batch {res['batch']}, solution {'yes' if x is not None else 'no'}",
              flush=True)
    assert max(r["batch"] for r, _ in in_mix) > 1
    for i, ((w, f, fp32), (res, x)) in enumerate(zip(reqs, in_mix)):
        alone_srv = Server(8 << 30, 1)
        (res1, x1), = _run(alone_srv, [(w, f, fp32)])
        alone_srv.close()
        print(f"  alone request {i} {w.name}: status {res1['status']}, {res1['iterations']} its", flush=True)
        assert res1["batch"] == 1
        assert res["status"] == 0 and res1["status"] == 0, (w.name, fp32, res["status"], res1["status"])
        assert res["rel_residual"] <= 1e-8
        assert res["iterations"] == res1["iterations"]
        assert np.array_equal(x, x1), w.name


def test_server_result_matches_direct_solve():
    """A served request (its load vector assembled on the device, the
    multi-column PCG of its batch) equals the one-column cmg_solve_multi on the
    device load vector bit for bit, in FP64 and FP32, and the single-column
    cmg_solve on the host-assembled load vector to the solver's tolerance."""
    from paper_2508_11608_amd import Problem, Server

    w = W.offcentre_ball(2, 3)
    f = W.fourier_modes(3, 7)
    srv = Server(4 << 30, 2)
    (res, x), (res32, x32) = _run(srv, [(w, f, False), (w, f, True)])
    srv.close()
    P = Problem(w)
    bd = P.rhs_fourier_device(*f)
    for fp32, r, xs in ((False, res, x), (True, res32, x32)):
        P.set_precision(fp32)
        xm, infos = P.solve_multi(bd[None, :].contiguous(), rtol=1e-8)
        assert r["iterations"] == infos[0]["iterations"], fp32
        assert np.array_equal(xs, xm[0].cpu().numpy()), fp32
    P.set_precision(False)
    xd, info = P.solve(torch.from_numpy(P.rhs_fourier(*f)).cuda(), rtol=1e-8)
    d = np.abs(x - xd.cpu().numpy()).max() / np.abs(xd.cpu().numpy()).max()
    print(f"\n  served FP64 vs direct solve: {res['iterations']} / {info['iterations']} its, max diff {d:.2e}")
    assert abs(res["iterations"] - info["iterations"]) <= 1 and d < 1e-7


def test_admission_under_a_small_budget():
    """A budget that holds one hierarchy at a time still finishes every request
    (eviction of idle hierarchies, waiting for memory)."""
    from paper_2508_11608_amd import Server, footprint

    ws = [W.offcentre_disc(2, 4), W.ellipse(2, 4), W.offcentre_disc(3, 3)]
    need = 0
    for w in ws:
        fb, n = footprint(w, fp32=True, multi=True)  # FP32 copies + multi-column buffers
        need = max(need, fb + 2 * 8 * 8 * n)          # + the batch's b and x columns
    srv = Server(int(need * 1.5), 2)
    reqs = [(w, W.fourier_modes(2, 50 + i), True) for i, w in enumerate(ws * 2)]
    res = _run(srv, reqs)
    srv.close()
    assert all(r["status"] == 0 and r["rel_residual"] <= 1e-8 for r, _ in res)


def test_request_larger_than_the_budget_is_refused_before_set_up():
    """Admission by footprint happens before the set-up: a request that cannot
    fit into the whole budget finishes with CMG_ENOMEM at once, and a request
    that fits still runs on the same server."""
    from paper_2508_11608_amd import Server, footprint

    big = W.ball_q2().with_levels(5)  # 64^3 cells: about 1 GB with the multi-column buffers
    small = W.offcentre_disc(2, 3)
    fb, _ = footprint(big, fp32=True, multi=True)
    fs, n = footprint(small, fp32=True, multi=True)
    budget = fs + 2 * 8 * 8 * n + (1 << 20)
    assert budget < fb
    print(f"\n[case] budget {budget} B, large request {fb} B", flush=True)
    srv = Server(budget, 1)
    t0 = time.perf_counter()
    (rb, xb), (rs, xs) = _run(srv, [(big, W.fourier_modes(3, 5), True), (small, W.fourier_modes(2, 6), True)])
    dt = time.perf_counter() - t0
    srv.close()
    print(f"  large: status {rb['status']}; small: status {rs['status']}, {rs['iterations']} its; {dt:.2f} s", flush=True)
    assert rb["status"] == -2 and xb is None
    assert rs["status"] == 0 and rs["rel_residual"] <= 1e-8


def test_single_requests_of_one_lattice_shape_are_grouped():
    """Single queued requests of different resident geometries of one lattice
    shape are solved by one grouped PCG (cmg_group_solve), and every result
    equals the same request alone on a fresh server, bit for bit."""
    from paper_2508_11608_amd import Server

    ws = [W.disc_q2(), W.offcentre_disc(2, 4), W.ellipse(2, 4), W.disc_union(2, 4)]
    print("\n[case] grouped serving: " + ", ".join(w.name for w in ws), flush=True)
    srv = Server(8 << 30, 1)
    _run(srv, [(w, W.fourier_modes(2, 3000 + i), True) for i, w in enumerate(ws)])  # all resident
    # a longer request first, so that the four single requests queue behind it
    reqs = [(W.offcentre_ball(2, 3), W.fourier_modes(3, 3099), True)]
    reqs += [(w, W.fourier_modes(2, 3100 + i), True) for i, w in enumerate(ws)]
    res = _run(srv, reqs)
    srv.close()
    print("  groups:", [r["group"] for r, _ in res], flush=True)
    assert max(r["group"] for r, _ in res[1:]) > 1
    for (w, f, fp32), (r, x) in zip(reqs[1:], res[1:]):
        alone = Server(8 << 30, 1)
        (r1, x1), = _run(alone, [(w, f, fp32)])
        alone.close()
        print(f"  {w.name}: group {r['group']}, {r['iterations']} its; alone {r1['iterations']} its", flush=True)
        assert r["status"] == 0 and r1["status"] == 0 and r1["group"] == 1
        assert r["iterations"] == r1["iterations"]
        assert np.array_equal(x, x1), w.name
