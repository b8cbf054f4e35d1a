"""Host-only parts of the C ABI, on the CPU: the footprint estimate before
set-up, the error statuses of bad geometries and parameters, the launch
policy setter, and the exported cut-cell quadrature against closed forms."""
import ctypes
import math
import os

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2508_11608_amd", "libcutmg.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libcutmg.so not built")

CMG_EINVAL, CMG_EGEOM, CMG_ENOTSPD = -1, -3, -4


@pytest.mark.parametrize("w", [W.disc_q2(), W.offcentre_ball(3, 2), W.ball_union(2, 3), W.sphere_union_8(3, 2),
                               W.ellipse(1, 4)], ids=lambda w: w.name)
def test_footprint_equals_device_bytes_of_the_set_up(w):
    """cmg_footprint counts without quadrature or factorisation; it must give
    exactly the bytes of the problem cmg_setup builds, for every flag set."""
    from paper_2508_11608_amd import Problem, footprint

    P = Problem(w, device=False)
    for fp32 in (False, True):
        for multi in (False, True):
            fb, nd = footprint(w, fp32=fp32, multi=multi)
            assert fb == P.device_bytes(fp32=fp32, multi=multi), (fp32, multi)
            assert nd == P.ndofs()
    P.close()


def _status(fn):
    from paper_2508_11608_amd import CutmgError

    try:
        fn()
    except CutmgError as e:
        return e.status
    return 0


def test_indefinite_form_is_enotspd():
    """A negative ghost penalty makes the bilinear form indefinite: the set-up
    stops at the first Cholesky factorisation that fails (CMG_ENOTSPD)."""
    from paper_2508_11608_amd import Problem

    w = W.Workload(**{**W.disc_q2().__dict__, "gamma_g": -0.5, "name": "negative-ghost"})
    assert _status(lambda: Problem(w, device=False)) == CMG_ENOTSPD


def test_geometry_outside_the_box_is_egeom():
    from paper_2508_11608_amd import Problem, footprint

    w = W.Workload("outside", 2, 2, 3, centers=((3.0, 3.0),), semi=((0.5, 0.5),))
    assert _status(lambda: Problem(w, device=False)) == CMG_EGEOM
    assert _status(lambda: footprint(w)) == CMG_EGEOM


@pytest.mark.parametrize("change", [{"k": 4}, {"k": 0}, {"n_levels": 0}, {"coarse_cells": 0}, {"n_c": -1},
                                    {"semi": ((0.0, 0.7),)}, {"dim": 4}, {"ghost_exp_mode": 2}],
                         ids=lambda c: next(iter(c)))
def test_bad_parameters_are_einval(change):
    from paper_2508_11608_amd import Problem, footprint

    w = W.Workload(**{**W.disc_q2().__dict__, **change})
    assert _status(lambda: Problem(w, device=False)) == CMG_EINVAL
    assert _status(lambda: footprint(w)) == CMG_EINVAL


def test_device_calls_on_a_host_problem_are_einval():
    from paper_2508_11608_amd import Problem, cutmg

    P = Problem(W.disc_q2().with_levels(2), device=False)
    lib = cutmg.load_library()
    assert lib.cmg_vcycle(P._h, None, None, None) == CMG_EINVAL
    assert lib.cmg_set_precision(P._h, 1) == CMG_EINVAL
    assert lib.cmg_set_launch(P._h, -1, 16) == CMG_EINVAL
    assert lib.cmg_set_launch(P._h, 0, 0) == CMG_EINVAL
    assert lib.cmg_set_launch(P._h, 0, 1) == 0
    assert lib.cmg_set_ghost_coupling(P._h, 2) == CMG_EINVAL
    assert lib.cmg_set_ghost_coupling(P._h, 1) == 0
    assert lib.cmg_set_ghost_coupling(P._h, 0) == 0
    P.close()


def _columns(P, level, d):
    """Parse the CMG_EXPORT_QUADRATURE layout into per-cell lists of columns."""
    q = P.export(level, 5, np.float64)
    cells, i = [], 0
    rec = 7 + 2 * d
    while i < len(q):
        m = int(q[i])
        cells.append(q[i + 1:i + 1 + m * rec].reshape(m, rec))
        i += 1 + m * rec
    return cells


@pytest.mark.parametrize("w,vol,area", [
    (W.disc_q2().with_levels(3), math.pi * 0.49, 2 * math.pi * 0.7),
    (W.ball_q2().with_levels(2), 4 / 3 * math.pi * 0.343, 4 * math.pi * 0.49),
], ids=["disc", "ball"])
def test_exported_quadrature_integrates_closed_forms(w, vol, area):
    """The library's own cut-cell rule (the columns its element matrices are
    built from) against the closed forms of the disc / ball: volume, surface,
    int_Gamma x.n = d |Omega| and int_Omega x_0^2 (exact along each column)."""
    from paper_2508_11608_amd import Problem

    d = w.dim
    P = Problem(w, device=False)
    L = w.n_levels - 1
    c = P.counts(L)
    cells = _columns(P, L, d)
    assert len(cells) == c["cut_cells"]
    V = S = XN = M2 = 0.0
    for cols in cells:
        e = cols[:, 0].astype(int)
        x = cols[:, 1:1 + d]
        wb, t0, t1, surf, ts, sw = (cols[:, 1 + d + j] for j in range(6))
        nrm = cols[:, 7 + d:7 + 2 * d]
        inside = t1 > t0
        V += np.sum(wb[inside] * (t1 - t0)[inside])
        # int x_0^2 along the column: exact for columns along x_0, else x_0^2 times the length
        along = inside & (e == 0)
        M2 += np.sum(wb[along] * (t1[along] ** 3 - t0[along] ** 3) / 3.0)
        across = inside & (e != 0)
        M2 += np.sum(wb[across] * x[across, 0] ** 2 * (t1 - t0)[across])
        s = surf > 0.5
        xs = x[s].copy()
        xs[np.arange(s.sum()), e[s]] = ts[s]
        S += np.sum(sw[s])
        XN += np.sum(sw[s] * np.sum(xs * nrm[s], axis=1))
    flags = P.export(L, 2, np.uint8)
    N = round(len(flags) ** (1.0 / d))
    h = (w.hi - w.lo) / N
    uncut = np.argwhere(((flags & 1) != 0) & ((flags & 2) == 0)).ravel()
    V += len(uncut) * h ** d
    x0 = w.lo + (uncut % N) * h
    M2 += np.sum(((x0 + h) ** 3 - x0 ** 3) / 3.0) * h ** (d - 1)
    r = 0.7
    m2 = math.pi * r ** 4 / 4 if d == 2 else 4 * math.pi * r ** 5 / 15
    assert abs(V / vol - 1) < 1e-13
    assert abs(S / area - 1) < 1e-13
    assert abs(XN / (d * vol) - 1) < 1e-12
    assert abs(M2 / m2 - 1) < 1e-13
    P.close()


def test_perm_export_is_the_lattice_order():
    """CMG_EXPORT_PERM: canonical DoF i sits at lattice node perm[i], ascending."""
    from paper_2508_11608_amd import Problem

    P = Problem(W.offcentre_disc(2, 3), device=False)
    perm = P.export(2, 1, np.int32)
    assert np.all(np.diff(perm) > 0)
    nn = P.counts(2)["nodes_per_dir"]
    assert perm[0] >= 0 and perm[-1] < nn ** 2
    P.close()


def test_group_arguments_are_checked_before_any_device_work():
    """cmg_group_create refuses bad member counts and problems that were set
    up on the host only (CMG_EINVAL); nothing is recorded or allocated."""
    from paper_2508_11608_amd import Group, Problem
    from paper_2508_11608_amd.cutmg import load_library

    lib = load_library()
    out = ctypes.c_void_p()
    assert lib.cmg_group_create(None, 1, ctypes.byref(out)) == CMG_EINVAL
    P = Problem(W.disc_q2().with_levels(2), device=False)
    try:
        arr = (ctypes.c_void_p * 9)(*([P._h.value] * 9))
        assert lib.cmg_group_create(arr, 0, ctypes.byref(out)) == CMG_EINVAL
        assert lib.cmg_group_create(arr, 9, ctypes.byref(out)) == CMG_EINVAL
        assert _status(lambda: Group([P])) == CMG_EINVAL  # host-only problem
        assert out.value is None
    finally:
        P.close()
