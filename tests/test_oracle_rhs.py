"""Pins of the oracle's Fourier load vector against closed forms.

With homogeneous Dirichlet data the load vector is b_i = (f, phi_i)_Omega
(weak equation, Section 2.1).  The nodal basis of Q_k reproduces every
polynomial of degree <= 1 exactly on the active cells, so

    sum_i b_i            = int_Omega f,
    sum_i b_i x_{i,j}    = int_Omega f x_j       (x_i: coordinates of DoF i).

For f = cos(w . x + theta) on a ball |x - c| < r the integrals are closed forms
of the Fourier transform I(s) of the ball's indicator, s = |w|:

    int cos(w.x + theta)       = cos(phi) I(s),                    phi = w.c + theta,
    int x_j cos(w.x + theta)   = c_j cos(phi) I(s) + sin(phi) I'(s) w_j / s,
    I_2(s) = 2 pi r J_1(s r) / s,       I_3(s) = 4 pi (sin(s r) - s r cos(s r)) / s^3.

The ball is off-centre, so a wrong sign of the phase or of w . x, a sine for the
cosine, a missing pi or a dropped mode all change these sums.
"""
import math

import numpy as np
import pytest
from scipy.special import j0, j1

import workloads as W
from oracle import problem
from oracle.geometry import build_levels


def _ft_ball(dim, r, s):
    """I(s) and I'(s) of the indicator of a ball of radius r."""
    if dim == 2:
        I = 2 * math.pi * r * j1(s * r) / s
        dI = 2 * math.pi * r * (r * s * j0(s * r) - 2 * j1(s * r)) / s ** 2
    else:
        F = math.sin(s * r) - s * r * math.cos(s * r)
        I = 4 * math.pi * F / s ** 3
        dI = 4 * math.pi * (r * r * math.sin(s * r) / s ** 2 - 3 * F / s ** 4)
    return I, dI


def _closed_forms(c, r, kappa, amp, theta):
    """int_Omega f and int_Omega f x_j for f = sum_q a_q cos(pi kappa_q . x + theta_q)."""
    dim = len(c)
    tot = 0.0
    mom = np.zeros(dim)
    for kq, aq, tq in zip(kappa, amp, theta):
        w = math.pi * np.asarray(kq, dtype=np.float64)
        s = float(np.linalg.norm(w))
        I, dI = _ft_ball(dim, r, s)
        phi = float(w @ c) + tq
        tot += aq * math.cos(phi) * I
        mom += aq * (c * math.cos(phi) * I + math.sin(phi) * dI * w / s)
    return tot, mom


def _sums(w, L, kappa, amp, theta):
    lev = build_levels(problem.shapes_of(w), w.dim, w.k, L, w.coarse_cells, w.lo, w.hi)[-1]
    b = problem.rhs_fourier(w, lev, kappa, amp, theta)
    X = lev.dof_coords()
    return b.sum(), X.T @ b


def test_fourier_load_vector_disc():
    w = W.offcentre_disc(k=2)
    c, r = np.array(w.centers[0]), w.semi[0][0]
    for seed in (1000, 1001, 1007):
        kappa, amp, theta = W.fourier_modes(2, seed)
        tot, mom = _sums(w, 5, kappa, amp, theta)  # 64^2 cells
        tot_x, mom_x = _closed_forms(c, r, kappa, amp, theta)
        scale = np.abs(amp).sum() * math.pi * r * r
        assert abs(tot - tot_x) < 1e-12 * scale, (seed, tot, tot_x)
        assert np.abs(mom - mom_x).max() < 1e-12 * scale, (seed, mom, mom_x)


def test_fourier_load_vector_single_modes_disc():
    """One mode at a time, including the largest wave numbers of the generator."""
    w = W.offcentre_disc(k=3)
    c, r = np.array(w.centers[0]), w.semi[0][0]
    for kq, tq in (((1, 0), 0.3), ((0, 3), 2.1), ((4, 4), 4.4), ((2, 3), 5.9)):
        kappa, amp, theta = np.array([kq]), np.array([1.0]), np.array([tq])
        tot, mom = _sums(w, 5, kappa, amp, theta)
        tot_x, mom_x = _closed_forms(c, r, kappa, amp, theta)
        assert abs(tot - tot_x) < 1e-12 * math.pi * r * r, (kq, tot, tot_x)
        assert np.abs(mom - mom_x).max() < 1e-12 * math.pi * r * r, (kq, mom, mom_x)


def test_fourier_load_vector_ball():
    """3-D, 16^3 cells, Q3: the seeded generator's modes (wave numbers up to 4
    per direction) and a hand-picked set."""
    w = W.offcentre_ball(k=3)
    c, r = np.array(w.centers[0]), w.semi[0][0]
    cases = [W.fourier_modes(3, 1000), W.fourier_modes(3, 1005),
             (np.array([(1, 0, 0), (0, 1, 1), (1, 1, 1), (1, 0, 1)]), np.array([0.7, -1.3, 0.4, 0.9]),
              np.array([0.2, 1.9, 3.7, 5.1]))]
    for kappa, amp, theta in cases:
        tot, mom = _sums(w, 3, kappa, amp, theta)
        tot_x, mom_x = _closed_forms(c, r, kappa, amp, theta)
        scale = np.abs(amp).sum() * 4 / 3 * math.pi * r ** 3
        assert abs(tot - tot_x) < 1e-12 * scale, (tot, tot_x)
        assert np.abs(mom - mom_x).max() < 1e-12 * scale, (mom, mom_x)


@pytest.mark.parametrize("flaw", ["sin", "no_pi", "phase_sign"])
def test_closed_forms_tell_plausible_flaws_apart(flaw):
    """The sums above are sensitive to each plausible mistake: a flawed f of
    the same modes misses the closed form by far more than the tolerance."""
    w = W.offcentre_disc(k=2)
    c, r = np.array(w.centers[0]), w.semi[0][0]
    kappa, amp, theta = W.fourier_modes(2, 1000)
    lev = build_levels(problem.shapes_of(w), 2, 2, 4, w.coarse_cells, w.lo, w.hi)[-1]
    kap = kappa.astype(np.float64)

    def f_bad(x):
        if flaw == "sin":
            return np.sin(math.pi * x @ kap.T + theta) @ amp
        if flaw == "no_pi":
            return np.cos(x @ kap.T + theta) @ amp
        return np.cos(math.pi * x @ kap.T - theta) @ amp

    from oracle.assemble import load_vector

    b = load_vector(lev, problem.shapes_of(w), problem.form_params(w), f_bad, None)
    tot_x, mom_x = _closed_forms(c, r, kappa, amp, theta)
    scale = np.abs(amp).sum() * math.pi * r * r
    miss = max(abs(b.sum() - tot_x), np.abs(lev.dof_coords().T @ b - mom_x).max())
    assert miss > 1e-4 * scale
