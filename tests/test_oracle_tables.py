"""Pins of the oracle's tables (eqs. 11-24, Sec. V.C-D) against the
geometry they discretise: rounding bounds, symmetries, bijectivity and
exact edge-length sums (Lemma 4/5)."""
import math

import numpy as np
import pytest

import oracle
from tests.pins.graph import Graph

CASES = [(64, 64, 10.0, 1), (64, 64, 10.0, 0), (48, 128, 12.0, 1), (40, 256, 100.0, 1), (96, 512, 12.0, 1),
         (64, 72, 7.5, 1), (30, 24, 3.0, 0)]


def _prob(N, L, R, hc):
    return oracle.Problem(N, L, R, hc, ct=[1024] * 6, gear=[256, 256, 384, 256, 384, 384])


@pytest.mark.parametrize("N,L,R,hc", CASES)
def test_turn_rounding_error(N, L, R, hc):
    """eq. (14): beta + Psi represents R sin(theta) within 1/4 cell with the
    half-cell representation, within 1/2 with plain rounding."""
    tb = oracle.tables(_prob(N, L, R, hc))
    alpha = np.array([R * math.sin(2 * math.pi * T / L) for T in range(L)])
    rep = tb["beta"] + 0.5 * tb["psi"]
    bound = 0.25 if hc else 0.5
    assert np.all(np.abs(rep - alpha) <= bound + 1e-9)
    if not hc:
        assert np.all(tb["psi"] == 0)


@pytest.mark.parametrize("N,L,R,hc", CASES)
def test_turn_symmetries(N, L, R, hc):
    """alpha(T + L/2) = -alpha(T) and alpha(L/2 - T) = alpha(T) hold exactly for
    the rounded tables; Psi_2 = Psi_0 and Psi_3 = Psi_1 (text after eq. 14)."""
    tb = oracle.tables(_prob(N, L, R, hc))
    z = 2 * tb["beta"] + tb["psi"]  # twice the represented offset
    T = np.arange(L)
    assert np.array_equal(z[(T + L // 2) % L], -z)
    assert np.array_equal(z[(L // 2 - T) % L], z)
    psi = tb["psi"]
    assert np.array_equal(psi[(T + L // 2) % L], psi)  # Psi_2 = Psi_0
    assert np.array_equal(psi[(T + 3 * L // 4) % L], psi[(T + L // 4) % L])  # Psi_3 = Psi_1


@pytest.mark.parametrize("N,L,R,hc", CASES)
def test_unit_turn_steps(N, L, R, hc):
    """With N_theta >= 2 pi R successive planes shift by at most one cell
    (the end of Sec. V.C)."""
    tb = oracle.tables(_prob(N, L, R, hc))
    step = np.abs(np.diff(np.r_[tb["beta"], tb["beta"][0]]))
    if L >= 2 * math.pi * R:
        assert step.max() <= 1
    else:
        assert step.max() >= 2  # the reduced-angle case really jumps


@pytest.mark.parametrize("N,L,R,hc", CASES)
def test_straight_tables(N, L, R, hc):
    """eqs. (19)-(24): the family follows |tan| <= 1, B(y', T) rounds y' K
    within 1/2 cell and moves at most one cell per step, J is the sign of
    the major direction."""
    tb = oracle.tables(_prob(N, L, R, hc))
    for T in range(L):
        th = 2 * math.pi * T / L
        c, s = math.cos(th), math.sin(th)
        if abs(abs(c) - abs(s)) > 1e-9:
            assert tb["I"][T] == (0 if abs(c) > abs(s) else 1)
        K = s / c if tb["I"][T] == 0 else c / s
        assert abs(K) <= 1 + 1e-12
        y = np.arange(N)
        assert np.all(np.abs(tb["Bsk"][T] - y * K) <= 0.5 + 1e-9)
        assert np.all(np.abs(np.diff(tb["Bsk"][T])) <= 1)
        assert tb["J"][T] == (np.sign(c) if tb["I"][T] == 0 else np.sign(s))
    # the x-major family is exactly the planes within 45 degrees of 0 or 180
    assert int((tb["I"] == 0).sum()) == L // 2 + 2


@pytest.mark.parametrize("N,L,R,hc", CASES)
def test_edge_lengths(N, L, R, hc):
    """Lemma 4: a full circle of turn edges sums to 2 pi R (here within the
    rounding of L edges); Sec. V.D: a straight edge is 1/max(|cos|, |sin|)."""
    prob = _prob(N, L, R, hc)
    tb = oracle.tables(prob)
    for mu in (oracle.LF, oracle.RB, oracle.RF, oracle.LB):
        g = prob.gear[mu] / 256.0
        assert abs(L * int(tb["Lq"][mu, 0]) - 2 * math.pi * R * 1024 * g) <= L / 2 + 1e-6
        assert np.all(tb["Lq"][mu] == tb["Lq"][mu, 0])
    for mu in (oracle.SF, oracle.SB):
        g = prob.gear[mu] / 256.0
        for T in range(L):
            th = 2 * math.pi * T / L
            exact = 1024 * g / max(abs(math.cos(th)), abs(math.sin(th)))
            assert abs(int(tb["Lq"][mu, T]) - exact) <= 0.5 + 1e-6


@pytest.mark.parametrize("N,L,R,hc", CASES[:5])
def test_edges_are_bijective_and_follow_curves(N, L, R, hc):
    """Every maneuver's edge map is a permutation of the volume (Sec. V.C:
    curves of one maneuver partition the volume), the forward/backward maps
    of a maneuver type are inverse, and a turn edge moves one plane."""
    prob = _prob(N, L, R, hc)
    tb = oracle.tables(prob)
    B = np.zeros((L, N, N), np.uint8)
    g = Graph(N, L, tb, B, prob.ct)
    for mu in range(6):
        assert g.is_permutation(mu)
    NR = N * N * L
    ar = np.arange(NR)
    assert np.array_equal(g.succ[oracle.LB][g.succ[oracle.LF]], ar)
    assert np.array_equal(g.succ[oracle.RB][g.succ[oracle.RF]], ar)
    assert np.array_equal(g.succ[oracle.SB][g.succ[oracle.SF]], ar)
    T = ar // (N * N)
    assert np.array_equal(g.succ[oracle.LF] // (N * N), (T + 1) % L)
    assert np.array_equal(g.succ[oracle.RF] // (N * N), (T - 1) % L)


@pytest.mark.parametrize("N,L,R", [(64, 64, 10.0), (80, 128, 12.0)])
def test_turn_edges_move_along_the_circle(N, L, R):
    """A LEFT-FORWARD edge moves the represented point (eq. 16) along the
    heading by about one arc step and turns left (positive theta); a
    RIGHT-FORWARD edge turns right.  The chord direction matches the mean
    heading of the edge within the rounding (Lemma 4: at most 1/4 cell per
    end)."""
    prob = _prob(N, L, R, 1)
    tb = oracle.tables(prob)
    B = np.zeros((L, N, N), np.uint8)
    g = Graph(N, L, tb, B, prob.ct)
    psi = tb["psi"]
    step = 2 * math.pi * R / L
    for mu, sgn in ((oracle.LF, 1), (oracle.RF, -1)):
        for T in range(L):
            x = (T * N + N // 2) * N + N // 2
            y = int(g.succ[mu][x])
            T2 = y // (N * N)
            assert (T2 - T) % L == (1 if sgn > 0 else L - 1)
            p0 = np.array([N // 2 + 0.5 * psi[T], N // 2 + 0.5 * psi[(T + L // 4) % L]])
            j2, i2 = (y // N) % N, y % N
            p1 = np.array([i2 + 0.5 * psi[T2], j2 + 0.5 * psi[(T2 + L // 4) % L]])
            d = p1 - p0
            mid = 2 * math.pi * (T + 0.5 * sgn) / L
            exact = step * np.array([math.cos(mid), math.sin(mid)]) * (2 * math.sin(math.pi / L) / (2 * math.pi / L))
            assert np.all(np.abs(d - exact) <= 0.5 + 1e-9)
