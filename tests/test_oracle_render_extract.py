"""Pins of the oracle's obstacle rendering (Sec. VI), goal search (Sec. IX)
and back-tracking (Sec. X): closed-form box dilation at the axis headings,
a rasterised rotated box at other headings, brute-force goal window, and
replay of the extracted plan through the explicit graph."""
import math

import numpy as np
import pytest
from scipy.ndimage import maximum_filter

import oracle
from paper_2306_01301_amd import scenes
from tests.common import cell, oracle_volumes, problem_of
from tests.pins import graph as G

INF = oracle.INF


def _walled(img):
    w = img.copy()
    w[0, :] = 255
    w[:, 0] = 255
    return w


@pytest.mark.parametrize("f,r,s", [(4, 1, 1), (7, 2, 2), (0, 0, 0), (10, 3, 4)])
def test_axis_headings_are_box_dilations(f, r, s):
    """At theta = 0, 90, 180, 270 degrees the footprint is an axis-aligned box
    and the volume is a plain maximum filter of the walled image."""
    N, L = 48, 32
    rng = np.random.default_rng(f * 7 + s)
    img = rng.integers(0, 255, size=(N, N)).astype(np.uint8)
    img[rng.random((N, N)) < 0.02] = 255
    prob = oracle.Problem(N, L, 5.0, 0)
    B = oracle.render(prob, img, f, r, s)
    w = _walled(img)
    # heading +x: rows j-s..j+s, columns i-r..i+f; the other three axes rotate it
    for T, (dy0, dy1, dx0, dx1) in {0: (-s, s, -r, f), L // 4: (-r, f, -s, s),
                                    L // 2: (-s, s, -f, r), 3 * L // 4: (-f, r, -s, s)}.items():
        want = np.zeros_like(w)
        for dy in range(dy0, dy1 + 1):
            for dx in range(dx0, dx1 + 1):
                want = np.maximum(want, np.roll(np.roll(w, -dy, 0), -dx, 1))
        want[0, :] = 255
        want[:, 0] = 255
        assert np.array_equal(B[T], want), T
        # scipy's maximum filter (window centred, so shift by the box centre) agrees
        if (dy1 - dy0) % 2 == 0 and (dx1 - dx0) % 2 == 0:
            mf = maximum_filter(np.roll(np.roll(w, -(dy0 + dy1) // 2, 0), -(dx0 + dx1) // 2, 1),
                                size=(dy1 - dy0 + 1, dx1 - dx0 + 1), mode="wrap")
            mf[0, :] = 255
            mf[:, 0] = 255
            assert np.array_equal(B[T], mf), T


def _rect_pixels(cx, cy, th, f, r, s, grow):
    """Pixels whose centre lies in the rotated rectangle [-r-grow, f+grow] x
    [-s-grow, s+grow] around (cx, cy) with heading th."""
    c, sn = math.cos(th), math.sin(th)
    ext = int(math.ceil(max(f, r) + s + grow)) + 2
    out = []
    for dy in range(-ext, ext + 1):
        for dx in range(-ext, ext + 1):
            u = dx * c + dy * sn      # along the heading
            v = -dx * sn + dy * c     # along the left normal
            if -r - grow <= u <= f + grow and -s - grow <= v <= s + grow:
                out.append((dx, dy))
    return out


@pytest.mark.parametrize("T", [3, 5, 8, 13, 21, 30])
def test_oblique_headings_follow_the_rotated_box(T):
    """Sound within one cell: a hard vertex has a hard pixel inside the box
    grown by one cell; a 3 x 3 hard block well inside the box is never
    missed."""
    N, L, f, r, s = 40, 64, 6, 2, 2
    rng = np.random.default_rng(T)
    img = np.zeros((N, N), np.uint8)
    for _ in range(6):
        x, y = rng.integers(4, N - 7, 2)
        img[y:y + 3, x:x + 3] = 255
    prob = oracle.Problem(N, L, 5.0, 0)
    B = oracle.render(prob, img, f, r, s)
    th = 2 * math.pi * T / L
    grown = _rect_pixels(0, 0, th, f, r, s, 1.0)
    inner = _rect_pixels(0, 0, th, f, r, s, -1.5)
    w = _walled(img)
    for j in range(12, N - 12):
        for i in range(12, N - 12):
            hard = B[T, j, i] == 255
            near = any(w[j + dy, i + dx] == 255 for dx, dy in grown)
            if hard:
                assert near, (i, j)
            blocks = [(dx, dy) for dx, dy in inner
                      if all((dx + a, dy + b) in set(inner) for a in (-1, 0, 1) for b in (-1, 0, 1))]
            if any(np.all(w[j + dy - 1:j + dy + 2, i + dx - 1:i + dx + 2] == 255) for dx, dy in blocks):
                assert hard, (i, j)


def test_walls_and_start_rules():
    sc = scenes.plain_64()
    prob, B, V = oracle_volumes(sc, 0)
    assert np.all(B[:, 0, :] == 255) and np.all(B[:, :, 0] == 255)
    assert V[sc.start[2], sc.start[1], sc.start[0]] == 0
    assert np.count_nonzero(V != INF) == 1
    with pytest.raises(oracle.OracleError) as e:
        oracle.init(prob, B, (0, 5, 0))
    assert e.value.rc == oracle.ESTART


def test_goal_search_brute_force():
    sc = scenes.random_small(71, n=24, nt=16, R=3.0)
    prob, B, V = oracle_volumes(sc, 2)
    N, L = sc.nx, sc.nt
    for d, wxy, wt in [(0, 0, 0), (1, 1024, 512), (2, 300, 4000), (3, 0, 0)]:
        gi, gj, gt = sc.goal
        cands = []
        for dt in range(-d, d + 1):
            for dy in range(-d, d + 1):
                for dx in range(-d, d + 1):
                    i, j, t = (gi + dx) % N, (gj + dy) % N, (gt + dt) % L
                    if B[t, j, i] == 255 or V[t, j, i] == INF:
                        continue
                    sc_ = min(int(V[t, j, i]) + wxy * (abs(dx) + abs(dy)) + wt * abs(dt), INF)
                    cands.append(((sc_, abs(dx) + abs(dy) + abs(dt), dt, dy, dx), (i, j, t)))
        if not cands:
            with pytest.raises(oracle.OracleError):
                oracle.goal_search(prob, B, V, sc.goal, d, wxy, wt)
            continue
        key, best = min(cands)
        got, score = oracle.goal_search(prob, B, V, sc.goal, d, wxy, wt)
        assert got == best and score == key[0]


@pytest.mark.parametrize("seed,converge", [(81, False), (82, True), (83, True), (84, False)])
def test_backtrack_replays_through_the_explicit_graph(seed, converge):
    sc = scenes.random_small(seed, n=24, nt=16, R=2.5)
    prob = problem_of(sc)
    B = oracle.render(prob, sc.image, *sc.vehicle)
    V = oracle.init(prob, B, sc.start)
    if converge:
        prev = None
        while prev is None or not np.array_equal(prev, V):
            prev = V.copy()
            oracle.cycles(prob, B, V, 1)
    else:
        oracle.cycles(prob, B, V, 2)
    g = G.Graph(sc.nx, sc.nt, oracle.tables(prob), B, sc.ct)
    try:
        best, score = oracle.goal_search(prob, B, V, sc.goal, 3, 0, 0)
    except oracle.OracleError:
        pytest.skip("goal not reached")
    steps = oracle.backtrack(prob, B, V, sc.start, best)
    N = sc.nx
    x = cell(N, *sc.start)
    total = 0
    for st in steps:
        assert cell(N, *st.frm) == x
        (y, c), = G.path_cost(g, x, [(st.maneuver, st.steps)])
        assert y == cell(N, *st.to) and c == st.cost
        # the step's candidate value never exceeds the value it explains
        assert int(V.reshape(-1)[x]) + c <= int(V.reshape(-1)[y])
        total += c
        x = y
    assert x == cell(N, *best)
    vb = int(V.reshape(-1)[x])
    assert total <= vb
    if converge:
        assert total == vb  # at a fixed point the minimum is the value itself (Sec. X)
