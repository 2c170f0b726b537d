"""Helpers shared by the tests (argument plumbing only)."""
import numpy as np

import oracle


def problem_of(sc):
    return oracle.Problem(sc.nx, sc.nt, sc.R, sc.half_cell, list(sc.schedule), list(sc.ct), list(sc.gear))


def oracle_volumes(sc, n_cycles=None):
    """Oracle B and V after `n_cycles` (default: the scene's) for a scene."""
    prob = problem_of(sc)
    f, r, s = sc.vehicle
    B = oracle.render(prob, sc.image, f, r, s)
    V = oracle.init(prob, B, sc.start)
    oracle.cycles(prob, B, V, sc.n_cycles if n_cycles is None else n_cycles)
    return prob, B, V


def cell(N, i, j, T):
    return (T * N + j) * N + i
