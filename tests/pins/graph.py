"""The planner's graph written out explicitly, from the edge maps of
Sec. V.D, eqs. (25)-(31), and the Star transition subgraph of Sec. V.A.

This is a second code route to the same graph: the oracle walks curves with
the curve parametrisations (18) and (23); here every vertex gets its one
successor per maneuver from the beta and B differences of eqs. (25)-(31).
Only the integer tables (beta, B, I, J, edge lengths) come from the oracle;
they are pinned separately.

Edge weights (the cost model, Sec. VI): the edge leaving vertex X in
maneuver mu costs (Lq_mu(T) * (256 + 4 kappa(X)) + 128) >> 8 in 1/1024 cell,
infinite when X is hard (kappa = 255).
"""
from __future__ import annotations

import heapq

import numpy as np

INF = 0xFFFFFFFF
HARD = 255
LF, SF, RB, RF, SB, LB = range(6)


def idx(N, i, j, T):
    return (T * N + j) * N + i


class Graph:
    def __init__(self, N: int, L: int, tb: dict, B: np.ndarray, ct, gear_unused=None):
        self.N, self.L, self.tb = N, L, tb
        self.B = B.reshape(-1)
        self.ct = [int(c) for c in ct]
        NR = N * N * L
        T, j, i = np.meshgrid(np.arange(L), np.arange(N), np.arange(N), indexing="ij")
        T, j, i = T.reshape(-1), j.reshape(-1), i.reshape(-1)
        self.Tc, self.jc, self.ic = T, j, i
        beta = tb["beta"].astype(np.int64)
        q = L // 4

        def bk(k, t):
            return beta[(t + k * q) % L]

        Tp, Tm = (T + 1) % L, (T - 1) % L
        # beta_k^+(T) = beta_k(T+1) - beta_k(T), beta_k^-(T) = beta_k(T-1) - beta_k(T)
        succ = np.zeros((6, NR), np.int64)
        succ[LF] = idx(N, (i + bk(0, Tp) - bk(0, T)) % N, (j + bk(3, Tp) - bk(3, T)) % N, Tp)  # (25)
        succ[LB] = idx(N, (i + bk(0, Tm) - bk(0, T)) % N, (j + bk(3, Tm) - bk(3, T)) % N, Tm)  # (26)
        succ[RF] = idx(N, (i + bk(2, Tm) - bk(2, T)) % N, (j + bk(1, Tm) - bk(1, T)) % N, Tm)  # (27)
        succ[RB] = idx(N, (i + bk(2, Tp) - bk(2, T)) % N, (j + bk(1, Tp) - bk(1, T)) % N, Tp)  # (28)
        Bsk = tb["Bsk"].astype(np.int64)
        Ifam = tb["I"][T]
        J = tb["J"][T]
        ip, im = (i + 1) % N, (i - 1) % N
        jp, jm = (j + 1) % N, (j - 1) % N
        # (30): I = 0: (i+, j + B(i+) - B(i)); I = 1: (i + B(j+) - B(j), j+)
        plus = np.where(Ifam == 0,
                        idx(N, ip, (j + Bsk[T, ip] - Bsk[T, i]) % N, T),
                        idx(N, (i + Bsk[T, jp] - Bsk[T, j]) % N, jp, T))
        # (31): the same with i-, j-
        minus = np.where(Ifam == 0,
                         idx(N, im, (j + Bsk[T, im] - Bsk[T, i]) % N, T),
                         idx(N, (i + Bsk[T, jm] - Bsk[T, j]) % N, jm, T))
        # (30) is the forward direction when J >= 0, (31) otherwise
        succ[SF] = np.where(J >= 0, plus, minus)
        succ[SB] = np.where(J >= 0, minus, plus)
        self.succ = succ
        kappa = self.B.astype(np.int64)
        Lq = tb["Lq"].astype(np.int64)
        w = np.zeros((6, NR), np.int64)
        for mu in range(6):
            ww = (Lq[mu, T] * (256 + 4 * kappa) + 128) >> 8
            w[mu] = np.where(kappa == HARD, INF, np.minimum(ww, INF))
        self.w = w
        self.pred = np.zeros_like(succ)
        for mu in range(6):
            p = np.empty(NR, np.int64)
            p[succ[mu]] = np.arange(NR)
            self.pred[mu] = p

    def is_permutation(self, mu: int) -> bool:
        return np.unique(self.succ[mu]).size == self.succ[mu].size


def sat(a):
    return np.minimum(a, INF)


def schedule_dp_sweep(g: Graph, mu: int, V: np.ndarray) -> np.ndarray:
    """The effect of one maneuver kernel, written as a fixed point over the
    explicit mu-edges: m(X) = best value of being inside maneuver mu at X
    (entered from the transition state somewhere upstream, Sec. VIII.B);
    the new transition value is min(V, value carried in along the edge)."""
    V0 = V.reshape(-1).astype(np.int64)
    ct = g.ct[mu]
    pred, w = g.pred[mu], g.w[mu]
    m = sat(V0 + ct)
    while True:
        carried = sat(m[pred] + w[pred])
        m2 = np.minimum(m, carried)
        if np.array_equal(m2, m):
            break
        m = m2
    carried = sat(m[pred] + w[pred])
    out = np.minimum(V0, carried)
    out[g.B == HARD] = INF
    return out.astype(np.uint32).reshape(V.shape)


def schedule_dp(g: Graph, schedule, V: np.ndarray, n_cycles: int) -> np.ndarray:
    for _ in range(n_cycles):
        for mu in schedule:
            V = schedule_dp_sweep(g, mu, V)
    return V


def star_dijkstra(g: Graph, schedule, start: int) -> np.ndarray:
    """Shortest distances to the transition vertices of the Star graph
    (Sec. V.A): T(X) -> M_mu(X) costs ct_mu, M_mu(X) -> T(X) costs 0, and
    M_mu(X) -> M_mu(succ_mu(X)) costs w_mu(X)."""
    NR = g.succ.shape[1]
    mus = sorted(set(int(m) for m in schedule))
    dist = {}
    dT = np.full(NR, INF, np.int64)
    dM = {mu: np.full(NR, INF, np.int64) for mu in mus}
    heap = [(0, 0, start)]  # (d, kind, x): kind 0 = transition, 1 + mu = maneuver
    dT[start] = 0
    succ = {mu: g.succ[mu] for mu in mus}
    w = {mu: g.w[mu] for mu in mus}
    while heap:
        d, kind, x = heapq.heappop(heap)
        if kind == 0:
            if d != dT[x]:
                continue
            for mu in mus:
                nd = d + g.ct[mu]
                if nd < dM[mu][x]:
                    dM[mu][x] = nd
                    heapq.heappush(heap, (nd, 1 + mu, x))
        else:
            mu = kind - 1
            if d != dM[mu][x]:
                continue
            if d < dT[x]:
                dT[x] = d
                heapq.heappush(heap, (d, 0, x))
            we = int(w[mu][x])
            if we < INF:
                y = int(succ[mu][x])
                nd = d + we
                if nd < dM[mu][y]:
                    dM[mu][y] = nd
                    heapq.heappush(heap, (nd, 1 + mu, y))
    del dist
    return np.minimum(dT, INF)


def compact_dijkstra(g: Graph, start: int, ct_left: int, ct_right: int) -> np.ndarray:
    """Shortest distances in the Compact graph (Sec. V.A, Fig. 12): three
    vertices per pose (LEFT, STRAIGHT, RIGHT), the transition state merged
    with STRAIGHT; STRAIGHT -> LEFT/RIGHT costs ct, back costs 0; LEFT holds
    the LF and LB edges, STRAIGHT SF and SB, RIGHT RF and RB."""
    NR = g.succ.shape[1]
    d = np.full((3, NR), INF, np.int64)  # 0 LEFT, 1 STRAIGHT, 2 RIGHT
    d[1, start] = 0
    heap = [(0, 1, start)]
    edges = {0: (LF, LB), 1: (SF, SB), 2: (RF, RB)}
    while heap:
        dd, v, x = heapq.heappop(heap)
        if dd != d[v, x]:
            continue
        nbrs = []
        if v == 1:
            nbrs += [(0, x, ct_left), (2, x, ct_right)]
        else:
            nbrs.append((1, x, 0))
        for mu in edges[v]:
            we = int(g.w[mu][x])
            if we < INF:
                nbrs.append((v, int(g.succ[mu][x]), we))
        for v2, y, c in nbrs:
            nd = dd + c
            if nd < d[v2, y]:
                d[v2, y] = nd
                heapq.heappush(heap, (nd, v2, y))
    return np.minimum(d[1], INF)


def enumerate_paths(g: Graph, start: int, sequence_options, max_steps: dict):
    """Brute force: every path from `start` that uses, in order, a sub-sequence
    of `sequence_options` (each used at most once, each for 1..max_steps
    edges).  Returns per-vertex minimum cost over all enumerated paths."""
    NR = g.succ.shape[1]
    ends = np.array([start], np.int64)
    costs = np.array([0], np.int64)
    for mu in sequence_options:
        new_e, new_c = [ends], [costs]
        cur, E = ends.copy(), np.zeros_like(costs)
        ok = np.ones_like(costs, bool)
        for k in range(1, max_steps[mu] + 1):
            E = E + g.w[mu][cur]
            ok &= E < INF
            cur = g.succ[mu][cur]
            new_e.append(cur[ok])
            new_c.append(sat(costs[ok] + g.ct[mu] + E[ok]))
        ends, costs = np.concatenate(new_e), np.concatenate(new_c)
    best = np.full(NR, INF, np.int64)
    np.minimum.at(best, ends, costs)
    return best


def path_cost(g: Graph, start: int, steps) -> list:
    """Replays (maneuver, k) steps through the explicit graph and returns the
    vertex reached and the cost of each step."""
    x, out = start, []
    for mu, k in steps:
        E = 0
        for _ in range(k):
            E += int(g.w[mu][x])
            x = int(g.succ[mu][x])
        out.append((x, min(E + g.ct[mu], INF)))
    return out


def star_dijkstra_sources(g: Graph, schedule, sources) -> np.ndarray:
    """Star-graph Dijkstra from several sources: (x, d, mu) puts distance d
    on the transition vertex of x (mu < 0) or on its maneuver-mu vertex
    (a maneuver already in progress: it continues along mu's edges, and
    leaving it costs nothing).  Transition -> maneuver edges exist for the
    scheduled maneuvers only."""
    NR = g.succ.shape[1]
    sched = sorted(set(int(m) for m in schedule))
    mus = sorted(set(sched) | {int(m) for _, _, m in sources if m >= 0})
    dT = np.full(NR, INF, np.int64)
    dM = {mu: np.full(NR, INF, np.int64) for mu in mus}
    heap = []
    for x, d, mu in sources:
        if mu < 0:
            if d < dT[x]:
                dT[x] = d
                heapq.heappush(heap, (d, 0, x))
        elif d < dM[mu][x]:
            dM[mu][x] = d
            heapq.heappush(heap, (d, 1 + mu, x))
    while heap:
        d, kind, x = heapq.heappop(heap)
        if kind == 0:
            if d != dT[x]:
                continue
            for mu in sched:
                nd = d + g.ct[mu]
                if nd < dM[mu][x]:
                    dM[mu][x] = nd
                    heapq.heappush(heap, (nd, 1 + mu, x))
        else:
            mu = kind - 1
            if d != dM[mu][x]:
                continue
            if d < dT[x] and g.B[x] != HARD:
                dT[x] = d
                heapq.heappush(heap, (d, 0, x))
            we = int(g.w[mu][x])
            if we < INF:
                y = int(g.succ[mu][x])
                nd = d + we
                if nd < dM[mu][y]:
                    dM[mu][y] = nd
                    heapq.heappush(heap, (nd, 1 + mu, y))
    out = np.minimum(dT, INF)
    out[g.B == HARD] = INF
    return out
