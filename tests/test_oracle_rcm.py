"""Pins of the oracle's reverse Cuthill-McKee (fixed tie-break): hand-derived
orders, bandwidths of special graphs, brute-force minimum bandwidth, the
level structure of the Cuthill-McKee BFS, and the characterisation of the
order inside each level that the parallel GPU formulation relies on."""
import itertools
import json
import os
from collections import deque

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import oracle
import synth


def graph_of(L):
    n = L.n
    rows = np.repeat(np.arange(n), np.diff(L.rowptr))
    A = sp.coo_matrix((np.ones(L.nnz), (rows, L.col)), shape=(n, n)).tocsr()
    A = ((A + A.T) > 0).astype(np.int8).tocsr()
    return A


def nbrs(A, v):
    return A.indices[A.indptr[v]:A.indptr[v + 1]]


def rcm_bandwidth(L, perm):
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(len(perm), dtype=perm.dtype)
    rows = np.repeat(np.arange(L.n), np.diff(L.rowptr))
    if L.nnz == 0:
        return 0
    return int(np.abs(iperm[rows] - iperm[L.col]).max())


def from_edge_list(n, edges):
    return synth.from_edges(n, edges, seed=0, values="ones")


@pytest.mark.parametrize("name", ["grid3x3_rcm.json", "star_rcm.json"])
def test_hand_derived(golden_dir, name):
    g = json.load(open(os.path.join(golden_dir, name)))
    L = from_edge_list(g["n"], g["edges"])
    perm = oracle.rcm(L)
    assert perm.tolist() == g["perm"]
    assert rcm_bandwidth(L, perm) == g["bandwidth"]


def brute_min_bandwidth(n, edges):
    if not edges:
        return 0
    e = np.array(edges)
    best = n
    for p in itertools.permutations(range(n)):
        pos = np.array(p)
        best = min(best, int(np.abs(pos[e[:, 0]] - pos[e[:, 1]]).max()))
    return best


SPECIAL = {
    "path6": (6, [(i, i + 1) for i in range(5)]),
    "cycle7": (7, [(i, (i + 1) % 7) for i in range(7)]),
    "k5": (5, [(i, j) for i in range(5) for j in range(i)]),
    "grid2": (4, [(0, 1), (2, 3), (0, 2), (1, 3)]),
}


@pytest.mark.parametrize("name", sorted(SPECIAL))
def test_special_graphs_reach_optimum(name):
    n, edges = SPECIAL[name]
    L = from_edge_list(n, edges)
    bw = rcm_bandwidth(L, oracle.rcm(L))
    assert bw == brute_min_bandwidth(n, edges)
    assert bw == {"path6": 1, "cycle7": 2, "k5": 4, "grid2": 2}[name]


@pytest.mark.parametrize("seed", range(12))
def test_never_below_brute_force_minimum(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 8))
    edges = [(i, j) for i in range(n) for j in range(i) if rng.random() < 0.4]
    L = from_edge_list(n, edges)
    perm = oracle.rcm(L)
    assert sorted(perm.tolist()) == list(range(n))
    assert rcm_bandwidth(L, perm) >= brute_min_bandwidth(n, edges)


def bfs_dist(A, s):
    dist = {s: 0}
    q = deque([s])
    while q:
        v = q.popleft()
        for u in nbrs(A, v):
            if u not in dist:
                dist[u] = dist[v] + 1
                q.append(u)
    return dist


def check_cm_structure(L, perm):
    """Checks, from definitions only, what the fixed-tie-break RCM must give."""
    n = L.n
    A = graph_of(L)
    deg = np.diff(A.indptr)
    order = perm[::-1]  # Cuthill-McKee order
    pos = np.empty(n, np.int64)
    pos[order] = np.arange(n)
    assert sorted(order.tolist()) == list(range(n))
    ncomp, lab = connected_components(A, directed=False)
    # components are contiguous in CM order and appear by their min (deg, index) key
    seen, keys = [], []
    for v in order:
        if not seen or seen[-1] != lab[v]:
            assert lab[v] not in seen
            seen.append(lab[v])
    for c in seen:
        nodes = np.flatnonzero(lab == c)
        keys.append(min((int(deg[v]), int(v)) for v in nodes))
    assert keys == sorted(keys)
    start = 0
    for c in seen:
        size = int((lab == c).sum())
        comp = order[start:start + size]
        s = int(comp[0])
        dist = bfs_dist(A, s)
        lev = np.array([dist[int(v)] for v in comp])
        # BFS order: levels are non-decreasing along the order
        assert np.all(np.diff(lev) >= 0)
        # George-Liu termination: the minimum of the last level is no further
        ecc = int(lev.max())
        last = [int(v) for v in comp if dist[int(v)] == ecc]
        u = min(last, key=lambda v: (int(deg[v]), v))
        assert max(bfs_dist(A, u).values()) <= ecc
        # the start is at least as eccentric as the minimum (deg, index) node
        s0 = min((int(v) for v in comp), key=lambda v: (int(deg[v]), v))
        assert ecc >= max(bfs_dist(A, s0).values())
        # inside level l+1 the order is lexicographic in
        # (min CM position of a level-l neighbour, deg, index)
        for l in range(1, ecc + 1):
            nodes = [int(v) for v in comp if dist[int(v)] == l]
            keyf = lambda v: (min(int(pos[u]) for u in nbrs(A, v) if dist[int(u)] == l - 1), int(deg[v]), v)
            assert nodes == sorted(nodes, key=keyf)
        # level bound on every edge inside the component
        sizes = np.bincount(lev)
        for v in comp:
            for u in nbrs(A, int(v)):
                lv, lu = dist[int(v)], dist[int(u)]
                assert abs(lv - lu) <= 1
                lo = min(lv, lu)
                span = sizes[lo] + (sizes[lo + 1] if lo + 1 < len(sizes) else 0) - 1
                assert abs(int(pos[v]) - int(pos[u])) <= span
        start += size


@pytest.mark.parametrize("maker", [
    lambda: synth.grid2d(12, 5),
    lambda: synth.grid3d(5, 6),
    lambda: synth.rgg2d(400, 6.0, 7),
    lambda: synth.chung_lu(500, 4.0, 2.5, 8),
    lambda: synth.from_edges(10, [(0, 1), (2, 3), (3, 4), (7, 9)], relabel=True, seed=3),
    lambda: synth.from_edges(5, [], seed=1),
])
def test_cm_structure(maker):
    L = maker()
    check_cm_structure(L, oracle.rcm(L))


def test_isolated_nodes_last():
    L = synth.from_edges(6, [(0, 1), (1, 2)], seed=0)
    perm = oracle.rcm(L)
    # isolated nodes 3,4,5 have degree 0: first in CM order, so last after reversal
    assert perm[-3:].tolist() == [5, 4, 3]


def test_workload0_band():
    L = synth.workload(0)
    perm = oracle.rcm(L)
    B = oracle.permute(L, perm)
    beta = oracle.bandwidth(B)
    assert beta <= 199
    assert beta >= 100  # the grid's minimum bandwidth is its side length
