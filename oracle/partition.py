"""Oracle: grain grids, contact interfaces and contact grids.  TEST
INFRASTRUCTURE ONLY.

Follows Sec. 3.1 (non-overlapping grain grids Omega^{g_i}, contact interfaces
Gamma^{c_j} shared by neighbouring grain grids, contact grids Omega^{zeta_k}
obtained by dilating each interface) and Sec. 3.2 (the sets C^{g_i}, G^{c_j})
of the paper, applied to a voxel partition with FEM nodes on voxel corners.

Readings:
* R1 (interfaces).  The adjacent-grain set S(v) of a free node v is the set of
  labels of the solid voxels touching v.  |S(v)| = 1 makes v an interior node
  of that grain.  |S(v)| >= 2 makes v an interface node; an interface is a
  connected set of interface nodes with identical S, two nodes being
  connected when both are corners of one solid voxel.  Where only two grains
  meet this is the paper's pairwise contact; box partitions also produce edge
  and corner interfaces with |S| up to 8.  Interfaces are numbered by their
  smallest free-node index; their nodes are listed in ascending order.
* R5 (contact grids).  One contact grid per interface (the paper has
  N^zeta = N^c); its node set is every free node within Chebyshev lattice
  distance w of a node of the interface (the morphological dilation), in
  ascending order.
"""
from __future__ import annotations

import numpy as np

from .fem import LOCAL_NODES


class Partition:
    """Result of the classification.

    node_grain[v]: grain id of an interior node, or -1 for an interface node.
    grain_nodes[i]: ascending free-node indices of grain i's interior.
    iface_nodes[c]: ascending free-node indices of interface c.
    iface_grains[c]: sorted tuple S of grains sharing interface c.
    node_iface[v]: interface id of interface node v, or -1.
    contact_nodes[c]: ascending free-node indices of contact grid c.
    """


def adjacent_sets(problem, mesh):
    """S(v) for every free node, as a list of sorted tuples."""
    sets = [set() for _ in range(mesh.n)]
    nz, ny, nx = problem.solid.shape
    lab = problem.labels
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if not problem.solid[k, j, i]:
                    continue
                g = int(lab[k, j, i])
                for cx, cy, cz in LOCAL_NODES:
                    f = mesh.lat2free[mesh.lattice_id(i + cx, j + cy, k + cz)]
                    if f >= 0:
                        sets[f].add(g)
    return [tuple(sorted(s)) for s in sets]


def classify(problem, mesh):
    """Grain interiors and interfaces (reading R1)."""
    S = adjacent_sets(problem, mesh)
    n = mesh.n
    node_grain = -np.ones(n, dtype=np.int64)
    for v in range(n):
        if len(S[v]) == 1:
            node_grain[v] = S[v][0]
    # union-find over interface nodes sharing a solid voxel and the same S
    parent = np.arange(n)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    nz, ny, nx = problem.solid.shape
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if not problem.solid[k, j, i]:
                    continue
                corner = []
                for cx, cy, cz in LOCAL_NODES:
                    f = mesh.lat2free[mesh.lattice_id(i + cx, j + cy, k + cz)]
                    if f >= 0 and node_grain[f] < 0:
                        corner.append(int(f))
                for a in corner:
                    for b in corner:
                        if a < b and S[a] == S[b]:
                            ra, rb = find(a), find(b)
                            if ra != rb:
                                parent[max(ra, rb)] = min(ra, rb)
    roots = {}
    for v in range(n):
        if node_grain[v] < 0:
            r = find(v)
            roots.setdefault(r, []).append(v)
    # number interfaces by smallest member
    groups = sorted(roots.values(), key=lambda g: min(g))
    P = Partition()
    P.n_grains = problem.n_grains
    P.node_grain = node_grain
    P.iface_nodes = [np.array(sorted(g), dtype=np.int64) for g in groups]
    P.iface_grains = [S[g[0]] for g in groups]
    P.node_iface = -np.ones(n, dtype=np.int64)
    for c, g in enumerate(P.iface_nodes):
        P.node_iface[g] = c
    P.grain_nodes = [np.flatnonzero(node_grain == i) for i in range(problem.n_grains)]
    P.S = S
    return P


def contact_grids(P, mesh, w):
    """Dilation of each interface by Chebyshev distance w (reading R5)."""
    key = {}
    for v in range(mesh.n):
        key[tuple(mesh.xyz[v])] = v
    out = []
    for nodes in P.iface_nodes:
        sel = set()
        for v in nodes:
            x, y, z = mesh.xyz[v]
            for dz in range(-w, w + 1):
                for dy in range(-w, w + 1):
                    for dx in range(-w, w + 1):
                        u = key.get((x + dx, y + dy, z + dz))
                        if u is not None:
                            sel.add(u)
        out.append(np.array(sorted(sel), dtype=np.int64))
    P.contact_nodes = out
    return out
