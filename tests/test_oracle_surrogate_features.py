"""Pins of the surrogate oracle's input features (`grain_features`,
`sample_inputs`, `coupled_interfaces`), CPU only.

Two independent routes to the same channels:

* hand-derived values on a full 16^3 block with 8^3 boxes
  (`tests/golden/surrogate_features_block16_box8.json`, derivation inside):
  interior masks, voxel counts behind the log-trace channel, neighbour counts
  behind the fill channel, the coupled interfaces of a corner grain, and the
  mortar channel placed at the interface's lattice points (n = 1, where every
  Gaussian weight is 1, Eq. 8);
* on a porous block with a lognormal modulus, the channels recomputed from
  the voxel geometry alone: the trace of a node's diagonal 3x3 block is
  t0 * sum of E over the solid voxels touching it (every element matrix is
  E Khat(nu) and the trace of Khat's corner blocks is the same for all eight
  corners), so the log-trace channel is log(sum E) minus its grain mean; the
  stored blocks of a node row are the free nodes that share a solid voxel
  with the node (the Q1 assembly pattern of Eq. 4).

A wrong lattice origin, a swapped axis or channel, a wrong neighbour count or a
dropped interface fails one of them.
"""
import json
import os
import types

import numpy as np
import pytest

from oracle import fem, mortar as mortar_mod, partition as part_mod, surrogate as sg
from paper_2509_19777_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "surrogate_features_block16_box8.json")


def _setup(problem, n):
    A, b, mesh = fem.assemble(problem)
    P = part_mod.classify(problem, mesh)
    mortar_mod.build_mortars(P, mesh, n, problem.beta)
    return A.tocsr(), mesh, P


@pytest.fixture(scope="module")
def block16():
    p = synth.config_block(16, 16, 16, 8, n_mortar=1)
    A, mesh, P = _setup(p, 1)
    return p, A, mesh, P, json.load(open(GOLD))


def _grain_of_box(problem, mesh, P, origin):
    i, j, k = origin
    lab = int(problem.labels[k, j, i])
    return lab


def test_block16_interior_and_log_trace(block16):
    p, A, mesh, P, gold = block16
    for key in ("grain0", "grain7"):
        g = gold[key]
        o = np.array(g["origin"])
        gi = _grain_of_box(p, mesh, P, o)
        nodes = P.grain_nodes[gi]
        assert len(nodes) == g["n_interior"]
        adj = sg.coupled_interfaces(A, P, gi)
        f = sg.grain_features(A, mesh.xyz, nodes, [P.iface_nodes[q] for q in adj], o)
        assert f.shape == (sg.G, sg.G, sg.G, 3)
        # channel 0: exactly the interior lattice points, indexed [z, y, x]
        ch0 = np.zeros((sg.G,) * 3)
        top = 16
        for (i, j, k) in mesh.xyz[nodes]:
            ch0[k - o[2], j - o[1], i - o[0]] = 1.0
        assert np.array_equal(f[..., 0], ch0)
        assert f[..., 0].sum() == g["n_interior"]
        # channel 1 from the voxel count m of each interior node
        by_m = {int(k): v for k, v in g["channel1_by_m"].items()}
        for (i, j, k) in mesh.xyz[nodes]:
            m = 1
            for c, lo in ((i, o[0]), (j, o[1]), (k, o[2])):
                m *= 1 if (c == 0 or c == top) else 2
            assert abs(f[k - o[2], j - o[1], i - o[0], 1] - by_m[m]) <= 1e-12
        # channel 1 vanishes off the interior
        assert np.all(f[..., 1][ch0 == 0] == 0.0)


def test_block16_fill_channel(block16):
    p, A, mesh, P, gold = block16
    g = gold["grain0"]
    gi = _grain_of_box(p, mesh, P, g["origin"])
    adj = sg.coupled_interfaces(A, P, gi)
    f = sg.grain_features(A, mesh.xyz, P.grain_nodes[gi], [P.iface_nodes[q] for q in adj], np.zeros(3, int))
    for s in g["channel2_spot"]:
        i, j, k = s["ijk"]
        assert abs(f[k, j, i, 2] - s["value"]) <= 1e-15, s
    # the whole channel from the per-axis counts: 3 neighbours per axis, 2 on
    # the faces i = 0, j = 0 and at k = 1 (its k = 0 neighbours are clamped)
    cnt = lambda c, lo_clamped: (2 if c == 0 else 3) if not lo_clamped else (2 if c == 1 else 3)
    covered = 0
    for nodes in [P.grain_nodes[gi]] + [P.iface_nodes[q] for q in adj]:
        for (i, j, k) in mesh.xyz[nodes]:
            if max(i, j, k) > 8:
                continue
            ref = cnt(i, False) * cnt(j, False) * cnt(k, True) / 27.0
            assert abs(f[k, j, i, 2] - ref) <= 1e-15
            covered += 1
    # every lattice point of the 9^3 window above the clamped plane is either
    # interior to grain 0 or on one of its coupled interfaces
    assert covered == 9 * 9 * 8
    assert np.all(f[0, :, :, 2] == 0.0)   # the clamped plane holds no free node


def test_block16_coupled_interfaces(block16):
    p, A, mesh, P, gold = block16
    g = gold["grain0"]
    gi = _grain_of_box(p, mesh, P, g["origin"])
    adj = sg.coupled_interfaces(A, P, gi)
    sets = sorted([sorted(P.iface_grains[c]) for c in adj], key=lambda s: (len(s), s))
    want = sorted(g["coupled_grain_sets"], key=lambda s: (len(s), s))
    assert sets == want
    assert adj == sorted(adj)
    face = next(c for c in adj if sorted(P.iface_grains[c]) == [0, 1])
    assert len(P.iface_nodes[face]) == g["face01_nodes"]


def test_block16_mortar_channel_at_n1(block16):
    # n = 1: H_c = 1 on every node of interface c (Eq. 8), so channel 3 is the
    # indicator of the interface's lattice points in the grain's window
    p, A, mesh, P, gold = block16
    g = gold["grain0"]
    gi = _grain_of_box(p, mesh, P, g["origin"])
    H = types.SimpleNamespace(part=P)
    for c in sg.coupled_interfaces(A, P, gi):
        assert P.H[c].shape[1] == 1 and np.all(P.H[c] == 1.0)
        x, origin = sg.sample_inputs(H, A, mesh, gi, c, 0)
        assert np.array_equal(origin, np.zeros(3))
        ind = np.zeros((sg.G,) * 3)
        for (i, j, k) in mesh.xyz[P.iface_nodes[c]]:
            ind[k, j, i] = 1.0
        assert np.array_equal(x[..., 3], ind)
    # the {0, 1} face sits on the plane i = 8: x index 8, y 0..7, z 1..7
    face = next(c for c in sg.coupled_interfaces(A, P, gi) if sorted(P.iface_grains[c]) == [0, 1])
    x, _ = sg.sample_inputs(H, A, mesh, gi, face, 0)
    assert x[1:8, 0:8, 8, 3].sum() == 56 and x[..., 3].sum() == 56


@pytest.fixture(scope="module")
def porous():
    p = synth.config_pores_lognormal(16, 8, seed=5, n_mortar=2)
    A, mesh, P = _setup(p, 2)
    return p, A, mesh, P


def _geometry_channels(p, mesh, nodes, origin):
    """Channels 1 and 2 at the given nodes from the voxel grid alone."""
    nz, ny, nx = p.solid.shape
    out1, out2 = {}, {}
    for v in nodes:
        i, j, k = (int(t) for t in mesh.xyz[v])
        esum = 0.0
        neigh = set()
        for dk in (-1, 0):
            for dj in (-1, 0):
                for di in (-1, 0):
                    a, bb, c = i + di, j + dj, k + dk
                    if not (0 <= a < nx and 0 <= bb < ny and 0 <= c < nz) or not p.solid[c, bb, a]:
                        continue
                    esum += p.E[c, bb, a]
                    for ck in (0, 1):
                        for cj in (0, 1):
                            for ci in (0, 1):
                                w = mesh.lat2free[mesh.lattice_id(a + ci, bb + cj, c + ck)]
                                if w >= 0:
                                    neigh.add(int(w))
        out1[v] = np.log(esum)
        out2[v] = len(neigh) / 27.0
    return out1, out2


def test_porous_channels_from_voxel_geometry(porous):
    p, A, mesh, P = porous
    checked = 0
    for gi, nodes in enumerate(P.grain_nodes):
        if len(nodes) < 20:
            continue
        origin = (mesh.xyz[nodes].min(axis=0) // 8) * 8
        adj = sg.coupled_interfaces(A, P, gi)
        ifn = [P.iface_nodes[q] for q in adj]
        f = sg.grain_features(A, mesh.xyz, nodes, ifn, origin)
        l1, c2 = _geometry_channels(p, mesh, list(nodes) + [v for q in ifn for v in q], origin)
        mean = np.mean([l1[v] for v in nodes])
        for v in nodes:
            i, j, k = mesh.xyz[v] - origin
            assert f[k, j, i, 0] == 1.0
            assert abs(f[k, j, i, 1] - (l1[v] - mean)) <= 1e-12
            assert abs(f[k, j, i, 2] - c2[v]) <= 1e-15
        for q in ifn:
            for v in q:
                i, j, k = mesh.xyz[v] - origin
                if max(i, j, k) < sg.G and min(i, j, k) >= 0:
                    assert f[k, j, i, 0] == 0.0 and f[k, j, i, 1] == 0.0
                    assert abs(f[k, j, i, 2] - c2[v]) <= 1e-15
        checked += 1
    assert checked >= 4


def test_porous_coupled_interfaces_by_voxels(porous):
    # an interface is coupled to grain g exactly when one of its nodes is a
    # corner of a solid voxel that also has an interior node of g as a corner
    p, A, mesh, P = porous
    nz, ny, nx = p.solid.shape
    for gi, nodes in enumerate(P.grain_nodes):
        if len(nodes) == 0:
            continue
        want = set()
        interior = set(int(v) for v in nodes)
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    if not p.solid[k, j, i]:
                        continue
                    corners = [mesh.lat2free[mesh.lattice_id(i + ci, j + cj, k + ck)]
                               for ck in (0, 1) for cj in (0, 1) for ci in (0, 1)]
                    corners = [int(c) for c in corners if c >= 0]
                    if any(c in interior for c in corners):
                        want.update(int(P.node_iface[c]) for c in corners if P.node_iface[c] >= 0)
        assert sg.coupled_interfaces(A, P, gi) == sorted(want)


def test_porous_mortar_channel_is_the_weight_column(porous):
    # channel 3 of sample (g, c, a) holds column a of H_c at interface c's
    # lattice points and nothing else; the weights of a node sum to 1 over a
    # (partition of unity, Eq. 8)
    p, A, mesh, P = porous
    H = types.SimpleNamespace(part=P)
    gi = max(range(len(P.grain_nodes)), key=lambda g: len(P.grain_nodes[g]))
    for c in sg.coupled_interfaces(A, P, gi)[:6]:
        tot = np.zeros((sg.G,) * 3)
        for a in range(P.H[c].shape[1]):
            x, origin = sg.sample_inputs(H, A, mesh, gi, c, a)
            ref = np.zeros((sg.G,) * 3)
            for row, v in enumerate(P.iface_nodes[c]):
                i, j, k = mesh.xyz[v] - origin
                ref[k, j, i] = P.H[c][row, a]
            assert np.array_equal(x[..., 3], ref)
            tot += x[..., 3]
        for v in P.iface_nodes[c]:
            i, j, k = mesh.xyz[v] - origin
            assert abs(tot[k, j, i] - 1.0) <= 1e-14
