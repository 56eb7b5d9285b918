"""Pins of the oracle's decomposition (paper Sec. 3.1-3.2, reading R1/R5)
and mortars (Sec. 3.3, Eqs. 7-8, readings R6-R8)."""
import json
import os

import numpy as np
import pytest

from oracle import fem, mortar, partition
from paper_2509_19777_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def block8():
    p = synth.config_block(8, 8, 8, 4)
    A, b, mesh = fem.assemble(p)
    P = partition.classify(p, mesh)
    return p, A, b, mesh, P


def test_block_partition_matches_hand_count(block8):
    g = json.load(open(os.path.join(GOLD, "partition_block8_box4.json")))
    p, A, b, mesh, P = block8
    assert mesh.n == g["n_free_nodes"]
    assert [len(x) for x in P.grain_nodes] == g["grain_interior_nodes"]
    assert len(P.iface_nodes) == g["n_interfaces"]
    by = {}
    for nodes, S in zip(P.iface_nodes, P.iface_grains):
        by.setdefault(str(len(S)), []).append(len(nodes))
    for k, v in g["interface_sizes_by_grain_count"].items():
        assert sorted(by[k]) == v
    f = g["face_x4_lowest"]
    c = [i for i, S in enumerate(P.iface_grains) if list(S) == f["grains"]][0]
    nodes = P.iface_nodes[c]
    assert len(nodes) == f["n_nodes"]
    idx = mortar.place_mortars(mesh.xyz[nodes], 2)
    assert sorted(idx) == f["farthest_pair_local"]
    assert mesh.xyz[nodes[idx]].tolist() == f["farthest_pair_xyz"]


def test_every_free_node_in_exactly_one_block():
    p = synth.config_pores(16, 4, seed=2)
    A, b, mesh = fem.assemble(p)
    P = partition.classify(p, mesh)
    owner = np.zeros(mesh.n, dtype=int)
    for nodes in P.grain_nodes:
        owner[nodes] += 1
    for nodes in P.iface_nodes:
        owner[nodes] += 1
    assert np.all(owner == 1)
    for nodes, S in zip(P.iface_nodes, P.iface_grains):
        assert len(S) >= 2
        assert all(P.S[v] == S for v in nodes)


def test_grain_blocks_are_decoupled():
    """A_gg is block diagonal (Eq. 20): no stiffness couples interior nodes of
    two different grains."""
    p = synth.config_pores(16, 4, seed=2)
    A, b, mesh = fem.assemble(p)
    P = partition.classify(p, mesh)
    Ac = A.tocoo()
    gi = P.node_grain[Ac.row // 3]
    gj = P.node_grain[Ac.col // 3]
    both = (gi >= 0) & (gj >= 0)
    assert np.all(gi[both] == gj[both])
    # interface nodes only touch grains of their own grain set
    for r, c in zip(Ac.row // 3, Ac.col // 3):
        if P.node_grain[r] >= 0 and P.node_grain[c] < 0:
            assert P.node_grain[r] in P.S[c]


def test_contact_grid_is_dilation(block8):
    p, A, b, mesh, P = block8
    Z = partition.contact_grids(P, mesh, 1)
    for nodes, cz in zip(P.iface_nodes, Z):
        X = mesh.xyz[nodes]
        for v in range(mesh.n):
            d = np.abs(X - mesh.xyz[v]).max(axis=1).min()
            assert (v in set(cz.tolist())) == (d <= 1)
        break  # one interface is enough for the brute force
    assert all(set(P.iface_nodes[c]).issubset(set(Z[c])) for c in range(len(Z)))


def test_gaussian_weights_partition_of_unity_and_values():
    pos = np.array([[x, y, 5] for y in range(5) for x in range(7)])
    idx = mortar.place_mortars(pos, 4)
    H = mortar.gaussian_weights(pos, idx, beta=4.0)
    assert np.allclose(H.sum(axis=1), 1.0, atol=1e-15, rtol=0)
    assert np.all(H > 0)
    # two mortars at distance d: the weight of mortar 0 at its own node is
    # 1 / (1 + exp(-1/beta))  (Eq. 8 with min distance d)
    pos2 = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [3, 0, 0]])
    idx2 = mortar.place_mortars(pos2, 2)
    assert sorted(idx2) == [0, 3]
    H2 = mortar.gaussian_weights(pos2, idx2, beta=4.0)
    assert H2[0, idx2.index(0)] == pytest.approx(1.0 / (1.0 + np.exp(-0.25)), rel=1e-15)
    # midpoint-symmetric node pair gets mirrored weights
    assert H2[1, 0] == pytest.approx(H2[2, 1], rel=1e-15)


def test_plmm_limit_and_identity_limit():
    pos = np.array([[x, y, 0] for y in range(3) for x in range(3)])
    assert np.all(mortar.gaussian_weights(pos, mortar.place_mortars(pos, 1)) == 1.0)
    idx = mortar.place_mortars(pos, 9)
    assert idx == list(range(9))
    assert np.array_equal(mortar.gaussian_weights(pos, idx), np.eye(9))


def test_placement_is_a_fixed_point_of_the_sweep():
    """After placement no single mortar can lower its potential (Eq. 7 sweep)."""
    rng = np.random.default_rng(0)
    pos = np.unique(rng.integers(0, 9, size=(60, 3)), axis=0)
    pos[:, 2] = 0
    pos = np.unique(pos, axis=0)
    for nu in (3, 4, 6):
        idx = mortar.place_mortars(pos, nu)
        assert len(set(idx)) == nu
        for m in range(nu):
            others = idx[:m] + idx[m + 1:]
            cur = sum(1.0 / np.linalg.norm(pos[idx[m]] - pos[j]) for j in others)
            for y in range(len(pos)):
                if y in others:
                    continue
                val = sum(1.0 / np.linalg.norm(pos[y] - pos[j]) for j in others)
                assert val >= cur * (1 - 1e-9)
