"""Oracle for the learned basis surrogate.  TEST INFRASTRUCTURE ONLY.

The surrogate is a small 3D convolutional network on the 9 x 9 x 9 node
lattice of an 8^3-voxel box subdomain.  For one sample = (grain, interface c,
mortar a) it maps four input channels per node

    0  1 on the grain's interior nodes, else 0
    1  log of the trace of the node's diagonal 3x3 block of A, minus its mean
       over the grain's interior nodes (a stiffness proxy: the trace is
       proportional to the sum of E over the node's solid voxels), 0 elsewhere
    2  (stored 3x3 blocks in the node's row of A) / 27 on interior and
       interface nodes (a fill proxy), 0 elsewhere
    3  the Gaussian weight H_c[row(v), a] on the nodes v of interface c
       (the mortar mode's boundary trace, Eq. 8), 0 elsewhere

to nine output channels: the shape vectors of the three components gamma of
that mortar node, p_k = -A_gi^-1 Abar_gi,m e_k with k = 3a + gamma (Eq. 23,
the grain-interior response to the boundary displacement H_c[., a] e_gamma),
written at the interior nodes as (u_x, u_y, u_z) for gamma = x, y, z.

Network: four 3x3x3 'same' convolutions (zero padding) with bias; ReLU after
the first three.  Loss: the mean over samples of the masked squared error of
the nine outputs on interior nodes divided by the masked squared norm of the
target (plus 1e-30).

Everything is float64 NumPy written from the definitions: a convolution is
the sum over the 27 kernel offsets of shifted channel products; gradients
follow from the chain rule.  Pinned in tests by central finite differences
(an independent route to the same derivative), a delta kernel (identity), a
shifted delta (shift with zero fill), and linearity.
"""
from __future__ import annotations

import numpy as np

G = 9                 # nodes per side of an 8^3-voxel box
N_IN, N_OUT = 4, 9
CHANNELS = (N_IN, 32, 32, 32, N_OUT)
OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def init_params(rng, channels=CHANNELS, scale=1.0):
    """He-style initial weights w[l]: (3, 3, 3, cin, cout), biases zero."""
    params = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        std = scale * np.sqrt(2.0 / (27 * cin))
        params.append((rng.standard_normal((3, 3, 3, cin, cout)) * std, np.zeros(cout)))
    return params


def _shift(x, dz, dy, dx):
    """y[s, z, y, x, :] = x[s, z+dz, y+dy, x+dx, :], zero outside the grid."""
    out = np.zeros_like(x)
    n = x.shape[1]
    zs, ys, xs = slice(max(0, -dz), n - max(0, dz)), slice(max(0, -dy), n - max(0, dy)), slice(max(0, -dx), n - max(0, dx))
    zs2, ys2, xs2 = slice(max(0, dz), n - max(0, -dz)), slice(max(0, dy), n - max(0, -dy)), slice(max(0, dx), n - max(0, -dx))
    out[:, zs, ys, xs, :] = x[:, zs2, ys2, xs2, :]
    return out


def conv3d(x, w, b):
    """out[s, p, co] = b[co] + sum_{offset d, ci} w[d, ci, co] x[s, p + d, ci]."""
    out = np.zeros(x.shape[:4] + (w.shape[-1],))
    for dz, dy, dx in OFFSETS:
        out += _shift(x, dz, dy, dx) @ w[dz + 1, dy + 1, dx + 1]
    return out + b


def conv3d_backward(x, w, gout):
    """Gradients of sum(gout * conv3d(x, w, b)) w.r.t. x, w and b."""
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for dz, dy, dx in OFFSETS:
        xs = _shift(x, dz, dy, dx)
        gw[dz + 1, dy + 1, dx + 1] = np.einsum("szyxi,szyxo->io", xs, gout)
        # x[p + d] feeds out[p]: the adjoint shifts back by -d
        gx += _shift(gout @ w[dz + 1, dy + 1, dx + 1].T, -dz, -dy, -dx)
    gb = gout.sum(axis=(0, 1, 2, 3))
    return gx, gw, gb


def forward(params, x):
    """Returns the list of layer outputs (after ReLU for hidden layers)."""
    acts = [x]
    for l, (w, b) in enumerate(params):
        z = conv3d(acts[-1], w, b)
        acts.append(np.maximum(z, 0.0) if l < len(params) - 1 else z)
    return acts


def forward_bf16(params, x):
    """The inference the GPU runs with bfloat16 operands: every layer's input
    activations and weights rounded to bfloat16 (to nearest even, via
    float32), the convolution summed exactly (FP64 here), the float32 bias
    added, ReLU on hidden layers.  Returns the last layer's output."""
    from .precision import round_bf16, round_f32
    a = x
    for l, (w, b) in enumerate(params):
        z = conv3d(round_bf16(a), round_bf16(w), round_f32(b))
        a = np.maximum(z, 0.0) if l < len(params) - 1 else z
    return a


def loss(pred, y, mask):
    """Mean over samples of |m (pred - y)|^2 / (|m y|^2 + 1e-30)."""
    m = mask[..., None]
    num = (((pred - y) * m) ** 2).sum(axis=(1, 2, 3, 4))
    den = ((y * m) ** 2).sum(axis=(1, 2, 3, 4)) + 1e-30
    return float((num / den).mean())


def loss_grad(pred, y, mask):
    m = mask[..., None]
    den = ((y * m) ** 2).sum(axis=(1, 2, 3, 4)) + 1e-30
    return 2.0 * (pred - y) * m * m / (den[:, None, None, None, None] * pred.shape[0])


def backward(params, acts, gpred):
    """Gradients of the loss w.r.t. every (w, b), given d loss / d output."""
    grads = [None] * len(params)
    g = gpred
    for l in range(len(params) - 1, -1, -1):
        w, _ = params[l]
        if l < len(params) - 1:
            g = g * (acts[l + 1] > 0.0)
        gx, gw, gb = conv3d_backward(acts[l], w, g)
        grads[l] = (gw, gb)
        g = gx
    return grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected); state = {'t': int, 'm': [...], 'v': [...]}."""
    state["t"] += 1
    t = state["t"]
    out = []
    for i, ((w, b), (gw, gb)) in enumerate(zip(params, grads)):
        new = []
        for j, (p, g) in enumerate(((w, gw), (b, gb))):
            k = 2 * i + j
            state["m"][k] = beta1 * state["m"][k] + (1 - beta1) * g
            state["v"][k] = beta2 * state["v"][k] + (1 - beta2) * g * g
            mh = state["m"][k] / (1 - beta1 ** t)
            vh = state["v"][k] / (1 - beta2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
        out.append(tuple(new))
    return out


# ---- features of a box grain from the assembled system --------------------------------
def grain_features(A, node_xyz, interior_nodes, iface_nodes_list, origin, row_nnzb=None):
    """Channels 0-2 of every sample of one grain on its 9^3 lattice.

    A: scipy CSR of the free dofs (node-major, 3 dofs per node);
    interior_nodes: the grain's interior node ids; iface_nodes_list: node id
    arrays of the grain's adjacent interfaces; origin: lattice coordinates of
    the box's lowest corner.  Returns (G, G, G, 3) float64.
    """
    A = A.tocsr()
    f = np.zeros((G, G, G, 3))
    diag = A.diagonal()
    tr = {v: diag[3 * v] + diag[3 * v + 1] + diag[3 * v + 2] for v in interior_nodes}
    logs = np.array([np.log(tr[v]) for v in interior_nodes])
    mean = logs.mean() if len(logs) else 0.0
    if row_nnzb is None:
        # stored blocks of node row v = distinct neighbour nodes in dof row 3v
        indptr, indices = A.indptr, A.indices
        row_nnzb = lambda v: float(len(np.unique(indices[indptr[3 * v]:indptr[3 * v + 1]] // 3)))
    for v, lv in zip(interior_nodes, logs):
        x, y, z = (int(t) for t in node_xyz[v] - origin)
        f[z, y, x, 0] = 1.0
        f[z, y, x, 1] = lv - mean
        f[z, y, x, 2] = row_nnzb(v) / 27.0
    for nodes in iface_nodes_list:
        for v in nodes:
            x, y, z = (int(t) for t in node_xyz[v] - origin)
            f[z, y, x, 2] = row_nnzb(v) / 27.0
    return f


# ---- features of every sample and the Galerkin product with predicted shape vectors --
def sample_inputs(H, A, mesh, g, c, a):
    """Network input (9, 9, 9, 4) of sample (grain g, interface c, mortar a) of
    an oracle HPLMM object H (channels as in the module docstring)."""
    P = H.part
    nodes = P.grain_nodes[g]
    adj = coupled_interfaces(A, P, g)
    origin = (mesh.xyz[nodes].min(axis=0) // 8) * 8
    x = np.zeros((G, G, G, N_IN))
    x[..., :3] = grain_features(A, mesh.xyz, nodes, [P.iface_nodes[q] for q in adj], origin)
    for row, v in enumerate(P.iface_nodes[c]):
        i, j, k = mesh.xyz[v] - origin
        x[k, j, i, 3] = P.H[c][row, a]
    return x, origin


def coupled_interfaces(A, P, g):
    """Interfaces with a node coupled to grain g's interior through A, ascending."""
    A = A.tocsr()
    out = set()
    for v in P.grain_nodes[g]:
        for w in A.indices[A.indptr[3 * v]:A.indptr[3 * v + 1]] // 3:
            if P.node_iface[w] >= 0:
                out.add(int(P.node_iface[w]))
    return sorted(out)


def predicted_blocks(H, A, mesh, params, grains):
    """Shape-vector blocks B~_g (rows: the grain's dofs, columns: the global
    mortar dofs of its coupled interfaces, ascending) predicted by the network
    for the given grains."""
    P = H.part
    out = {}
    for g in grains:
        nodes = P.grain_nodes[g]
        cols, blocks = [], []
        for c in coupled_interfaces(A, P, g):
            for a in range(P.H[c].shape[1]):
                x, origin = sample_inputs(H, A, mesh, g, c, a)
                y = forward(params, x[None])[-1][0]
                for gm in range(3):
                    col = np.zeros(3 * len(nodes))
                    for li, v in enumerate(nodes):
                        i, j, k = mesh.xyz[v] - origin
                        col[3 * li:3 * li + 3] = y[k, j, i, 3 * gm:3 * gm + 3]
                    cols.append(H.moff[c] + 3 * a + gm)
                    blocks.append(col)
        out[g] = (np.asarray(cols), np.stack(blocks, axis=1))
    return out


def galerkin_mortar_block(H, blocks):
    """Mortar block of P~^T A_M P~ (Eq. 18 with P = [B; I], A_M = Q^T W^T A W Q),
    B taken from `blocks` for the grains it holds and exact for the others."""
    import scipy.sparse as sp
    Ngf, Nmo = H.Ngf, H.Nmo
    rows, cols, vals = [], [], []
    for g, off in enumerate(H.goff):
        if g in blocks:
            cg, Bg = blocks[g]
        elif H.B_blocks[g] is not None:
            cg, Bg = H.B_blocks[g]
        else:
            continue
        r = np.repeat(np.arange(off, off + Bg.shape[0]), cg.size)
        rows.append(r)
        cols.append(np.tile(cg, Bg.shape[0]))
        vals.append(Bg.ravel())
    B = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(Ngf, Nmo))
    Pm = sp.vstack([B, sp.identity(Nmo, format="csr")]).tocsr()
    AM = (H.Q.T @ (H.W.T @ H.A @ H.W) @ H.Q).tocsr()
    return (Pm.T @ AM @ Pm).toarray()
