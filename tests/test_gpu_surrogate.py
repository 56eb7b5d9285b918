"""GPU surrogate network (HIP kernels through the C ABI) against the float64
oracle: forward outputs, loss, every parameter gradient and one Adam step.

Tolerances: float32 arithmetic with float32 accumulation over at most
27 x 32 = 864 products per output (forward) and 729 x n x 27 products per
weight gradient; normwise relative error bounds 2e-5 (forward, loss) and
2e-4 (gradients) leave a wide margin over the ~1e-6 expected."""
import numpy as np
import pytest

from oracle import surrogate as osg

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _case(channels, n, seed):
    rng = np.random.default_rng(seed)
    params = osg.init_params(rng, channels)
    params = [(w, 0.1 * rng.standard_normal(b.shape)) for w, b in params]
    x = rng.standard_normal((n, 9, 9, 9, channels[0]))
    x[..., 0] = (rng.random((n, 9, 9, 9)) < 0.6).astype(float)
    y = rng.standard_normal((n, 9, 9, 9, channels[-1]))
    return params, x, y


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


@pytest.mark.parametrize("channels,n", [((4, 8, 8, 8, 9), 3), ((4, 32, 32, 32, 9), 2), ((4, 5, 17, 3, 9), 1)])
def test_forward_matches_oracle(channels, n):
    torch = _torch()
    from paper_2509_19777_amd import hplmm as hp
    params, x, y = _case(channels, n, 1)
    net = hp.SurrogateNet(channels, max_batch=4)
    net.set_params(hp.flatten_params(params))
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    out = net.forward(xt).cpu().numpy().astype(np.float64)
    ref = osg.forward(params, x)[-1]
    assert _rel(out, ref) <= 2e-5


@pytest.mark.parametrize("channels,n", [((4, 8, 8, 8, 9), 3), ((4, 32, 32, 32, 9), 2), ((4, 5, 17, 3, 9), 1)])
def test_bf16_inference_matches_emulation(channels, n):
    # bfloat16 operands on the matrix cores against the oracle's emulation
    # (each layer's inputs and weights rounded to bfloat16, exact sums): the
    # first layer differs only by FP32 summation (<= 864 u32 of the
    # magnitudes), later layers also where the two sides' activations straddle
    # a bfloat16 rounding boundary (a fraction ~1e-3 of the entries, one
    # ulp = 2^-8 each): ~1e-3 expected, bar 1e-2
    torch = _torch()
    from paper_2509_19777_amd import hplmm as hp
    params, x, y = _case(channels, n, 2)
    net = hp.SurrogateNet(channels, max_batch=4)
    net.set_params(hp.flatten_params(params))
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    out32 = net.forward(xt).cpu().numpy().astype(np.float64)
    net.set_inference_precision(16)
    out16 = net.forward(xt).cpu().numpy().astype(np.float64)
    p32 = [(w.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for w, b in params]
    ref = osg.forward_bf16(p32, x.astype(np.float32).astype(np.float64))
    print(f"bf16 inference {channels}: {_rel(out16, ref):.2e} from the emulation, {_rel(out16, out32):.2e} from FP32")
    assert _rel(out16, ref) <= 1e-2
    assert _rel(out16, out32) > 1e-5          # the operands really are rounded
    net.set_inference_precision(32)
    assert np.array_equal(net.forward(xt).cpu().numpy().astype(np.float64), out32)
    with pytest.raises(hp.HplmmError):
        net.set_inference_precision(8)


@pytest.mark.parametrize("channels,n", [((4, 8, 8, 8, 9), 3), ((4, 32, 32, 32, 9), 2)])
def test_gradients_match_oracle(channels, n):
    torch = _torch()
    from paper_2509_19777_amd import hplmm as hp
    params, x, y = _case(channels, n, 2)
    net = hp.SurrogateNet(channels, max_batch=n)
    net.set_params(hp.flatten_params(params))
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    yt = torch.from_numpy(y.astype(np.float32)).cuda()
    loss = net.gradient(xt, yt)
    acts = osg.forward(params, x)
    mask = (x[..., 0] > 0.5).astype(float)
    ref_loss = osg.loss(acts[-1], y, mask)
    assert abs(loss - ref_loss) <= 2e-5 * ref_loss
    ref = osg.backward(params, acts, osg.loss_grad(acts[-1], y, mask))
    got = hp.unflatten_params(net.get_grads(), channels)
    for l, ((gw, gb), (rw, rb)) in enumerate(zip(got, ref)):
        assert _rel(gw, rw) <= 2e-4, (l, _rel(gw, rw))
        assert _rel(gb, rb) <= 2e-4, (l, _rel(gb, rb))


def test_adam_step_matches_oracle():
    torch = _torch()
    from paper_2509_19777_amd import hplmm as hp
    channels = (4, 8, 8, 8, 9)
    params, x, y = _case(channels, 2, 3)
    net = hp.SurrogateNet(channels, max_batch=2)
    net.set_params(hp.flatten_params(params))
    net.gradient(torch.from_numpy(x.astype(np.float32)).cuda(), torch.from_numpy(y.astype(np.float32)).cuda())
    lr = 1e-3
    net.adam(lr)
    got = net.get_params()
    acts = osg.forward(params, x)
    mask = (x[..., 0] > 0.5).astype(float)
    grads = osg.backward(params, acts, osg.loss_grad(acts[-1], y, mask))
    st = {"t": 0, "m": [0.0] * 8, "v": [0.0] * 8}
    ref = hp.flatten_params(osg.adam_step(params, grads, st, lr)).astype(np.float64)
    g = hp.flatten_params(grads).astype(np.float64)
    p0 = hp.flatten_params(params).astype(np.float64)
    # the first step is -lr g / (|g| + eps): compare where the gradient is not tiny (sign-stable)
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    assert np.all(np.abs(got[big] - ref[big]) <= 1e-3 * lr + 1e-6 * np.abs(p0[big]))
    assert np.all(np.abs(got - p0) <= 1.01 * lr + 1e-6 * np.abs(p0))


def test_bad_arguments_raise():
    _torch()
    from paper_2509_19777_amd import hplmm as hp
    with pytest.raises(hp.HplmmError):
        hp.SurrogateNet((4, 33, 8, 8, 9))
    net = hp.SurrogateNet((4, 8, 8, 8, 9), max_batch=2)
    with pytest.raises(hp.HplmmError):
        net.set_params(np.zeros(net.n_params + 1, dtype=np.float32))


@pytest.fixture(scope="module")
def small_problem():
    torch = _torch()
    from oracle import fem, hplmm as oh
    from paper_2509_19777_amd import hplmm as hp, synth
    p = synth.config_pores_lognormal(16, 8, seed=3, n_mortar=2)
    A, b, mesh = fem.assemble(p)
    H = oh.HPLMM(p, A=A, b=b, mesh=mesh, n=2)
    sysm, part = hp.build_problem(p)
    S = hp.Solver(sysm, part, n_mortar=2)
    S.setup()
    torch.cuda.synchronize()
    return p, A, mesh, H, S


def test_samples_match_oracle_features_and_basis(small_problem):
    from paper_2509_19777_amd import hplmm as hp
    p, A, mesh, H, S = small_problem
    x, y, meta = hp.surrogate_samples(S)
    x, y = x.cpu().numpy().astype(np.float64), y.cpu().numpy().astype(np.float64)
    P = H.part
    grains = [g for g in range(len(P.grain_nodes)) if len(P.grain_nodes[g])]
    assert x.shape[0] == sum(
        sum(P.H[c].shape[1] for c in np.unique(P.node_iface[_coupled(A, P, g)])) for g in grains)
    checked = 0
    for s, (m, c, a) in enumerate(meta):
        g = grains[m]
        nodes = P.grain_nodes[g]
        adj = np.unique(P.node_iface[_coupled(A, P, g)])
        origin = (mesh.xyz[nodes].min(axis=0) // 8) * 8
        f = osg.grain_features(A, mesh.xyz, nodes, [P.iface_nodes[q] for q in adj], origin)
        assert np.array_equal(x[s, ..., 0], f[..., 0])
        assert np.allclose(x[s, ..., 1], f[..., 1], rtol=0, atol=2e-6)
        assert np.allclose(x[s, ..., 2], f[..., 2], rtol=0, atol=1e-7)
        ref3 = np.zeros((9, 9, 9))
        for row, v in enumerate(P.iface_nodes[c]):
            i, j, k = mesh.xyz[v] - origin
            ref3[k, j, i] = P.H[c][row, a]
        assert np.allclose(x[s, ..., 3], ref3, rtol=0, atol=1e-7)
        # targets: the shape vectors B e_k for the global mortar dofs moff_c + 3a + gamma
        cols, Bi = H.B_blocks[g]
        for gm in range(3):
            k = H.moff[c] + 3 * a + gm
            col = Bi[:, np.flatnonzero(cols == k)[0]] if np.any(cols == k) else np.zeros(3 * len(nodes))
            ref = np.zeros((9, 9, 9, 3))
            for li, v in enumerate(nodes):
                i, j, kk = mesh.xyz[v] - origin
                ref[kk, j, i] = col[3 * li:3 * li + 3]
            got = y[s, ..., 3 * gm:3 * gm + 3]
            assert np.abs(got - ref).max() <= 1e-6 * max(1.0, np.abs(ref).max())
        checked += 1
    assert checked == x.shape[0] > 0


def _coupled(A, P, g):
    """Interface nodes coupled to grain g's interior through A."""
    A = A.tocsr()
    nodes = P.grain_nodes[g]
    nb = set()
    for v in nodes:
        cols = A.indices[A.indptr[3 * v]:A.indptr[3 * v + 1]] // 3
        nb.update(int(w) for w in cols if P.node_iface[w] >= 0)
    return np.array(sorted(nb), dtype=np.int64)


def _random_net(channels=(4, 8, 8, 8, 9), scale=0.3, seed=12):
    """A network with seeded random weights (drawn here, in the test)."""
    from paper_2509_19777_amd import hplmm as hp
    rng = np.random.default_rng(seed)
    params = []
    for ci, co in zip(channels[:-1], channels[1:]):
        params.append((rng.standard_normal((3, 3, 3, ci, co)) * scale / np.sqrt(27 * ci),
                       0.01 * rng.standard_normal(co)))
    net = hp.SurrogateNet(channels, max_batch=64)
    net.set_params(hp.flatten_params(params))
    return net, params


def test_surrogate_setup_with_zero_threshold_is_the_exact_setup(small_problem):
    p, A, mesh, H, S = small_problem
    ref = S.coarse_matrix().copy()
    net, _ = _random_net()
    st = S.setup_surrogate(net, 0.0)
    assert st["accepted"] == 0 and st["fallback"] == st["grains"] > 0
    got = S.coarse_matrix()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    S.setup()   # leave the fixture's solver in its exact state


def test_surrogate_galerkin_block_matches_oracle(small_problem):
    p, A, mesh, H, S = small_problem
    net, params = _random_net()
    st = S.setup_surrogate(net, 1e300)
    loaded = {g for g in H.corr_grains}
    grains = [g for g in range(len(H.B_blocks)) if H.B_blocks[g] is not None and g not in loaded]
    assert st["accepted"] == len(grains) and st["fallback"] == st["loaded"]
    blocks = osg.predicted_blocks(H, A, mesh, params, grains)
    ref = osg.galerkin_mortar_block(H, blocks)
    got = S.coarse_matrix()[:H.Nmo, :H.Nmo]
    assert np.abs(got - ref).max() <= 1e-4 * np.abs(ref).max(), np.abs(got - ref).max() / np.abs(ref).max()
    # the correction pivots stay exact
    nc = len(H.corr_grains)
    if nc:
        assert np.allclose(np.diag(S.coarse_matrix())[H.Nmo:], np.diag(H.Acoarse)[H.Nmo:], rtol=1e-12, atol=0)
    # the preconditioner stays SPD: FGMRES still reaches the FP64 tolerance
    x, info = S.solve(rtol=1e-8, restart=50, maxit=300)
    assert info["status"] == "OK"
    assert np.linalg.norm(p_rhs(S) - A @ x.cpu().numpy()) <= 1e-8 * np.linalg.norm(p_rhs(S))
    S.setup()


def p_rhs(S):
    return S.b.cpu().numpy()
