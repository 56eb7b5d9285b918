"""Pins of the surrogate oracle (network algebra and features), CPU only."""
import numpy as np
import pytest

from oracle import surrogate as sg


def _rng(seed=0):
    return np.random.default_rng(seed)


def test_delta_kernel_is_identity():
    rng = _rng(1)
    x = rng.standard_normal((2, 5, 5, 5, 3))
    w = np.zeros((3, 3, 3, 3, 3))
    w[1, 1, 1] = np.eye(3)
    assert np.array_equal(sg.conv3d(x, w, np.zeros(3)), x)


@pytest.mark.parametrize("d", [(1, 0, 0), (0, -1, 1), (-1, 1, -1)])
def test_shifted_delta_shifts_with_zero_fill(d):
    rng = _rng(2)
    x = rng.standard_normal((1, 4, 4, 4, 2))
    w = np.zeros((3, 3, 3, 2, 2))
    w[d[0] + 1, d[1] + 1, d[2] + 1] = np.eye(2)
    out = sg.conv3d(x, w, np.zeros(2))
    n = 4
    for z in range(n):
        for y in range(n):
            for xx in range(n):
                zz, yy, x2 = z + d[0], y + d[1], xx + d[2]
                inside = 0 <= zz < n and 0 <= yy < n and 0 <= x2 < n
                ref = x[0, zz, yy, x2] if inside else np.zeros(2)
                assert np.array_equal(out[0, z, y, xx], ref)


def test_conv_is_linear_in_input_and_bias_adds():
    rng = _rng(3)
    x1, x2 = rng.standard_normal((2, 1, 4, 4, 4, 3))
    w = rng.standard_normal((3, 3, 3, 3, 2))
    b = rng.standard_normal(2)
    lhs = sg.conv3d(2.0 * x1 - 0.5 * x2, w, np.zeros(2))
    rhs = 2.0 * sg.conv3d(x1, w, np.zeros(2)) - 0.5 * sg.conv3d(x2, w, np.zeros(2))
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-12)
    assert np.allclose(sg.conv3d(x1, w, b) - sg.conv3d(x1, w, np.zeros(2)), b, atol=1e-12)


def _tiny():
    rng = _rng(4)
    ch = (2, 3, 3, 2)
    params = sg.init_params(rng, ch)
    params = [(w, rng.standard_normal(b.shape) * 0.1) for w, b in params]
    x = rng.standard_normal((2, 4, 4, 4, 2))
    y = rng.standard_normal((2, 4, 4, 4, 2))
    mask = (rng.random((2, 4, 4, 4)) < 0.7).astype(float)
    return params, x, y, mask


def _loss_of(params, x, y, mask):
    return sg.loss(sg.forward(params, x)[-1], y, mask)


def test_gradients_match_central_differences():
    params, x, y, mask = _tiny()
    acts = sg.forward(params, x)
    grads = sg.backward(params, acts, sg.loss_grad(acts[-1], y, mask))
    rng = _rng(5)
    h = 1e-6
    for l, (w, b) in enumerate(params):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in w.shape)
            wp, wm = w.copy(), w.copy()
            wp[idx] += h
            wm[idx] -= h
            pp = list(params); pp[l] = (wp, b)
            pm = list(params); pm[l] = (wm, b)
            fd = (_loss_of(pp, x, y, mask) - _loss_of(pm, x, y, mask)) / (2 * h)
            assert abs(fd - grads[l][0][idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx, fd, grads[l][0][idx])
        j = int(rng.integers(0, b.shape[0]))
        bp, bm = b.copy(), b.copy()
        bp[j] += h
        bm[j] -= h
        pp = list(params); pp[l] = (w, bp)
        pm = list(params); pm[l] = (w, bm)
        fd = (_loss_of(pp, x, y, mask) - _loss_of(pm, x, y, mask)) / (2 * h)
        assert abs(fd - grads[l][1][j]) <= 1e-6 * max(1.0, abs(fd))


def test_input_gradient_matches_central_differences():
    params, x, y, mask = _tiny()
    w, b = params[0]
    g = _rng(6).standard_normal((2, 4, 4, 4, 3))
    gx, _, _ = sg.conv3d_backward(x, w, g)
    h = 1e-6
    for idx in [(0, 1, 2, 3, 0), (1, 0, 0, 0, 1), (1, 3, 3, 3, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = ((g * sg.conv3d(xp, w, b)).sum() - (g * sg.conv3d(xm, w, b)).sum()) / (2 * h)
        assert abs(fd - gx[idx]) <= 1e-6 * max(1.0, abs(fd))


def test_first_adam_step_has_length_lr():
    # bias correction makes the first step -lr * g / (|g| + eps) elementwise
    params = [(np.array([[3.0, -2.0]]), np.array([0.5]))]
    grads = [(np.array([[4.0, -1e-3]]), np.array([2.0]))]
    st = {"t": 0, "m": [0.0, 0.0], "v": [0.0, 0.0]}
    out = sg.adam_step(params, grads, st, lr=0.1)
    assert np.allclose(out[0][0], [[2.9, -1.9]], atol=1e-6)
    assert np.allclose(out[0][1], [0.4], atol=1e-9)


def test_loss_is_zero_at_target_and_scale_invariant():
    rng = _rng(7)
    y = rng.standard_normal((3, 4, 4, 4, 2))
    mask = np.ones((3, 4, 4, 4))
    assert sg.loss(y, y, mask) == 0.0
    p = y + 0.1 * rng.standard_normal(y.shape)
    assert np.isclose(sg.loss(p, y, mask), sg.loss(5 * p, 5 * y, mask), rtol=1e-12)


@pytest.fixture(scope="module")
def small_oracle():
    from oracle import fem, hplmm as oh
    from paper_2509_19777_amd import synth
    p = synth.config_pores_lognormal(16, 8, seed=3, n_mortar=2)
    A, b, mesh = fem.assemble(p)
    return A, mesh, oh.HPLMM(p, A=A, b=b, mesh=mesh, n=2)


def test_galerkin_with_exact_blocks_is_the_coarse_operator(small_oracle):
    A, mesh, H = small_oracle
    S = sg.galerkin_mortar_block(H, {})
    ref = H.Acoarse[:H.Nmo, :H.Nmo]
    assert np.abs(S - ref).max() <= 1e-12 * np.abs(ref).max()


def test_exact_shape_vectors_minimise_the_coarse_energy(small_oracle):
    # the harmonic extension minimises the energy of P for fixed interface
    # values, so any other grain block raises P^T A P by a PSD matrix
    A, mesh, H = small_oracle
    rng = _rng(8)
    pert = {}
    for g, blk in enumerate(H.B_blocks):
        if blk is not None:
            cols, B = blk
            pert[g] = (cols, B + 0.05 * rng.standard_normal(B.shape))
    d = sg.galerkin_mortar_block(H, pert) - sg.galerkin_mortar_block(H, {})
    ev = np.linalg.eigvalsh(0.5 * (d + d.T))
    assert ev.min() >= -1e-10 * abs(ev).max()
    assert ev.max() > 0


def test_predicted_blocks_cover_every_mortar_column(small_oracle):
    A, mesh, H = small_oracle
    params = sg.init_params(_rng(9), (4, 4, 4, 4, 9))
    g = next(i for i, b in enumerate(H.B_blocks) if b is not None)
    blocks = sg.predicted_blocks(H, A, mesh, params, [g])
    cols, B = blocks[g]
    ecols, EB = H.B_blocks[g]
    assert np.array_equal(np.sort(cols), np.sort(ecols)) and B.shape == EB.shape


def test_bf16_forward_emulation():
    """forward_bf16 equals forward exactly when the inputs, weights and
    biases are already bfloat16 values and the net has one layer (nothing
    left to round), and stays within the bfloat16 rounding bound of forward
    otherwise (a relative error of a few u16 = 2^-9 per layer)."""
    from oracle import precision as prec
    rng = np.random.default_rng(3)
    params = sg.init_params(rng, (4, 5))
    params = [(prec.round_bf16(w), prec.round_bf16(rng.standard_normal(b.shape))) for w, b in params]
    x = prec.round_bf16(rng.standard_normal((2, 9, 9, 9, 4)))
    assert np.array_equal(sg.forward_bf16(params, x), sg.forward(params, x)[-1])
    params = sg.init_params(rng, (4, 8, 8, 8, 9))
    x = rng.standard_normal((2, 9, 9, 9, 4))
    ref = sg.forward(params, x)[-1]
    rel = np.linalg.norm(sg.forward_bf16(params, x) - ref) / np.linalg.norm(ref)
    assert 1e-5 < rel < 4 * 4 * 2.0 ** -9
