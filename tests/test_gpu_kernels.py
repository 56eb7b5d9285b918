"""GPU checks of single dense kernels (through the test hooks of the C ABI)
and of intermediate set-up state, against NumPy/oracle references."""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_2509_19777_amd import synth

pytestmark = pytest.mark.gpu

TS = 64


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _tiles(mats, dtype):
    """numpy (n, 64, 64) matrices -> CUDA tensor holding column-major tiles."""
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(np.transpose(mats, (0, 2, 1)))).to(dtype).cuda()


def _untile(t):
    return np.transpose(t.cpu().numpy().astype(np.float64), (0, 2, 1)) if t.dim() == 3 else t.cpu().numpy().T


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("npairs", [3, 0])
@pytest.mark.parametrize("flags", [0, 1, 2, 3, 4 | 8, 2 | 4 | 8, 16 | 8, 1 | 16, 32, 2 | 4 | 8 | 32, 1 | 8 | 32])
def test_tile_gemm(prec, flags, npairs):
    torch = _torch()
    from paper_2509_19777_amd import hplmm as hp
    dt = torch.float64 if prec == 64 else torch.float32
    if npairs == 0 and not flags & 32:
        pytest.skip("an empty sum is only meaningful with a right factor")
    rng = np.random.default_rng(flags + prec + npairs)
    A = rng.standard_normal((max(npairs, 1), TS, TS))
    B = rng.standard_normal((max(npairs, 1), TS, TS))
    C0 = rng.standard_normal((TS, TS))
    Pm = rng.standard_normal((TS, TS))
    ref = np.zeros((TS, TS))
    for p in range(npairs):
        ref += (A[p].T if flags & 1 else A[p]) @ (B[p].T if flags & 2 else B[p])
    if flags & 16:
        ref = Pm @ ref
    if flags & 8:
        ref = -ref
    if (flags & 4) and not (flags & 16):
        ref = C0 + ref
    if flags & 32:
        ref = ref @ Pm
    Ct = _tiles(C0[None], dt)[0].contiguous()
    hp.debug_tile_gemm(_tiles(A, dt)[:npairs] if npairs else _tiles(A, dt), _tiles(B, dt), Ct, flags,
                       _tiles(Pm[None], dt)[0].contiguous(), npairs=npairs)
    got = _untile(Ct)
    tol = 1e-13 if prec == 64 else 2e-5
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("flags", [0, 1, 2, 3, 4, 1 | 4 | 8])
def test_tile_gemm_bf16(flags):
    # bfloat16 operands on the matrix cores with FP32 accumulation: against
    # the exact FP64 sum of the same bfloat16 values, within the bound of an
    # FP32 sum of 64 npairs products, (64 npairs + 2) u32 sum |a b| (plus the
    # accumulated C)
    torch = _torch()
    from oracle import precision as prec
    from paper_2509_19777_amd import hplmm as hp
    npairs = 5
    rng = np.random.default_rng(40 + flags)
    A = prec.round_bf16(rng.standard_normal((npairs, TS, TS)))
    B = prec.round_bf16(rng.standard_normal((npairs, TS, TS)))
    C0 = prec.round_f32(rng.standard_normal((TS, TS)))
    ref = np.zeros((TS, TS))
    mag = np.zeros((TS, TS))
    for p in range(npairs):
        a, b = (A[p].T if flags & 1 else A[p]), (B[p].T if flags & 2 else B[p])
        ref += a @ b
        mag += np.abs(a) @ np.abs(b)
    if flags & 8:
        ref = -ref
    if flags & 4:
        ref = C0 + ref
        mag += np.abs(C0)

    def bits(x):   # column-major tiles of bfloat16 bit patterns
        f = np.ascontiguousarray(np.swapaxes(x, -1, -2)).astype(np.float32)
        return torch.from_numpy((f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)).cuda()
    Ct = _tiles(C0[None], torch.float32)[0].contiguous()
    hp.debug_tile_gemm(bits(A), bits(B), Ct, flags)
    got = _untile(Ct)
    err = np.abs(got - ref)
    assert np.all(err <= (64 * npairs + 2) * 2.0 ** -24 * mag), err.max()


@pytest.mark.parametrize("prec", [64, 32])
def test_diag_factor_and_inverse(prec):
    torch = _torch()
    from paper_2509_19777_amd import hplmm as hp
    dt = torch.float64 if prec == 64 else torch.float32
    rng = np.random.default_rng(3)
    M = rng.standard_normal((TS, TS))
    Aspd = M @ M.T + TS * np.eye(TS)
    At = _tiles(Aspd[None], dt)[0].contiguous()
    L, W, Wt = hp.debug_diag(At)
    Lr = np.linalg.cholesky(Aspd)
    tol = 1e-13 if prec == 64 else 1e-5
    assert np.abs(_untile(L) - Lr).max() <= tol * np.abs(Lr).max()
    Wr = np.linalg.inv(Lr)
    assert np.abs(_untile(W) - Wr).max() <= tol * 10 * np.abs(Wr).max()
    assert np.array_equal(_untile(Wt), _untile(W).T)


@pytest.mark.parametrize("prec", [64, 32])
def test_diag_subtracts_panel_term(prec):
    # the last term of a left-looking diagonal update: factor of A - P P^T
    torch = _torch()
    from paper_2509_19777_amd import hplmm as hp
    dt = torch.float64 if prec == 64 else torch.float32
    rng = np.random.default_rng(5)
    M = rng.standard_normal((TS, TS))
    S = M @ M.T + TS * np.eye(TS)
    P = rng.standard_normal((TS, TS))
    At = _tiles((S + P @ P.T)[None], dt)[0].contiguous()
    Pt = _tiles(P[None], dt)[0].contiguous()
    L, W, Wt = hp.debug_diag(At, Pt)
    Lr = np.linalg.cholesky(S)
    tol = 1e-12 if prec == 64 else 1e-4
    assert np.abs(_untile(L) - Lr).max() <= tol * np.abs(Lr).max()
    Wr = np.linalg.inv(Lr)
    assert np.abs(_untile(W) - Wr).max() <= tol * 10 * np.abs(Wr).max()
    assert np.array_equal(_untile(Wt), _untile(W).T)


def test_diag_reports_indefinite():
    torch = _torch()
    from paper_2509_19777_amd import hplmm as hp
    A = -np.eye(TS)
    with pytest.raises(hp.HplmmError) as e:
        hp.debug_diag(_tiles(A[None], torch.float64)[0].contiguous())
    assert e.value.code == -3


def _dense_from_packed(tiles_flat, n, nt):
    D = np.zeros((nt * TS, nt * TS))
    for I in range(nt):
        for J in range(I + 1):
            t = tiles_flat[(I * (I + 1) // 2 + J) * TS * TS:(I * (I + 1) // 2 + J + 1) * TS * TS]
            D[I * TS:(I + 1) * TS, J * TS:(J + 1) * TS] = t.reshape(TS, TS).T
    return D


def _dense_from_rect(tiles_flat, nt, ntc):
    D = np.zeros((nt * TS, ntc * TS))
    for C in range(ntc):
        for I in range(nt):
            k = C * nt + I
            D[I * TS:(I + 1) * TS, C * TS:(C + 1) * TS] = tiles_flat[k * TS * TS:(k + 1) * TS * TS].reshape(TS, TS).T
    return D


@pytest.fixture(scope="module")
def staged():
    torch = _torch()
    from oracle import fem, hplmm as oh
    from paper_2509_19777_amd import hplmm as hp
    p = synth.config_pores(12, 4, seed=3)
    A, b, mesh = fem.assemble(p)
    H = oh.HPLMM(p, A=A, b=b, mesh=mesh, n=2)
    sysm, part = hp.build_problem(p)
    S = hp.Solver(sysm, part, n_mortar=2)
    return p, A, b, mesh, H, S, hp


def test_stage_gather_and_factor(staged):
    p, A, b, mesh, H, S, hp = staged
    lay = hp.debug_grain_layout(S)
    hp.debug_setup_stage(S, 0)
    blocks = {}
    for (g, n, nt, ncol, ntc, ao, wo, wto, ro, yo, ko) in lay:
        Ad = _dense_from_packed(hp.debug_read_arena(S, 0, ao, nt * (nt + 1) // 2 * TS * TS), n, nt)
        o = H.goff[g]
        Ao = H.A_gg[o:o + n, o:o + n].toarray()
        low = np.tril(Ad[:n, :n])
        assert np.allclose(low, np.tril(Ao), rtol=0, atol=1e-14 * np.abs(Ao).max()), g
        if ntc:
            R = _dense_from_rect(hp.debug_read_arena(S, 0, ro, nt * ntc * TS * TS), nt, ntc)
            cols, _ = H.B_blocks[g]
            Abar = H.Abar_gm[o:o + n].toarray()[:, cols]
            k = len(cols)
            assert np.allclose(R[:n, :k], -Abar, rtol=0, atol=1e-14 * max(1, np.abs(Abar).max())), g
        blocks[g] = Ao
    hp.debug_setup_stage(S, 1)
    for (g, n, nt, ncol, ntc, ao, wo, wto, ro, yo, ko) in lay:
        L = _dense_from_packed(hp.debug_read_arena(S, 0, ao, nt * (nt + 1) // 2 * TS * TS), n, nt)[:n, :n]
        W = _dense_from_packed(hp.debug_read_arena(S, 0, wo, nt * (nt + 1) // 2 * TS * TS), n, nt)[:n, :n]
        Lr = np.linalg.cholesky(blocks[g])
        assert np.abs(np.tril(L) - Lr).max() <= 1e-12 * np.abs(Lr).max(), g
        assert np.abs(np.tril(W) @ Lr - np.eye(n)).max() <= 1e-11, g


@pytest.mark.gpu
@pytest.mark.parametrize("n", [1, 7, 4096 * 3 + 5, 1 << 22])
def test_stream_triad(n):
    # the bandwidth reference: a = b + s c, one multiply-add per element (the
    # kernel may fuse it: within one rounding of the product of the two-step sum)
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_19777_amd import hplmm as hp
    g = torch.Generator().manual_seed(n)
    b = torch.randn(n, generator=g, dtype=torch.float64)
    c = torch.randn(n, generator=g, dtype=torch.float64)
    a = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    hp.stream_triad(a, b.cuda(), c.cuda(), -1.5)
    prod = (-1.5) * c.numpy()
    ref = b.numpy() + prod
    assert np.all(np.abs(a.cpu().numpy() - ref) <= 2.0 ** -52 * (np.abs(prod) + np.abs(ref)))
