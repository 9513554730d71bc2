"""GPU parity of the building blocks against the oracle (FP64) and numpy,
called through the C ABI: MFMA lane layout, GEMM (all transposes, ragged
tails, FP32 / BF16 operands), the two-site effective Hamiltonian (small
shapes and the L=100, chi=1024 block shape), environment updates, the Jacobi
SVD split and the GMRES local solve."""
import numpy as np
import pytest

import paper_2606_02930_amd as ite
from oracle import mps as omps, mpo as ompo
from tests.gpu_util import require_gpu, dev, host, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = require_gpu()
    ctx = ite.ite_ctx_create(0)
    yield torch, ctx
    torch.cuda.synchronize()
    ite.ite_ctx_destroy(ctx)


def test_mfma_f64_lane_layout(env):
    torch, ctx = env
    out = ite.ite_debug_mfma_probe(ctx, 0)
    A = np.array([[1.0 + i + 16 * k for k in range(4)] for i in range(16)])
    B = np.array([[1.0 / (1.0 + j + 16 * k) for j in range(16)] for k in range(4)])
    D = A @ B
    # FP64 16x16x4: accumulator element r of lane l is D[4 r + l // 16][l % 16]
    for lane in range(64):
        for r in range(4):
            row, col = 4 * r + lane // 16, lane % 16
            assert abs(out[lane * 4 + r] - D[row, col]) < 1e-13 * abs(D[row, col]), (lane, r)


GEMM_SHAPES = [(1, 1, 1), (37, 61, 23), (128, 128, 16), (129, 255, 300), (300, 17, 1000), (256, 384, 64)]


@pytest.mark.parametrize("tA", [0, 1])
@pytest.mark.parametrize("tB", [0, 1])
@pytest.mark.parametrize("shape", GEMM_SHAPES)
def test_gemm_f64(env, tA, tB, shape):
    torch, ctx = env
    M, N, K = shape
    rng = np.random.default_rng(M * 7 + N * 3 + K + 100 * tA + 10 * tB)
    A = rng.standard_normal((K, M) if tA else (M, K))
    B = rng.standard_normal((N, K) if tB else (K, N))
    Cm = rng.standard_normal((M, N))
    want = 0.7 * ((A.T if tA else A) @ (B.T if tB else B)) - 1.3 * Cm
    dA, dB, dC = dev(torch, A), dev(torch, B), dev(torch, Cm)
    dD = torch.zeros((M, N), dtype=torch.float64, device="cuda")
    ite.ite_debug_gemm(ctx, tA, tB, M, N, K, 0.7, dA, A.shape[1], dB, B.shape[1], -1.3, dC, N, dD, N, 0)
    assert rel_err(host(dD), want) < 1e-13
    # in-place accumulate D = alpha AB + beta D
    ite.ite_debug_gemm(ctx, tA, tB, M, N, K, 1.0, dA, A.shape[1], dB, B.shape[1], 1.0, dD, N, dD, N, 0)
    assert rel_err(host(dD), want + (A.T if tA else A) @ (B.T if tB else B)) < 1e-13


@pytest.mark.parametrize("tA,tB", [(0, 0), (0, 1), (1, 0)])
@pytest.mark.parametrize("shape", [(5120, 2048, 1024), (4096, 1024, 5120), (5000, 2048, 1024)])
def test_gemm_large_dispatch(env, tA, tB, shape):
    # the library's FP64 dispatch at the block sizes of the 1024 bond: 640
    # tiles on 512 workgroup slots (5000 rows: the last tile row partial) in
    # one launch; 256 tiles with K = 5120 (half the slots): two K parts
    # summed in a fixed order
    torch, ctx = env
    M, N, K = shape
    rng = np.random.default_rng(M + N + K + 3 * tA + tB)
    A = rng.standard_normal((K, M) if tA else (M, K))
    B = rng.standard_normal((N, K) if tB else (K, N))
    C = rng.standard_normal((M, N))
    want = 0.75 * (A.T if tA else A) @ (B.T if tB else B) - 0.5 * C
    dA, dB, dC = dev(torch, A), dev(torch, B), dev(torch, C)
    dD = torch.zeros((M, N), dtype=torch.float64, device="cuda")
    ite.ite_debug_gemm(ctx, tA, tB, M, N, K, 0.75, dA, A.shape[1], dB, B.shape[1], -0.5, dC, N, dD, N, 0)
    assert rel_err(host(dD), want) < 1e-13


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("tA,tB", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("shape", [(200, 136, 520), (37, 133, 517), (256, 128, 1024), (136, 200, 72)])
def test_gemm_low_precision(env, prec, tA, tB, shape):
    # aligned rows take the 16-byte operand loads (ragged edges element by
    # element), the 517-wide shape the element loads throughout; K = 72 ends
    # in a partial K slice
    torch, ctx = env
    M, N, K = shape
    rng = np.random.default_rng(11 + prec + tB + 2 * tA)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((N, K) if tB else (K, N))
    # operands rounded to nearest even directly from FP64 (FP32: 24 bits,
    # BF16: 8 significant bits), computed independently of the library
    if prec == 1:
        rnd = lambda x: x.astype(np.float32).astype(np.float64)
    else:
        def rnd(x):
            m, e = np.frexp(x)
            return np.ldexp(np.round(m * 256.0) / 256.0, e)
    Ar, Br = rnd(A), rnd(B)
    want = Ar @ (Br.T if tB else Br)
    dD = torch.zeros((M, N), dtype=torch.float64, device="cuda")
    Ain = np.ascontiguousarray(A.T) if tA else A
    ite.ite_debug_gemm(ctx, tA, tB, M, N, K, 1.0, dev(torch, Ain), Ain.shape[1], dev(torch, B), B.shape[1], 0.0, None,
                       N, dD, N, prec)
    # FP32 accumulation of exactly rounded operands
    assert rel_err(host(dD), want) < 2e-5
    exact = A @ (B.T if tB else B)
    assert rel_err(host(dD), exact) < (1e-5 if prec == 1 else 3e-2)


def _heff_case(rng, Dxl, Dyl, Dxr, Dyr, d, W1, W2):
    w0, w2 = W1.shape[0], W2.shape[1]
    Lm = rng.standard_normal((Dxl, w0, Dyl))
    Rm = rng.standard_normal((Dxr, w2, Dyr))
    th = rng.standard_normal((Dyl, d, d, Dyr))
    return Lm, Rm, th


@pytest.mark.parametrize("dims", [(1, 1, 2, 2), (3, 5, 4, 2), (16, 16, 16, 16), (37, 29, 70, 130), (130, 130, 64, 64)])
def test_heff_apply_matches_oracle(env, dims):
    torch, ctx = env
    Dxl, Dyl, Dxr, Dyr = dims
    rng = np.random.default_rng(sum(dims))
    W = ompo.heisenberg_mpo(4, Jz=0.9)
    W1, W2 = W[1], W[2]
    Lm, Rm, th = _heff_case(rng, Dxl, Dyl, Dxr, Dyr, 2, W1, W2)
    want = omps.heff_apply(Lm, W1, W2, Rm, th)
    y = torch.zeros((Dxl, 2, 2, Dxr), dtype=torch.float64, device="cuda")
    ite.ite_debug_heff_apply(ctx, dev(torch, Lm), W1, W2, dev(torch, Rm), dev(torch, th), 0.0, 1.0, y)
    assert rel_err(host(y), want) < 1e-13
    if Dxl == Dyl and Dxr == Dyr:
        ite.ite_debug_heff_apply(ctx, dev(torch, Lm), W1, W2, dev(torch, Rm), dev(torch, th), 0.3, -0.25, y)
        assert rel_err(host(y), 0.3 * th - 0.25 * want) < 1e-13


def test_heff_apply_fermionic_boundary_blocks(env):
    torch, ctx = env
    rng = np.random.default_rng(5)
    W = ompo.aim_mpo(4.0, -2.0, np.array([-0.5, 0.0, 0.5]), np.array([0.2, 0.3, 0.1]))
    for j in range(3):
        W1, W2 = W[j], W[j + 1]
        Lm, Rm, th = _heff_case(rng, 12, 12, 9, 9, 4, W1, W2)
        want = omps.heff_apply(Lm, W1, W2, Rm, th)
        y = torch.zeros((12, 4, 4, 9), dtype=torch.float64, device="cuda")
        ite.ite_debug_heff_apply(ctx, dev(torch, Lm), W1, W2, dev(torch, Rm), dev(torch, th), 0.0, 1.0, y)
        assert rel_err(host(y), want) < 1e-13


@pytest.mark.parametrize("w,d", [(10, 4), (16, 8)])
def test_heff_apply_wide_mpo(env, w, d):
    # MPO bond dimension up to the loader's limits: the two-site stage then has
    # w d^2 = 160 (the impurity model's allowed w = 10 at d = 4) and 1024 inputs
    torch, ctx = env
    rng = np.random.default_rng(w * d)
    W1 = rng.standard_normal((w, w, d, d))
    W2 = rng.standard_normal((w, w, d, d))
    Lm, Rm, th = _heff_case(rng, 9, 7, 11, 6, d, W1, W2)
    want = omps.heff_apply(Lm, W1, W2, Rm, th)
    y = torch.zeros((9, d, d, 11), dtype=torch.float64, device="cuda")
    ite.ite_debug_heff_apply(ctx, dev(torch, Lm), W1, W2, dev(torch, Rm), dev(torch, th), 0.0, 1.0, y)
    assert rel_err(host(y), want) < 1e-13


def test_heff_apply_full_block_shape(env):
    # the L=100, chi=1024 Heisenberg block: L, R [1024][5][1024], theta [1024][2][2][1024]
    torch, ctx = env
    D = 1024
    g = torch.Generator(device="cuda").manual_seed(1234)
    Lm = torch.randn((D, 5, D), dtype=torch.float64, device="cuda", generator=g)
    Rm = torch.randn((D, 5, D), dtype=torch.float64, device="cuda", generator=g)
    th = torch.randn((D, 2, 2, D), dtype=torch.float64, device="cuda", generator=g)
    W = ompo.heisenberg_mpo(4)
    y = torch.zeros_like(th)
    ite.ite_debug_heff_apply(ctx, Lm, W[1], W[2], Rm, th, 0.5, 2.0, y)
    want = 0.5 * host(th) + 2.0 * omps.heff_apply(host(Lm), W[1], W[2], host(Rm), host(th))
    assert rel_err(host(y), want) < 1e-12


@pytest.mark.parametrize("with_mpo", [True, False])
@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("dims", [(1, 1, 2, 2), (5, 3, 7, 6), (64, 48, 100, 90)])
def test_env_update_matches_oracle(env, with_mpo, direction, dims):
    torch, ctx = env
    Dxa, Dya, Dxb, Dyb = dims
    rng = np.random.default_rng(3 * sum(dims) + direction + 2 * with_mpo)
    d = 2
    Wfull = ompo.heisenberg_mpo(4, Jz=0.7)[1]
    W = Wfull if with_mpo else None
    wl, wr = (5, 5) if with_mpo else (1, 1)
    if direction == 0:
        E = rng.standard_normal((Dxa, wl, Dya)) if with_mpo else rng.standard_normal((Dxa, Dya))
        X = rng.standard_normal((Dxa, d, Dxb))
        Y = rng.standard_normal((Dya, d, Dyb))
        want = omps.env_left_h(E, X, W, Y) if with_mpo else omps.env_left_o(E, X, Y)
    else:
        E = rng.standard_normal((Dxa, wr, Dya)) if with_mpo else rng.standard_normal((Dxa, Dya))
        X = rng.standard_normal((Dxb, d, Dxa))
        Y = rng.standard_normal((Dyb, d, Dya))
        want = omps.env_right_h(E, X, W, Y) if with_mpo else omps.env_right_o(E, X, Y)
    out = torch.zeros(want.shape, dtype=torch.float64, device="cuda")
    ite.ite_debug_env_update(ctx, direction, dev(torch, E), dev(torch, X), W, dev(torch, Y), out)
    assert rel_err(host(out), want) < 1e-13


# from p >= 256 rows the Jacobi runs on the Householder R factor: square,
# more rows than columns (rows of R beyond q vanish) and fewer rows
# up to 64 rows the whole Jacobi runs in one launch (16-row blocks up to 32
# rows, 32-row blocks up to 64); from 256 rows on with Householder
# preconditioning
SPLIT_SHAPES = [(1, 2, 2, 1), (1, 2, 2, 2), (3, 2, 2, 5), (8, 2, 2, 3), (16, 2, 2, 16), (24, 2, 2, 20),
                (32, 2, 2, 32), (33, 2, 2, 17), (64, 4, 4, 64), (256, 2, 2, 256), (200, 2, 2, 64),
                (64, 2, 2, 300), (130, 2, 2, 150), (512, 2, 2, 512)]


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("shape", SPLIT_SHAPES)
def test_svd_split_matches_numpy(env, direction, shape):
    torch, ctx = env
    Dl, d1, d2, Dr = shape
    m, n = Dl * d1, d2 * Dr
    rng = np.random.default_rng(m * 31 + n + direction)
    # graded spectrum so that truncation decisions are well separated
    r = min(m, n)
    U, _ = np.linalg.qr(rng.standard_normal((m, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n, r)))
    s_true = np.exp(-np.linspace(0, 12, r))
    theta = ((U * s_true) @ V.T).reshape(Dl, d1, d2, Dr)
    chi = max(1, r - 2)
    A1o, A2o, info = omps.split_two_site(theta, "lr" if direction == 0 else "rl", 1e-14, chi, 1e-13)
    k_o = info["k"]
    A1 = torch.zeros((Dl, d1, r), dtype=torch.float64, device="cuda")
    A2 = torch.zeros((r, d2, Dr), dtype=torch.float64, device="cuda")
    k, sig, disc = ite.ite_debug_svd_split(ctx, direction, dev(torch, theta), chi, 1e-14, 1e-13, A1, A2)
    a1 = host(A1).reshape(-1)[: Dl * d1 * k].reshape(Dl, d1, k)
    a2 = host(A2).reshape(-1)[: k * d2 * Dr].reshape(k, d2, Dr)
    diag = dict(k=k, k_o=k_o, sig_err=float(np.abs(sig - info["sigma"]).max()),
                worst=int(np.abs(sig - info["sigma"]).argmax()),
                recon=rel_err(omps.two_site(a1, a2), omps.two_site(A1o, A2o)),
                orth=(omps.left_orthonormality_error(a1) if direction == 0 else omps.right_orthonormality_error(a2)))
    assert k == k_o, diag
    assert np.allclose(sig, info["sigma"], rtol=0, atol=1e-13 * s_true[0]), diag
    assert abs(disc - info["disc"]) < 1e-12, diag
    # the kept rank-k approximation is unique (gauge-free) and equals the oracle's
    assert diag["recon"] < 1e-12, diag
    assert diag["orth"] < 5e-13, diag


@pytest.mark.parametrize("shape", [(64, 2, 2, 64), (100, 2, 2, 100), (256, 2, 2, 256), (1024, 2, 2, 1024)])
def test_svd_split_wide_dynamic_range(env, shape):
    # singular values from 1 down to 1e-30: the pair Grams span 60 decades,
    # beyond single precision, which the first Jacobi sweeps use for their
    # rotation angles; the result must still be FP64-accurate (128 and 200
    # rows: 16-row blocks without preconditioning; 512 rows: Householder and
    # the fused rotation; 2048 x 2048: the full-size bond split of the
    # benchmark)
    torch, ctx = env
    Dl, d1, d2, Dr = shape
    m, n = Dl * d1, d2 * Dr
    rng = np.random.default_rng(m + 5)
    r = min(m, n)
    U, _ = np.linalg.qr(rng.standard_normal((m, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n, r)))
    s_true = np.logspace(0, -30, r)
    theta = ((U * s_true) @ V.T).reshape(Dl, d1, d2, Dr)
    chi = r
    A1o, A2o, info = omps.split_two_site(theta, "lr", 1e-14, chi, 1e-13)
    A1 = torch.zeros((Dl, d1, r), dtype=torch.float64, device="cuda")
    A2 = torch.zeros((r, d2, Dr), dtype=torch.float64, device="cuda")
    k, sig, disc = ite.ite_debug_svd_split(ctx, 0, dev(torch, theta), chi, 1e-14, 1e-13, A1, A2)
    a1 = host(A1).reshape(-1)[: Dl * d1 * k].reshape(Dl, d1, k)
    a2 = host(A2).reshape(-1)[: k * d2 * Dr].reshape(k, d2, Dr)
    diag = dict(k=k, k_o=info["k"], sig_err=float(np.abs(sig - info["sigma"]).max()))
    assert k == info["k"], diag
    assert np.allclose(sig, info["sigma"], rtol=0, atol=1e-13), diag
    assert rel_err(omps.two_site(a1, a2), omps.two_site(A1o, A2o)) < 1e-12, diag
    assert omps.left_orthonormality_error(a1) < 5e-13, diag


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("D", [4, 128])
def test_svd_split_keeps_complete_basis_with_zeros(env, direction, D):
    # cutoff 0 keeps min(rows, cols, chi) values including exact zeros; the
    # factor that becomes the canonical tensor must still be orthonormal
    # (D = 128: 256 rows, through the Householder-preconditioned path)
    torch, ctx = env
    rng = np.random.default_rng(77)
    Dl, d, Dr = D, 2, D
    m = Dl * d
    u = rng.standard_normal((m, 2))
    v = rng.standard_normal((2, d * Dr))
    theta = (u @ v).reshape(Dl, d, d, Dr)       # rank 2
    A1 = torch.zeros((Dl, d, m), dtype=torch.float64, device="cuda")
    A2 = torch.zeros((m, d, Dr), dtype=torch.float64, device="cuda")
    k, sig, disc = ite.ite_debug_svd_split(ctx, direction, dev(torch, theta), m, 0.0, 1e-13, A1, A2)
    assert k == m and np.all(sig[2:] < 1e-13 * sig[0])
    a1 = host(A1).reshape(Dl, d, m)
    a2 = host(A2).reshape(m, d, Dr)
    assert rel_err(omps.two_site(a1, a2), theta) < 1e-13
    if direction == 0:
        assert omps.left_orthonormality_error(a1) < 1e-13
    else:
        assert omps.right_orthonormality_error(a2) < 1e-13


def _symmetric_envs(rng, D, W1, W2):
    """Environments of a random MPS so that H_eff is symmetric."""
    Wall = ompo.heisenberg_mpo(6)
    A = [rng.standard_normal((1, 2, 2)), rng.standard_normal((2, 2, D))]
    Lm = np.ones((1, 1, 1))
    for j in range(2):
        Lm = omps.env_left_h(Lm, A[j], Wall[j], A[j])
    B = [rng.standard_normal((D, 2, 2)), rng.standard_normal((2, 2, 1))]
    Rm = np.ones((1, 1, 1))
    for j in (5, 4):
        a = B[j - 4]
        Rm = omps.env_right_h(Rm, a, Wall[j], a)
    return Lm / np.abs(Lm).max(), Rm / np.abs(Rm).max(), Wall[2], Wall[3]


@pytest.mark.parametrize("budget", ["paper", "tol"])
def test_local_solve_matches_oracle(env, budget):
    torch, ctx = env
    rng = np.random.default_rng(9)
    Lm, Rm, W1, W2 = _symmetric_envs(rng, 4, None, None)
    Dl, Dr = Lm.shape[0], Rm.shape[0]
    h, s = 0.3, -1.0
    alpha, beta = 1.0 - h * s, h
    b = rng.standard_normal((Dl, 2, 2, Dr))
    x0 = rng.standard_normal((Dl, 2, 2, Dr))
    op = lambda v: alpha * v + beta * omps.heff_apply(Lm, W1, W2, Rm, v)
    if budget == "paper":
        m, cyc, tol = 10, 1, 0.0
    else:
        m, cyc, tol = 4, 100, 1e-13
    want, info = omps.gmres(op, b, x0, m, cyc, tol)
    x = torch.zeros(b.shape, dtype=torch.float64, device="cuda")
    mv, res = ite.ite_debug_local_solve(ctx, dev(torch, Lm), W1, W2, dev(torch, Rm), alpha, beta, dev(torch, b),
                                        dev(torch, x0), x, krylov_dim=m, max_cycles=cyc, tol=tol)
    got = host(x)
    if budget == "paper":
        assert mv == info["matvecs"] == 11
        assert rel_err(got, want) < 1e-10
    else:
        exact = np.linalg.solve(np.column_stack([op(e.reshape(b.shape)).reshape(-1) for e in np.eye(b.size)]),
                                b.reshape(-1)).reshape(b.shape)
        assert rel_err(got, exact) < 1e-11
        assert res <= 1e-13


@pytest.mark.parametrize("D", [40, 48])
def test_local_solve_paper_budget_longer_vectors(env, D):
    # n = 6400 (both Gram-Schmidt passes in one launch) and n = 9216 (the
    # multi-workgroup reductions): the same GMRES iterate as the oracle's
    torch, ctx = env
    rng = np.random.default_rng(90 + D)
    Lm, Rm, W1, W2 = _symmetric_envs(rng, D, None, None)
    Dl, Dr = Lm.shape[0], Rm.shape[0]
    h, s = 0.2, -1.5
    alpha, beta = 1.0 - h * s, h
    b = rng.standard_normal((Dl, 2, 2, Dr))
    x0 = rng.standard_normal((Dl, 2, 2, Dr))
    op = lambda v: alpha * v + beta * omps.heff_apply(Lm, W1, W2, Rm, v)
    want, info = omps.gmres(op, b, x0, 10, 1, 0.0)
    x = torch.zeros(b.shape, dtype=torch.float64, device="cuda")
    mv, res = ite.ite_debug_local_solve(ctx, dev(torch, Lm), W1, W2, dev(torch, Rm), alpha, beta, dev(torch, b),
                                        dev(torch, x0), x, krylov_dim=10, max_cycles=1, tol=0.0)
    assert mv == info["matvecs"] == 11
    assert rel_err(host(x), want) < 1e-10


def test_local_solve_paper_budget_full_block(env):
    # the L=100, chi=1024 block: n = 4 194 304 (the reductions run on their
    # capped grid of 1024 workgroups), paper budget, against the oracle's GMRES
    torch, ctx = env
    D = 1024
    rng = np.random.default_rng(1024)
    W = ompo.heisenberg_mpo(4)
    Lm = rng.standard_normal((D, 5, D)) / np.sqrt(D)
    Rm = rng.standard_normal((D, 5, D)) / np.sqrt(D)
    b = rng.standard_normal((D, 2, 2, D))
    x0 = b + 0.1 * rng.standard_normal((D, 2, 2, D))
    alpha, beta = 2.5, 0.3
    op = lambda v: alpha * v + beta * omps.heff_apply(Lm, W[1], W[2], Rm, v)
    want, info = omps.gmres(op, b, x0, 10, 1, 0.0)
    x = torch.zeros(b.shape, dtype=torch.float64, device="cuda")
    mv, res = ite.ite_debug_local_solve(ctx, dev(torch, Lm), W[1], W[2], dev(torch, Rm), alpha, beta,
                                        dev(torch, b), dev(torch, x0), x, krylov_dim=10, max_cycles=1, tol=0.0)
    assert mv == info["matvecs"] == 11
    assert rel_err(host(x), want) < 1e-10
    assert abs(res - info["res_rel"]) <= 1e-8 * info["res_rel"]


@pytest.mark.parametrize("prec,bound", [(1, 2e-6), (2, 3e-2)])
@pytest.mark.parametrize("dims", [(3, 5, 4, 2), (37, 29, 70, 130), (130, 130, 64, 64)])
def test_heff_apply_low_precision(env, prec, bound, dims):
    # FP32 / BF16 operands with FP32 accumulation: error of the order of the
    # operand rounding (2^-24 resp. 2^-9 relative per operand, three roundings)
    torch, ctx = env
    Dxl, Dyl, Dxr, Dyr = dims
    rng = np.random.default_rng(100 + sum(dims))
    W = ompo.heisenberg_mpo(4, Jz=0.9)
    Lm, Rm, th = _heff_case(rng, Dxl, Dyl, Dxr, Dyr, 2, W[1], W[2])
    want = omps.heff_apply(Lm, W[1], W[2], Rm, th)
    y = torch.zeros((Dxl, 2, 2, Dxr), dtype=torch.float64, device="cuda")
    ite.ite_debug_heff_apply(ctx, dev(torch, Lm), W[1], W[2], dev(torch, Rm), dev(torch, th), 0.0, 1.0, y, prec=prec)
    err = rel_err(host(y), want)
    assert err < bound
    assert err > 0.0    # the products really ran in the lower precision
    # the timing entry runs the same product (environments rounded once):
    # the same bits
    y2 = torch.zeros_like(y)
    ms = ite.ite_debug_heff_time(ctx, dev(torch, Lm), W[1], W[2], dev(torch, Rm), dev(torch, th), 0.0, 1.0, y2,
                                 prec=prec, reps=2)
    assert ms > 0.0
    assert torch.equal(y2, y)
    if Dxl == Dyl and Dxr == Dyr:
        ite.ite_debug_heff_apply(ctx, dev(torch, Lm), W[1], W[2], dev(torch, Rm), dev(torch, th), 0.3, -0.25, y,
                                 prec=prec)
        assert rel_err(host(y), 0.3 * th - 0.25 * want) < bound


@pytest.mark.parametrize("prec,bound", [(1, 1e-5), (2, 3e-2)])
def test_heff_apply_low_precision_full_block_shape(env, prec, bound):
    # the L=100, chi=1024 block in FP32 / BF16 operands: the second
    # contraction (M=4096, N=1024, K=5120) fills half the GPU's workgroup
    # slots, so the FP32 product runs it in two K parts summed in FP64.  For
    # random operands the FP32 accumulation error grows like sqrt(K) 2^-24
    # (K = 1024 and 2 x 2560 here: about 6e-6 for both contractions together)
    torch, ctx = env
    D = 1024
    g = torch.Generator(device="cuda").manual_seed(4321)
    Lm = torch.randn((D, 5, D), dtype=torch.float64, device="cuda", generator=g)
    Rm = torch.randn((D, 5, D), dtype=torch.float64, device="cuda", generator=g)
    th = torch.randn((D, 2, 2, D), dtype=torch.float64, device="cuda", generator=g)
    W = ompo.heisenberg_mpo(4)
    y = torch.zeros_like(th)
    ite.ite_debug_heff_apply(ctx, Lm, W[1], W[2], Rm, th, 0.5, 2.0, y, prec=prec)
    want = 0.5 * host(th) + 2.0 * omps.heff_apply(host(Lm), W[1], W[2], host(Rm), host(th))
    err = rel_err(host(y), want)
    assert 0.0 < err < bound
    y2 = torch.zeros_like(y)
    ite.ite_debug_heff_time(ctx, Lm, W[1], W[2], Rm, th, 0.5, 2.0, y2, prec=prec, reps=1)
    assert torch.equal(y2, y)


@pytest.mark.parametrize("prec", [1, 2])
def test_local_solve_refinement_reaches_fp64(env, prec):
    # mixed precision refinement: FP64 residuals, low-precision GMRES
    # corrections; the refined solution meets an FP64 residual target
    torch, ctx = env
    rng = np.random.default_rng(19)
    Lm, Rm, W1, W2 = _symmetric_envs(rng, 8, None, None)
    h, s = 0.3, -1.0
    alpha, beta = 1.0 - h * s, h
    b = rng.standard_normal((Lm.shape[0], 2, 2, Rm.shape[0]))
    x0 = np.zeros_like(b)
    op = lambda v: alpha * v + beta * omps.heff_apply(Lm, W1, W2, Rm, v)
    A = np.column_stack([op(e.reshape(b.shape)).reshape(-1) for e in np.eye(b.size)])
    exact = np.linalg.solve(A, b.reshape(-1)).reshape(b.shape)
    x = torch.zeros(b.shape, dtype=torch.float64, device="cuda")
    mv, res = ite.ite_debug_local_solve(ctx, dev(torch, Lm), W1, W2, dev(torch, Rm), alpha, beta, dev(torch, b),
                                        dev(torch, x0), x, krylov_dim=8, max_cycles=4, tol=1e-6, precision=prec,
                                        max_refine=20, tol_refine=1e-12)
    assert res <= 1e-12
    assert rel_err(host(x), exact) < 1e-11
    r = b - op(host(x))
    assert np.linalg.norm(r) <= 2e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("prec", [1, 2])
def test_local_solve_refinement_fixed_rounds(env, prec):
    # tol_refine = 0: exactly max_refine corrections of one GMRES(m) cycle
    # each; products: one FP64 residual before each correction and m - 1 + 1
    # = m low-precision products per correction (its first Krylov vector is
    # the residual itself); no FP64 residual after the last correction
    torch, ctx = env
    rng = np.random.default_rng(23)
    Lm, Rm, W1, W2 = _symmetric_envs(rng, 4, None, None)
    h, s = 0.3, -1.0
    alpha, beta = 1.0 - h * s, h
    b = rng.standard_normal((Lm.shape[0], 2, 2, Rm.shape[0]))
    x0 = rng.standard_normal(b.shape)
    op = lambda v: alpha * v + beta * omps.heff_apply(Lm, W1, W2, Rm, v)
    true_prev = None
    for rounds in (1, 2, 3):
        x = torch.zeros(b.shape, dtype=torch.float64, device="cuda")
        mv, res = ite.ite_debug_local_solve(ctx, dev(torch, Lm), W1, W2, dev(torch, Rm), alpha, beta,
                                            dev(torch, b), dev(torch, x0), x, krylov_dim=6, max_cycles=1, tol=0.0,
                                            precision=prec, max_refine=rounds, tol_refine=0.0)
        assert mv == rounds + rounds * 6
        true = np.linalg.norm(b - op(host(x))) / np.linalg.norm(b)
        if prec == 1 and rounds == 1:
            # the estimate is the FP32 system's residual: close to the true one
            # while it is far above the FP32 rounding level
            assert abs(res - true) <= 0.1 * true
        if true_prev is not None:
            assert true < true_prev
        true_prev = true
