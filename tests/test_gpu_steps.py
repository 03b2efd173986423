"""Step-level parity of the HIP path against the oracle (GPU, via the C ABI).

Each test generates seeded inputs with ``synth``, runs one phase through the
library and compares element by element with the oracle's FP64 step.  Sizes
span several 16/64-row tiles with ragged tails; the filter cases include
split-K partial sums and several column blocks.
"""
import numpy as np
import pytest

from oracle import eig, steps
from paper_2006_08498_amd import chase, synth
from tests.gpu_util import EPS, dev_block, dev_colmajor, dot_bound, host, torch_cuda

pytestmark = pytest.mark.gpu

FILTER_CASES = [(1, 1), (7, 3), (63, 16), (257, 5), (1000, 33), (1301, 140),
                (2049, 161), (4100, 16)]


@pytest.mark.parametrize("N,n", FILTER_CASES)
def test_filter_step_elementwise(N, n):
    torch_cuda()
    H = synth.dk_matrix(N, seed=N)
    Y = synth.random_block(N, n, seed=1)
    X = synth.random_block(N, n, seed=2)
    a, b, g = 0.37, -1.3, 0.55
    ref = steps.cheb_step(H, Y, X, a, b, g)
    W = host(chase.filter_step(dev_colmajor(H), dev_block(Y), dev_block(X), a, b, g))
    bound = abs(a) * dot_bound(np.abs(H), np.abs(Y), N) + 4 * EPS * (
        abs(b) * np.abs(Y) + abs(g) * np.abs(X)) + 1e-300
    err = np.abs(W - ref)
    assert np.all(err <= bound), (err / bound).max()


def test_filter_step_in_place_and_padded_ld():
    torch = torch_cuda()
    N, n, ld = 530, 21, 40
    H = synth.dk_matrix(N, seed=3)
    Yb = synth.random_block(N, ld, seed=4)
    Xb = synth.random_block(N, ld, seed=5)
    ref = steps.cheb_step(H, Yb[:, :n], Xb[:, :n], 2.0, -0.5, -1.0)
    dY, dX = dev_block(Yb), dev_block(Xb)
    out = chase.filter_step(dev_colmajor(H), dY[:, :n], dX[:, :n], 2.0, -0.5, -1.0,
                            W=dX[:, :n])
    got = host(dX)
    bound = 2.0 * dot_bound(np.abs(H), np.abs(Yb[:, :n]), N) + 8 * EPS * (
        np.abs(Yb[:, :n]) + np.abs(Xb[:, :n]))
    assert np.all(np.abs(got[:, :n] - ref) <= bound)
    assert np.array_equal(got[:, n:], Xb[:, n:])       # padding untouched
    assert out.data_ptr() == dX.data_ptr()
    torch.cuda.synchronize()


def test_filter_step_zero_g_without_X():
    torch_cuda()
    N, n = 300, 7
    H = synth.dk_matrix(N, seed=6)
    Y = synth.random_block(N, n, seed=6)
    ref = steps.cheb_step(H, Y, None, 1.0, 0.0, 0.0)
    W = host(chase.filter_step(dev_colmajor(H), dev_block(Y), None, 1.0, 0.0, 0.0))
    assert np.all(np.abs(W - ref) <= dot_bound(np.abs(H), np.abs(Y), N))


def test_filter_step_group_bitwise_equals_single_steps():
    """One grouped launch over steps of different N, n (tile widths 1..10,
    split and unsplit plans, several column blocks), with and without X, one
    of them in place: each result is bitwise the single step's, which the
    elementwise test above pins to the oracle."""
    torch = torch_cuda()
    shapes = [(1, 1), (63, 16), (700, 33), (1301, 140), (2049, 161), (4100, 16),
              (5000, 150), (3000, 9), (257, 64)]
    steps_g, singles = [], []
    for k, (N, n) in enumerate(shapes):
        H = dev_colmajor(synth.dk_matrix(N, seed=100 + k))
        Y = dev_block(synth.random_block(N, n, seed=200 + k))
        X = dev_block(synth.random_block(N, n, seed=300 + k))
        a, b, g = 0.37 + 0.01 * k, -1.3, (0.0 if k % 3 == 0 else 0.55)
        Xs = None if g == 0.0 else X
        singles.append(host(chase.filter_step(H, Y, Xs, a, b, g)))
        W = X if k == 4 else torch.empty_like(Y)      # one in-place update
        steps_g.append((H, Y, Xs, W, a, b, g))
    chase.filter_step_group(steps_g)
    for (H, Y, X, W, a, b, g), ref in zip(steps_g, singles):
        assert np.array_equal(host(W), ref)
    chase.filter_step_group([])                          # empty group is a no-op


@pytest.mark.parametrize("deg", [[2, 2, 4, 4, 6, 8, 10, 10, 12, 16, 20, 20],
                                 [1, 1, 1, 2, 2, 4, 6, 6, 8, 10, 12, 14]])
def test_filter_per_vector_degrees_vs_oracle_and_closed_form(deg):
    """Per-vector degrees, including degree-1 columns (their single step
    ends in the other buffer and is copied back)."""
    torch_cuda()
    N = 700
    H, lam, Q = synth.planted_matrix(N, seed=7, n_clusters=4, cluster_size=5)
    V = synth.random_block(N, 12, seed=7)
    deg = np.array(deg)
    mu1, alpha, beta = lam[0] - 0.01, lam[30], lam[-1] + 0.1
    ref = steps.cheb_filter(H, V, deg, mu1, alpha, beta)
    dV = dev_block(V)
    mv = chase.filter(dev_colmajor(H), dV, deg, mu1, alpha, beta)
    got = host(dV)
    assert mv == deg.sum()
    c, e = steps.interval(alpha, beta)
    t0 = (mu1 - c) / e
    for j, m in enumerate(deg):
        scale = np.linalg.norm(ref[:, j])
        assert np.linalg.norm(got[:, j] - ref[:, j]) <= 1e-12 * m * scale
        f = steps.chebyshev_T(m, (lam - c) / e) / steps.chebyshev_T(m, np.array([t0]))[0]
        closed = Q @ (f * (Q.conj().T @ V[:, j]))
        assert np.linalg.norm(got[:, j] - closed) <= 1e-11 * m * scale


def test_lanczos_vs_oracle():
    torch_cuda()
    N, r, k = 900, 4, 25
    H = synth.dk_matrix(N, seed=8)
    V0 = synth.random_block(N, r, seed=8)
    al, be = chase.lanczos(dev_colmajor(H), dev_block(V0), k)
    ral, rbe = steps.lanczos(H, V0, k)
    hn = np.abs(np.linalg.eigvalsh(H)).max()
    # The first steps agree to rounding; without re-orthogonalisation the
    # later coefficients drift apart as Ritz values converge, so those are
    # compared through the bounds they produce.
    assert np.abs(al[:8] - ral[:8]).max() <= 1e-12 * hn
    assert np.abs(be[:8] - rbe[:8]).max() <= 1e-12 * hn
    got = chase.lanczos_bounds(al, be, N, 30)
    ref = steps.lanczos_bounds(ral, rbe, N, 30)
    assert abs(got[0] - ref[0]) <= 1e-9 * hn      # mu1 (converged Ritz value)
    assert abs(got[3] - ref[3]) <= 1e-9 * hn      # largest |Ritz value|
    lam = np.linalg.eigvalsh(H)
    assert got[2] >= lam[-1] and got[0] >= lam[0] - 1e-12


@pytest.mark.parametrize("N,n,nlocked,graded", [(1000, 40, 0, 0), (777, 33, 0, 8),
                                                 (1200, 50, 17, 0), (64, 64, 0, 0),
                                                 (3000, 400, 100, 0), (1100, 1024, 0, 0),
                                                 (2000, 180, 0, 8), (2000, 181, 0, 0),
                                                 (500, 2, 0, 0), (500, 1, 0, 0),
                                                 (1500, 140, 0, 8), (1500, 141, 0, 0),
                                                 (900, 144, 5, 0), (1000, 60, 0, 12),
                                                 (1600, 200, 0, 12), (800, 16, 0, 0),
                                                 (800, 17, 0, 4), (900, 15, 2, 0),
                                                 (2500, 260, 0, 8), (3000, 400, 0, 12),
                                                 (3000, 400, 140, 8)])
def test_qr_vs_oracle(N, n, nlocked, graded):
    """graded: column norms fall from 1 to 10^-graded across the block."""
    torch_cuda()
    V = synth.random_block(N, n, seed=N + n)
    if graded:
        V = V * np.logspace(0, -graded, n)[None, :]
    if nlocked:
        V[:, :nlocked] = steps.qr_orth(V[:, :nlocked])
    dV = dev_block(V)
    chase.qr(dV, nlocked)
    got = host(dV)
    assert np.array_equal(got[:, :nlocked], V[:, :nlocked])
    Va = steps.orth_against(V[:, :nlocked], steps.orth_against(V[:, :nlocked], V[:, nlocked:]))
    ref = steps.qr_orth(Va)
    cond = np.linalg.cond(Va * (1.0 / np.linalg.norm(Va, axis=0))[None, :])
    assert np.abs(got[:, nlocked:] - ref).max() <= 1e-13 * max(cond, 1.0) * np.sqrt(N)
    Qa = got
    assert np.abs(Qa.conj().T @ Qa - np.eye(n)).max() <= 1e-14 * np.sqrt(N)


@pytest.mark.parametrize("n", [20, 140, 141, 300, 1024])
def test_qr_breakdown_names_the_dependent_column(n):
    # A zero column has a zero Gram diagonal, which the factor reports at
    # its own index whatever the block it falls in.
    torch_cuda()
    V = synth.random_block(max(700, n + 10), n, seed=n)
    V[:, 7] = 0.0
    with pytest.raises(chase.ChaseError, match="breakdown at column 7"):
        chase.qr(dev_block(V), 0)


def test_rayleigh_ritz_vs_oracle():
    torch_cuda()
    N, n = 600, 30
    H, lam, _ = synth.planted_matrix(N, seed=9, n_clusters=3, cluster_size=4)
    Q = steps.qr_orth(synth.random_block(N, n, seed=9))
    th_ref, V_ref, _ = steps.rayleigh_ritz(H, Q)
    res_ref = steps.residual_norms(H, V_ref, th_ref)
    dQ = dev_block(Q)
    th, res = chase.rayleigh_ritz(dev_colmajor(H), dQ)
    V = host(dQ)
    hn = lam.max()
    assert np.abs(th - th_ref).max() <= 1e-13 * hn
    gaps = np.diff(th_ref)
    sep = np.minimum(np.r_[np.inf, gaps], np.r_[gaps, np.inf])
    for j in range(n):
        ov = abs(np.vdot(V_ref[:, j], V[:, j]))
        assert ov >= 1.0 - 1e-13 * hn / sep[j] - 1e-13
    assert np.allclose(res, res_ref, rtol=1e-10, atol=1e-13 * hn)
    assert np.abs(V.conj().T @ V - np.eye(n)).max() <= 1e-13


@pytest.mark.parametrize("n", [1, 2, 3, 17, 32, 33, 64, 65, 100, 130, 139, 140, 141])
def test_heevj_vs_oracle(n):
    """Orders up to 64 take the one-launch LDS kernel, 65..140 the packed-LDS
    kernel with recorded rotations (130: an odd number of pairs per round,
    139: a phantom index), larger ones the per-round launches; all against
    the oracle."""
    torch_cuda()
    G = synth.random_block(n, n, seed=n)
    G = 0.5 * (G + G.conj().T)
    w, Y = chase.heevj(dev_block(G))
    Y = host(Y)
    w_ref, _ = eig.eigh_lowest(G, n)
    gn = max(np.abs(w_ref).max(), 1e-300)
    assert np.abs(w - w_ref).max() <= 1e-13 * gn * max(1.0, np.sqrt(n) / 4)
    assert np.abs(G @ Y - Y * w).max() <= 1e-13 * gn * np.sqrt(n)
    assert np.abs(Y.conj().T @ Y - np.eye(n)).max() <= 1e-13 * np.sqrt(n)


def test_heevj_reports_non_convergence(monkeypatch):
    """A sweep cap below what the matrix needs is reported as an error by
    all three Jacobi paths (the diagnostic override of the cap)."""
    torch_cuda()
    monkeypatch.setenv("CHASE_JACOBI_MAX_SWEEPS", "1")
    for n in (40, 100, 160):
        G = synth.random_block(n, n, seed=3)
        G = 0.5 * (G + G.conj().T)
        with pytest.raises(chase.ChaseError, match="did not converge in 1 sweeps"):
            chase.heevj(dev_block(G))


def test_heevj_degenerate_and_zero():
    torch_cuda()
    n = 12
    lamv = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 3.0, 3.0, 3.0, 3.0, 4.0, 5.0, 5.0])
    U = steps.qr_orth(synth.random_block(n, n, seed=3))
    G = (U * lamv) @ U.conj().T
    G = 0.5 * (G + G.conj().T)
    w, Y = chase.heevj(dev_block(G))
    Y = host(Y)
    assert np.abs(w - lamv).max() <= 1e-13 * 5
    assert np.abs(Y.conj().T @ Y - np.eye(n)).max() <= 1e-13
    w0, Y0 = chase.heevj(dev_block(np.zeros((5, 5), dtype=np.complex128)))
    assert np.array_equal(w0, np.zeros(5))
    assert np.abs(host(Y0).conj().T @ host(Y0) - np.eye(5)).max() == 0.0


def test_residuals_vs_oracle():
    torch_cuda()
    N, n = 500, 9
    H = synth.dk_matrix(N, seed=10)
    V = synth.random_block(N, n, seed=10)
    th = np.linspace(0.5, 2.0, n)
    got = chase.residuals(dev_colmajor(H), dev_block(V), th)
    ref = steps.residual_norms(H, V, th)
    assert np.allclose(got, ref, rtol=1e-12, atol=0)


def test_device_generator_matches_host_generator():
    torch = torch_cuda()
    N = 1500
    Hd = synth.dk_matrix_device(N, seed=5)
    assert Hd.stride() == (1, N)
    Hh = synth.dk_matrix(N, seed=5)
    got = Hd.cpu().numpy()
    assert np.abs(got - Hh).max() <= 1e-15 * np.abs(Hh).max()
    assert np.array_equal(got, got.conj().T)        # Hermitian to the bit
    G = synth.gaussian_matrix_device(300, 7, seed=2).cpu().numpy()
    Gh = synth.gaussian_matrix(300, 7, seed=2)
    assert np.abs(G - Gh).max() <= 1e-14
    torch.cuda.synchronize()


def test_filter_fused_bitwise_equals_each_job_alone():
    """Several whole filter calls (different N, column counts over one and
    several pieces, split and unsplit plans, degree-1 columns) run by the
    persistent filter engine in one launch: each job's block is bitwise the
    one chase_filter gives alone; an empty job and a repeat (a second launch
    of the engine) included."""
    torch = torch_cuda()
    specs = [(1000, 40, 3), (2049, 161, 4), (300, 7, 5), (4100, 90, 6), (700, 0, 7),
             (1536, 16, 8)]
    jobs, refs = [], []
    for N, n, seed in specs:
        H = synth.dk_matrix(N, seed=seed)
        V = synth.random_block(N, max(n, 1), seed=seed)[:, :n]
        rng = np.random.default_rng(seed)
        deg = np.sort(rng.choice([1, 2, 4, 6, 8, 12, 16], size=n)) if n else np.zeros(0, int)
        lam = np.linalg.eigvalsh(H) if N <= 2049 else None
        lo, hi = (lam[0], lam[-1]) if lam is not None else (0.8, 6.3)
        mu1, alpha, beta = lo - 0.01, lo + 0.3 * (hi - lo), hi + 0.1
        dH = dev_colmajor(H)
        Vref = dev_block(V)
        if n:
            chase.filter(dH, Vref, deg, mu1, alpha, beta)
        refs.append(host(Vref))
        jobs.append((dH, dev_block(V), deg, mu1, alpha, beta))
    for rep in range(2):
        blocks = [dev_block(r0) for r0 in [host(j[1]) for j in jobs]]
        mv = chase.filter_fused([(j[0], b, j[2], j[3], j[4], j[5])
                                 for j, b in zip(jobs, blocks)])
        assert mv == sum(int(np.sum(j[2])) for j in jobs)
        for b, r in zip(blocks, refs):
            assert np.array_equal(host(b), r)
    torch.cuda.synchronize()
