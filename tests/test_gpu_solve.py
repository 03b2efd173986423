"""End-to-end parity of the GPU solver with the oracle (GPU, via the C ABI).

Bar (per eigenpair): relative eigenvalue error <= 1e-10 against the oracle,
||H v - lambda v|| / ||H||_2 <= 1e-10, max |V^H V - I| <= 1e-12, and the
eigenvectors equal to the oracle's up to phase where eigenvalues are
separated (cluster subspaces where they are not).
"""
import numpy as np
import pytest

from oracle import brute, eig
from paper_2006_08498_amd import chase, synth
from tests.gpu_util import check_against_oracle as _check_against_oracle
from tests.gpu_util import dev_colmajor, host, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed", [0, 1])
def test_dk_2000_matches_oracle(seed):
    """The N = 2000 D + K workload (nev 20, nex 10, degree <= 20)."""
    torch_cuda()
    H = synth.dk_matrix(2000, seed=seed)
    r = chase.solve(dev_colmajor(H), 20, 10, tol=1e-10, degree_max=20)
    assert r.status == chase.CHASE_OK and r.info["nconv"] == 20
    _check_against_oracle(H, r, 20)
    assert 1 <= r.info["iterations"] <= 30
    assert r.info["matvecs_filter"] > 0
    assert r.info["beta"] >= np.linalg.eigvalsh(H)[-1]


def test_row_major_input_gives_same_eigenpairs():
    torch = torch_cuda()
    H = synth.dk_matrix(800, seed=3)
    rc = chase.solve(dev_colmajor(H), 8, 6)
    rr = chase.solve(torch.from_numpy(H).cuda(), 8, 6)
    assert np.abs(rc.eigvals - rr.eigvals).max() <= 1e-12
    _check_against_oracle(H, rr, 8)


@pytest.mark.parametrize("N,nev,nex", [(1, 1, 0), (2, 1, 1), (3, 2, 0), (8, 3, 2),
                                       (40, 10, 30), (257, 7, 9), (1001, 12, 5)])
def test_small_and_ragged_sizes(N, nev, nex):
    torch_cuda()
    if N <= 8:
        H = synth.gaussian_integer_hermitian(N, seed=N).astype(np.complex128)
        exact = np.array(brute.eigenvalues(H.tolist()))[:nev]
    else:
        H = synth.dk_matrix(N, seed=N)
        exact = None
    r = chase.solve(dev_colmajor(H), nev, nex, tol=1e-10, degree_max=20)
    assert r.status == chase.CHASE_OK
    _check_against_oracle(H, r, nev)
    if exact is not None:
        assert np.abs(r.eigvals - exact).max() <= 1e-10 * max(1.0, np.abs(exact).max())


def test_planted_clusters():
    torch_cuda()
    N = 1500
    H, lam, _ = synth.planted_matrix(N, seed=4, n_clusters=8, cluster_size=10)
    nev, nex = 40, 16
    r = chase.solve(dev_colmajor(H), nev, nex, tol=1e-10, degree_max=20)
    assert r.status == chase.CHASE_OK
    assert np.abs(r.eigvals - lam[:nev]).max() <= 1e-10 * lam[:nev].max()
    _check_against_oracle(H, r, nev, hn=lam.max())


def test_deterministic_repeat():
    torch_cuda()
    H = synth.dk_matrix(1200, seed=5)
    dH = dev_colmajor(H)
    a = chase.solve(dH, 10, 6)
    b = chase.solve(dH, 10, 6)
    assert np.array_equal(a.eigvals, b.eigvals)
    assert np.array_equal(host(a.V), host(b.V))
    for key in ("iterations", "matvecs_filter", "matvecs_total"):
        assert a.info[key] == b.info[key]


def test_warm_start_converges_fast():
    torch = torch_cuda()
    H = synth.dk_matrix(900, seed=6)
    nev, nex = 10, 5
    w, V = eig.eigh_lowest(H, nev + nex)
    r = chase.solve(dev_colmajor(H), nev, nex, V0=torch.from_numpy(V).cuda())
    # The warm start's Rayleigh-Ritz already meets tol: no filter at all.
    assert r.status == chase.CHASE_OK and r.info["iterations"] == 1
    assert r.info["matvecs_filter"] == 0
    _check_against_oracle(H, r, nev)


def test_failure_modes():
    torch = torch_cuda()
    H = synth.dk_matrix(300, seed=7)
    Hn = H.copy()
    Hn[17, 5] = np.nan
    Hn[5, 17] = np.nan
    with pytest.raises(chase.ChaseError) as ei:
        chase.solve(dev_colmajor(Hn), 5, 3)
    assert ei.value.status == chase.CHASE_ENONFINITE
    r = chase.solve(dev_colmajor(H), 5, 3, max_iter=1, initial_degree=2,
                    allow_noconv=True)
    assert r.status == chase.CHASE_ENOCONV and r.info["nconv"] < 5
    assert np.all(np.isfinite(r.eigvals)) and np.all(np.diff(r.eigvals) >= 0)
    with pytest.raises(chase.ChaseError) as ei:
        chase.solve(dev_colmajor(H), 200, 150)
    assert ei.value.status == chase.CHASE_EINVAL
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(chase.ChaseError) as ei:
        chase.solve(dev_colmajor(H), 5, 3, workspace=small)
    assert ei.value.status == chase.CHASE_ENOMEM


def test_caller_workspace_and_profile_counters():
    torch = torch_cuda()
    H = synth.dk_matrix(1000, seed=8)
    nbytes = chase.workspace_bytes(1000, 10, 6)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    r = chase.solve(dev_colmajor(H), 10, 6, workspace=ws, profile=1)
    _check_against_oracle(H, r, 10)
    assert r.info["filter_launches"] > 0 and r.info["t_filter_kernels"] > 0
    assert r.info["filter_flops"] == 8.0 * 1000 * 1000 * r.info["matvecs_filter"]
    # Every FP64 H-times-block launch is timed: filter steps plus the
    # Lanczos products plus one Rayleigh-Ritz product per iteration.
    lz = chase.default_opts()
    assert r.info["gemm_launches"] == (r.info["filter_launches"] + lz.lanczos_steps
                                       + r.info["iterations"])
    assert r.info["gemm_flops"] == 8.0 * 1000 * 1000 * r.info["matvecs_total"]
    assert r.info["gemm_time"] >= r.info["t_filter_kernels"] > 0


def test_iteration_callback_reports_and_stops():
    torch_cuda()
    H = synth.dk_matrix(1200, seed=9)
    dH = dev_colmajor(H)
    seen = []
    full = chase.solve(dH, 12, 6, on_iteration=lambda i: seen.append(dict(i)) and False)
    assert [s["iterations"] for s in seen] == list(range(1, full.info["iterations"] + 1))
    assert all(a["nconv"] <= b["nconv"] for a, b in zip(seen, seen[1:]))
    assert seen[-1]["nconv"] == 12
    # Same pairs as without a callback (the callback only observes).
    plain = chase.solve(dH, 12, 6)
    assert np.array_equal(plain.eigvals, full.eigvals)
    # A true return stops after that iteration with the best pairs so far.
    stop = chase.solve(dH, 12, 6, on_iteration=lambda i: i["iterations"] >= 2,
                       allow_noconv=True)
    assert stop.info["iterations"] == 2
    assert stop.status == (chase.CHASE_OK if seen[1]["nconv"] >= 12 else chase.CHASE_ENOCONV)
    assert stop.info["nconv"] == seen[1]["nconv"]


def test_stall_behind_locked_pairs_is_refined():
    """A served request (N = 16000 D + K, seed 1086) whose pair 117 stalled
    at 1.4e-10 * ||H|| behind pairs locked just under tol: the whole-block
    Rayleigh-Ritz step must let it converge, in both precisions."""
    torch_cuda()
    N, nev, nex = 16000, 119, 48
    H = synth.dk_matrix_device(N, seed=1086, std=0.02, decay=200.0)
    out = {}
    for prec in (chase.CHASE_MIXED, chase.CHASE_FP64):
        r = chase.solve(H, nev, nex, 1e-10, 20, precision=prec)
        assert r.status == chase.CHASE_OK and r.info["iterations"] < 60
        assert np.all(r.resid <= 1e-10 * r.info["hnorm_est"])
        out[prec] = r
    a, b = out[chase.CHASE_MIXED], out[chase.CHASE_FP64]
    assert np.abs(a.eigvals - b.eigvals).max() <= 1e-10 * np.abs(b.eigvals).max()


@pytest.mark.parametrize("N,nev,nex,seed", [(2000, 20, 10, 0), (1500, 40, 16, 4)])
def test_graph_replayed_jacobi_sweeps_match_direct_launches(N, nev, nex, seed):
    """Each Jacobi sweep replayed from a captured HIP graph (replayed many
    times per solve, with filter / QR work and host synchronisations in
    between) gives bitwise the result of launching its kernels one by one."""
    torch_cuda()
    if seed == 4:
        H, _, _ = synth.planted_matrix(N, seed=seed, n_clusters=8, cluster_size=10)
    else:
        H = synth.dk_matrix(N, seed=seed)
    dH = dev_colmajor(H)
    g = chase.solve(dH, nev, nex, graphs=1)
    d = chase.solve(dH, nev, nex, graphs=0)
    g2 = chase.solve(dH, nev, nex, graphs=1)
    for r in (d, g2):
        assert np.array_equal(g.eigvals, r.eigvals)
        assert np.array_equal(host(g.V), host(r.V))
        assert g.info["iterations"] == r.info["iterations"]
    _check_against_oracle(H, g, nev)


def test_largest_subspace_1024():
    """nev + nex at the ABI's maximum (1024): Jacobi at order 1024, filter
    products split into column pieces, the Cholesky factor at full size."""
    torch_cuda()
    N, nev, nex = 2600, 700, 324
    H = synth.dk_matrix(N, seed=21)
    r = chase.solve(dev_colmajor(H), nev, nex, 1e-10, 20)
    assert r.status == chase.CHASE_OK
    _check_against_oracle(H, r, nev)


def test_degenerate_eigenvalue_across_the_cut():
    """lambda_nev = lambda_{nev+1} exactly (a triple eigenvalue straddling
    the cut) and a 5-fold one inside the wanted set: any orthonormal basis
    of a degenerate eigenspace is correct, so eigenvalues, residuals and
    orthogonality are checked, and the returned vectors of each degenerate
    eigenvalue must lie in its planted eigenspace."""
    torch_cuda()
    N, nev, nex = 800, 12, 8
    rng = np.random.default_rng(3)
    lam = np.sort(np.concatenate([[1.0, 1.1], [1.3] * 5, [1.5, 1.6, 1.7, 1.8],
                                  [2.0] * 3, rng.uniform(2.5, 9.0, N - 14)]))
    H, lam, Q = synth.planted_matrix(N, seed=5, lam=lam)
    r = chase.solve(dev_colmajor(H), nev, nex, 1e-10, 20)
    assert r.status == chase.CHASE_OK
    assert np.abs(r.eigvals - lam[:nev]).max() <= 1e-10 * lam.max()
    V = host(r.V)
    res = np.linalg.norm(H @ V - V * r.eigvals[None, :], axis=0) / lam.max()
    assert res.max() <= 1e-10
    assert np.abs(V.conj().T @ V - np.eye(nev)).max() <= 1e-12
    for value in (1.3, 2.0):
        cols = np.nonzero(np.abs(r.eigvals - value) < 1e-6)[0]
        P = Q[:, np.abs(lam - value) < 1e-12]
        # residual / gap bounds the part outside the planted eigenspace
        out = np.linalg.norm(V[:, cols] - P @ (P.conj().T @ V[:, cols]), axis=0)
        assert out.max() <= 1e-8, out.max()


def test_scalar_matrix():
    """H = c I: every vector is an eigenvector, Lanczos breaks down at once
    and the filter interval is empty; the solve must return c with
    orthonormal vectors."""
    torch = torch_cuda()
    N, nev, nex = 300, 6, 4
    H = 3.25 * np.eye(N, dtype=np.complex128)
    r = chase.solve(dev_colmajor(H), nev, nex, 1e-10, 20)
    assert r.status == chase.CHASE_OK
    assert np.all(np.abs(r.eigvals - 3.25) <= 1e-12)
    V = host(r.V)
    assert np.abs(V.conj().T @ V - np.eye(nev)).max() <= 1e-12
    assert np.linalg.norm(H @ V - V * r.eigvals[None, :], axis=0).max() <= 1e-10 * 3.25


@pytest.mark.parametrize("precision", [chase.CHASE_FP64, chase.CHASE_MIXED])
def test_h_is_read_only_and_padding_is_ignored(precision):
    """H with leading dimension N + 5 (NaN in the padding rows): the solve
    reads only the N x N matrix and writes none of it."""
    torch = torch_cuda()
    N, ld = 700, 705
    H = synth.dk_matrix(N, seed=4)
    buf = torch.full((N, ld), complex("nan"), dtype=torch.complex128, device="cuda")
    dH = buf.t()[:N, :]                                 # column-major, ldh = 705
    dH.copy_(torch.from_numpy(H))
    before = torch.view_as_real(buf).view(torch.int64).clone()
    r = chase.solve(dH, 8, 6, precision=precision)
    assert r.status == chase.CHASE_OK
    assert torch.equal(torch.view_as_real(buf).view(torch.int64), before)
    _check_against_oracle(H, r, 8)


def test_minimal_chase_solve_call():
    """chase_solve, the minimal form: null stream, its own workspace, default
    options; H column-major with ldh = N, V column-major N x nev."""
    import ctypes
    torch = torch_cuda()
    N, nev, nex = 1200, 12, 8
    H = synth.dk_matrix(N, seed=21)
    dH = dev_colmajor(H)
    out = torch.empty((nev, N), dtype=torch.complex128, device="cuda")
    ev = np.zeros(nev)
    torch.cuda.synchronize()
    st = chase.lib().chase_solve(ctypes.c_void_p(dH.data_ptr()), N, nev, nex, 1e-10, 20,
                                 ev.ctypes.data_as(ctypes.c_void_p),
                                 ctypes.c_void_p(out.data_ptr()))
    assert st == chase.CHASE_OK, chase.last_error()
    res = chase.SolveResult(ev, out.t(), np.zeros(nev), st)
    _check_against_oracle(H, res, nev)
    full = chase.solve(dH, nev, nex, 1e-10, 20)       # chase_solve_ex, defaults
    assert np.array_equal(full.eigvals, ev)
    assert np.array_equal(host(full.V), host(out.t()))


def test_degree_max_one_single_step_filter():
    """degree_max = 1: one filter step per iteration (plain subspace
    iteration with the first Chebyshev polynomial); on a matrix with a wide
    gap below the unwanted part it still reaches the bar."""
    torch_cuda()
    N, nev, nex = 400, 4, 4
    lam = np.concatenate([[0.1, 0.2, 0.3, 0.4], np.linspace(5.0, 6.0, N - 4)])
    Q = synth.random_block(N, N, seed=7)
    Q, _ = np.linalg.qr(Q)
    H = (Q * lam[None, :]) @ Q.conj().T
    H = 0.5 * (H + H.conj().T)
    r = chase.solve(dev_colmajor(H), nev, nex, tol=1e-10, degree_max=1, max_iter=400)
    assert r.status == chase.CHASE_OK
    # at most one step per active column per iteration
    assert 0 < r.info["matvecs_filter"] <= r.info["iterations"] * (nev + nex)
    _check_against_oracle(H, r, nev)
    assert np.abs(r.eigvals - lam[:nev]).max() <= 1e-10 * 6.0
