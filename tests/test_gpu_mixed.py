"""Mixed-precision form (GPU, via the C ABI): the FP32 filter step, the
complex64 shadow of H, and mixed solves against the FP64 oracle at the same
accuracy bar as the plain FP64 path."""
import numpy as np
import pytest

from oracle import eig, steps
from paper_2006_08498_amd import chase, synth
from tests.gpu_util import dev_colmajor, host, torch_cuda

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _c64(A):
    return np.asarray(A).astype(np.complex64)


@pytest.mark.parametrize("N,n", [(5, 3), (63, 16), (700, 33), (1301, 140), (4100, 16),
                                 (2049, 161)])
def test_filter_step_fp32_elementwise(N, n):
    """Against FP64 arithmetic on the FP32-rounded inputs: the bound is the
    forward error of FP32 complex dot products of length N."""
    torch = torch_cuda()
    H = synth.dk_matrix(N, seed=N + 1)
    Y = _c64(synth.random_block(N, n, seed=3))
    X = _c64(synth.random_block(N, n, seed=4))
    a, b, g = np.float32(0.37), np.float32(-1.3), np.float32(0.55)
    Hc = chase.shadow_c(dev_colmajor(H))
    assert np.array_equal(host(Hc), _c64(H))                 # round to nearest
    W = host(chase.filter_step_c(Hc, torch.from_numpy(Y).cuda(),
                                 torch.from_numpy(X).cuda(), a, b, g))
    H64, Y64, X64 = (_c64(H).astype(np.complex128), Y.astype(np.complex128),
                     X.astype(np.complex128))
    ref = steps.cheb_step(H64, Y64, X64, float(a), float(b), float(g))
    bound = (4.0 * (N + 2) * U32 * abs(float(a)) * (np.abs(H64) @ np.abs(Y64))
             + 8 * U32 * (abs(float(b)) * np.abs(Y64) + abs(float(g)) * np.abs(X64)))
    err = np.abs(W.astype(np.complex128) - ref)
    assert np.all(err <= bound), (err / bound).max()


def _check(H, r, nev):
    w_ref, _ = eig.eigh_lowest(H, nev)
    hn = np.abs(np.linalg.eigvalsh(H)).max()
    V = host(r.V)
    rel = np.abs(r.eigvals - w_ref) / np.abs(w_ref)
    res = np.linalg.norm(H @ V - V * r.eigvals[None, :], axis=0) / hn
    assert rel.max() <= 1e-10, rel.max()
    assert res.max() <= 1e-10, res.max()
    assert np.abs(V.conj().T @ V - np.eye(nev)).max() <= 1e-12
    return rel, res


@pytest.mark.parametrize("N,nev,nex,seed", [(3000, 30, 10, 0), (1700, 12, 6, 1)])
def test_mixed_solve_matches_oracle(N, nev, nex, seed):
    """The D + K family of the mixed-precision workload (std 0.01, decay
    1000) at sizes the oracle finishes; per-eigenpair error is checked."""
    torch_cuda()
    H = synth.dk_matrix(N, seed=seed, std=0.01, decay=1000.0)
    dH = dev_colmajor(H)
    r = chase.solve(dH, nev, nex, 1e-10, 20, precision=chase.CHASE_MIXED)
    assert r.status == chase.CHASE_OK
    assert r.info["matvecs_filter_fp32"] > 0
    assert r.info["matvecs_filter_fp32"] <= r.info["matvecs_filter"]
    _check(H, r, nev)
    r64 = chase.solve(dH, nev, nex, 1e-10, 20)
    assert np.abs(r.eigvals - r64.eigvals).max() <= 1e-10 * np.abs(r64.eigvals).max()


def test_mixed_switch_tolerance_extremes():
    """switch_tol above every residual filters all in FP64; tiny switch_tol
    keeps FP32 until each vector stalls; both reach the same bar."""
    torch_cuda()
    H = synth.dk_matrix(1200, seed=5, std=0.01, decay=1000.0)
    dH = dev_colmajor(H)
    a = chase.solve(dH, 10, 6, 1e-10, 20, precision=chase.CHASE_MIXED, switch_tol=1e3)
    _check(H, a, 10)
    # First iteration always starts in FP32 (residuals unknown); after that
    # no column is above the switch tolerance.
    first_it = a.info["matvecs_filter_fp32"]
    assert first_it <= 16 * 20
    b = chase.solve(dH, 10, 6, 1e-10, 20, precision=chase.CHASE_MIXED, switch_tol=1e-14)
    _check(H, b, 10)
    assert b.info["matvecs_filter_fp32"] >= a.info["matvecs_filter_fp32"]


@pytest.mark.parametrize("switch_tol", [1e-7, 1e-9])
def test_mixed_switch_below_fp32_floor_still_converges(switch_tol):
    """A switch level at or below what FP32 filtering can reach: vectors
    that stall there must move to FP64 and the solve must still converge."""
    torch_cuda()
    H = synth.dk_matrix(4000, seed=2, std=0.01, decay=1000.0)
    r = chase.solve(dev_colmajor(H), 40, 16, 1e-10, 20, precision=chase.CHASE_MIXED,
                    switch_tol=switch_tol)
    assert r.status == chase.CHASE_OK
    assert r.info["matvecs_filter_fp32"] > 0
    _check(H, r, 40)
