"""Serving (continuous batching) on the GPU, via the C ABI.

Each request's result must be the same alone and in the mix (bitwise: every
kernel reduces in a fixed order and each solve has its own workspace), and
every served result must meet the end-to-end bar against the oracle;
admission must respect the memory budget; H may come from a caller buffer
or be produced at admission by a fill callback."""
import ctypes

import numpy as np
import pytest

from paper_2006_08498_amd import chase, synth
from tests.gpu_util import check_against_oracle, dev_colmajor, host, torch_cuda

pytestmark = pytest.mark.gpu

CASES = [(1500, 10, 4, 11), (2600, 20, 8, 12), (900, 8, 3, 13), (3000, 30, 12, 14)]


def _solo(H, nev, nex):
    return chase.solve(H, nev, nex, 1e-10, 20)


def test_results_same_alone_and_in_the_mix():
    torch_cuda()
    hmats = [synth.dk_matrix(N, seed=s) for N, _, _, s in CASES]
    mats = [dev_colmajor(H) for H in hmats]
    solo = [_solo(H, nev, nex) for H, (N, nev, nex, s) in zip(mats, CASES)]
    with chase.Server(slots=3) as srv:
        tickets = [srv.submit(H, nev, nex) for H, (N, nev, nex, s) in zip(mats, CASES)]
        outs = []
        for t in tickets:
            assert srv.wait(t, timeout=120.0)
            outs.append(srv.poll(t))
        st = srv.stats()
    assert st["peak_running"] >= 2          # the work overlapped
    for a, b in zip(solo, outs):
        assert np.array_equal(a.eigvals, b.eigvals)
        assert np.array_equal(host(a.V), host(b.V))
        assert a.info["iterations"] == b.info["iterations"]
        assert b.latency_s >= b.gpu_s >= 0 and b.queued_s >= 0
    for H, b, (N, nev, nex, _) in zip(hmats, outs, CASES):
        check_against_oracle(H, b, nev)


def test_fused_filter_same_results_and_fuses():
    """With cross-request filter fusion the results are bitwise the solo
    ones, and the grouped launches really held steps of several solves."""
    torch_cuda()
    hmats = [synth.dk_matrix(N, seed=s) for N, _, _, s in CASES]
    mats = [dev_colmajor(H) for H in hmats]
    solo = [_solo(H, nev, nex) for H, (N, nev, nex, s) in zip(mats, CASES)]
    with chase.Server(slots=4, fuse=True) as srv:
        tickets = [srv.submit(H, nev, nex) for H, (N, nev, nex, s) in zip(mats, CASES)]
        outs = []
        for t in tickets:
            assert srv.wait(t, timeout=120.0)
            outs.append(srv.poll(t))
        st = srv.stats()
    for a, b in zip(solo, outs):
        assert np.array_equal(a.eigvals, b.eigvals)
        assert np.array_equal(host(a.V), host(b.V))
    for H, b, (N, nev, nex, _) in zip(hmats, outs, CASES):
        check_against_oracle(H, b, nev)
    total = sum(r.info["matvecs_filter"] for r in outs)
    assert st["fused_ticks"] > 0 and st["fused_steps"] > st["fused_ticks"]
    assert st["fused_steps"] <= total


def test_budget_admits_one_at_a_time():
    torch = torch_cuda()
    same = [(2600, 20, 8, 31), (2600, 20, 8, 32), (2600, 20, 8, 33)]
    mats = [dev_colmajor(synth.dk_matrix(N, seed=s)) for N, _, _, s in same]
    # Budget for one footprint (H is the caller's, so: workspace, output and
    # alignment slack): three equal requests must run one by one.
    fp = chase.workspace_bytes(2600, 20, 8) + 16 * 2600 * 20 + 768
    budget = fp + 4096
    with chase.Server(budget_bytes=budget, slots=4) as srv:
        tickets = [srv.submit(H, nev, nex) for H, (N, nev, nex, s) in zip(mats, same)]
        for t in tickets:
            assert srv.wait(t, timeout=120.0)
            srv.poll(t)
        st = srv.stats()
        assert st["peak_bytes"] <= budget
        assert st["peak_running"] == 1
        # A request whose footprint exceeds the budget is refused at once.
        big = torch.empty((1, 1), dtype=torch.complex128, device="cuda")
        with pytest.raises(chase.ChaseError) as ei:
            srv.submit(dev_colmajor(synth.dk_matrix(4000, seed=1)), 200, 100)
        assert ei.value.status == chase.CHASE_ENOMEM
        del big


def test_fill_callback_generates_h_at_admission():
    torch_cuda()
    N, nev, nex, seed = 2200, 12, 6, 21
    lib = synth._slib()

    def fill(ptr, n, ld, stream):
        return lib.synth_dk(ctypes.c_void_p(ptr), ld, n, seed, 0.02, 200.0, 1.0, 6.0,
                            ctypes.c_void_p(stream))

    ref = _solo(synth.dk_matrix_device(N, seed=seed), nev, nex)
    with chase.Server(slots=2) as srv:
        t = srv.submit_fill(fill, N, nev, nex)
        assert srv.wait(t, timeout=120.0)
        out = srv.poll(t)
    assert np.array_equal(ref.eigvals, out.eigvals)
    assert np.array_equal(host(ref.V), host(out.V))
    check_against_oracle(synth.dk_matrix(N, seed=seed), out, nev)


def test_shortest_first_admission_and_aging():
    """One slot: after the first admission, shortest-first takes the queued
    requests by estimated work N^2 (nev + nex); with aging 0 every waiting
    request counts as aged and the order is arrival order.  Results are
    those of solo solves either way."""
    torch_cuda()
    reqs = [(3000, 30, 12, 41), (2800, 20, 8, 42), (1200, 10, 4, 43), (2000, 16, 6, 44)]
    hmats = [synth.dk_matrix(N, seed=s) for N, _, _, s in reqs]
    mats = [dev_colmajor(H) for H in hmats]
    solo = [_solo(H, nev, nex) for H, (N, nev, nex, s) in zip(mats, reqs)]
    work = [N * N * (nev + nex) for N, nev, nex, _ in reqs]
    for aging, expect_fifo in ((None, False), (0.0, True)):
        with chase.Server(slots=1, shortest_first=True, aging_s=aging) as srv:
            tickets = [srv.submit(H, nev, nex) for H, (N, nev, nex, s) in zip(mats, reqs)]
            outs = []
            for t in tickets:
                assert srv.wait(t, timeout=120.0)
                outs.append(srv.poll(t))
        order = sorted(range(len(reqs)), key=lambda i: outs[i].queued_s)
        if expect_fifo:
            assert order == list(range(len(reqs)))
        else:
            rest = order[1:]
            assert [work[i] for i in rest] == sorted(work[i] for i in rest)
        for a, b in zip(solo, outs):
            assert np.array_equal(a.eigvals, b.eigvals)
        for H, b, (N, nev, nex, _) in zip(hmats, outs, reqs):
            check_against_oracle(H, b, nev)


def test_device_h_written_by_an_async_kernel_without_host_sync():
    """H produced on the device by a kernel still running when submit is
    called (no synchronisation by the caller): the binding orders the
    server's read after it, and the result is the solo one."""
    torch_cuda()
    N, nev, nex, seed = 2400, 14, 6, 51
    ref = _solo(synth.dk_matrix_device(N, seed=seed), nev, nex)
    with chase.Server(slots=2) as srv:
        dH = synth.dk_matrix_device(N, seed=seed)   # enqueued, not synchronised
        t = srv.submit(dH, nev, nex)
        assert srv.wait(t, timeout=120.0)
        out = srv.poll(t)
    assert np.array_equal(ref.eigvals, out.eigvals)
    assert np.array_equal(host(ref.V), host(out.V))
    check_against_oracle(synth.dk_matrix(N, seed=seed), out, nev)


@pytest.mark.parametrize("kw,msg", [
    (dict(tol=float("inf")), "tol"),
    (dict(tol=0.0), "tol"),
    (dict(max_iter=0), "max_iter"),
    (dict(switch_tol=0.0), "switch_tol"),
    (dict(lanczos_runs=65), "lanczos_runs"),
    (dict(graphs=2), "graphs"),
    (dict(degree_max=65), "degree_max"),
])
def test_bad_requests_refused_at_submission(kw, msg):
    """A served request is checked like chase_solve_ex before it is queued."""
    torch_cuda()
    H = dev_colmajor(synth.dk_matrix(200, seed=1))
    tol = kw.pop("tol", 1e-10)
    dmax = kw.pop("degree_max", 20)
    with chase.Server(slots=1) as srv:
        with pytest.raises(chase.ChaseError) as ei:
            srv.submit(H, 4, 4, tol=tol, degree_max=dmax, **kw)
        assert ei.value.status == chase.CHASE_EINVAL
        assert msg in str(ei.value)
        assert srv.stats()["queued"] == 0 and srv.stats()["running"] == 0


def test_a_result_is_collected_once():
    """After one poll collects a result, the ticket is gone (a second poll is
    refused, not a second copy or free); a poll with no output buffer is
    refused and leaves the result to collect."""
    torch = torch_cuda()
    H = dev_colmajor(synth.dk_matrix(600, seed=2))
    with chase.Server(slots=1) as srv:
        t = srv.submit(H, 5, 4)
        assert srv.wait(t, timeout=120.0)
        ev = np.zeros(5)
        L = chase.lib()
        st = L.chase_server_poll(srv._s, t, ev.ctypes.data_as(ctypes.c_void_p), None, None, 600,
                                 None, None)
        assert st == chase.CHASE_EINVAL
        out = srv.poll(t)
        assert out is not None and out.status == chase.CHASE_OK
        dV = torch.empty((5, 600), dtype=torch.complex128, device="cuda")
        st = L.chase_server_poll(srv._s, t, ev.ctypes.data_as(ctypes.c_void_p), None,
                                 ctypes.c_void_p(dV.data_ptr()), 600, None, None)
        assert st == chase.CHASE_EINVAL
        assert b"unknown ticket" in L.chase_server_last_error()
