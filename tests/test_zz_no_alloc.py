"""The allocation-free reduced eigensolve (chase_heevj_noalloc) against the
allocating one (chase_heevj), through the C ABI on the GPU.

The two run the same kernels in the same order, so the eigenvalues and
eigenvectors must agree bit for bit.  Two calls in a row, the second on a
smaller matrix, check that the static scratch array keeps no state that
matters from one call to the next; both are also checked against the
oracle's eigenvalues (relative 1e-13 of the norm, the Jacobi accuracy)."""
import ctypes

import numpy as np
import pytest

from oracle import eig
from paper_2006_08498_amd import chase, synth
from tests.gpu_util import dev_block, host, torch_cuda

pytestmark = pytest.mark.gpu


def _hermitian(n, seed):
    A = synth.random_block(n, n, seed=seed)
    return 0.5 * (A + A.conj().T)


@pytest.mark.parametrize("sizes", [(300, 120), (512, 1)])
def test_noalloc_matches_allocating_call_twice(sizes):
    torch = torch_cuda()
    for k, n in enumerate(sizes):
        print(f"heevj_noalloc: call {k} n={n}", flush=True)
        G = _hermitian(n, seed=100 + n)
        dG = dev_block(G)
        w_ref, Y_ref = chase.heevj(dG)
        Y = torch.empty_like(dG)
        w, Y = chase.heevj_noalloc(dG, Y)
        assert np.array_equal(w, w_ref)
        assert np.array_equal(host(Y), host(Y_ref))
        assert np.array_equal(host(dG), G)            # G is not modified
        w_o = eig.eigh_lowest(G, n)[0]
        assert np.abs(w - w_o).max() <= 1e-13 * max(1.0, np.abs(w_o).max()) * n
        Yh = host(Y)
        assert np.abs(Yh.conj().T @ Yh - np.eye(n)).max() <= 1e-13 * n
        assert np.abs(G @ Yh - Yh * w[None, :]).max() <= 1e-12 * max(1.0, np.abs(w).max())


def test_noalloc_refuses_orders_above_the_scratch():
    torch = torch_cuda()
    dG = torch.zeros((513, 513), dtype=torch.complex128, device="cuda")
    w = np.zeros(513)
    st = chase.lib().chase_heevj_noalloc(ctypes.c_void_p(dG.data_ptr()), 513,
                                         w.ctypes.data_as(ctypes.c_void_p),
                                         ctypes.c_void_p(dG.data_ptr()), None)
    assert st == chase.CHASE_EINVAL
    assert "allocation-free" in chase.last_error()
