"""Ingesting H through the C ABI, bit for bit against the oracle's
completion of the stored triangle: row stripes from device and host memory
(ragged stripes, padded leading dimensions, several staging chunks) and
in-place completion from either triangle; at N = 24000, a device-generated
matrix must come back unchanged."""
import time

import numpy as np
import pytest

from oracle import steps
from paper_2006_08498_amd import chase, synth
from tests.gpu_util import host, torch_cuda

pytestmark = pytest.mark.gpu


def _bits(X):
    return np.ascontiguousarray(X).view(np.uint64)


def _colmajor_buffer(torch, N, ldh, fill):
    """A column-major N x N view (leading dimension ldh) of a buffer whose
    padding rows hold `fill` too."""
    buf = torch.full((N, ldh), fill, dtype=torch.complex128, device="cuda")
    return buf, buf.t()[:N, :]


def _random(N, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))


@pytest.mark.parametrize("N,ldh,pad", [(1000, 1000, 0), (1001, 1004, 5), (1, 1, 0), (33, 40, 2)])
def test_device_stripes_in_any_order(N, ldh, pad):
    torch = torch_cuda()
    A = _random(N, N)
    cuts = sorted({0, N} | {c for c in (1, 38, N // 2, (3 * N) // 4) if 0 < c < N})
    stripes = list(zip(cuts[:-1], cuts[1:]))[::-1]      # bottom stripe first
    buf, H = _colmajor_buffer(torch, N, ldh, complex("nan"))
    for r0, r1 in stripes:
        print(f"ingest N={N} rows {r0}:{r1}", flush=True)
        # rows r0..r1-1 with ldr = N + pad; columns right of the diagonal are
        # filled with NaN, which must never be read
        rows = np.full((r1 - r0, N + pad), complex("nan"))
        for r in range(r0, r1):
            rows[r - r0, :r + 1] = A[r, :r + 1]
        chase.ingest_rows(H, torch.from_numpy(rows).cuda(), r0)
    want = steps.hermitian_from_triangle(A, lower=True)
    assert np.array_equal(_bits(host(H)), _bits(want))
    assert torch.isnan(buf[:, N:]).all()                # padding untouched


@pytest.mark.parametrize("pinned", [False, True])
def test_host_stripes_stream_in_several_chunks(pinned):
    torch = torch_cuda()
    N = 6000                                    # 64 MiB chunks of 672 rows: 9 of them
    A = _random(N, 11)
    buf, H = _colmajor_buffer(torch, N, N, complex("nan"))
    # Two stripes, the upper one from a numpy array (pageable) or a pinned
    # tensor; each row holds its full width.
    for r0, r1 in ((2500, N), (0, 2500)):
        print(f"host ingest pinned={pinned} rows {r0}:{r1}", flush=True)
        rows = A[r0:r1]
        if pinned:
            t = torch.empty(rows.shape, dtype=torch.complex128, pin_memory=True)
            t.copy_(torch.from_numpy(np.ascontiguousarray(rows)))
            chase.ingest_rows(H, t, r0)
        else:
            chase.ingest_rows(H, np.ascontiguousarray(rows), r0)
    want = steps.hermitian_from_triangle(A, lower=True)
    assert np.array_equal(_bits(host(H)), _bits(want))


@pytest.mark.parametrize("N,ldh", [(1001, 1003), (64, 64), (1, 2)])
@pytest.mark.parametrize("uplo", ["L", "U"])
def test_complete_in_place_from_either_triangle(N, ldh, uplo):
    torch = torch_cuda()
    A = _random(N, 3 * N)
    print(f"complete N={N} ldh={ldh} uplo={uplo}", flush=True)
    buf, H = _colmajor_buffer(torch, N, ldh, complex("nan"))
    H.copy_(torch.from_numpy(A))
    chase.hermitian_complete(H, uplo)
    want = steps.hermitian_from_triangle(A, lower=(uplo == "L"))
    assert np.array_equal(_bits(host(H)), _bits(want))
    assert torch.isnan(buf[:, N:]).all()


def test_full_size_round_trip_24000():
    """A D + K matrix of N = 24000 generated on the device, sent back through
    host rows (pinned, streamed) and through one triangle completed in place,
    is unchanged to the bit."""
    torch = torch_cuda()
    N = 24000
    print("full size: generate", flush=True)
    H = synth.dk_matrix_device(N, seed=0)                # column-major
    rows = torch.empty((N, N), dtype=torch.complex128, pin_memory=True)
    rows.copy_(H)                                         # row-major host copy
    torch.cuda.synchronize()
    buf, H2 = _colmajor_buffer(torch, N, N, complex("nan"))
    print("full size: ingest from pinned host rows", flush=True)
    t0 = time.perf_counter()
    chase.ingest_rows(H2, rows, 0)
    dt = time.perf_counter() - t0
    print(f"full size: {8.0 * N * (N + 1) / dt / 1e9:.1f} GB/s of lower triangle from the host",
          flush=True)
    same = lambda X, Y: torch.equal(torch.view_as_real(X).view(torch.int64),
                                    torch.view_as_real(Y).view(torch.int64))
    assert same(H2, H)
    print("full size: complete from the upper triangle", flush=True)
    H2.copy_(torch.triu(H))                               # lower half zeroed
    chase.hermitian_complete(H2, "U")
    assert same(H2, H)
