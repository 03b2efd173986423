"""C ABI checks that need no GPU: exports, struct layout, validation before
device work, and the host-side control logic against the oracle."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import steps
from paper_2006_08498_amd import chase, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chase_mi355x.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chase_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_function_is_exported_and_bound():
    L = chase.lib()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert sorted(chase.SIGNATURES) == names


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "s.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "chase_mi355x.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(chase_opts),'
        ' sizeof(chase_info), offsetof(chase_opts, dV0),'
        ' offsetof(chase_info, t_total), sizeof(chase_z)); return 0;}\n')
    exe = tmp_path / "s"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True,
                                       check=True).stdout.split()))
    assert got == [ctypes.sizeof(chase.ChaseOpts), ctypes.sizeof(chase.ChaseInfo),
                   chase.ChaseOpts.dV0.offset, chase.ChaseInfo.t_total.offset, 16]


def test_defaults():
    o = chase.default_opts()
    assert (o.precision, o.max_iter, o.initial_degree, o.degree_extra,
            o.lanczos_steps, o.lanczos_runs, o.seed) == (0, 100, 20, 2, 25, 4, 0)
    assert o.switch_tol == 1e-7 and o.dV0 is None and o.profile == 0 and o.graphs == 1


@pytest.mark.parametrize("args,msg", [
    ((10, 20, 0, 1e-10, 20), "nev + nex"),
    ((0, 1, 0, 1e-10, 20), "N must be"),
    ((10, 0, 0, 1e-10, 20), "nev must be"),
    ((10, 2, -1, 1e-10, 20), "nex must be"),
    ((10, 2, 1, 0.0, 20), "tol"),
    ((10, 2, 1, 1e-10, 0), "degree_max"),
    ((10, 2, 1, float("inf"), 20), "tol"),
    ((10, 2, 1, 1e-10, 65), "degree_max"),
])
def test_invalid_arguments_rejected_before_device_work(args, msg):
    L = chase.lib()
    N, nev, nex, tol, dmax = args
    ev = np.zeros(max(nev, 1))
    # A non-null dummy device pointer: validation must fail before any use.
    st = L.chase_solve(ctypes.c_void_p(16), N, nev, nex, tol, dmax,
                       ev.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(16))
    assert st == chase.CHASE_EINVAL
    assert msg in chase.last_error()


def test_noalloc_eigensolve_rejects_orders_beyond_its_scratch_before_device_work():
    L = chase.lib()
    w = np.zeros(4)
    for n in (0, 513):
        st = L.chase_heevj_noalloc(ctypes.c_void_p(16), n, w.ctypes.data_as(ctypes.c_void_p),
                                   ctypes.c_void_p(16), None)
        assert st == chase.CHASE_EINVAL
        assert "allocation-free" in chase.last_error()


def test_null_pointers_rejected():
    L = chase.lib()
    ev = np.zeros(2)
    st = L.chase_solve(None, 10, 2, 1, 1e-10, 20, ev.ctypes.data_as(ctypes.c_void_p),
                       ctypes.c_void_p(16))
    assert st == chase.CHASE_EINVAL and "dH" in chase.last_error()


def test_mixed_precision_flag_validated():
    L = chase.lib()
    o = chase.default_opts(precision=7)
    ev = np.zeros(2)
    st = L.chase_solve_ex(ctypes.c_void_p(16), 10, 10, 2, 1, 1e-10, 20,
                          ev.ctypes.data_as(ctypes.c_void_p), None, ctypes.c_void_p(16),
                          10, None, 0, None, ctypes.byref(o), None)
    assert st == chase.CHASE_EINVAL


@pytest.mark.parametrize("kw,msg", [
    (dict(v0_cols=-1), "v0_cols"), (dict(v0_cols=4), "v0_cols"),
    (dict(out_cols=1), "out_cols"), (dict(out_cols=4), "out_cols"),
])
def test_sequence_columns_validated(kw, msg):
    L = chase.lib()
    o = chase.default_opts(**kw)
    ev = np.zeros(2)
    st = L.chase_solve_ex(ctypes.c_void_p(16), 10, 10, 2, 1, 1e-10, 20,
                          ev.ctypes.data_as(ctypes.c_void_p), None, ctypes.c_void_p(16),
                          10, None, 0, None, ctypes.byref(o), None)
    assert st == chase.CHASE_EINVAL and msg in chase.last_error()


def test_workspace_bytes():
    a = chase.workspace_bytes(2000, 20, 10)
    b = chase.workspace_bytes(4000, 20, 10)
    c = chase.workspace_bytes(24000, 100, 40)
    assert 0 < a < b < c
    # Four N x ne complex blocks dominate.
    assert c >= 4 * 24000 * 140 * 16
    assert chase.workspace_bytes(10, 20, 0) == 0


def test_degrees_match_oracle_exactly():
    rng = np.random.default_rng(0)
    n = 400
    alpha, beta = 3.7, 12.0
    c, e = steps.interval(alpha, beta)
    theta = np.sort(rng.uniform(1.0, 3.9, n))
    res = 10.0 ** rng.uniform(-12, 0, n)
    tol_abs = 1e-10 * 12.0
    for dmax, extra in [(20, 2), (30, 0), (21, 1), (2, 2)]:
        got = chase.degrees(theta, res, tol_abs, alpha, beta, dmax, extra)
        ref = [steps.degree(r, tol_abs, t, c, e, dmax, extra) for t, r in zip(theta, res)]
        assert np.array_equal(got, np.array(ref)), (dmax, extra)


def test_lanczos_bounds_match_oracle():
    N, ne = 3000, 30
    H = synth.dk_matrix(300, seed=11)
    V0 = synth.random_block(300, 4, seed=11)
    al, be = steps.lanczos(H, V0, 25)
    got = chase.lanczos_bounds(al, be, N, ne)
    ref = steps.lanczos_bounds(al, be, N, ne)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_group_and_server_arguments_rejected_without_device_work():
    L = chase.lib()
    assert L.chase_filter_step_group(None, -1, None) == chase.CHASE_EINVAL
    assert L.chase_filter_step_group(None, 2, None) == chase.CHASE_EINVAL
    bad = (chase.FilterCall * 1)()
    bad[0] = chase.FilterCall(16, 10, 5, 16, 4, None, 4, 32, 4, 4, 1.0, 0.0, 0.0)  # ldh < N
    assert L.chase_filter_step_group(ctypes.cast(bad, ctypes.c_void_p), 1, None) == \
        chase.CHASE_EINVAL
    assert "leading dimension" in chase.last_error()
    assert L.chase_server_create(0, 2, 8) is None
    assert b"flags" in L.chase_server_last_error()
    assert L.chase_server_create(0, 0, 0) is None


def test_nex_linear_matches_oracle_and_rejects_bad_input():
    from oracle import steps
    rng = np.random.default_rng(3)
    for _ in range(2000):
        lo, hi = (int(v) for v in rng.integers(0, 400, 2))
        e0 = float(rng.uniform(-5, 20))
        e1 = e0 + float(rng.uniform(0.01, 10))
        e = float(rng.uniform(e0 - 3, e1 + 3))
        assert chase.nex_linear(lo, hi, e0, e1, e) == steps.nex_linear(lo, hi, e0, e1, e)
    for bad in [(-1, 5, 0.0, 1.0, 0.5), (1, 5, 1.0, 1.0, 0.5), (1, 5, 0.0, float("nan"), 0.5)]:
        with pytest.raises(chase.ChaseError):
            chase.nex_linear(*bad)


@pytest.mark.parametrize("args,msg", [
    ((0, 0, 0, 0, 0), "N must be"),
    ((10, 9, 10, 0, 10), "ldh"),
    ((10, 10, 10, -1, 5), "r0"),
    ((10, 10, 10, 6, 5), "r0 + nrows"),
    ((10, 10, 7, 0, 8), "ldr"),
    ((200000, 200000, 200000, 0, 1), "N must be"),
])
def test_ingest_arguments_rejected_before_device_work(args, msg):
    L = chase.lib()
    N, ldh, ldr, r0, nrows = args
    for fn in (L.chase_ingest_rows, L.chase_ingest_rows_host):
        st = fn(ctypes.c_void_p(16), N, ldh, ctypes.c_void_p(16), ldr, r0, nrows, None)
        assert st == chase.CHASE_EINVAL and msg in chase.last_error()
    st = L.chase_hermitian_complete(ctypes.c_void_p(16), 10, 10, ord("X"), None)
    assert st == chase.CHASE_EINVAL and "uplo" in chase.last_error()
    st = L.chase_ingest_rows(None, 10, 10, ctypes.c_void_p(16), 10, 0, 3, None)
    assert st == chase.CHASE_EINVAL and "NULL" in chase.last_error()
