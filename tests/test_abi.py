"""CPU checks of the C ABI: the library loads, exports every function that
include/dwf.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "dwf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dwf_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    import paper_1101_0423_amd as dwf
    L = dwf.lib()
    names = declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(dwf.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", dwf.lib_path()], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(r" T " + n + r"$", out, flags=re.M), n


def test_default_params():
    import paper_1101_0423_amd as dwf
    p = dwf.default_params()
    assert p.tol == 1e-10 and p.inner_prec == dwf.PREC_FP32 and p.reliable == 1 and p.use_graph == 1


def _create(dims=(4, 4, 4, 4), ns=4, m0=1.8, mq=0.1, sigma=None, omega=None, gauge=True):
    import paper_1101_0423_amd as dwf
    L = dwf.lib()
    h = ctypes.c_void_p()
    sigma = np.zeros(ns) if sigma is None else np.asarray(sigma, float)
    omega = np.ones(ns) if omega is None else np.asarray(omega, float)
    g = np.zeros(4 * 18 * int(np.prod(dims))) if gauge else None
    dp = ctypes.POINTER(ctypes.c_double)
    d = (ctypes.c_int * 4)(*dims)
    rc = L.dwf_create(ctypes.byref(h), g.ctypes.data_as(dp) if gauge else None, d, ns, m0, mq,
                      sigma.ctypes.data_as(dp), omega.ctypes.data_as(dp), None)
    return rc, L.dwf_last_error().decode()


@pytest.mark.parametrize("kw,msg", [
    (dict(dims=(4, 4, 4, 3)), "even"),
    (dict(dims=(4, 0, 4, 4)), "even"),
    (dict(ns=0), "Ns"),
    (dict(ns=33), "Ns"),
    (dict(m0=0.0), "m0"),
    (dict(m0=2.0), "m0"),
    (dict(omega=[1, 1, 0, 1]), "omega"),
    (dict(gauge=False), "NULL"),
    # (1 + cL) singular: Ns = 1, 1 - kappa c = 0 with kappa = mq / (2 m0) = 0.1
    (dict(ns=1, m0=1.0, mq=0.2, sigma=[10.0], omega=[1.0]), "singular"),
])
def test_create_rejects_bad_arguments(kw, msg):
    import paper_1101_0423_amd as dwf
    rc, err = _create(**kw)
    assert rc == dwf.DWF_EINVAL
    assert msg in err


@pytest.mark.parametrize("dims,ns", [((128, 128, 128, 66), 16), ((128, 128, 128, 128), 32)])
def test_create_rejects_a_lattice_beyond_the_index_range(dims, ns):
    # the 5D half-lattice may hold at most 2^30 sites (V4 / 2 * Ns; 128^3 x 64
    # at Ns = 16 is exactly the limit); larger ones are refused before the
    # gauge field is read, so a short buffer stands in for it
    import paper_1101_0423_amd as dwf
    L = dwf.lib()
    h = ctypes.c_void_p()
    dp = ctypes.POINTER(ctypes.c_double)
    g, sigma, omega = np.zeros(16), np.zeros(ns), np.ones(ns)
    rc = L.dwf_create(ctypes.byref(h), g.ctypes.data_as(dp), (ctypes.c_int * 4)(*dims), ns, 1.8, 0.1,
                      sigma.ctypes.data_as(dp), omega.ctypes.data_as(dp), None)
    assert int(np.prod(dims)) // 2 * ns > 2 ** 30
    assert rc == dwf.DWF_EINVAL and h.value is None
    assert "too large" in L.dwf_last_error().decode()


def test_stream_copy_and_time_kernels_reject_bad_arguments():
    # checked before any HIP call, so small dummy addresses stand in for the
    # device buffers and the stream
    import paper_1101_0423_amd as dwf
    L = dwf.lib()
    a, b, s = ctypes.c_void_p(256), ctypes.c_void_p(512), ctypes.c_void_p(1024)
    assert L.dwf_stream_copy(None, b, 16, 0, 0, s) == dwf.DWF_EINVAL
    assert L.dwf_stream_copy(a, None, 16, 0, 0, s) == dwf.DWF_EINVAL
    assert L.dwf_stream_copy(a, b, 24, 0, 0, s) == dwf.DWF_EINVAL
    assert "multiple of 16" in L.dwf_last_error().decode()
    assert L.dwf_stream_copy(a, b, 16, 2, 0, s) == dwf.DWF_EINVAL
    assert L.dwf_stream_copy(a, b, 16, 0, 0, None) == dwf.DWF_EINVAL
    assert "stream" in L.dwf_last_error().decode()
    ms, by = np.zeros(5), np.zeros(5)
    dp = ctypes.POINTER(ctypes.c_double)
    p = dwf.default_params()
    assert L.dwf_time_kernels(None, ctypes.byref(p), 1, 1, ms.ctypes.data_as(dp), by.ctypes.data_as(dp)) \
        == dwf.DWF_EINVAL


def test_x_singular_rejected():
    """X = a + b L_+ with Ns = 1: a - kappa b = 0 makes X singular (Eq. (7))."""
    import paper_1101_0423_amd as dwf
    m0, om = 1.0, 1.0
    a = (4 - m0) * om + 1            # = 4
    # choose sigma so that b = (4 - m0) sigma - 1 and kappa = a / b
    sigma = 1.0
    b = (4 - m0) * sigma - 1         # = 2  -> kappa = 2 -> mq = 2 kappa m0 = 4
    rc, err = _create(ns=1, m0=m0, mq=2 * (a / b) * m0, sigma=[sigma], omega=[om])
    assert rc == dwf.DWF_EINVAL and "singular" in err


def test_null_arguments_everywhere():
    import paper_1101_0423_amd as dwf
    L = dwf.lib()
    assert L.dwf_apply(None, 0, 0, None, None, 1) == dwf.DWF_EINVAL
    assert L.dwf_solve(None, None, None, 1, None, None) == dwf.DWF_EINVAL
    assert L.dwf_solve_dev(None, None, None, 1, None, None, None) == dwf.DWF_EINVAL
    assert L.dwf_apply_dev(None, 0, 0, None, None, 1, None) == dwf.DWF_EINVAL
    L.dwf_destroy(None)


def test_missing_library_fails_loudly(tmp_path):
    """The binding never falls back to anything: without libdwf.so it raises."""
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_1101_0423_amd.binding as b\n"
        "b._LIB_PATH = %r\n"
        "try:\n    b.lib()\nexcept ImportError as e:\n    print('RAISED', e)\n"
    ) % (ROOT, str(tmp_path / "missing.so"))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True).stdout
    assert "RAISED" in out


def test_server_entry_points_without_a_device():
    """Ticket lookup, statistics and argument checks of the request server need
    no GPU: an unknown ticket is DWF_ENOTFOUND, NULL arguments DWF_EINVAL."""
    import paper_1101_0423_amd as dwf
    L = dwf.lib()
    st = dwf.SolveStats()
    assert L.dwf_poll(ctypes.c_uint64(123456789), None, ctypes.byref(st), 0) == dwf.DWF_ENOTFOUND
    assert "ticket" in L.dwf_last_error().decode()
    t = ctypes.c_uint64()
    assert L.dwf_submit(None, None, None, ctypes.byref(t)) == dwf.DWF_EINVAL
    assert L.dwf_submit_mass(None, None, 0.1, None, ctypes.byref(t)) == dwf.DWF_EINVAL
    assert L.dwf_server_stats_get(None, 0) == dwf.DWF_EINVAL
    s = dwf.server_stats(reset=True)
    assert s["completed"] == 0 and s["waits_for_memory"] == 0 and s["p99_latency"] == 0.0


def test_unknown_system_rejected():
    import paper_1101_0423_amd as dwf
    L = dwf.lib()
    p = dwf.default_params(system=2)
    assert L.dwf_solve_dev(ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.c_void_p(1), 1, ctypes.byref(p),
                           None, None) == dwf.DWF_EINVAL
    assert "system" in L.dwf_last_error().decode()


def test_one_hip_runtime_per_process():
    """The binding loads torch (when installed) before libdwf.so, so that both
    use the HIP and HSA runtimes torch ships: a process that had loaded the
    system runtimes first would hold two HSA runtimes, and the second cannot
    open the GPU (torch then reports no device)."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_1101_0423_amd as dwf\n"
            "dwf.lib()\n"
            "import torch\n"
            "m = sorted({l.split()[-1] for l in open('/proc/self/maps')"
            " if 'libamdhip64' in l or 'libhsa-runtime64' in l})\n"
            "print('\\n'.join(m))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    libs = out.stdout.split()
    assert sum("libamdhip64" in p for p in libs) == 1, libs
    assert sum("libhsa-runtime64" in p for p in libs) == 1, libs


def test_su3_deviation_check():
    """The host-side check behind 12-real links: an SU(3) field passes; the same
    field times a phase e^{i phi} (a U(3) field) deviates by
    |1 - e^{-3 i phi}| max_b |U_2b| (row 2 picks up e^{i phi}, the conjugated
    cross product of rows 0 and 1 e^{-2 i phi}); a non-finite entry gives inf."""
    import dwf_inputs as inp
    import paper_1101_0423_amd as dwf
    dims = (4, 2, 2, 6)
    U = inp.gauge_field(dims, 0.5, seed=3)
    assert dwf.gauge_su3_deviation(U, dims) < 1e-14
    phi = 0.013
    z = (U[..., 0] + 1j * U[..., 1]) * np.exp(1j * phi)
    Up = np.stack([z.real, z.imag], axis=-1)
    dev = dwf.gauge_su3_deviation(Up, dims)
    expect = abs(1 - np.exp(-3j * phi)) * np.max(np.abs(U[..., 2, :, 0] + 1j * U[..., 2, :, 1]))
    assert abs(dev - expect) <= 1e-12 * expect and dev > dwf.SU3_TOL
    Un = U.copy()
    Un[1, 0, 1, 2, 3, 0, 2, 1] = np.nan
    assert dwf.gauge_su3_deviation(Un, dims) == np.inf
    with pytest.raises(ValueError):
        dwf.gauge_su3_deviation(U, (4, 2, 2, 4))
    L = dwf.lib()
    out = ctypes.c_double()
    d = (ctypes.c_int * 4)(4, 2, 3, 6)
    assert L.dwf_gauge_su3_deviation(U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), d,
                                     ctypes.byref(out)) == dwf.DWF_EINVAL


def test_binding_rejects_mismatched_arrays():
    """Shapes, dtypes, devices and sizes are checked in the binding before a
    pointer reaches the library (a short or misplaced buffer would be read or
    written out of bounds)."""
    import torch

    import dwf_inputs as inp
    import paper_1101_0423_amd as dwf
    dims, ns = (4, 2, 2, 6), 3
    one = dwf.spinor_shape(dims, ns)
    a, n = dwf.check_host_spinors(np.zeros(one), dims, ns)
    assert n == 1 and a.flags.c_contiguous
    a, n = dwf.check_host_spinors(np.zeros((2,) + one), dims, ns)
    assert n == 2
    for bad in (np.zeros(one[:-1] + (12,)), np.zeros((4, 2, 2, 6, ns, 24)), np.zeros(int(np.prod(one))),
                np.zeros((0,) + one)):
        with pytest.raises(ValueError):
            dwf.check_host_spinors(bad, dims, ns)
    n = int(np.prod(one))
    for t in (torch.zeros(n, dtype=torch.float64),                 # not on the GPU
              torch.zeros(n, dtype=torch.float32),                 # wrong dtype
              torch.zeros(2 * n, dtype=torch.float64)[::2],        # not contiguous
              np.zeros(n)):                                        # not a tensor
        with pytest.raises(ValueError):
            dwf.check_device_spinors(t, dims, ns, 1, 0)
    # the context refuses a gauge field or weights of the wrong shape before any library call
    U = inp.gauge_field(dims, 0.5, seed=3)
    with pytest.raises(ValueError):
        dwf.Context(U.reshape(-1), dims, ns, 1.8, 0.1, np.zeros(ns), np.ones(ns))
    with pytest.raises(ValueError):
        dwf.Context(U, dims, ns, 1.8, 0.1, np.zeros(ns + 1), np.ones(ns))
