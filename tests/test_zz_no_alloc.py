"""fk_solve_noalloc: pipelined CG whose work vectors, reduction scratch and
device state live in the library's static per-device array, against fk_solve
with the same options (solver handle, library-allocated workspace).  Both
enqueue the same kernels in the same order, so x, k and the residual must be
equal bit for bit.  Calls follow one another on the same array, each
smaller than the last, so a call that read what the previous one left there
(counters, partials, state, stale vector entries) would show up as a
difference.  Also: the size limit and the options the entry point refuses."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import dev, host
from paper_1410_4054_amd import fk, problems as P

pytestmark = pytest.mark.gpu


def _both(A, b, x0=None, **kw):
    """(noalloc result, x) and (fk_solve result, x) on the same inputs."""
    M = fk.Matrix(A)
    x0 = np.zeros(A.n) if x0 is None else x0
    bd = dev(b)
    xa = dev(x0)
    ra = fk.solve_noalloc(M, bd, xa, **kw)
    xs = dev(x0)
    small = kw.pop("small", True)
    rs = fk.solve(M, bd, xs, method="cg_pipelined", record_history=False, small=small, **kw)
    M.close()
    return ra, host(xa), rs, host(xs)


def _same(name, ra, xa, rs, xs):
    print(f"[result] {name}: noalloc k={ra.k} {ra.status} rel={ra.rel_res:.3e}; "
          f"fk_solve k={rs.k} {rs.status} rel={rs.rel_res:.3e}", flush=True)
    assert ra.status == rs.status
    assert ra.k == rs.k
    assert ra.rel_res == rs.rel_res
    assert np.array_equal(xa, xs)


def test_noalloc_matches_fk_solve(device):
    # 1. the largest system the array holds (n = FK_NOALLOC_MAX_N), grid path
    A, b, _ = P.workload("poisson2d_1024")
    assert A.n == fk.NOALLOC_MAX_N
    print(f"\n[case] noalloc poisson2d_1024 n={A.n} rtol 1e-6", flush=True)
    _same("poisson2d_1024", *_both(A, b, rtol=1e-6))
    # 2. a smaller grid-path system right after it, with a warm start
    A, b, _ = P.workload("poisson3d_32")
    x0 = np.random.default_rng(3).uniform(-0.1, 0.1, A.n)
    print(f"[case] noalloc poisson3d_32 n={A.n} warm start", flush=True)
    ra, xa, rs, xs = _both(A, b, x0=x0, rtol=1e-9, unroll=7)
    _same("poisson3d_32", ra, xa, rs, xs)
    assert ra.status == "converged"
    # 3. smaller again: the multi-kernel path forced, then the single-workgroup path
    A, b, _ = P.workload("poisson2d_40")
    print(f"[case] noalloc poisson2d_40 n={A.n} multi-kernel and single-workgroup", flush=True)
    ra, xa, rs, xs = _both(A, b, rtol=1e-8, small=False)
    _same("poisson2d_40 grid", ra, xa, rs, xs)
    ref = oracle.solve(A, b, method="cg_pipelined", rtol=1e-8)
    assert ra.k == ref.k and np.array_equal(xa, ref.x)
    _same("poisson2d_40 small", *_both(A, b, rtol=1e-8))
    # 4. iteration budget, b = 0 (x set to 0 on both paths), max_iter 0
    A, b, _ = P.workload("poisson3d_20")
    print(f"[case] noalloc poisson3d_20 n={A.n} limits", flush=True)
    ra, xa, rs, xs = _both(A, b, rtol=1e-12, max_iter=13, unroll=5)
    _same("poisson3d_20 max_iter 13", ra, xa, rs, xs)
    assert ra.status == "not_converged" and ra.k == 13
    ones = np.ones(A.n)
    for small in (True, False):
        ra, xa, rs, xs = _both(A, np.zeros(A.n), x0=ones, small=small)
        _same(f"poisson3d_20 b=0 small={small}", ra, xa, rs, xs)
        assert ra.status == "converged" and ra.k == 0 and not xa.any()
    ra, xa, rs, xs = _both(A, b, max_iter=0)
    _same("poisson3d_20 max_iter 0", ra, xa, rs, xs)


def test_noalloc_refuses(device):
    L = fk.lib()
    # one row more than the array holds
    big = P.scaled_identity(fk.NOALLOC_MAX_N + 1, 2.0)
    M = fk.Matrix(big)
    b = dev(np.ones(big.n))
    x = dev(np.zeros(big.n))
    with pytest.raises(fk.FkError) as e:
        fk.solve_noalloc(M, b, x)
    assert e.value.status == fk.E_ARG
    M.close()
    A, bb, _ = P.workload("poisson2d_16")
    M = fk.Matrix(A)
    b, x = dev(bb), dev(np.zeros(A.n))
    k, rel = ctypes.c_int32(), ctypes.c_double()
    for method, rh, flags in ((fk.METHODS["bicgstab_pipelined"], 0, 0), (0, 1, 0), (0, 0, fk.FLAG_GRAPH)):
        o = fk._Opts(method, 1e-8, 100, rh, 0, flags, 0.0, 0, 0)
        st = L.fk_solve_noalloc(M.handle, ctypes.byref(o), ctypes.c_void_p(b.data_ptr()),
                                ctypes.c_void_p(x.data_ptr()), None, ctypes.byref(k), ctypes.byref(rel))
        assert st == fk.E_ARG
    M.close()
