"""The OpenMP timing build of the oracle (used only to time the oracle on
the host's cores): its classical CG is Algorithm 1 with the same steps as
the parity oracle's, so at any thread count it takes the same iterations on
a well-conditioned problem, reaches the sine-transform solution within
kappa * rtol, and stays within roundoff of the parity oracle's iterate."""
import numpy as np
import pytest
import scipy.fft

import oracle
from oracle.build import build_timing
from paper_1410_4054_amd import problems as P


@pytest.fixture(scope="module")
def timing(tmp_path_factory):
    path = str(tmp_path_factory.mktemp("omp") / "liboracle_omp.so")
    return oracle.TimingOracle(build_timing(path))


def test_timing_build_matches_parity_oracle(timing):
    n = 31
    A, b, _ = P.workload(f"poisson2d_{n}")
    t = np.pi * np.arange(1, n + 1) / (n + 1)
    lam = 4.0 - 2.0 * np.cos(t)[:, None] - 2.0 * np.cos(t)[None, :]
    xs = scipy.fft.idstn(scipy.fft.dstn(b.reshape(n, n), type=1, norm="ortho") / lam, type=1,
                         norm="ortho").ravel()
    kappa = lam.max() / lam.min()
    ref = oracle.solve(A, b, method="cg_classical", rtol=1e-10)
    for threads in (1, 3, 8):
        st, k, x = timing.cg_classical(A, b, threads, rtol=1e-10)
        assert st == ref.status == "converged"
        assert abs(k - ref.k) <= 1, (threads, k, ref.k)
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * 1e-10
        assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) <= 1e-9
    st, k, x = timing.cg_classical(A, b, 4, rtol=0.0, max_iter=7)
    r7 = oracle.solve(A, b, method="cg_classical", rtol=0.0, max_iter=7)
    assert st == "not_converged" and k == 7
    assert np.linalg.norm(x - r7.x) / np.linalg.norm(r7.x) <= 1e-12
    st, k, x = timing.cg_classical(A, np.zeros(A.n), 2)
    assert st == "converged" and k == 0 and not x.any()
