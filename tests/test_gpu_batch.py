"""Batched solves (fk_batch_*) against the oracle's refinement run system by
system (oracle.solve_mixed) on the same seeded inputs.

A system is solved by one workgroup or by a team of workgroups, either way
with the arithmetic of the single-system mixed method, so status, inner
iterations, sweeps, the last relative residual and the iterate must equal
the oracle's bit for bit, whatever the workgroup size, the LDS limit, the
team size or graph replay."""
import numpy as np
import pytest

import oracle
from gpu_util import dev, host
from paper_1410_4054_amd import fk, problems as P

pytestmark = pytest.mark.gpu

STATUS = {0: "converged", 1: "not_converged", 2: "breakdown", 3: "unsolved"}


def oracle_batch(A, sp, b, x0=None, **kw):
    out = []
    for s in range(len(sp) - 1):
        r0, r1 = int(sp[s]), int(sp[s + 1])
        As = P.system_of(A, sp, s)
        out.append(oracle.solve_mixed(As, b[r0:r1], x0=None if x0 is None else x0[r0:r1], **kw))
    return out


def assert_batch_equal(B, x, refs, sp, label=""):
    res = B.results()
    for s, ref in enumerate(refs):
        r0, r1 = int(sp[s]), int(sp[s + 1])
        got = (STATUS[int(res.status[s])], int(res.iterations[s]), int(res.sweeps[s]))
        assert got == (ref.status, ref.k, ref.sweeps), (label, s, got, ref.status, ref.k, ref.sweeps)
        assert res.rel_res[s] == ref.hist[-1], (label, s, res.rel_res[s], ref.hist[-1])
        assert np.array_equal(x[r0:r1], ref.x), (label, s, np.abs(x[r0:r1] - ref.x).max())


@pytest.fixture(scope="module")
def small():
    A, sp, b = P.batch_problem(40, seed=3, nmin=1, nmax=70)
    refs = oracle_batch(A, sp, b, rtol=1e-10, inner_rtol=1e-4)
    return A, sp, b, refs


@pytest.mark.parametrize("workgroup", [256, 512, 1024])
@pytest.mark.parametrize("lds_rows", [0, -1, 1000], ids=["lds", "global", "split"])
def test_batch_matches_oracle(small, workgroup, lds_rows, device):
    A, sp, b, refs = small
    print(f"\n[case] batch 40 systems wg={workgroup} lds_rows={lds_rows}", flush=True)
    B = fk.Batch(A, sp)
    xd = dev(np.zeros(A.n))
    B.solve(dev(b), xd, rtol=1e-10, inner_rtol=1e-4, workgroup=workgroup, lds_rows=lds_rows)
    assert_batch_equal(B, host(xd), refs, sp, f"wg{workgroup}/lds{lds_rows}")
    assert all(r.status == "converged" for r in refs)


@pytest.mark.parametrize("lds_rows", [-1, 0], ids=["teams", "dissolve"])
@pytest.mark.parametrize("team,teams", [(2, 3), (3, 5), (8, 2), (8, 1000)],
                         ids=["t2x3", "t3x5", "t8x2", "t8-all"])
def test_batch_teams_match_oracle(small, team, teams, lds_rows, device):
    """Teams take the largest systems and single workgroups the smallest;
    teams=1000 is clamped to the resident workgroups, so teams take
    everything.  With lds_rows=-1 no system fits LDS and teams solve them;
    with the default limit every system here fits, so each team dissolves
    at its first claim and its members go on alone."""
    A, sp, b, refs = small
    print(f"\n[case] batch 40 systems team={team} teams={teams} lds_rows={lds_rows}", flush=True)
    B = fk.Batch(A, sp)
    xd = dev(np.zeros(A.n))
    B.solve(dev(b), xd, rtol=1e-10, inner_rtol=1e-4, team=team, teams=teams, lds_rows=lds_rows)
    assert_batch_equal(B, host(xd), refs, sp, f"team{team}x{teams}/lds{lds_rows}")


def test_batch_team_gives_up(small, device):
    """A team wait bounded at two polls gives up: the kernel still ends, the
    call reports the error, the systems it left have status 3 and the rest
    equal the oracle; the next solve with the default patience is whole."""
    A, sp, b, refs = small
    print("\n[case] batch 40 systems team=4 spin_limit=1", flush=True)
    B = fk.Batch(A, sp)
    xd = dev(np.zeros(A.n))
    with pytest.raises(RuntimeError, match="team wait"):
        B.solve(dev(b), xd, rtol=1e-10, inner_rtol=1e-4, team=4, teams=4, spin_limit=1, lds_rows=-1)
    res = B.results()
    assert set(np.unique(res.status)) <= {0, 3} and (res.status == 3).any(), res.status
    x = host(xd)
    for s, ref in enumerate(refs):
        if res.status[s] == 0:
            r0, r1 = int(sp[s]), int(sp[s + 1])
            assert np.array_equal(x[r0:r1], ref.x), s
    xd = dev(np.zeros(A.n))
    B.solve(dev(b), xd, rtol=1e-10, inner_rtol=1e-4, team=4, teams=4, lds_rows=-1)
    assert_batch_equal(B, host(xd), refs, sp, "after give-up")


def test_batch_graph_replay(small, device):
    """The captured launch replayed several times, with other work and
    synchronisation between replays, gives the eager result every time."""
    import torch

    A, sp, b, refs = small
    B = fk.Batch(A, sp)
    bd = dev(b)
    stream = torch.cuda.Stream()
    for rep in range(4):
        team = 4 if rep >= 2 else 0
        xd = dev(np.zeros(A.n))
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            B.solve(bd, xd, rtol=1e-10, inner_rtol=1e-4, graph=True, stream=stream, team=team, teams=3)
        torch.cuda.synchronize()
        assert_batch_equal(B, host(xd), refs, sp, f"replay {rep} team {team}")
        junk = torch.ones(1 << 20, device="cuda")
        junk.mul_(2.0)
        torch.cuda.synchronize()


@pytest.mark.parametrize("team", [0, 3])
def test_batch_edge_cases(team, device):
    """b_s = 0, a one-row system, an indefinite system (breakdown), a start
    from a nonzero x0, a tight iteration budget and too few sweeps; alone
    and with teams of 3 (uneven row chunks, empty chunks on one-row
    systems)."""
    mats = [P.poisson2d(5), P.scaled_identity(1, 3.0), P.dense_to_csr(np.diag([1.0, -1.0, 2.0, -2.0])),
            P.poisson2d(9), P.heat2d(12), P.poisson2d(20)]
    A, sp = P.block_diagonal(mats)
    rng = np.random.default_rng(4)
    b = rng.uniform(-1, 1, A.n)
    b[sp[0]:sp[1]] = 0.0
    x0 = np.zeros(A.n)
    x0[sp[3]:sp[4]] = rng.uniform(-1, 1, sp[4] - sp[3])
    x0[sp[0]:sp[1]] = 1.0
    B = fk.Batch(A, sp)
    for kw in ({}, {"max_iter": 7}, {"max_outer": 1}, {"inner_rtol": 2.0}):
        opts = {"rtol": 1e-10, "inner_rtol": 1e-4, **kw}
        refs = oracle_batch(A, sp, b, x0=x0, **opts)
        xd = dev(x0)
        B.solve(dev(b), xd, team=team, teams=6 if team else 0, lds_rows=-1 if team else 0, **opts)
        assert_batch_equal(B, host(xd), refs, sp, f"team {team} {kw}")
        if not kw:
            assert refs[0].status == "converged" and not host(xd)[sp[0]:sp[1]].any()
            assert refs[2].status == "breakdown"
        if "inner_rtol" in kw:
            assert all(r.status == "not_converged" for r in refs if r.k == 0 and r.hist[0] > 0)


@pytest.mark.parametrize("team", [0, 8])
def test_batch_config_full(team, device):
    """The uneven batch of 512 shifted Laplacians (n_s in [16, 512]) to 1e-10
    in one launch, alone and with teams of 8: every system converges;
    sampled systems (the largest, solved by a team when there are teams,
    among them) equal the oracle bit for bit; the true residual of every
    system, from the oracle's CSR product, is within the tolerance."""
    A, sp, b = P.batch_problem()
    print(f"\n[case] batch 512 systems n={A.n} nnz={A.nnz} team={team}", flush=True)
    B = fk.Batch(A, sp)
    xd = dev(np.zeros(A.n))
    B.solve(dev(b), xd, rtol=1e-10, team=team)
    x = host(xd)
    res = B.results()
    assert (res.status == 0).all(), np.unique(res.status, return_counts=True)
    assert (res.rel_res <= 1e-10).all()
    sizes = np.diff(sp)
    picks = [int(np.argmin(sizes)), int(np.argsort(sizes)[40]), int(np.argsort(sizes)[100]),
             int(np.argmax(sizes))]
    for s in picks:
        r0, r1 = int(sp[s]), int(sp[s + 1])
        ref = oracle.solve_mixed(P.system_of(A, sp, s), b[r0:r1], rtol=1e-10, inner_rtol=1e-4)
        assert (int(res.iterations[s]), int(res.sweeps[s])) == (ref.k, ref.sweeps), s
        assert np.array_equal(x[r0:r1], ref.x), s
    r = b - oracle.spmv(A, x)
    rn = np.sqrt(np.add.reduceat(r * r, sp[:-1]))
    bn = np.sqrt(np.add.reduceat(b * b, sp[:-1]))
    assert (rn / bn <= 1.0000001e-10).all(), (rn / bn).max()
    print(f"[result] inner iterations per system: min {res.iterations.min()} median "
          f"{int(np.median(res.iterations))} max {res.iterations.max()}; sweeps max {res.sweeps.max()}",
          flush=True)
