"""Batched persistent solve (ipm_solve_batch): every instance of an uneven
batch against the CPU oracle, in float64 and float32 operator storage."""
import numpy as np
import pytest

import oracle as O
from paper_2308_00637_amd import workloads as W
from tests.helpers import from_masked

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def uneven_batch(count=24, seed=7, nmin=20, nmax=160, round_f32=False):
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        if i % 3 == 0:
            sp = W.random_bounded_qp(100 + i, n, int(rng.integers(0, 2 * n)), 0, max(2, n // 3),
                                     h_kind="lowrank" if i % 2 else "dense")
            sp.A = None if sp.A.shape[0] == 0 else np.asarray(sp.A)
            if sp.A is None:
                sp.lA = sp.uA = None
        else:
            m = int(rng.integers(n, 2 * n + 1))
            sp = W.dense_qp(rng, n, m, n // 2, round_f32=round_f32, name=f"dense{i}")
        specs.append(sp)
    return specs


def to_f32(sp):
    """Round every operator and vector of a spec to float32 values, so that
    float32 storage holds the problem exactly."""
    r = lambda a: None if a is None else np.asarray(a, dtype=np.float32).astype(np.float64)
    for f in ("c", "H", "h0", "U", "wd", "A", "lA", "uA", "lx", "ux"):
        v = getattr(sp, f)
        if v is not None:
            setattr(sp, f, r(v))
    return sp


def check(specs, infos, qb, tol_obj=1e-6):
    for i, sp in enumerate(specs):
        prob = O.from_spec(sp)
        ref = O.solve(prob)
        f = infos[i]
        x, lam, s = qb.solution(i)
        st = from_masked(prob, x.cpu().numpy(), lam.cpu().numpy(), s.cpu().numpy())
        kkt = O.stacked_norm(O.residuals(prob, st, f.mu_final))
        err = abs(f.objective - ref.objective) / max(1.0, abs(ref.objective))
        assert f.result == 0 and ref.status == "converged", (i, f.result)
        assert err <= tol_obj, (i, err)
        # the residual at convergence is a cancellation of O(1..100) terms, so
        # the device's and the oracle's evaluations agree to rounding in absolute terms
        assert kkt <= 1e-6 and abs(kkt - f.rnorm) <= 1e-10, (i, kkt, f.rnorm)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_matches_oracle_per_instance(prec):
    from paper_2308_00637_amd.qpk import QPBatch
    specs = uneven_batch()
    if prec == "fp32":
        specs = [to_f32(sp) for sp in specs]
    qb = QPBatch(specs, precision=prec)
    infos, st = qb.solve()
    print(f"batch {prec}: {len(specs)} instances in {infos[0].time_ms:.1f} ms, "
          f"ipm iters {[f.iterations for f in infos]}", flush=True)
    assert st == 0
    check(specs, infos, qb)


def test_batch_of_one_tiny_dense_matches_oracle_and_single_path():
    """The 200-variable case: one persistent launch vs the multi-kernel path."""
    from paper_2308_00637_amd.qpk import QP, QPBatch
    spec = W.tiny_dense(0)
    qb = QPBatch([spec])
    infos, st = qb.solve()
    out = QP(spec).solve()
    print(f"tiny_dense: batch {infos[0].time_ms:.1f} ms ({infos[0].iterations} ipm, "
          f"{infos[0].total_cg_iters} cg) vs multi-kernel {out['info'].time_ms:.1f} ms "
          f"({out['info'].iterations} ipm, {out['info'].total_cg_iters} cg)", flush=True)
    check([spec], infos, qb)


def test_batch_rejects_unsupported_inputs():
    from paper_2308_00637_amd.qpk import QPBatch, QPError, QP_ERR_UNSUPPORTED
    with pytest.raises(QPError) as e:
        QPBatch([W.rt_qp(5, 100, 10, 0.1, 5)])
    assert e.value.status == QP_ERR_UNSUPPORTED


def test_teams_of_workgroups_match_one_workgroup_per_instance_and_the_oracle():
    """Teams of 2, 4 and 8 workgroups (and teams of one beside them, each size
    with its own queue) in one cooperative launch: per instance the same
    optimum as one workgroup per instance and as the oracle.  The teams add
    the same products in another order (reductions over the members'
    partials in rank order, column sums over row slabs), and these Newton
    systems often run the PCG to its 5,000-iteration cap, where an inexact
    step's rounding can steer the IPM path: the iteration counts may differ
    by a few (never more than 15%), the optima may not."""
    from paper_2308_00637_amd.qpk import QPBatch
    rng = np.random.default_rng(31)
    specs = []
    for i in range(12):
        n = int(rng.integers(150, 420))
        specs.append(W.dense_qp(rng, n, int(rng.integers(n, 2 * n + 1)), n // 2, name=f"t{i}"))
    sizes = [8, 4, 2, 1] * 3
    qb = QPBatch(specs)
    solo, st0 = qb.solve()
    qb.set_teams(sizes)
    team, st1 = qb.solve()
    wg, teams = qb.launch_shape()
    print(f"teams: {wg} workgroups in {teams} teams, {team[0].time_ms:.1f} ms "
          f"(one workgroup each: {solo[0].time_ms:.1f} ms)", flush=True)
    assert st0 == 0 and st1 == 0
    assert 4 <= teams <= wg <= 1024
    t0, t1, g = qb.instance_times()
    assert min(t0) == 0.0 and all(0.0 <= a <= b for a, b in zip(t0, t1))
    assert max(t1) <= team[0].time_ms + 1.0
    assert all(gi >= si for gi, si in zip(g, sizes))   # its own queue's team, or a larger one helping
    for i, (a, b) in enumerate(zip(team, solo)):
        rel = abs(a.objective - b.objective) / max(1.0, abs(b.objective))
        print(f"  {i}: n={specs[i].n} team {sizes[i]}: ipm {a.iterations}/{b.iterations} "
              f"cg {a.total_cg_iters}/{b.total_cg_iters} obj rel {rel:.1e}", flush=True)
        assert a.result == 0 and abs(a.iterations - b.iterations) <= max(1, 0.15 * b.iterations)
        assert rel <= 1e-9
    check(specs, team, qb)


def test_team_barrier_give_up_is_reported_and_the_next_launch_is_clean(monkeypatch):
    """A barrier spin limit of one poll (set from the host) makes the team
    barriers give up: the launch drains at once and reports QP_ERR_HIP
    instead of running on; the next launch with the normal limit solves the
    same batch as one workgroup per instance."""
    import time
    from paper_2308_00637_amd.qpk import QPBatch, QPError, QP_ERR_HIP
    rng = np.random.default_rng(7)
    specs = [W.dense_qp(rng, n, n + 40, n // 2, name=f"g{n}") for n in (220, 180, 150)]
    qb = QPBatch(specs)
    solo, st0 = qb.solve()
    assert st0 == 0
    qb.set_teams([4, 2, 1])
    monkeypatch.setenv("QPK_BATCH_SPIN", "1")
    t0 = time.perf_counter()
    with pytest.raises(QPError) as e:
        qb.solve()
    took = time.perf_counter() - t0
    print(f"forced give-up reported in {took:.2f} s: {e.value}", flush=True)
    assert e.value.status == QP_ERR_HIP
    assert took < 20.0
    monkeypatch.delenv("QPK_BATCH_SPIN")
    team, st1 = qb.solve()
    assert st1 == 0
    for a, b in zip(team, solo):   # the same optima (iteration counts as in the test above)
        assert a.result == 0 and abs(a.iterations - b.iterations) <= max(1, 0.15 * b.iterations)
        assert abs(a.objective - b.objective) <= 1e-9 * max(1.0, abs(b.objective))


def test_team_sizes_are_checked():
    from paper_2308_00637_amd.qpk import QPBatch, QPError, QP_ERR_ARG
    qb = QPBatch([W.tiny_dense(0)])
    for bad in ([3], [0], [128]):
        with pytest.raises(QPError) as e:
            qb.set_teams(bad)
        assert e.value.status == QP_ERR_ARG
    qb.set_teams([64])
    infos, st = qb.solve()
    assert st == 0 and infos[0].result == 0
    assert qb.launch_shape() == (64, 1)


def test_autotune_picks_teams_from_measurements_and_reuses_its_table(tmp_path):
    """qp_batch_autotune times each size class's largest instance with teams
    of 1, 2, 4, ... workgroups, keeps the times in a table and gives the
    largest instances the largest teams; a second batch with the same
    classes reads the table and measures nothing.  With the tuned teams one
    IPM iteration whose PCG runs exactly 30 iterations agrees with one
    workgroup per instance to rounding (the two add the same products in
    other orders; a PCG stopped by its tolerance instead could stop one
    iteration apart and steer the IPM path)."""
    from paper_2308_00637_amd.qpk import QPBatch, default_ipm_options, default_pcg_options
    rng = np.random.default_rng(41)
    specs = [W.dense_qp(rng, n, int(1.5 * n), n // 2, name=f"a{n}")
             for n in (1500, 900, 400, 150, 150, 150)]
    table = tmp_path / "teams.txt"
    qb = QPBatch(specs)
    sizes, probes = qb.autotune(table)
    lines = table.read_text().splitlines()
    print(f"tuned team sizes {sizes} after {probes} measurements:\n" + "\n".join(lines), flush=True)
    assert probes >= 4 and len(lines) == probes
    assert sizes[0] == max(sizes) and sizes[0] >= 4 and sizes[3] <= sizes[0]
    sizes2, probes2 = QPBatch(specs).autotune(table)
    assert probes2 == 0 and sizes2 == sizes
    o = default_ipm_options(max_iter=1, pcg=default_pcg_options(tol=1e-300, maxit=30))
    tuned, st = qb.solve(o)
    qb.set_teams(None)
    solo, st0 = qb.solve(o)
    assert st == 0 and st0 == 0
    for a, b in zip(tuned, solo):
        assert a.iterations == b.iterations == 1 and a.total_cg_iters == b.total_cg_iters == 30
        assert a.rnorm == pytest.approx(b.rnorm, rel=1e-8)
        assert a.objective == pytest.approx(b.objective, rel=1e-8)


def test_wide_column_tiles_split_over_a_team_against_oracle_pcg():
    """Operators wide enough for 1,024-column tiles on every member of a
    team (A of n = 1,600 on two workgroups, n = 3,100 on four: the members
    take alternate tiles, the last one partial), and narrower ones whose
    column sums the team splits into row slabs (A of n = 1,200 on four, and
    every H factor of n/2 columns here): one IPM iteration with 30 PCG
    iterations against the oracle's step driven by its own Jacobi PCG, and
    the same instances on one workgroup each."""
    from paper_2308_00637_amd.qpk import QPBatch, default_ipm_options, default_pcg_options
    from oracle.pcg import pcg
    rng = np.random.default_rng(17)
    specs = [W.dense_qp(rng, n, m, n // 2, round_f32=True, name=f"w{n}")
             for n, m in ((1600, 1900), (3100, 3300), (1200, 1500))]
    opts = default_ipm_options(max_iter=1, pcg=default_pcg_options(tol=1e-300, maxit=30))

    def direction(prob, st_, mu, res):
        rhs, _ = O.newton_rhs_doubly(prob, st_, mu)
        dg = O.jacobi_diagonal(prob, st_, mu)
        sol, _, _, _ = pcg(lambda v: O.kkt_matvec(prob, st_, mu, v), rhs, dg, tol=1e-300, maxit=30)
        return O.direction_from_solution(prob, st_, res, sol)

    refs = [O.solve(O.from_spec(sp), O.IPMOptions(max_iter=1), direction=direction) for sp in specs]
    for teams in ([2, 4, 4], None):
        qb = QPBatch(specs, precision="fp32")
        qb.set_teams(teams)
        infos, st = qb.solve(opts)
        assert st == 0
        for i, sp in enumerate(specs):
            prob = O.from_spec(sp)
            ref = refs[i]
            x, lam, s = qb.solution(i)
            gst = from_masked(prob, x.cpu().numpy(), lam.cpu().numpy(), s.cpu().numpy())
            ex = np.max(np.abs(gst.x - ref.state.x)) / max(1.0, np.max(np.abs(ref.state.x)))
            es = np.max(np.abs(gst.s_lA - ref.state.s_lA)) / max(1.0, np.max(np.abs(ref.state.s_lA)))
            print(f"teams {teams} n={sp.n} m={sp.m}: x {ex:.1e}, s {es:.1e}, "
                  f"rnorm {infos[i].rnorm:.6g} / {ref.log[0]['rnorm']:.6g}", flush=True)
            assert infos[i].total_cg_iters == 30
            assert ex <= 1e-8 and es <= 1e-8
            assert infos[i].rnorm == pytest.approx(ref.log[0]["rnorm"], rel=1e-8)


@pytest.mark.parametrize("teams", [[1, 4, 16], None])
def test_uneven_batch_shapes_first_iteration_against_oracle_pcg(teams):
    """Instances of the 256-instance uneven batch at their real shapes (the
    three smallest of 32 strata, n from 627 to 1,159) in teams of 1, 4 and
    16 workgroups (column products in 64-column tiles), then one workgroup
    each (the two wider ones take the 1024-column tiles): one IPM iteration
    whose PCG runs 30 iterations, against the oracle's step driven by its
    own Jacobi PCG for 30 iterations.  The data are float32 values, stored
    as such on the GPU and summed in float64 on both sides."""
    from paper_2308_00637_amd.qpk import QPBatch, default_ipm_options, default_pcg_options
    from oracle.pcg import pcg
    specs = W.batch_stratified(3, 256, 32, strata=[0, 1, 2])
    qb = QPBatch(specs, precision="fp32")
    qb.set_teams(teams)
    opts = default_ipm_options(max_iter=1, pcg=default_pcg_options(tol=1e-300, maxit=30))
    infos, st = qb.solve(opts)
    assert st == 0

    def direction(prob, st_, mu, res):
        rhs, _ = O.newton_rhs_doubly(prob, st_, mu)
        dg = O.jacobi_diagonal(prob, st_, mu)
        sol, _, _, _ = pcg(lambda v: O.kkt_matvec(prob, st_, mu, v), rhs, dg, tol=1e-300, maxit=30)
        return O.direction_from_solution(prob, st_, res, sol)

    for i, sp in enumerate(specs):
        prob = O.from_spec(sp)
        ref = O.solve(prob, O.IPMOptions(max_iter=1), direction=direction)
        x, lam, s = qb.solution(i)
        gst = from_masked(prob, x.cpu().numpy(), lam.cpu().numpy(), s.cpu().numpy())
        ex = np.max(np.abs(gst.x - ref.state.x)) / max(1.0, np.max(np.abs(ref.state.x)))
        es = np.max(np.abs(gst.s_lA - ref.state.s_lA)) / max(1.0, np.max(np.abs(ref.state.s_lA)))
        print(f"n={sp.n} m={sp.m}: cg {infos[i].total_cg_iters}, x {ex:.1e}, s {es:.1e}, "
              f"rnorm {infos[i].rnorm:.6g} / {ref.log[0]['rnorm']:.6g}", flush=True)
        assert infos[i].total_cg_iters == 30
        assert ex <= 1e-8 and es <= 1e-8
        assert infos[i].rnorm == pytest.approx(ref.log[0]["rnorm"], rel=1e-8)
