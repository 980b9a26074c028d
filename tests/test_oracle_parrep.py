"""Pins of the oracle's Gen.ParRep bookkeeping (Sec. 2.4): the Gelman-Rubin statistic
(Eq. 3), Fleming-Viot branching (Sec. 2.4.1), the exit-time formula (Eq. 5) and the clock
(Eq. 6), and the method as a whole against brute-force direct simulation."""
import numpy as np
import pytest
from scipy import stats

import gpr_synth as G
import oracle
from helpers import direct_exits, gen_parrep_exits


# ------------------------------------------------------------------ Eq. 3
def test_rhat_is_pooled_over_within_variance():
    """With equal sample counts, the numerator of Eq. 3 is the variance of all samples
    pooled and the denominator the mean per-trajectory variance (law of total variance):
    R-hat = 1 + var(trajectory means) / mean(within variance) >= 1."""
    rng = np.random.default_rng(1)
    for nw, n, no in ((7, 50, 3), (63, 20, 6), (1, 5, 1), (255, 4, 8)):
        O = rng.normal(size=(nw, n, no)) + rng.normal(size=(nw, 1, no)) * 0.3 + 5.0
        c = O[0, 0]                                   # any common shift
        S1 = (O - c).sum(1)
        S2 = ((O - c) ** 2).sum(1)
        rh = oracle.rhat(n, S1, S2)
        pooled = O.reshape(nw * n, no).var(0)
        within = O.var(1).mean(0)
        assert rh == pytest.approx(pooled / within, rel=1e-9)
        assert np.all(rh >= 1.0 - 1e-12)
        between = O.mean(1).var(0)
        assert rh == pytest.approx(1 + between / within, rel=1e-9)


def test_rhat_identical_workers_is_one_and_degenerate_is_inf():
    S1 = np.tile([[3.0, -1.0]], (5, 1))
    S2 = np.tile([[7.0, 2.0]], (5, 1))
    assert oracle.rhat(4, S1, S2) == pytest.approx([1.0, 1.0], abs=1e-15)
    # zero within-variance: R-hat undefined -> +inf (never converged)
    S2z = S1 ** 2 / 4
    assert np.all(np.isinf(oracle.rhat(4, S1, S2z)))


# ------------------------------------------------------------------ F-V branching
def test_fv_plan_invariants_and_uniform_donors():
    rng = np.random.default_rng(2)
    R = 16
    ranks = []
    for step in range(4000):
        ex = rng.random(R) < 0.3
        ex[0] = rng.random() < 0.5          # the reference flag is ignored
        d = oracle.fv_plan(77, step, ex)
        surv = [r for r in range(1, R) if not ex[r]]
        if not surv:
            assert np.all(d == -2)
            continue
        assert d[0] == -1
        for r in range(1, R):
            if ex[r]:
                assert d[r] in surv          # donors are survivors, never the reference
                ranks.append((surv.index(d[r]) + rng.random()) / len(surv))
            else:
                assert d[r] == -1            # survivors are not killed
    # each survivor is drawn with probability 1/|S|: the jittered rank is U(0, 1)
    assert stats.kstest(ranks, "uniform").pvalue > 1e-3


def test_fv_plan_donor_frequencies_chi2():
    ex = np.zeros(9, np.uint8)
    ex[[2, 5]] = 1
    surv = [1, 3, 4, 6, 7, 8]
    hist = np.zeros(9)
    for step in range(6000):
        d = oracle.fv_plan(3, step, ex)
        hist[d[2]] += 1
        hist[d[5]] += 1
    obs = hist[surv]
    assert stats.chisquare(obs).pvalue > 1e-3
    assert hist[[0, 2, 5]].sum() == 0


def test_fv_plan_deterministic_and_step_dependent():
    ex = np.array([0, 1, 0, 1, 0, 0, 1, 0], np.uint8)
    a = oracle.fv_plan(5, 100, ex)
    assert np.array_equal(a, oracle.fv_plan(5, 100, ex))
    diff = sum(not np.array_equal(a, oracle.fv_plan(5, 100 + k, ex)) for k in range(1, 20))
    assert diff > 10


# ------------------------------------------------------------------ Eq. 5
def test_exit_vote_enumerated():
    # N = 4, exits at the third check for replicas 2 and 4 (1-based): M = 3, k = 2,
    # tau = (4 * 2 + 2) t_check
    assert oracle.exit_vote([0, 3, 0, 3], 10) == (3, 2, 100)
    assert oracle.exit_vote([5, 0, 2, 2], 7) == (2, 3, (4 * 1 + 3) * 7)
    assert oracle.exit_vote([1, 1, 1], 1) == (1, 1, 1)
    assert oracle.exit_vote([0, 0, 0], 10) is None


def test_exit_vote_samples_geometric_law():
    """If each replica exits independently at each check with probability p, the index
    L = N (M - 1) + k of Eq. 5 is exactly Geometric(p): replica-checks are visited in
    the order (check 1: replicas 1..N), (check 2: ...), and L is the first success."""
    rng = np.random.default_rng(3)
    N, p, trials = 5, 0.07, 20000
    L = np.zeros(trials, np.int64)
    for t in range(trials):
        fec = np.zeros(N, np.int64)
        fec[:] = rng.geometric(p, N)
        M, k, tau = oracle.exit_vote(fec, 1)
        L[t] = tau
    assert L.mean() == pytest.approx(1 / p, rel=0.03)
    kmax = 60
    obs = np.array([(L == x).sum() for x in range(1, kmax)] + [(L >= kmax).sum()])
    pm = np.array([(1 - p) ** (x - 1) * p for x in range(1, kmax)] + [(1 - p) ** (kmax - 1)])
    assert stats.chisquare(obs, pm * trials).pvalue > 1e-3


# ------------------------------------------------------------------ the method
def test_parallel_step_requires_converged_dephasing():
    s = oracle.System(G.toy2d())
    with pytest.raises(oracle.OracleError):
        s.parallel_step()


def test_forced_reference_exit_during_dephasing():
    s = oracle.System(G.toy2d())
    rc, ev = s.decorrelate(0)
    assert rc == 0 and ev["kind"] == 0 and ev["to_state"] == 0
    q, v = s.get_state(0)
    q[0, 0] = 1.5                                    # reference walker put in state 1
    s.set_state(0, q, v)
    t0 = s.simulated_steps()
    rc, o = s.dephase()
    assert rc == 0 and o["outcome"] == 1 and o["to_state"] == 1
    assert o["t_steps"] == 10                        # detected at the first check (t_ref)
    assert s.simulated_steps() - t0 == 10            # t_sim += t_ref
    assert s.current_state() == 1


def test_clock_rules_and_resumable_budgets():
    """t_sim grows by the steps of the transient step, by t_FV or t_ref after the
    convergence step and by tau (Eq. 6) after the parallel step; a call interrupted by its
    budget resumes exactly where it stopped."""
    def run(chunked):
        s = oracle.System(G.toy2d(seed=21))
        log = []
        for _ in range(6):
            t0 = s.simulated_steps()
            if chunked:
                while True:
                    rc, ev = s.decorrelate(100, max_steps=30)
                    if rc == 0:
                        break
            else:
                rc, ev = s.decorrelate(100)
            assert s.simulated_steps() - t0 == ev["steps_taken"]
            log.append(("d", ev["kind"], ev["steps_taken"]))
            if ev["kind"] == 1:
                continue
            t0 = s.simulated_steps()
            if chunked:
                while True:
                    rc, o = s.dephase(max_steps=37)
                    if rc == 0:
                        break
            else:
                rc, o = s.dephase()
            assert s.simulated_steps() - t0 == o["t_steps"]
            log.append(("f", o["outcome"], o["t_steps"], o["n_branch"], tuple(np.round(o["rhat"], 12))))
            if o["outcome"] == 1:
                continue
            t0 = s.simulated_steps()
            if chunked:
                while True:
                    rc, e = s.parallel_step(max_checks=3)
                    if rc == 0:
                        break
            else:
                rc, e = s.parallel_step()
            assert e["tau_steps"] == (8 * (e["M"] - 1) + e["k"]) * 10
            assert s.simulated_steps() - t0 == e["tau_steps"]
            log.append(("p", e["M"], e["k"], e["tau_steps"], e["to_state"]))
        return log, s.get_state(0)[0]
    a, qa = run(False)
    b, qb = run(True)
    assert a == b
    assert np.array_equal(qa, qb)


@pytest.mark.slow
def test_toy_gen_parrep_matches_direct_simulation():
    """The method's claim (Sec. 2.4): exit events sampled by Gen.ParRep have the law of
    those of direct simulation.  Two-sample KS on the exit durations from the left well,
    with the same exit-check period on both sides; exit states agree; the exit times tau
    of the parallel step, which start from (approximate) QSD samples, have exponential law
    (QSD property 3, Sec. 2.3); the two 95 % confidence intervals of Sec. 4 overlap."""
    n = 600
    d = direct_exits(oracle.System(G.toy2d(seed=101)), n)
    g = gen_parrep_exits(oracle.System(G.toy2d(seed=202)), n, t_corr=100)
    dd = np.array([x[0] for x in d], float)
    gg = np.array([x[0] for x in g], float)
    assert stats.ks_2samp(dd, gg).pvalue > 0.05
    assert all(x[2] == 1 - x[1] for x in g) and all(x[2] == 1 - x[1] for x in d)
    kinds = {x[3] for x in g}
    assert "parallel" in kinds
    tau = np.array([x[4] for x in g if x[3] == "parallel"], float)
    assert len(tau) > n // 2
    assert stats.kstest(tau, "expon", args=(0, tau.mean())).pvalue > 0.01

    def ci(x):
        m = len(x)
        return (2 * m * x.mean() / stats.chi2.ppf(0.975, 2 * m), 2 * m * x.mean() / stats.chi2.ppf(0.025, 2 * m))
    a, b = ci(dd), ci(gg)
    assert a[0] < b[1] and b[0] < a[1]


def _chain6(seed):
    """The chain of the 22-atom workload cut to six atoms (phi = (1,2,3,4), psi = (2,3,4,5),
    the same force field and state = (phi, psi) quadrant; chain seed 5) with the n = 2 terms
    raised to k2 = 10 kJ/mol, so that each quadrant is metastable with exits every ~6,000
    steps into both neighbouring quadrants (the 22-atom chain exits every ~4e5 steps, out of
    reach of a CPU test, and almost only through psi).  ``seed`` is the noise seed."""
    return dict(G.chain(seed=5, n_atoms=6, n_replicas=8, k2=10.0, t_gr=10, t_check=50, t_check_parallel=50),
                seed=seed)


@pytest.mark.slow
def test_chain_exit_states_match_direct_simulation():
    """Exit states (Sec. 2.2: the quadrant the walker leaves into) sampled by Gen.ParRep have
    the law of those of direct simulation.  For each state left, a chi-square test of
    homogeneity of the destination counts of the two runs (destinations seen fewer than ten
    times in both runs together pooled); the statistics and degrees of freedom are summed over
    the four states into one test.  Same exit-check period on both sides; the exit durations
    agree by a two-sample KS test."""
    from collections import Counter
    n = 400
    d = direct_exits(oracle.System(_chain6(105)), n)
    g = gen_parrep_exits(oracle.System(_chain6(205)), n, t_corr=3000)
    cd = Counter((x[1], x[2]) for x in d)
    cg = Counter((x[1], x[2]) for x in g)
    assert all(a != b for a, b in list(cd) + list(cg))
    stat, dof, multi = 0.0, 0, 0
    for f in range(4):
        dests = sorted({b for a, b in list(cd) + list(cg) if a == f})
        main = [b for b in dests if cd[(f, b)] + cg[(f, b)] >= 10]
        rest = [b for b in dests if b not in main]
        rows = [[c[(f, b)] for b in main] + ([sum(c[(f, b)] for b in rest)] if rest else []) for c in (cd, cg)]
        table = np.array(rows)
        table = table[:, table.sum(0) > 0]
        if table.shape[1] < 2:
            continue
        multi += 1
        c2, _, k, _ = stats.chi2_contingency(table, correction=False)
        stat += c2
        dof += k
    assert multi == 4                                  # every state has two or more destinations
    assert stats.chi2.sf(stat, dof) > 0.01, (stat, dof, cd, cg)
    kinds = Counter(x[3] for x in g)
    assert kinds["parallel"] > n // 10 and kinds["dephase"] > n // 10
    dd = np.array([x[0] for x in d], float)
    gg = np.array([x[0] for x in g], float)
    assert stats.ks_2samp(dd, gg).pvalue > 0.01
