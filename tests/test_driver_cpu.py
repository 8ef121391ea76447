"""Host logic of the OF-MLMC driver (no GPU): the ledger keeps the solves of
a run stopped at its deadline, including pair members whose partner had not
run yet, so that the resumed run solves only what is missing."""
import json

import pytest

from paper_1705_04374_amd import driver
from workloads.configs import MASTER_SEED, cloud_spec, solver_config


def fake_qoi(spec, bubbles):
    v = float(spec.n) * 1e6 + float(sum(sum(b) for b in bubbles))
    return dict(p_max=v, x=(0.5, 0.5, 0.0), t_at_max=1e-4, t=2e-4, argmax=0, steps=spec.n, status=0,
                p_sensor=v / 2, t_p_sensor=1e-4, gas_min=0.01, t_gas_min=1e-4, c_max=1500.0,
                peak_distance=0.0)


def make(tmp_path, log):
    cfg = solver_config("cloud2d", 16)
    return driver.OFMLMC(None, cfg, cloud_spec("cloud2d"), [16, 32], "f32", t_end=1e-4, seed=MASTER_SEED,
                         ledger=str(tmp_path / "ledger.jsonl"), log=log)


def test_stopped_run_keeps_unpaired_members(tmp_path, monkeypatch):
    calls = []

    def stop_after_fine(ctx, specs, bubbles, max_batch_bytes, log, deadline=None, done=None):
        calls.append(sorted(s.n for s in specs))
        big = [i for i, s in enumerate(specs) if s.n == 32]
        done(big, [fake_qoi(specs[i], bubbles[i]) for i in big], [2.0] * len(big))
        raise driver.Deadline("stop")

    monkeypatch.setattr(driver, "solve_many", stop_after_fine)
    mc = make(tmp_path, log=lambda *a: None)
    with pytest.raises(driver.Deadline):
        mc.sample_terms([3, 2])
    # term 1 pairs (32, 16): only their fine members ran; nothing is settled
    rows = [json.loads(l) for l in open(tmp_path / "ledger.jsonl")]
    assert sorted((r["term"], r["index"], r["member"]) for r in rows) == [(1, 0, "f"), (1, 1, "f")]

    seen = []

    def run_rest(ctx, specs, bubbles, max_batch_bytes, log, deadline=None, done=None):
        seen.append(sorted(s.n for s in specs))
        done(list(range(len(specs))), [fake_qoi(s, b) for s, b in zip(specs, bubbles)], [1.0] * len(specs))

    monkeypatch.setattr(driver, "solve_many", run_rest)
    mc2 = make(tmp_path, log=lambda *a: None)
    mc2.sample_terms([3, 2])
    assert seen == [[16, 16, 16, 16, 16]]          # 3 term-0 solves + 2 coarse members, no fine again
    assert mc2.count == [3, 2]
    # the pairs carry the first run's fine QoIs and this run's coarse ones
    for i in range(2):
        r = mc2.ledger.have(1, i)
        m = mc2.ledger.have_member(1, i, "f")
        assert r["qf"] == m["q"]["p_max"] and r["seconds"] == 2.0 + 1.0 and r["ok"]
        assert r["qc"] != r["qf"]
    # a third driver finds everything in the ledger and solves nothing
    monkeypatch.setattr(driver, "solve_many", lambda *a, **k: pytest.fail("solved again"))
    mc3 = make(tmp_path, log=lambda *a: None)
    mc3.sample_terms([3, 2])
    assert mc3.q[1]["f"] == mc2.q[1]["f"] and mc3.q[0]["f"] == mc2.q[0]["f"]


def test_plain_mc_comparison_closed_form(tmp_path):
    """eq. (speedup) with the square: M = ceil(var / eps^2) finest solves at
    (steps x FP64 seconds per step) each, against the OF-MLMC cost plus the
    learned level's training."""
    mc = make(tmp_path, log=lambda *a: None)
    mc.q[1] = dict(f=[1.0, 2.0, 3.0, 4.0, 99.0], c=[0.0] * 5, ok=[1, 1, 1, 1, 0])
    mc.count = [0, 5]
    mc.ledger.add([dict(term=1, index=i, qf=0.0, qc=0.0, ok=i < 4, steps_f=100 + 10 * i, steps_c=50,
                        seconds=1.0) for i in range(5)])
    r = driver.plain_mc_comparison(mc, dict(E=-100.0, eps=0.9, tau=1.0, cost_seconds=10.0), 0.01, 0.5,
                                   dict(solve_seconds_charged=4.0, fit_seconds=6.0))
    var = 5.0 / 3.0                                 # sample variance of 1, 2, 3, 4
    assert r["finest_samples"] == 4 and abs(r["var_finest"] - var) < 1e-15
    assert r["eps"] == 1.0 and r["M_mc"] == 2
    assert r["steps_per_sample"] == 115.0 and r["seconds_per_sample"] == 57.5
    assert r["mc_seconds"] == 115.0 and r["speedup"] == 115.0 / 20.0
    assert r["speedup_without_training"] == 11.5 and r["ofmlmc_converged"]
    # a run that stopped above the tolerance is charged the cost of the
    # allocation it ended with (counts x measured cost per sample)
    r = driver.plain_mc_comparison(mc, dict(E=-100.0, eps=2.0, tau=1.0, cost_seconds=10.0, next_counts=[8, 20],
                                            W=[0.5, 2.0]), 0.01, 0.5, dict(solve_seconds_charged=4.0, fit_seconds=6.0))
    assert not r["ofmlmc_converged"] and r["ofmlmc_seconds_spent"] == 10.0
    assert r["ofmlmc_seconds"] == 44.0 and r["speedup"] == 115.0 / 54.0


def test_fit_warmup_takes_one_finest_sample(tmp_path, monkeypatch):
    """eq. (warmup) counts, with a single finest sample when its variances
    are to be inferred (App. A.1) and at least two solver differences lie
    below it; without the fit every term keeps at least two."""
    asked = []

    def fake_solve(ctx, specs, bubbles, max_batch_bytes, log, deadline=None, done=None):
        asked.append(sorted(s.n for s in specs))
        done(list(range(len(specs))), [fake_qoi(s, b) for s, b in zip(specs, bubbles)], [1.0] * len(specs))

    monkeypatch.setattr(driver, "solve_many", fake_solve)
    cfg = solver_config("cloud2d", 16)
    W_model = [1.0, 9.0, 72.0, 576.0]
    for fit, last in ((True, 1), (False, 2)):
        mc = driver.OFMLMC(None, cfg, cloud_spec("cloud2d"), [16, 32, 64, 128], "f32", t_end=1e-4,
                           seed=MASTER_SEED, log=lambda *a: None)
        seen = {}

        def fake_eval(W, classical=False, qoi=None, fit=False, m_floor=2, mc=mc):
            seen["fit"] = fit
            seen["m_floor"] = m_floor
            return dict(E=1.0, eps=0.0, alpha=[1.0] * 4, sigma_t2=[0.0] * 4, M=list(mc.count), fit_flag=0)

        monkeypatch.setattr(mc, "evaluate", fake_eval)
        mc.run(rel_tol=0.01, W_model=W_model, fit=fit)
        # W_L / W_l / 2^(L - l): 576/1/8 = 72, 576/9/4 = 16, 576/72/2 = 4, 1
        assert mc.count == [72, 16, 4, last] and seen["fit"] is fit
        assert seen["m_floor"] == 2
    # with a sample floor above two, the fit keeps the inferred difference
    # variance as a floor of the terms below it: the floor reaches the fit
    mc = driver.OFMLMC(None, cfg, cloud_spec("cloud2d"), [16, 32, 64, 128], "f32", t_end=1e-4,
                       seed=MASTER_SEED, log=lambda *a: None)

    def fake_eval6(W, classical=False, qoi=None, fit=False, m_floor=2, mc=mc):
        seen["m_floor"] = m_floor
        return dict(E=1.0, eps=0.0, alpha=[1.0] * 4, sigma_t2=[0.0] * 4, M=list(mc.count), fit_flag=0)

    monkeypatch.setattr(mc, "evaluate", fake_eval6)
    mc.run(rel_tol=0.01, W_model=W_model, fit=True, min_samples=6)
    assert mc.count == [72, 16, 6, 1] and seen["m_floor"] == 6


def test_term_without_variance_is_not_converged(tmp_path, monkeypatch):
    """A term with fewer than two usable samples has no variance (its moments
    report 0, so its error term would be 0).  Unless the indicator fit filled
    it in, the loop must not stop on that estimate: the error is unknown and
    the term gets samples until it has two."""
    def fake_solve(ctx, specs, bubbles, max_batch_bytes, log, deadline=None, done=None):
        done(list(range(len(specs))), [fake_qoi(s, b) for s, b in zip(specs, bubbles)], [1.0] * len(specs))

    monkeypatch.setattr(driver, "solve_many", fake_solve)
    cfg = solver_config("cloud2d", 16)
    W_model = [1.0, 9.0, 72.0, 576.0]
    for fit_flag in (driver.capi.OFM_ESINGULAR, 0):
        mc = driver.OFMLMC(None, cfg, cloud_spec("cloud2d"), [16, 32, 64, 128], "f32", t_end=1e-4,
                           seed=MASTER_SEED, log=lambda *a: None)
        calls = []

        def fake_eval(W, classical=False, qoi=None, fit=False, m_floor=2, mc=mc, fit_flag=fit_flag):
            calls.append(list(mc.count))
            # every term reports a tiny error: only the missing variance can keep the loop going
            return dict(E=1.0, eps=1e-9, alpha=[1.0] * 4, sigma_t2=[0.0] * 4, M=list(mc.count),
                        fit_flag=fit_flag)

        monkeypatch.setattr(mc, "evaluate", fake_eval)
        monkeypatch.setattr(mc, "allocate", lambda *a, **k: pytest.fail("allocated on an unknown error"))
        out = mc.run(rel_tol=0.01, W_model=W_model, fit=True)
        if fit_flag == 0:
            # the fit completed the single finest sample: converged at once
            assert calls == [[72, 16, 4, 1]] and out["converged"]
        else:
            # the fit failed: not converged on one sample; a second finest
            # sample is asked for, then the estimate stands
            assert calls == [[72, 16, 4, 1], [72, 16, 4, 2]]
            assert out["history"][0]["eps"] == float("inf") and out["history"][0]["unfilled"] == [3]
            assert out["converged"] and mc.count == [72, 16, 4, 2]
    # without the fit a single sample per term cannot be asked for
    mc = driver.OFMLMC(None, cfg, cloud_spec("cloud2d"), [16, 32], "f32", t_end=1e-4, seed=MASTER_SEED,
                       log=lambda *a: None)
    with pytest.raises(ValueError):
        mc.run(rel_tol=0.01, W_model=[1.0, 9.0], min_samples=1)
    with pytest.raises(SystemExit):
        driver.main(["mlmc2d", "--min-samples", "1", "--dir", str(tmp_path)])


def test_failed_samples_count_against_the_two_sample_floor(tmp_path, monkeypatch):
    """Two solves of which one failed leave one usable sample: still no
    variance; the term gets another solve."""
    mc = make(tmp_path, log=lambda *a: None)
    res = dict(M=[5, 1], fit_flag=None)
    assert mc.unfilled_terms(res, fit=False) == [1]
    assert mc.unfilled_terms(dict(M=[5, 1], fit_flag=0), fit=True) == []
    assert mc.unfilled_terms(dict(M=[1, 3], fit_flag=0), fit=True) == [0]     # below the fit's first term


def test_plain_mc_run_times_each_solve_and_resumes(tmp_path, monkeypatch):
    """The capped plain Monte Carlo comparator: independent clouds of their
    own stream, one solve each, every solve timed; the QoIs' mean and sample
    variance over the solves; the comparator's cost model (mean steps x
    seconds per step) beside the measured seconds; a rerun reads the ledger
    and solves only samples it does not hold."""
    import numpy as np
    seen = []

    def fake_solve(ctx, spec, bubbles):
        seen.append([tuple(b) for b in bubbles])
        return fake_qoi(spec, bubbles)

    monkeypatch.setattr(driver.capi, "ofm_solve", fake_solve)
    monkeypatch.setattr(driver, "step_seconds", lambda *a, **k: 1e-3)
    cfg = solver_config("cloud2d", 16)
    cloud = cloud_spec("cloud2d")
    led = str(tmp_path / "mc.jsonl")
    r = driver.plain_mc_run(None, cfg, cloud, 16, "f64", 1e-4, MASTER_SEED, 5, led, log=lambda *a: None)
    assert len(seen) == 5 and r["samples"] == 5 and r["failed"] == 0 and r["steps"] == [16] * 5
    assert r["model_seconds_per_sample"] == pytest.approx(16e-3)
    # every sample is its own cloud, none of them an estimator term's
    assert len(set(map(tuple, seen))) == 5
    term0 = [tuple(b) for b in driver.capi.ofm_sample_cloud(cloud, MASTER_SEED, 0, 0)]
    assert all(s != term0 for s in seen)
    p = np.array([fake_qoi(type("S", (), {"n": 16})(), [list(b) for b in s])["p_max"] for s in seen])
    assert r["p_max"]["mean"] == pytest.approx(p.mean(), rel=1e-15)
    assert r["p_max"]["var"] == pytest.approx(np.var(p, ddof=1), rel=1e-12)
    assert r["measured_step_seconds"] == pytest.approx(sum(r["seconds"]) / 80.0)
    # rerun: nothing solved again; a larger count solves only the new samples
    seen.clear()
    r2 = driver.plain_mc_run(None, cfg, cloud, 16, "f64", 1e-4, MASTER_SEED, 5, led, log=lambda *a: None)
    assert seen == [] and r2["p_max"] == r["p_max"] and r2["seconds"] == r["seconds"]
    r3 = driver.plain_mc_run(None, cfg, cloud, 16, "f64", 1e-4, MASTER_SEED, 7, led, log=lambda *a: None)
    assert len(seen) == 2 and r3["samples"] == 7 and r3["seconds"][:5] == r["seconds"]


def test_plain_mc_run_in_portions(tmp_path, monkeypatch):
    """Large grids advance each solve in portions (a progress line after
    each); the QoIs are the run's at its end."""
    class FakeRun:
        def __init__(self, ctx, specs, bubbles):
            self.spec, self.b, self.k = specs[0], bubbles[0], 0

        def advance(self, max_steps):
            self.k += 1
            return self.k == 3

        def status(self):
            return dict(qoi=[fake_qoi(self.spec, self.b)], steps=self.k * 500)

        def close(self):
            pass

    monkeypatch.setattr(driver.capi, "Run", FakeRun)
    monkeypatch.setattr(driver.capi, "ofm_solve", lambda *a: pytest.fail("not in portions"))
    monkeypatch.setattr(driver, "step_seconds", lambda *a, **k: 1e-3)
    lines = []
    cfg = solver_config("cloud2d", 16)
    r = driver.plain_mc_run(None, cfg, cloud_spec("cloud2d"), 16, "f64", 1e-4, MASTER_SEED, 2,
                            str(tmp_path / "mc.jsonl"), log=lines.append, portion_steps=500)
    assert r["samples"] == 2 and r["steps"] == [16, 16]
    assert sum("500 steps" in x for x in lines) == 2 and sum("1000 steps" in x for x in lines) == 2


def test_plainmc_command_line(tmp_path, monkeypatch):
    """`driver plainmc`: the grid and count from the command line reach the
    run, each grid keeps its own ledger, and the result file is named by the
    grid."""
    seen = {}

    class FakeCtx:
        def __init__(self, device):
            pass

        def close(self):
            pass

    def fake_run(ctx, cfg, cloud, n, precision, T, seed, count, ledger_path, log=print, deadline=None,
                 portion_steps=0):
        seen.update(n=n, count=count, ledger=ledger_path, precision=precision, portion=portion_steps)
        return dict(n=n, samples=count)

    monkeypatch.setattr(driver.capi, "Context", FakeCtx)
    monkeypatch.setattr(driver, "plain_mc_run", fake_run)
    out = driver.main(["plainmc", "--n", "512", "--samples", "3", "--dir", str(tmp_path)])
    assert seen == dict(n=512, count=3, ledger=str(tmp_path / "ledger_plainmc_512.jsonl"), precision="f64",
                        portion=500)
    assert out["plain_mc"] == dict(n=512, samples=3)
    assert json.load(open(tmp_path / "result_plainmc_512.json"))["plain_mc"]["n"] == 512
    driver.main(["plainmc", "--dir", str(tmp_path)])
    assert seen["n"] == 256 and seen["count"] == 16 and seen["portion"] == 0
    assert (tmp_path / "result_plainmc_256.json").exists()
