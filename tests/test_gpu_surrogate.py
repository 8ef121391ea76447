"""The learned level end to end: trained on the GPU by the library's own
forward/backward/Adam kernels on QoIs the solver produced, then used as the
cheapest level of OF-MLMC.  What it gains over the method without it: the
pair term (solver level, network) with the estimator's coefficient has a
smaller variance than the solver level alone, and the estimate stays that of
the solver level."""
import math
import sys

import numpy as np
import pytest

from workloads.configs import MASTER_SEED, cloud_spec, solver_config, t_end

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_learned_level_reduces_the_pair_variance(tmp_path):
    from paper_1705_04374_amd import capi
    from paper_1705_04374_amd.driver import OFMLMC, load_surrogate, save_surrogate, train_level, variance_reduction
    ctx = capi.Context(0)
    cloud = cloud_spec("cloud2d")
    T = t_end("cloud2d")
    cfg = solver_config("cloud2d", 32)
    say("training set and fit")
    sur, info = train_level(ctx, cloud, cfg, 32, 1024, T, MASTER_SEED, "f32", log=say, epochs=150)
    say("  ", {k: info[k] for k in ("n_train", "epochs", "best_epoch", "val_corr_pmax", "val_loss", "train_loss")})
    assert info["val_corr_pmax"] > 0.5        # validation correlation of the p_max prediction
    # persistence round trip gives the same predictions
    path = str(tmp_path / "net.npz")
    save_surrogate(sur, path)
    again = load_surrogate(ctx, cloud, path, seed=MASTER_SEED)
    probe = [capi.ofm_sample_cloud(cloud, MASTER_SEED, 99, i) for i in range(8)]
    assert np.array_equal(sur.predict(probe), again.predict(probe))
    say("estimator with the learned level")
    mc = OFMLMC(ctx, cfg, cloud, [32], "f32", t_end=T, seed=MASTER_SEED, net=sur, log=say)
    mc.sample_terms([4096, 256])
    r = mc.evaluate(mc.work())
    vr = variance_reduction(r, 1)
    say("  ", vr, "alpha", r["alpha"])
    assert vr["correlation"] > 0.5
    assert vr["factor"] > 1.5
    # the coefficient is the optimal one for the pair: Cov / Var of the
    # network (the term-0 variance enters the alpha system too, with its own
    # tiny cost, so only approximately)
    a_pair = r["cov"][1] / r["var_c"][1]
    assert abs(r["alpha"][0] - a_pair) <= 0.05 * abs(a_pair) + 0.05
    # unbiased: the OF-MLMC estimate agrees with the solver level's own mean
    # on the pair samples within the statistical errors
    q = np.array(mc.q[1]["f"])
    se = math.sqrt(np.var(q, ddof=1) / q.size + r["eps"] ** 2)
    assert abs(r["E"] - q.mean()) <= 4 * se
    ctx.close()
