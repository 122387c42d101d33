"""Surrogate training on FMM-made data and serving with the FMM as judge and fallback
(small runs)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained(tmp_path_factory):
    from paper_2006_03515_amd import surrogate_tasks as T
    ck = str(tmp_path_factory.mktemp("sur") / "s.npz")
    rep = T.main(["train", "--n-train", "48", "--n-test", "8", "--epochs", "3", "--batch", "8",
                  "--workers", "1", "--checkpoint", ck])
    return ck, rep


def test_training_improves_on_the_untrained_network(trained):
    ck, rep = trained
    assert rep["held_out_rel_l2"]["mean"] < rep["untrained_rel_l2_mean"]
    assert rep["loss_history"][-1] < rep["loss_history"][0]
    assert rep["params"] > 1_000_000


def test_serving_fallback_branches(trained):
    from paper_2006_03515_amd import surrogate_tasks as T
    ck, _ = trained
    # a zero tolerance forces the FMM fallback on every step, and the served field is then
    # the FMM's (error at the sampled cells = the FMM's own error)
    srv = T.main(["serve", "--checkpoint", ck, "--steps", "6", "--tol", "0", "--check-targets", "256"])
    assert srv["fallback_rate"] == 1.0
    assert srv["served_rel_err_max"] == pytest.approx(srv["fmm_rel_err_max"], rel=1e-12)
    # the judge's own error at sampled cells (which weigh the dim background: 3e-4 measured)
    # stays below the serving tolerance of 1e-3
    assert srv["fmm_rel_err_max"] < 5e-4
    # an infinite tolerance never falls back: the served field is the prediction, whose error
    # against the exact sum is its error against the judge up to the FMM's own error
    srv = T.main(["serve", "--checkpoint", ck, "--steps", "6", "--tol", "1e30", "--check-targets", "256"])
    assert srv["fallback_rate"] == 0.0
    assert srv["served_rel_err_max_prediction"] == pytest.approx(srv["surrogate_rel_err"]["max"], rel=1e-2)


def test_serving_gain_over_the_fmm_alone(trained, record_property):
    # the time-stepped loop at the configured tolerance (1e-3 on 1,024 sampled cells): the
    # served field never misses the tolerance by more than the judge's own error, whichever
    # branch served it, and the gain of the surrogate path over the FMM alone (the same fast
    # configuration) is recorded -- below 1 here: the check alone (an FMM at the sampled
    # leaves) costs about as much as the FMM it guards
    from paper_2006_03515_amd import surrogate_tasks as T
    ck, _ = trained
    srv = T.main(["serve", "--checkpoint", ck, "--steps", "20", "--tol", "1e-3", "--check-targets", "1024"])
    for k in ("fallback_rate", "surrogate_path_steps_per_s", "fmm_only_steps_per_s", "gain_over_fmm_only",
              "served_rel_err_max", "fmm_rel_err_max"):
        record_property(k, srv[k])
    print({k: srv[k] for k in ("fallback_rate", "surrogate_path_steps_per_s", "fmm_only_steps_per_s",
                                "gain_over_fmm_only", "served_rel_err_max")})
    tol = 1e-3
    assert srv["fmm_rel_err_max"] < 5e-4
    if srv["served_rel_err_max_fallback"] is not None:
        assert srv["served_rel_err_max_fallback"] <= srv["fmm_rel_err_max"] * (1 + 1e-9)
    if srv["served_rel_err_max_prediction"] is not None:
        assert srv["served_rel_err_max_prediction"] <= tol + 2 * srv["fmm_rel_err_max"]
    assert 0.0 <= srv["fallback_rate"] <= 1.0
    assert np.isfinite(srv["gain_over_fmm_only"]) and srv["gain_over_fmm_only"] > 0
