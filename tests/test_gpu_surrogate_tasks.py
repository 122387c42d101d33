"""Surrogate training on FMM-made data and serving with FMM fallback (small runs)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_training_improves_on_the_untrained_network(tmp_path):
    from paper_2006_03515_amd import surrogate_tasks as T
    ck = str(tmp_path / "s.npz")
    rep = T.main(["train", "--n-train", "48", "--n-test", "8", "--epochs", "3", "--batch", "8",
                  "--workers", "1", "--checkpoint", ck])
    assert rep["held_out_rel_l2"]["mean"] < rep["untrained_rel_l2_mean"]
    assert rep["loss_history"][-1] < rep["loss_history"][0]
    assert rep["params"] > 1_000_000
    # serving: a zero tolerance forces the FMM fallback on every step, and the served
    # field is then the FMM's (error at the sampled cells = the FMM's own error)
    srv = T.main(["serve", "--checkpoint", ck, "--steps", "6", "--tol", "0", "--check-targets", "256"])
    assert srv["fallback_rate"] == 1.0
    assert srv["served_rel_err_max"] == pytest.approx(srv["fmm_rel_err_max"], rel=1e-12)
    assert srv["fmm_rel_err_max"] < 1e-3
    # an infinite tolerance never falls back: the served field is the surrogate's
    srv = T.main(["serve", "--checkpoint", ck, "--steps", "6", "--tol", "1e30", "--check-targets", "256"])
    assert srv["fallback_rate"] == 0.0
    assert srv["served_rel_err_max"] == pytest.approx(srv["surrogate_rel_err"]["max"], rel=1e-6) or \
        srv["served_rel_err_max"] <= srv["surrogate_rel_err"]["max"] * 1.0001
