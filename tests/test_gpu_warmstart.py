"""The learned warm start end to end (not in the paper; Lemma 1 makes any
starting point valid): DROT solves training pairs of grid histograms with the
batched solver, the library's MLP kernels learn the map from the marginals to
the (gauge-fixed, double c-transformed) duals, and DROT warm-started from the
predictions must need fewer iterations than cold DROT on held-out pairs and
reach the same objective.  A 16 x 16 grid keeps the test short; the 32 x 32
experiment is `python -m paper_2110_11738_amd.warmstart`."""
import pytest

pytestmark = pytest.mark.gpu


def test_learned_warm_start_reduces_iterations():
    from paper_2110_11738_amd import warmstart
    rep = warmstart.run(n_train=768, n_test=64, epochs=150, batch=128, lr=1e-3, tol=1e-3,
                        hidden=256, rho0=2.0, side=16, quiet=True)
    print(f"[warm start] cold {rep['cold_iters_mean']:.0f} / warm {rep['warm_iters_mean']:.0f} "
          f"iterations, dual RMSE {rep['test_rmse_duals']:.3e} "
          f"(mean predictor {rep['test_rmse_of_mean_predictor']:.3e})", flush=True)
    assert rep["train_unconverged"] == 0
    assert rep["warm_fallbacks"] == 0
    assert rep["test_rmse_duals"] < 0.5 * rep["test_rmse_of_mean_predictor"]
    assert rep["iteration_ratio_mean"] < 0.9
    # Both runs stop at the 1e-3 relative test: their objectives agree to it.
    assert rep["objective_rel_diff_warm_vs_cold_max"] < 5e-3
